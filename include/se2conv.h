/*
 * se2conv — convolutional finite Fourier series on Z^2\SE(2) for AMD gfx950.
 *
 * Computes, on the sampling grid Omega_L (paper Sec. 3.2, eq. (OmL)):
 *   x_i = -1/2 + i/Nx, y_j = -1/2 + j/Ny, theta_l = 2 pi l / M   (0-based),
 * the convolutional finite Fourier series (Sec. 5.2, eq. (SKfg); matrix form of
 * Sec. 6.1 with N = L):
 *   S_K[f, rho_1 .. rho_q](w) = sum_k f^[k; L] * prod_j rho_j^[k; L] * phi_k(w),
 * i.e. the real field f convolved on the right with a chain of kernels that are
 * radial in translations (Thm. f*gP: then every convolution is a product of
 * finite Fourier coefficients; Sec. 6.3 for chains and powers).
 *
 * Memory layout of every field: real samples F[b][theta][y][x], x fastest
 * (the order of the paper's F(i, j, l) with i fastest).  All pointers marked
 * "device" are HIP device pointers of the plan's device; the caller owns them.
 * All calls are asynchronous on the given stream; argument errors are detected
 * on the host before anything is enqueued and leave no partial state.
 * Supported sizes: 8 <= Nx, Ny <= 512; 2 <= M <= 512; Nx Ny M < 2^30.  Any
 * length: the paper's odd grids L = 2K+1 (Sec. 3.2) and even grids alike.  The
 * frequency of DFT index t is the signed one, t for t <= (L-1)/2, else t - L (for
 * odd L the paper's set |k| <= K; for even L the reading {-L/2, ..., L/2-1}), and
 * the sign (-1)^{k1+k2} of eq. (FkLv) uses it.  Lengths 2^a 3^b run on radix
 * 16/8/4/3/2 Stockham stages; prime factors 5 and 7 have codelets; a prime
 * length p above 7 runs by Rader's algorithm (a cyclic convolution of length p - 1
 * on the same stages, its kernel spectrum tabulated in FP64 at plan creation); any
 * other prime factor p of a composite length is one direct-summation stage (O(p)
 * work per point).  With odd Nx or Ny every chain runs on the field-pair passes.
 */
#ifndef SE2CONV_H
#define SE2CONV_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SE2CONV_ABI_VERSION 1

typedef struct se2conv_plan_s* se2conv_plan_t;

typedef enum {
    SE2CONV_OK = 0,
    SE2CONV_ERR_INVALID_ARG = 1,      /* null/misaligned pointer, bad index, foreign table, bad flag */
    SE2CONV_ERR_UNSUPPORTED_SIZE = 2, /* grid size outside the supported set */
    SE2CONV_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed inside the plan */
    SE2CONV_ERR_DEVICE = 4,           /* HIP runtime error (launch, no device, host-only plan) */
    SE2CONV_ERR_INTERNAL = 5
} se2conv_status;

typedef enum { SE2CONV_F32 = 0, SE2CONV_F64 = 1 } se2conv_dtype;

/* Omega_L sizes (eq. (OmL)): Nx x Ny spatial points, M angular points. */
typedef struct {
    int32_t nx, ny, m;
} se2conv_shape;

/* ---- plan flags */
#define SE2CONV_PLAN_HOST_ONLY 0x1u /* validation-only plan: no device resources; every
                                       call that would enqueue work returns ERR_DEVICE
                                       after validating its arguments */
#define SE2CONV_PLAN_GENERIC 0x2u   /* use only the general LDS-Stockham pass kernels (no
                                       shape-specialised register kernels); for testing and tuning */

/*
 * se2conv_plan: create a plan for a list of grid shapes and a compute dtype.
 *   shapes[n_shapes]  host array, copied.
 *   dtype             SE2CONV_F32: FP32 butterflies and products with FP64-generated
 *                     twiddles; SE2CONV_F64: FP64 throughout.
 *   out               receives the plan handle (owned by the caller, released with
 *                     se2conv_plan_destroy).
 * The plan allocates twiddle tables (generated in FP64 on the device, eq. (3DFT)
 * roots e^{-2 pi i j/L}), the tables of Rader's algorithm for every prime length
 * above 7 (computed in FP64 on the host and copied), and a workspace of one real
 * plane of the largest shape, on the current HIP device.  Returns ERR_UNSUPPORTED_SIZE for a bad shape,
 * ERR_DEVICE when no device is usable.
 */
se2conv_status se2conv_plan(const se2conv_shape* shapes, int32_t n_shapes, se2conv_dtype dtype, uint32_t flags,
                            se2conv_plan_t* out);

/* Release a plan and its device resources (synchronises the plan's device).  Resource
 * management of this library; it computes nothing of the paper's method. */
se2conv_status se2conv_plan_destroy(se2conv_plan_t plan);

/* ---- kernels rho (radial in translations, Sec. 5.1 footnote to Thm. f*gP) */
typedef enum {
    /* rho(x, theta) = exp(-|x|^2 / (2 sigma^2)) * exp(kappa cos(theta - theta0)),
       periodized over the lattice (eq. (TH)).  Separable: its table is the outer
       product of three 1-D coefficient vectors. */
    SE2CONV_K_GAUSS_VM = 0,
    /* arbitrary kernel samples P[theta][y][x] on Omega_L: device FP64 array `data`.
       The operator is S_K with these coefficients whether or not the kernel is
       radial; only for radial kernels is it the SE(2) convolution. */
    SE2CONV_K_SAMPLES = 1,
    /* radial profile: P[l][j][i] = sum_images sum_q prof[q][l] hat_q(|x_ij + image|),
       hat_q piecewise-linear with knots r_q = q r_max/(n_knots-1); `data` is the
       device FP64 array prof[n_knots][M]; 0 < r_max <= 1. */
    SE2CONV_K_RADIAL_PROFILE = 2,
    /* exponential-coordinates Gaussian (Sec. 6.3, eq. (gbS0)):
       rho(x, R_theta) = exp(-||log(x, R_theta)^v||^2 / (2 sigma^2)) with the principal
       logarithm, ||log^v||^2 = ((theta/2) / sin(theta/2))^2 |x|^2 + theta^2, theta
       wrapped to (-pi, pi]; periodized over the lattice.  Radial in translations, not
       separable: its table is FULL.  Uses `sigma` (> 0). */
    SE2CONV_K_EXP_GAUSS = 3
} se2conv_kernel_kind;

/* normalisation (kernel flags, bits 0..1) */
#define SE2CONV_KNORM_DISCRETE 0u   /* samples scaled so that rho^[0; L] = mean(P) = 1 (default) */
#define SE2CONV_KNORM_CONTINUOUS 1u /* GAUSS_VM only: unit Haar mass (1/2pi) int int rho = 1, eq. (dg) */
#define SE2CONV_KNORM_NONE 2u       /* raw samples */

typedef struct {
    int32_t kind;      /* se2conv_kernel_kind */
    uint32_t flags;    /* SE2CONV_KNORM_* */
    double sigma;      /* GAUSS_VM: translational width (> 0); EXP_GAUSS: width (> 0) */
    double kappa;      /* GAUSS_VM: von Mises concentration (>= 0) */
    double theta0;     /* GAUSS_VM: angular centre */
    const void* data;  /* SAMPLES / RADIAL_PROFILE: device FP64 array (see kind) */
    int32_t n_knots;   /* RADIAL_PROFILE: >= 2 */
    double r_max;      /* RADIAL_PROFILE */
} se2conv_kernel_desc;

/* Table kinds reported by se2conv_table_info. */
#define SE2CONV_TABLE_SEPARABLE 0 /* layout: Tx[Nx] | Ty[Ny] | Tt[M], complex (re, im) of the plan dtype;
                                     rho^[k; L] = Tx[k1] Ty[k2] Tt[k3] */
#define SE2CONV_TABLE_FULL 1      /* layout: T[M][Ny][Nx] complex of the plan dtype, T[k3][k2][k1] = rho^[k; L] */
#define SE2CONV_TABLE_SHIFT 2     /* se2conv_shift_table: J plane sets Q_j[M][Ny][Nx] complex of the plan dtype
                                     (one per distinct roll, in order of first appearance) */
#define SE2CONV_TABLE_QUARTER 3   /* se2conv_table_quarter: T[M][Ny/2+1][Nx/2+1] complex of the plan dtype,
                                     T[k3][|k2|][|k1|] = rho^[k; L] (signed frequencies, integer halves) */

/*
 * se2conv_coeffs: finite Fourier coefficients of a kernel chain (eq. (FkLv)),
 *   rho^[k; L] = prod_j (-1)^{k1+k2} P_j^[k] / norm_j, stored at array index tau(k)
 *   (tau_L(k) = k mod L).
 * Computed in FP64 on the device (samples, DFT, sign, normalisation, chain product)
 * and rounded once to the plan dtype.  All GAUSS_VM chains give a SEPARABLE table;
 * a chain containing SAMPLES or RADIAL_PROFILE gives a FULL table.
 *   kernels[n_kernels]  host array of descriptors (1 <= n_kernels <= 64).
 *   d_table             device buffer of *table_bytes bytes, 16-byte aligned, or NULL to
 *                       query the size into *table_bytes.
 * The plan records the table (its address, shape and kind); se2conv_apply rejects
 * tables it did not produce.  Uses the plan's FP64 scratch (allocated on first use).
 */
se2conv_status se2conv_coeffs(se2conv_plan_t plan, int32_t shape_idx, const se2conv_kernel_desc* kernels,
                              int32_t n_kernels, void* d_table, size_t* table_bytes, hipStream_t stream);

/*
 * se2conv_coeffs_sum: coefficients of a weighted sum of kernels, rho = sum_k w_k rho_k
 * (the paper's outlook of Sec. 1: a general kernel approximated by a sum of radial
 * ones), rho^[k; L] = sum_k w_k rho_k^[k; L] by linearity of eq. (FkLv).  Each term is one
 * kernel descriptor (validated as in se2conv_coeffs, normalised by its own flags); the
 * terms' tables are formed in FP64 on the device, accumulated in FP64 and rounded once.
 * The result is a FULL table (M*Ny*Nx complex of the plan dtype).
 *   kernels[n_terms], weights[n_terms]  host arrays, 1 <= n_terms <= 64, finite weights.
 *   d_table, table_bytes                as in se2conv_coeffs (NULL d_table: size query).
 * Uses the plan's FP64 scratch and an FP64 accumulator of M*Ny*Nx complex values
 * (allocated on first use).
 */
se2conv_status se2conv_coeffs_sum(se2conv_plan_t plan, int32_t shape_idx, const se2conv_kernel_desc* kernels,
                                  const double* weights, int32_t n_terms, void* d_table, size_t* table_bytes,
                                  hipStream_t stream);

/*
 * se2conv_table_quarter: a FULL table folded by the symmetries of a radial kernel.
 * A kernel radial in translations (Sec. 5.1, the footnote to Thm. f*gP) sampled on the
 * lattice of Omega_L is unchanged by x1 -> -x1 and by x2 -> -x2 (the grid is symmetric
 * modulo the period), so its coefficients satisfy rho^[k1, k2, k3] = rho^[-k1, k2, k3] =
 * rho^[k1, -k2, k3]: the table is fixed by its entries at nonnegative signed frequencies
 * 0 <= k1 <= Nx/2, 0 <= k2 <= Ny/2 (every k3), about a quarter of the FULL table.  (On a
 * square grid the diagonal reflection k1 <-> k2 of the same symmetry group holds as well;
 * it is not used for storage, as the y pass would read half of such a table across
 * columns.)  The result is usable wherever a FULL table is (apply, chain, powers, padded,
 * complex, save/backward, shifted sums).
 *   d_full      a FULL table this plan produced for shape_idx's shape.
 *   d_quarter   device buffer of *quarter_bytes bytes (M (Ny/2+1) (Nx/2+1) complex values
 *               of the plan dtype), 16-byte aligned, or NULL to query the size; it must
 *               not overlap d_full.
 * The symmetry is checked on the device: ERR_INVALID_ARG (nothing recorded) when some
 * |T[k] - T[|k1|, |k2|, k3]| exceeds 1e-5 max |T| (FP32 plan) or 1e-12 max |T| (FP64), the
 * rounding level of a table generated in FP64 and rounded once, as for a kernel that is not
 * radial.  Synchronises the stream for that check (not for graph capture).
 */
se2conv_status se2conv_table_quarter(se2conv_plan_t plan, const void* d_full, void* d_quarter, size_t* quarter_bytes,
                                     hipStream_t stream);

/* Kind (SE2CONV_TABLE_*) and byte size of a table produced by this plan. */
se2conv_status se2conv_table_info(se2conv_plan_t plan, const void* d_table, int32_t* kind, int32_t* shape_idx,
                                  size_t* bytes);

/*
 * se2conv_table_release: the plan forgets a table it recorded (se2conv_coeffs,
 * se2conv_coeffs_sum, se2conv_field_coeffs), together with every cached se2conv_chain
 * submission that names it (waiting for that submission's last enqueued use).  Call it
 * before the table's buffer is freed, so that a later buffer at the same address is not
 * taken for this table and the plan's record of tables stays bounded in a training loop.
 * Later calls that pass the address fail with ERR_INVALID_ARG until a table is produced
 * there again.  Host-side bookkeeping: nothing is enqueued.  ERR_INVALID_ARG when the
 * address is not a recorded table of this plan.
 */
se2conv_status se2conv_table_release(se2conv_plan_t plan, const void* d_table);

/*
 * Kernels that are sums of SE(2)-shifts of one kernel radial in translations (the outlook of
 * Sec. 1: a general f2 approximated by sum_k a_k rho_k, the rho_k shifts of one radial rho).
 * A shift acts on the left (group law eq. (SE2law)): rho_k(g) = rho(s_k^{-1} o g) with
 * s_k = (t_k, R_phi_k).  Radiality of rho gives f * rho_k = f_k * rho with
 * f_k(y, alpha) = f(y - R_{alpha - phi_k} t_k, alpha - phi_k): every theta-slice alpha of f
 * translated by R_alpha t_k, the field shifted by phi_k in theta; after that, Thm. f*gP's
 * product of coefficients applies.  On the spatial finite Fourier coefficients of a slice
 * the translation is the phase e^{-2 pi i (k1, k2) . R_alpha t_k} (signed frequencies; for
 * an even length the Nyquist index holds +-L/2 in halves, phase cos(pi L tau)), exact for
 * the trigonometric polynomial.  The rotation phi_k must be a grid angle: phi_k = 2 pi roll / M.
 */
typedef struct {
    double tx, ty;  /* translation t_k (any real values, |t| <= 1e6) */
    double weight;  /* a_k */
    int32_t roll;   /* phi_k = 2 pi roll / M, 0 <= roll < M */
} se2conv_shift;

/*
 * se2conv_shift_table: the translation-phase tables of a shift sum, computed in FP64 on the
 * device and rounded once: for each distinct roll r_j (at most 8),
 *   Q_j[alpha][t2][t1] = sum_{k: roll_k = r_j} a_k e^{-2 pi i (k1, k2) . R_alpha t_k}.
 *   shifts[n_shifts]  host array, 1 <= n_shifts <= 64.
 *   d_table           device buffer of *table_bytes bytes (J * M*Ny*Nx complex of the plan
 *                     dtype), 16-byte aligned, or NULL to query the size.
 * The plan records it as a SE2CONV_TABLE_SHIFT table (usable only with se2conv_apply_shifted).
 */
se2conv_status se2conv_shift_table(se2conv_plan_t plan, int32_t shape_idx, const se2conv_shift* shifts,
                                   int32_t n_shifts, void* d_table, size_t* table_bytes, hipStream_t stream);

/*
 * se2conv_apply_shifted: out[b] = Re S_K[f[b], sum_k a_k rho_k] with the shifts of d_shift_table
 * and rho the chain of kernel_tables (SEPARABLE or FULL tables of this plan and shape; for
 * the result to be the SE(2) convolution rho must be radial in translations):
 *   f^_shift[k] = sum_j DFT_theta( F2[k1, k2, alpha - r_j] Q_j[alpha - r_j][k2][k1] )[k3],
 *   out = Re synthesis of f^_shift . prod rho^   (eq. (SKfg)),
 * F2 the spatial FFCs of the theta-slices.  Five passes on pairs of fields: x and y forward,
 * theta lines (shift mix, forward transform, product, inverse), y and x inverse.
 *   d_f, d_out  device [batch][M][Ny][Nx] of the plan dtype, 16-byte aligned; d_out == d_f allowed.
 * Uses the plan workspace for an odd batch: calls on one plan must not overlap on different
 * streams.  Flags: SE2CONV_TIMING.
 */
se2conv_status se2conv_apply_shifted(se2conv_plan_t plan, int32_t shape_idx, const void* d_f,
                                     const void* d_shift_table, const void* const* kernel_tables,
                                     int32_t n_kernel_tables, void* d_out, int32_t batch, uint32_t flags,
                                     hipStream_t stream);

/* Diagnostics: number of tables the plan records and of cached se2conv_chain submissions. */
se2conv_status se2conv_plan_counts(se2conv_plan_t plan, int64_t* n_tables, int64_t* n_submissions);

/*
 * se2conv_field_coeffs: finite Fourier coefficient tables f^[k; L] = (-1)^{k1+k2} F^[k] / n
 * (eq. (FkLv)) of real fields, in the plan dtype, one FULL table per field.  They serve as
 * the checkpointed forward spectra of a field: the gradient of a loss with respect to the
 * kernel samples is the adjoint apply of dL/dout with this table (dL/dP = Re S_K[g, conj f^]).
 *   d_f         device [batch][M][Ny][Nx] real samples (plan dtype).
 *   d_tables    device buffer; table b starts at d_tables + b * table_stride (bytes), each
 *               M*Ny*Nx complex values; table_stride >= that size and a multiple of 16.
 * Every table is recorded by the plan (usable with se2conv_apply / se2conv_chain).
 * Uses two workspace planes of the largest shape (allocated on first use).
 */
se2conv_status se2conv_field_coeffs(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, int32_t batch,
                                    void* d_tables, size_t table_stride, hipStream_t stream);

/*
 * se2conv_kernel_grad: gradient of a loss with respect to the samples P of one kernel,
 * summed over a batch: for out_b = Re S_K[f_b, rho] and g_b = dL/dout_b,
 *   dP = sum_b Re S_K[g_b, conj f_b^] = Re iDFT( sum_b G_b^ . conj(f_b^) ),
 * accumulated in the spectral domain (two g fields per complex FFT, separated by Hermitian
 * symmetry) and inverted once.
 *   d_g           device [batch][M][Ny][Nx] (plan dtype).
 *   d_ftables     the fields' FFC tables from se2conv_field_coeffs (table b at
 *                 d_ftables + b * table_stride); for a kernel chain pass tables that already
 *                 include the other kernels' coefficients.
 *   d_grad        device [M][Ny][Nx] (plan dtype), overwritten.
 * Uses four workspace planes of the largest shape (allocated on first use).
 */
se2conv_status se2conv_kernel_grad(se2conv_plan_t plan, int32_t shape_idx, const void* d_g, const void* d_ftables,
                                   size_t table_stride, int32_t batch, void* d_grad, hipStream_t stream);

/*
 * se2conv_profile_grad: transpose of the RADIAL_PROFILE sample expansion, summed over a
 * batch: grad_prof[q][l] = sum_b sum_{j,i} H_q(x_ij) dP_b[l][j][i], where
 * H_q(x) = sum_images max(0, 1 - | |x + image| / h - q |), h = r_max / (n_knots - 1).
 *   d_grad_samples  device [batch][M][Ny][Nx] gradients w.r.t. kernel samples (plan dtype).
 *   d_grad_prof     device FP64 [n_knots][M], overwritten.
 * Computed in FP64 with fixed-order reductions (bitwise reproducible).  Uses the plan's
 * FP64 scratch.
 */
se2conv_status se2conv_profile_grad(se2conv_plan_t plan, int32_t shape_idx, const void* d_grad_samples,
                                    int32_t batch, int32_t n_knots, double r_max, double* d_grad_prof,
                                    hipStream_t stream);

/* ---- apply flags */
#define SE2CONV_ADJOINT 0x1u /* apply the transpose (conjugate coefficients: correlation with the kernels) */
#define SE2CONV_GRAPH 0x2u   /* se2conv_chain only: capture the submission once in a HIP graph and replay it */
#define SE2CONV_TIMING 0x4u  /* record a HIP event on the stream before the first and after every pass
                                launch; read the per-pass durations with se2conv_pass_times */

/*
 * se2conv_apply: out[b] = Re S_K[f[b], chain] for b = 0 .. batch-1.
 *   d_f, d_out  device arrays [batch][M][Ny][Nx] of the plan dtype, 16-byte aligned;
 *               d_out == d_f (in place) is allowed, other overlaps are not.
 *   d_table     a table produced for this plan and shape (se2conv_coeffs,
 *               se2conv_coeffs_sum or se2conv_field_coeffs).
 * Separable tables run two passes (x-theta slabs, then y pencils) when a slab fits
 * in LDS, three otherwise; full tables run forward / product / inverse passes on
 * pairs of fields.  Uses the plan workspace when batch is odd and the table is
 * FULL: calls on one plan must not overlap on different streams.  The environment
 * variable SE2CONV_SEP_CHUNK = k splits the separable two-pass schedule into launches
 * of k fields (tuning only; the default is the whole batch).
 */
se2conv_status se2conv_apply(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, const void* d_table,
                             void* d_out, int32_t batch, uint32_t flags, hipStream_t stream);

/*
 * se2conv_apply_complex: out[b] = S_K[f[b], chain] for complex-valued fields
 * f: SE(2) -> C (the paper's setting, Sec. 3.2).  Every kernel kind is real in space,
 * so S_K[a + i b] = S_K[a] + i S_K[b]: the real and imaginary parts of one field are
 * the two planes of one pair of the full-table passes, read and written interleaved.
 *   d_f, d_out  device arrays [batch][M][Ny][Nx] of complex values (re, im adjacent;
 *               complex64 for F32 plans, complex128 for F64), 16-byte aligned;
 *               d_out == d_f (in place) is allowed, other overlaps are not.
 *   d_table     a table produced for this plan and shape (as for se2conv_apply).
 * Runs on the generic passes (every size).  Flags: SE2CONV_ADJOINT, SE2CONV_TIMING.
 */
se2conv_status se2conv_apply_complex(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, const void* d_table,
                                     void* d_out, int32_t batch, uint32_t flags, hipStream_t stream);

/*
 * se2conv_apply_padded: out[b] = Re S_K[f[b], chain] evaluated on a finer grid
 * (paper Sec. 4.1 eq. (MatSKfonG), Sec. 6.1 eq. (MatSKfgonG), Prop. LtoN1D: the
 * iDFT of the zero-padded product spectrum).
 *   shape_idx       the sampling grid L of d_f and d_table.
 *   out_shape_idx   another shape of the same plan, the evaluation grid N, with
 *                   N >= L on every axis (N = L gives se2conv_apply's result).
 *   d_f             device [batch][Lm][Ly][Lx], d_out device [batch][Nm][Ny][Nx], plan
 *                   dtype, 16-byte aligned, not overlapping.
 * Every coefficient keeps its signed frequency k (|k| <= K for odd L = 2K+1); the
 * rest of the N-spectrum is zero.  For even L (a reading: the paper states odd L)
 * the index L/2 carries +-L/2 together and is split in halves between the two on a
 * finer grid, so real fields give real values.  Runs on the field-pair passes, one
 * pair at a time, with the plan workspace: calls on one plan must not overlap on
 * different streams.  Flags: SE2CONV_ADJOINT, SE2CONV_TIMING.
 */
se2conv_status se2conv_apply_padded(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, const void* d_table,
                                    int32_t out_shape_idx, void* d_out, int32_t batch, uint32_t flags,
                                    hipStream_t stream);

/*
 * Fused differentiation (FP32 plans on shapes with register kernels, see
 * se2conv_fused_supported; other plans use se2conv_field_coeffs + se2conv_kernel_grad).
 *
 * Field spectra: the 3-D DFT (eq. (3DFT), no sign factor, no 1/n) of the batch's fields
 * taken two at a time as z_p = f_{2p} + i f_{2p+1}: plane 2p holds Re Z_p and plane 2p+1
 * holds Im Z_p, each [M][Ny][Nx] FP32 in frequency order [k3][k2][k1].  With an odd batch
 * the last field is paired with zero.  A buffer of spectra is 2 * ceil(batch / 2) planes.
 *
 * The kernel-sample gradient of a loss over the batch follows from eqs. (FkLv), (SKfg):
 * for out_b = S_K[f_b, rho] with rho^ = (-1)^{k1+k2} P^ / n and g_b = dL/dout_b,
 *   dL/dP = sum_b (1/n^2) iDFT( (-1)^{k1+k2} G_b^ conj(F_b^) )   (unnormalised iDFT)
 *         = (1/n^2) Re iDFT( (-1)^{k1+k2} sum_p Z_{g,p} conj(Z_{f,p}) ),
 * the pair form following from the Hermitian symmetry of real fields' spectra.
 */

/* Nonzero when the fused entry points below support this plan and shape. */
int32_t se2conv_fused_supported(se2conv_plan_t plan, int32_t shape_idx);

/*
 * se2conv_field_spectra: field spectra of d_f (device [batch][M][Ny][Nx] FP32) into
 * d_spectra (device, 2 * ceil(batch / 2) planes, caller-owned).
 */
se2conv_status se2conv_field_spectra(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, int32_t batch,
                                     void* d_spectra, hipStream_t stream);

/*
 * se2conv_apply_save: se2conv_apply (forward, one table) that also writes the field
 * spectra of d_f to d_spectra (the checkpoint of the backward pass) from inside its y
 * pass.  d_out == d_f is allowed; d_spectra must not overlap either.
 */
se2conv_status se2conv_apply_save(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, const void* d_table,
                                  void* d_out, int32_t batch, void* d_spectra, hipStream_t stream);

/*
 * se2conv_backward: both gradients of a loss through out = S_K[f, rho] (one table):
 *   d_grad_f  device [batch][M][Ny][Nx]: dL/df_b = S_K[g_b, conj rho] (the adjoint apply);
 *   d_grad_p  device [M][Ny][Nx]: dL/dP summed over the batch, P the samples of the kernel
 *             whose FFC table is d_table;
 * from d_g = dL/dout (device [batch][M][Ny][Nx]) and the field spectra d_spectra of the
 * forward's fields.  Four passes: x-theta forward of g, one y pass (adjoint product and
 * gradient accumulation), x-theta inverses of both results.  d_grad_f may equal d_g.
 * Uses three workspace planes of the largest shape (allocated on first use).
 */
se2conv_status se2conv_backward(se2conv_plan_t plan, int32_t shape_idx, const void* d_g, const void* d_table,
                                const void* d_spectra, int32_t batch, void* d_grad_f, void* d_grad_p,
                                hipStream_t stream);

/* One problem of a heterogeneous submission: out = Re S_K[f, tables[0] * ... ], the chain form
 * f * rho_1 * ... * rho_q of Sec. 6.3 (Algorithm 4, eq. (MatSqKfgG) with distinct kernels: the
 * coefficients of the kernels multiply, Thm. f*gP (2)). */
typedef struct {
    int32_t shape_idx;
    int32_t batch;
    const void* f;              /* device [batch][M][Ny][Nx] */
    void* out;                  /* device, same shape (may equal f) */
    const void* const* tables;  /* host array of n_tables device tables of this plan/shape */
    int32_t n_tables;           /* 1 .. 8; coefficients multiplied in the plan dtype */
} se2conv_problem;

/*
 * se2conv_chain: run n_probs problems (different shapes and kernel chains allowed),
 * ordered after earlier work on the stream; the call's work is complete when the stream
 * reaches the point after it.  Problems whose tables are all SEPARABLE are grouped by
 * shape.  On FP32 plans, when every class has the multi-class register kernels (N in 32,
 * 48, 64, 96, 128, 256 with M 16, 32, 64), the classes of 2^k points take one launch per
 * pass and those of 3 * 2^k another, the second kind on one of the plan's auxiliary
 * streams (forked from and joined back into `stream`; on `stream` alone with
 * SE2CONV_TIMING).  Otherwise each class takes one launch per pass, the classes one after
 * another on `stream` (the environment variable SE2CONV_CHAIN_STREAMS = 2..4 forks them
 * over that many auxiliary streams; not with SE2CONV_TIMING).  Problems with FULL tables
 * follow one at a time.  A problem's output
 * must not overlap another problem's input or output.  With SE2CONV_GRAPH the
 * submission (forks included) is captured into a HIP graph on first use and replayed
 * on later calls with the same problem list (same pointers, sizes and table kinds).
 * SE2CONV_ADJOINT applies to every problem.  The plan caches up to 64 problem lists (their
 * device item arrays and graphs); the oldest is dropped first, after its last enqueued
 * use has finished on whatever stream it went to.  A list enqueued on a stream that the
 * caller is capturing stays cached until the plan is destroyed or one of its tables is
 * released, since the caller's graph refers to its item array.  Calls may come from
 * several threads and streams.
 */
se2conv_status se2conv_chain(se2conv_plan_t plan, const se2conv_problem* probs, int32_t n_probs, uint32_t flags,
                             hipStream_t stream);

/*
 * se2conv_chain_noalloc: se2conv_chain for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same result as se2conv_chain on the same problems (the same pass kernels), but the
 * per-field item lists (input, output, table chain) go into a fixed device array of the
 * library instead of a cached allocation: no hipMalloc, hipFree or allocating library
 * call, no graph, nothing cached.  The items are written by small kernels that carry them
 * in their arguments, then each shape class runs its passes on them, all on `stream`.
 *   probs[n_probs]  as for se2conv_chain, restricted to problems whose tables are all
 *                   SEPARABLE on shapes with even Nx and Ny (others: ERR_INVALID_ARG).
 *   flags           0 or SE2CONV_ADJOINT.
 * Limit: at most 4096 fields (the sum of the problems' batches) per call; more gives
 * ERR_INVALID_ARG and enqueues nothing.  The array (4096 items, about 360 KB) is held by
 * every device the library runs on until the process ends; its address is looked up at
 * plan creation with that device current, and the plan's device must be current here.
 * Every call on one device shares that array and overwrites it: calls that overlap on
 * one device (different streams, or threads without ordering) race and must not be
 * issued; calls ordered on one stream are safe.
 */
se2conv_status se2conv_chain_noalloc(se2conv_plan_t plan, const se2conv_problem* probs, int32_t n_probs,
                                     uint32_t flags, hipStream_t stream);

/*
 * se2conv_pass_times: durations of the passes enqueued with SE2CONV_TIMING since the
 * last read, in launch order.  Synchronises on the last recorded event.
 *   ms[cap], kinds[cap]   host arrays; kinds: 0 = x-theta slab pass, 1 = y pencil,
 *                         2 = theta pencil, 3 = x-row pass.
 *   n                     receives the number of passes recorded (may exceed cap;
 *                         only the first cap are written).  The record is cleared.
 */
se2conv_status se2conv_pass_times(se2conv_plan_t plan, float* ms, int32_t* kinds, int32_t cap, int32_t* n);

/*
 * se2conv_autotune: choose the launch schedule of one shape by timing candidates on
 * synthetic data (batch fields, one Gaussian x von Mises kernel): generic pencil tile width
 * (4..32 columns), blocks per CU of the persistent fast pencil (2, 4, 8) and x-row tile size
 * of the three-pass schedule.  The fastest schedule is kept in the plan and, when the
 * environment variable SE2CONV_TUNE_CACHE names a file, appended to it as a JSON line; plans
 * created later load that file (malformed lines are ignored).  Allocates and frees its own
 * buffers; synchronises the stream.
 */
se2conv_status se2conv_autotune(se2conv_plan_t plan, int32_t shape_idx, int32_t batch, hipStream_t stream);

/*
 * se2conv_sample_bumps: samples on Omega_L (eq. (OmL)) of a field made of Gaussian x von
 * Mises bumps periodized over the lattice (eq. (TH)):
 *   f(x, y, theta) = sum_b w_b G(x - cx_b) G(y - cy_b) exp(kappa cos(theta - theta0_b)),
 *   G(u) = sum_{l=-3..3} exp(-(u + l)^2 / (2 s^2)),
 * evaluated in FP64 and rounded to the plan dtype.
 *   d_params  device FP64 [n_bumps][4] = (cx, cy, theta0, w).
 *   d_out     device [M][Ny][Nx] (one field).
 * For s <= 0.1 the omitted images are below 1e-21 of the peak.  Uses the plan's FP64 scratch.
 */
se2conv_status se2conv_sample_bumps(se2conv_plan_t plan, int32_t shape_idx, const double* d_params,
                                    int32_t n_bumps, double s, double kappa, void* d_out, hipStream_t stream);

/*
 * se2conv_powers: every intermediate convolution of Algorithm 7 (Sec. 6.3),
 *   out[p-1][b] = Re S_K[f_b, rho^(p)],  p = 1 .. q,
 * with rho^(p) the p-fold self-convolution of the kernel chain in d_table (coefficients
 * rho^[k]^p; Thm. f*gP(2) and eq. (SqKfg)).  One forward 3-D transform of f, then for each p
 * a running Hadamard product H_p = H_{p-1} . rho^ and one inverse transform, as the paper's
 * fast loop does.
 *   d_out   device [q][batch][M][Ny][Nx] of the plan dtype (must not overlap d_f); the last
 *           slot holds the running spectrum until the final step.
 *   q       1 .. 4096.  flags: SE2CONV_ADJOINT conjugates the table.
 * Uses the plan workspace (and two more planes for odd batches).
 */
se2conv_status se2conv_powers(se2conv_plan_t plan, int32_t shape_idx, const void* d_f, const void* d_table,
                              int32_t q, void* d_out, int32_t batch, uint32_t flags, hipStream_t stream);

/* Static description of a status code (error reporting of this library; no passage of the paper). */
const char* se2conv_status_string(se2conv_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* se2conv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SE2CONV_H */
