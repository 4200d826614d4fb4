// Host side of the se2conv C ABI: plans, argument validation, table registry,
// pass scheduling and HIP-graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <set>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/se2conv.h"
#include "coeffs.hpp"
#include "passes.hpp"
#include "sep_fast.hpp"
#include "full_fast.hpp"
#include "grad.hpp"
#include "sample.hpp"
#include "shift.hpp"
#include "sep_fast64.hpp"

using namespace se2c;

namespace {

thread_local std::string g_last_error;

se2conv_status fail(se2conv_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

se2conv_status ok() {
    g_last_error.clear();
    return SE2CONV_OK;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(SE2CONV_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool shape_supported(const se2conv_shape& s, std::string* why) {
    if (s.nx < 8 || s.nx > 512 || s.ny < 8 || s.ny > 512) {
        *why = "Nx and Ny must lie in [8, 512]";
        return false;
    }
    if ((long long)s.nx * s.ny * s.m >= (1LL << 30)) {
        *why = "Nx * Ny * M must be below 2^30 points per field";
        return false;
    }
    if (s.m < 2 || s.m > 512) {
        *why = "M must lie in [2, 512]";
        return false;
    }
    return true;
}

// Even Nx and Ny allow the pair packings of the separable passes (two rows or two
// columns of one field as one complex line); other shapes run every chain on the
// field-pair (plane) passes.
bool pair_layout(const se2conv_shape& s) { return !(s.nx & 1) && !(s.ny & 1); }

bool is_prime(int n) {
    if (n < 2) return false;
    for (int f = 2; f * f <= n; ++f)
        if (n % f == 0) return false;
    return true;
}

// Stockham radices of one length: 16/8/4/2 for the power of two, codelets 3, 5, 7,
// and direct-summation stages for any other prime factor; largest radices first
// (the first stage needs no twiddles).  A prime length above 7 runs by Rader's
// algorithm on the stages of L - 1 (its tables are attached by radix_plan_of).
RadixPlan make_radix_plan(int L) {
    RadixPlan p{};
    p.L = L;
    p.nst = 0;
    p.rader = (L > 7 && is_prime(L)) ? 1 : 0;
    p.rtab = nullptr;
    int n = p.rader ? L - 1 : L, p2 = 1;
    while (n % 2 == 0) {
        n /= 2;
        p2 *= 2;
    }
    while (p2 >= 16) {
        p.r[p.nst++] = 16;
        p2 /= 16;
    }
    if (p2 > 1) p.r[p.nst++] = p2;
    for (int f = 3; f * f <= n || n > 1; f += 2) {
        if (f * f > n) f = n;  // the rest is prime
        while (n % f == 0) {
            p.r[p.nst++] = f;
            n /= f;
        }
    }
    std::sort(p.r, p.r + p.nst, [](int a, int b) { return a > b; });
    return p;
}

constexpr size_t kMaxLds = 160 * 1024;

// A length with a prime factor above 3 runs on the kernels with the radix-5/7 and
// direct stages, which are limited to 512 threads per workgroup (as FP64 is).
bool odd_len(int L) {
    while (L % 2 == 0) L /= 2;
    while (L % 3 == 0) L /= 3;
    return L != 1;
}

int max_threads(bool d, bool odd = false) { return (d || odd) ? 512 : 1024; }

// Complex values per thread per stage of the generic kernels.
int maxv(bool d, bool odd) { return odd ? SE2C_MAXV_ODD : (d ? SE2C_MAXV_F64 : SE2C_MAXV); }

// Points one generic tile can hold.
long long tile_capacity(bool d, bool odd) { return (long long)maxv(d, odd) * max_threads(d, odd); }

int threads_for(long long P, bool d, bool odd) {
    long long t = (P + maxv(d, odd) - 1) / maxv(d, odd);
    t = ((t + 63) / 64) * 64;
    if (t < 64) t = 64;
    if (t > max_threads(d, odd)) t = max_threads(d, odd);
    return (int)t;
}

// Tunable launch parameters of one shape (se2conv_autotune picks them by timing).
struct Schedule {
    int pencil_w = 16;          // generic pencils: columns per tile (clamped to the LDS/thread limits)
    int fast_blocks_per_cu = 8; // persistent register pencils (capped by occupancy)
    int xrow_points = 4096;     // three-pass schedule: points per x-row tile
    bool tuned = false;
};

// Untuned defaults per dtype (the autotuner's usual picks on MI355X: narrower generic
// pencils and longer x-row tiles for FP64).
Schedule default_schedule(bool d) {
    Schedule s;
    if (d) {
        s.pencil_w = 8;
        s.xrow_points = 8192;
    }
    return s;
}

struct TableRec {
    int32_t shape_idx;
    int32_t kind;
    size_t bytes;
    std::vector<int> rolls;  // SE2CONV_TABLE_SHIFT: theta roll of each plane set
};

// A problem list seen by se2conv_chain: its device item arrays (one group of
// fields per shape with separable chains) and, with SE2CONV_GRAPH, its graph.
// Records are shared: a call keeps its own reference while it enqueues work, so
// an eviction by another thread cannot free a record in use.  The device resources
// are released by the destructor, after the last enqueued use has finished.
struct SubmissionRec {
    std::vector<uint64_t> key;
    uint64_t key_hash = 0;                         // FNV-1a of key, compared first
    std::vector<uintptr_t> tabs;                   // every table address the list names
    void* d_items = nullptr;                       // all groups' SepItem arrays
    std::vector<std::pair<int, int>> groups;       // (shape_idx, first item) per group
    std::vector<int> group_counts;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // recorded after every enqueue of the record's work (eager or graph launch) on the
    // stream it went to; waited on before the record's device resources are freed
    hipEvent_t done = nullptr;
    bool used = false;       // done has been recorded at least once
    // enqueued on a stream under someone else's capture: the captured graph refers to
    // d_items for as long as that graph lives, so the record is never evicted
    bool pinned = false;
    SubmissionRec() = default;
    SubmissionRec(const SubmissionRec&) = delete;
    SubmissionRec& operator=(const SubmissionRec&) = delete;
    ~SubmissionRec() {
        if (done && used) (void)hipEventSynchronize(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_items) (void)hipFree(d_items);
        if (done) (void)hipEventDestroy(done);
    }
};

// Device scratch of se2conv_chain_noalloc: the per-field item lists (input, output,
// table chain) of one call, written by fill_items_kernel from kernel arguments.  Every
// device the library runs on holds one copy until the process ends.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returned for the current device (noalloc_scratch_of).
constexpr int kNoAllocMaxItems = 4096;
static __device__ __align__(256) SepItem scratch[kNoAllocMaxItems];

std::mutex g_scratch_mu;
std::map<int, SepItem*> g_scratch_ptr;  // device -> address of that device's copy

// Looks up the scratch's device address once per device, with that device current.
se2conv_status noalloc_scratch_setup(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return SE2CONV_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(SE2CONV_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                    hipGetErrorString(e));
    g_scratch_ptr[device] = reinterpret_cast<SepItem*>(ptr);
    return SE2CONV_OK;
}

SepItem* noalloc_scratch_of(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// Up to kFillBatch items travel by value in the kernel arguments (no host buffer, no
// copy engine) and are stored at dst[first .. first + n).
constexpr int kFillBatch = 32;
struct ItemBatch {
    SepItem it[kFillBatch];
    int first;
    int n;
};
static_assert(sizeof(ItemBatch) <= 4000, "kernel argument size");

__global__ void fill_items_kernel(SepItem* dst, ItemBatch b) {
    const int i = threadIdx.x;
    if (i < b.n) dst[b.first + i] = b.it[i];
}

}  // namespace

struct se2conv_plan_s {
    int device = -1;
    int num_cus = 256;
    se2conv_dtype dtype = SE2CONV_F32;
    uint32_t flags = 0;
    bool host_only = false;
    std::vector<se2conv_shape> shapes;
    std::vector<Schedule> sched;       // one per shape
    std::map<int, void*> tw32, tw64;   // length -> device twiddle table
    std::map<int, void*> rader32, rader64;  // prime length > 7 -> device Rader tables
    void* ws = nullptr;                // one real plane of the largest shape (plan dtype)
    size_t ws_bytes = 0;
    void* ws2 = nullptr;               // two more planes (field tables), allocated on first use
    void* ws4 = nullptr;               // four more planes (kernel gradient), allocated on first use
    void* scratch64 = nullptr;         // FP64 scratch for se2conv_coeffs
    size_t scratch64_bytes = 0;
    void* qstat = nullptr;             // two u64 of se2conv_table_quarter's symmetry check, on first use
    void* sum64 = nullptr;             // FP64 accumulator of se2conv_coeffs_sum, allocated on first use
    size_t sum64_bytes = 0;
    void* pad_ws = nullptr;            // sampling-grid product spectra of se2conv_apply_padded
    size_t pad_ws_bytes = 0;
    // hat basis of the last radial-profile geometry used by se2conv_profile_grad
    double* basis = nullptr;
    size_t basis_bytes = 0;
    int basis_shape = -1, basis_knots = 0;
    double basis_rmax = 0.0;
    // its real 2-D DFT on the quadrant k1 <= Nx/2, k2 <= Ny/2 (radial-profile tables in
    // se2conv_coeffs), same geometry key
    double* basis_hat = nullptr;
    size_t basis_hat_bytes = 0;
    int bh_shape = -1, bh_knots = 0;
    double bh_rmax = 0.0;
    std::unordered_map<uintptr_t, TableRec> tables;
    std::list<std::shared_ptr<SubmissionRec>> subs;  // se2conv_chain's cache, oldest first
    // concurrent shape classes in se2conv_chain: auxiliary streams (default priority)
    // and the fork / join events around them, created on first use
    std::vector<hipStream_t> aux;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    std::mutex mu;
    std::mutex fork_mu;  // one fork / join on the auxiliary streams at a time
    // pass timing (SE2CONV_TIMING)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<hipEvent_t> ev_rec;   // recorded events in order
    std::vector<int> ev_kind;         // kind of each timed pass, in order
    std::set<size_t> ev_sub_start;    // indices in ev_rec that open a new submission
};

namespace {

bool dbl(const se2conv_plan_s* p) { return p->dtype == SE2CONV_F64; }
size_t real_bytes(const se2conv_plan_s* p) { return dbl(p) ? 8 : 4; }
size_t cplx_bytes(const se2conv_plan_s* p) { return dbl(p) ? 16 : 8; }

// Drops the cached chain submissions whose problem list names a table address: the
// address is being registered again (possibly as a table of the other kind) or
// released, so the cached grouping of that list may no longer hold.  A record still
// in use by another call stays alive through that call's reference.  Caller holds p->mu.
void purge_subs_naming(se2conv_plan_s* p, uintptr_t addr) {
    for (auto it = p->subs.begin(); it != p->subs.end();) {
        const std::vector<uintptr_t>& t = (*it)->tabs;
        if (std::find(t.begin(), t.end(), addr) != t.end())
            it = p->subs.erase(it);
        else
            ++it;
    }
}

// Records a table produced by the plan (caller holds p->mu).
void register_table(se2conv_plan_s* p, const void* addr, const TableRec& rec) {
    purge_subs_naming(p, reinterpret_cast<uintptr_t>(addr));
    p->tables[reinterpret_cast<uintptr_t>(addr)] = rec;
}

const void* tw_of(se2conv_plan_s* p, int L, bool use64) { return use64 ? p->tw64.at(L) : p->tw32.at(L); }

// Radix plan of one axis for the generic passes, with its Rader tables attached.
RadixPlan radix_plan_of(se2conv_plan_s* p, int L, bool use64) {
    RadixPlan r = make_radix_plan(L);
    if (r.rader) r.rtab = use64 ? p->rader64.at(L) : p->rader32.at(L);
    return r;
}

// The twiddle table the plan's stages read: w_L, or w_{L-1} (first block of the
// Rader tables) for a prime length.
const void* stage_tw_of(se2conv_plan_s* p, const RadixPlan& r, bool use64) {
    return r.rader ? r.rtab : tw_of(p, r.L, use64);
}

// Rader tables of a prime length L (see RadixPlan), computed in FP64 on the host and
// stored in FP64 and rounded to FP32: twiddles w_{L-1}^j, the spectra
// B[k] = (1/(L-1)) sum_j w_L^{+-g^-j} w_{L-1}^{jk} for the forward (-) and inverse (+)
// transforms, and the index maps g^q, g^-q mod L for the smallest generator g.
// Angles come from exactly reduced integer products.
void rader_tables(int L, std::vector<unsigned char>& b64, std::vector<unsigned char>& b32) {
    const int n = L - 1;
    std::vector<int> fac;
    for (int f = 2, m = n; m > 1; ++f)
        if (m % f == 0) {
            fac.push_back(f);
            while (m % f == 0) m /= f;
        }
    auto powmod = [L](long long a, long long e) {
        long long r = 1;
        a %= L;
        for (; e > 0; e >>= 1, a = a * a % L)
            if (e & 1) r = r * a % L;
        return r;
    };
    int g = 2;
    for (;; ++g) {
        bool gen = true;
        for (int f : fac) gen = gen && powmod(g, n / f) != 1;
        if (gen) break;
    }
    const long long ginv = powmod(g, L - 2);
    std::vector<int> pin(n), pout(n);
    for (int q = 0; q < n; ++q) {
        pin[q] = (int)powmod(g, q);
        pout[q] = (int)powmod(ginv, q);
    }
    const double two_pi = 6.283185307179586476925286766559;
    // w_N^r = exp(-2 pi i r / N), exact at the quarter turns
    auto w = [&](long long r, long long N, double& c, double& sn) {
        r %= N;
        if ((4 * r) % N == 0) {
            const int q = (int)((4 * r) / N) & 3;
            c = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
            sn = q == 1 ? -1.0 : (q == 3 ? 1.0 : 0.0);
            return;
        }
        const double a = two_pi * (double)r / (double)N;
        c = std::cos(a);
        sn = -std::sin(a);
    };
    std::vector<double> tab(2 * 3 * (size_t)n), bre(n), bim(n);
    for (int j = 0; j < n; ++j) {
        w(j, n, tab[2 * j], tab[2 * j + 1]);
        w(pout[j], L, bre[j], bim[j]);
    }
    for (int dir = 0; dir < 2; ++dir) {
        for (int k = 0; k < n; ++k) {
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < n; ++j) {
                const double bc = bre[j], bs = dir == 1 ? -bim[j] : bim[j];
                const size_t r = (size_t)(((long long)j * k) % n);
                const double tc = tab[2 * r], ts = tab[2 * r + 1];
                sr += bc * tc - bs * ts;
                si += bc * ts + bs * tc;
            }
            tab[2 * ((size_t)(1 + dir) * n + k)] = sr / n;
            tab[2 * ((size_t)(1 + dir) * n + k) + 1] = si / n;
        }
    }
    const size_t ib = sizeof(int) * 2 * (size_t)n;
    b64.assign(sizeof(double) * tab.size() + ib, 0);
    b32.assign(sizeof(float) * tab.size() + ib, 0);
    std::memcpy(b64.data(), tab.data(), sizeof(double) * tab.size());
    std::vector<float> t32(tab.begin(), tab.end());
    std::memcpy(b32.data(), t32.data(), sizeof(float) * t32.size());
    for (auto* b : {&b64, &b32}) {
        unsigned char* ip = b->data() + (b->size() - ib);
        std::memcpy(ip, pin.data(), sizeof(int) * n);
        std::memcpy(ip + sizeof(int) * n, pout.data(), sizeof(int) * n);
    }
}

bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0; }

// Current plan for pass timing (set by the entry points while they enqueue).
thread_local se2conv_plan_s* g_timing_plan = nullptr;

hipError_t record_event(se2conv_plan_s* p, hipStream_t st, bool submission_start = false) {
    hipEvent_t ev;
    if (submission_start && !p->ev_rec.empty()) p->ev_sub_start.insert(p->ev_rec.size());
    if (!p->ev_pool.empty()) {
        ev = p->ev_pool.back();
        p->ev_pool.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
    }
    p->ev_rec.push_back(ev);
    return hipEventRecord(ev, st);
}

hipError_t after_pass(int kind, hipStream_t st) {
    se2conv_plan_s* p = g_timing_plan;
    if (!p) return hipSuccess;
    if (p->ev_rec.empty()) return hipErrorInvalidValue;
    p->ev_kind.push_back(kind);
    return record_event(p, st);
}

// ------------------------------------------------------------ pass schedules
struct Chain {
    int ntab = 0;
    int kind[SE2C_MAX_TABLES];
    const void* ptr[SE2C_MAX_TABLES];
};

bool slab_fits(const se2conv_shape& s, bool d) {
    SlabArgs a{};
    a.nx = s.nx;
    a.m = s.m;
    a.rows_per_tile = s.m;
    a.pad = 0;
    a.px = make_radix_plan(s.nx);  // their LDS tables count
    a.pt = make_radix_plan(s.m);
    const long long P = (long long)s.nx * s.m;
    const bool odd = odd_len(s.nx) || odd_len(s.m);
    return P <= tile_capacity(d, odd) && slab_lds_bytes(a, d) <= kMaxLds;
}

// Fields per launch of the separable two-pass schedule.  Measured on MI355X at
// 256x256x64: chunks small enough to keep the intermediate in the memory-side
// cache (8, 4, 2 fields) were not faster than one launch over the whole batch,
// so the default is the whole batch.  SE2CONV_SEP_CHUNK overrides (tuning only).
int sep_chunk_fields(const se2conv_plan_s* p, const se2conv_shape& s, int batch) {
    (void)p;
    (void)s;
    static const int env_chunk = [] {
        const char* e = std::getenv("SE2CONV_SEP_CHUNK");
        return e ? std::atoi(e) : 0;
    }();
    if (env_chunk > 0) return std::min(env_chunk, batch);
    return batch;
}

// Theta rows per x-row tile: the largest divisor of M within the point budget (capped
// by what one tile holds), or, when M has no divisor near the budget (a prime M, say),
// equal chunks of at most the budget with a shorter last one.
int rows_for_xpass(const se2conv_shape& s, bool d, int points = 4096) {
    points = (int)std::min<long long>(points, tile_capacity(d, odd_len(s.nx)));
    const int rmax = std::max(1, std::min(s.m, points / s.nx));
    int best = 1;
    for (int r = 1; r <= rmax; ++r)
        if (s.m % r == 0) best = r;
    if (2 * best >= rmax) return best;
    const int nt = (s.m + rmax - 1) / rmax;
    return (s.m + nt - 1) / nt;
}

// The schedule of a shape (shapes are looked up by value: passes receive the shape).
const Schedule& sched_of(const se2conv_plan_s* p, const se2conv_shape& s) {
    static const Schedule dflt32 = default_schedule(false), dflt64 = default_schedule(true);
    for (size_t i = 0; i < p->shapes.size(); ++i)
        if (p->shapes[i].nx == s.nx && p->shapes[i].ny == s.ny && p->shapes[i].m == s.m) return p->sched[i];
    return dbl(p) ? dflt64 : dflt32;
}

int pencil_width(int ncols, int L, bool d, int want = 16) {
    int W = want;
    while (W > 1 && (long long)W * L > tile_capacity(d, odd_len(L))) W /= 2;
    if (ncols < W) W = ncols;
    return W;
}

hipError_t run_slab(const se2conv_plan_s* p, SlabArgs a, bool d, hipStream_t st) {
    // x rows of a prime length with register kernels (planes; one direction, or forward,
    // 1-D product and inverse): Rader's algorithm in registers, unless the plan asks for
    // the generic kernels
    if (!(p->flags & SE2CONV_PLAN_GENERIC) && !a.do_t && a.in_mode == 1 && a.out_mode == 1 && !a.items &&
        a.px.rader && rader_fast_supported(a.px.L, d) &&
        ((a.mul == 0 && a.fwd != a.inv) || (a.mul == 1 && a.fwd && a.inv))) {
        PencilArgs r{};
        r.in0 = a.in0;
        r.in1 = a.in1;
        r.out0 = a.out0;
        r.out1 = a.out1;
        r.lone_in1 = a.lone_in1;
        r.lone_out1 = a.lone_out1;
        r.item_stride_in = a.item_stride_in;
        r.item_stride_out = a.item_stride_out;
        r.nitems = a.nitems;
        r.mode = 1;
        r.axis = 0;
        r.nx = a.nx;
        r.ny = a.ny;
        r.m = a.m;
        r.ncols = a.ny;
        r.fwd = a.fwd;
        r.inv = a.inv;
        r.mul = a.mul;
        r.ntab = a.mul ? a.ntab : 0;
        for (int j = 0; j < r.ntab; ++j) r.tab1[j] = a.tx[j];
        r.conj_tab = a.conj_tab;
        r.scale = a.scale;
        r.p = a.px;
        r.cplx = a.cplx;
        hipError_t e = launch_rader_pencil(r, d, st);
        if (e != hipSuccess) return e;
        return after_pass(3, st);
    }
    const long long P = (long long)a.rows_per_tile * a.nx;
    const bool odd = odd_len(a.nx) || (a.do_t && odd_len(a.m));
    const int nthr = threads_for(P, d, odd);
    if (P > (long long)maxv(d, odd) * nthr) return hipErrorInvalidConfiguration;  // tile larger than the workgroup covers
    const long long ntiles = (long long)a.nslab * a.ntile_t * a.nitems;
    const int nb = (int)std::min<long long>(ntiles, 1 << 20);
    hipError_t e = launch_slab(a, d, nthr, nb, st);
    if (e != hipSuccess) return e;
    return after_pass(a.do_t ? 0 : 3, st);
}

hipError_t run_pencil(const se2conv_plan_s* p, PencilArgs a, bool d, hipStream_t st) {
    // prime lengths with register kernels: Rader's algorithm in registers, unless the plan
    // asks for the generic kernels
    if (!(p->flags & SE2CONV_PLAN_GENERIC) && a.p.rader && rader_fast_supported(a.p.L, d) && a.mode == 1 &&
        !a.items &&
        ((a.fwd && a.inv && (a.mul == 2 || a.mul == 1)) || (a.fwd != a.inv && a.mul == 0))) {
        hipError_t e = launch_rader_pencil(a, d, st);
        if (e != hipSuccess) return e;
        return after_pass(a.axis == 1 ? 1 : 2, st);
    }
    const long long P = (long long)a.p.L * a.W;
    const bool odd = odd_len(a.p.L);
    // the shift-mix pencils hold fewer values per thread (SE2C_MAXV_SHIFT)
    const int mv = a.mul == 3 && !odd ? SE2C_MAXV_SHIFT : maxv(d, odd);
    long long nt = (P + mv - 1) / mv;
    nt = std::max<long long>(64, (nt + 63) / 64 * 64);
    const int nthr = (int)std::min<long long>(nt, a.mul == 3 ? 512 : max_threads(d, odd));
    if (P > (long long)mv * nthr) return hipErrorInvalidConfiguration;
    const int ncol_tiles = (a.ncols + a.W - 1) / a.W;
    const int nother = a.axis == 1 ? a.m : a.ny;
    const long long ntiles = (long long)ncol_tiles * nother * a.nitems;
    const int nb = (int)std::min<long long>(ntiles, 1 << 20);
    hipError_t e = launch_pencil(a, d, nthr, nb, st);
    if (e != hipSuccess) return e;
    return after_pass(a.axis == 1 ? 1 : 2, st);
}

// Separable chain: every table SEPARABLE.  f, out: [batch][m][ny][nx] real.
// Separable FP32 chain on shapes whose x-theta slab does not fit in LDS: three
// register-kernel passes (x rows, y pencils, theta pencils), each a 1-D circular
// convolution along its axis; the second and third run in place on the output.
se2conv_status enqueue_three_pass_fast(se2conv_plan_s* p, const se2conv_shape& s, const FastSepArgs& fa,
                                       hipStream_t st) {
    FastSepArgs r = fa;
    r.tw = reinterpret_cast<const float2*>(tw_of(p, s.nx, false));
    HIPCHK(launch_rows_fast(r, st));
    HIPCHK(after_pass(3, st));
    FastSepArgs y = fa;
    y.in = fa.out;
    y.axis = 1;
    y.tw = reinterpret_cast<const float2*>(tw_of(p, s.ny, false));
    HIPCHK(launch_pencil_fast(y, st));
    HIPCHK(after_pass(1, st));
    FastSepArgs t = y;
    t.axis = 2;
    t.tw = reinterpret_cast<const float2*>(tw_of(p, s.m, false));
    HIPCHK(launch_pencil_fast(t, st));
    HIPCHK(after_pass(2, st));
    return SE2CONV_OK;
}

se2conv_status enqueue_sep(se2conv_plan_s* p, const se2conv_shape& s, const void* f, void* out, int batch,
                           const Chain& ch, bool conj, hipStream_t st) {
    const bool d = dbl(p);
    const long long n = (long long)s.nx * s.ny * s.m;
    const RadixPlan px = radix_plan_of(p, s.nx, d), py = radix_plan_of(p, s.ny, d), pt = radix_plan_of(p, s.m, d);
    const size_t cb = cplx_bytes(p);
    auto fx = [&](int j) { return ch.ptr[j]; };
    auto fy = [&](int j) { return (const void*)((const char*)ch.ptr[j] + cb * s.nx); };
    auto ftt = [&](int j) { return (const void*)((const char*)ch.ptr[j] + cb * (s.nx + s.ny)); };

    // pass 1: x (and theta) on y-pair slabs, real -> real
    SlabArgs a{};
    a.in0 = f;
    a.out0 = out;
    a.item_stride_in = n;
    a.item_stride_out = n;
    a.nitems = batch;
    a.in_mode = 0;
    a.out_mode = 0;
    a.nx = s.nx;
    a.ny = s.ny;
    a.m = s.m;
    a.nslab = s.ny / 2;
    a.pad = 0;
    a.fwd = 1;
    a.inv = 1;
    a.mul = 1;
    a.ntab = ch.ntab;
    a.conj_tab = conj ? 1 : 0;
    a.px = px;
    a.pt = pt;
    a.twx = stage_tw_of(p, px, d);
    a.twt = stage_tw_of(p, pt, d);
    for (int j = 0; j < ch.ntab; ++j) {
        a.tx[j] = fx(j);
        a.tt[j] = ftt(j);
    }
    const bool two_pass = slab_fits(s, d);
    const bool generic_only = (p->flags & SE2CONV_PLAN_GENERIC) != 0;
    FastSepArgs fa{};
    fa.in = reinterpret_cast<const float*>(f);
    fa.out = reinterpret_cast<float*>(out);
    fa.n = n;
    fa.nitems = batch;
    fa.nx = s.nx;
    fa.ny = s.ny;
    fa.m = s.m;
    fa.ntab = ch.ntab;
    fa.conj_tab = conj ? 1 : 0;
    fa.grid_blocks = p->num_cus * sched_of(p, s).fast_blocks_per_cu;
    fa.cus = p->num_cus;
    for (int j = 0; j < ch.ntab; ++j) {
        fa.tx[j] = fx(j);
        fa.ty[j] = fy(j);
        fa.tt[j] = ftt(j);
    }
    fa.axis = 1;
    const bool fast_slab = !d && !generic_only && two_pass && slab_fast_supported(s.nx, s.m);
    const bool fast_pencil = !d && !generic_only && two_pass && pencil_fast_supported(s.nx, s.ny);
    if (!d && !generic_only && !two_pass && three_pass_fast_supported(s.nx, s.ny, s.m))
        return enqueue_three_pass_fast(p, s, fa, st);
    if (d && !generic_only && !two_pass && fast64_supported(s.nx, s.ny, s.m)) {
        // FP64 register kernels: x rows, then y and theta pencils in place
        Fast64Args g{};
        g.in = reinterpret_cast<const double*>(f);
        g.out = reinterpret_cast<double*>(out);
        g.n = n;
        g.nitems = batch;
        g.nx = s.nx;
        g.ny = s.ny;
        g.m = s.m;
        g.ntab = ch.ntab;
        g.conj_tab = conj ? 1 : 0;
        for (int j = 0; j < ch.ntab; ++j) g.tab[j] = fx(j);
        g.tw = reinterpret_cast<const double2*>(tw_of(p, s.nx, true));
        HIPCHK(launch_rows_f64(g, st));
        HIPCHK(after_pass(3, st));
        g.in = g.out;
        g.axis = 1;
        for (int j = 0; j < ch.ntab; ++j) g.tab[j] = fy(j);
        g.tw = reinterpret_cast<const double2*>(tw_of(p, s.ny, true));
        HIPCHK(launch_pencil_f64(g, st));
        HIPCHK(after_pass(1, st));
        g.axis = 2;
        for (int j = 0; j < ch.ntab; ++j) g.tab[j] = ftt(j);
        g.tw = reinterpret_cast<const double2*>(tw_of(p, s.m, true));
        HIPCHK(launch_pencil_f64(g, st));
        HIPCHK(after_pass(2, st));
        return SE2CONV_OK;
    }
    if (fast_slab && fast_pencil) {
        // Fields per launch pair (the whole batch unless SE2CONV_SEP_CHUNK says
        // otherwise; see sep_chunk_fields).
        const int chunk = sep_chunk_fields(p, s, batch);
        for (int c0 = 0; c0 < batch; c0 += chunk) {
            FastSepArgs ca = fa;
            ca.in = reinterpret_cast<const float*>(f) + (long long)c0 * n;
            ca.out = reinterpret_cast<float*>(out) + (long long)c0 * n;
            ca.nitems = std::min(chunk, batch - c0);
            ca.tw = reinterpret_cast<const float2*>(tw_of(p, s.nx, false));
            ca.twt = reinterpret_cast<const float2*>(tw_of(p, s.m, false));
            HIPCHK(launch_slab_fast(ca, st));
            HIPCHK(after_pass(0, st));
            FastSepArgs cb = ca;
            cb.in = ca.out;
            cb.tw = reinterpret_cast<const float2*>(tw_of(p, s.ny, false));
            HIPCHK(launch_pencil_fast(cb, st));
            HIPCHK(after_pass(1, st));
        }
        return SE2CONV_OK;
    }
    if (fast_slab) {
        fa.tw = reinterpret_cast<const float2*>(tw_of(p, s.nx, false));
        fa.twt = reinterpret_cast<const float2*>(tw_of(p, s.m, false));
        HIPCHK(launch_slab_fast(fa, st));
        HIPCHK(after_pass(0, st));
    }
    if (two_pass) {
        a.rows_per_tile = s.m;
        a.ntile_t = 1;
        a.do_t = 1;
        a.scale = 1.0 / ((double)s.nx * s.m);
    } else {
        a.rows_per_tile = rows_for_xpass(s, d, sched_of(p, s).xrow_points);
        a.ntile_t = (s.m + a.rows_per_tile - 1) / a.rows_per_tile;
        a.do_t = 0;
        a.scale = 1.0 / (double)s.nx;
    }
    if (!fast_slab) HIPCHK(run_slab(p, a, d, st));

    // pass 2 (and 3): y pencils (and theta pencils) on x-pairs, in place on out
    auto pencil = [&](int axis) -> se2conv_status {
        PencilArgs b{};
        b.in0 = out;
        b.out0 = out;
        b.item_stride_in = n;
        b.item_stride_out = n;
        b.nitems = batch;
        b.mode = 0;
        b.axis = axis;
        b.nx = s.nx;
        b.ny = s.ny;
        b.m = s.m;
        b.ncols = s.nx / 2;
        const int L = axis == 1 ? s.ny : s.m;
        b.W = pencil_width(b.ncols, L, d, sched_of(p, s).pencil_w);
        b.pad = 0;
        b.fwd = 1;
        b.inv = 1;
        b.mul = 1;
        b.ntab = ch.ntab;
        for (int j = 0; j < ch.ntab; ++j) b.tab1[j] = axis == 1 ? fy(j) : ftt(j);
        b.conj_tab = conj ? 1 : 0;
        b.scale = 1.0 / (double)L;
        b.p = axis == 1 ? py : pt;
        b.tw = stage_tw_of(p, b.p, d);
        HIPCHK(run_pencil(p, b, d, st));
        return SE2CONV_OK;
    };
    se2conv_status r = SE2CONV_OK;
    if (fast_pencil) {
        FastSepArgs fb = fa;
        fb.in = reinterpret_cast<const float*>(out);
        fb.tw = reinterpret_cast<const float2*>(tw_of(p, s.ny, false));
        HIPCHK(launch_pencil_fast(fb, st));
        HIPCHK(after_pass(1, st));
    } else {
        r = pencil(1);
        if (r != SE2CONV_OK) return r;
    }
    if (!two_pass) {
        r = pencil(2);
        if (r != SE2CONV_OK) return r;
    }
    return SE2CONV_OK;
}

// Separable chains given as a device item list (one SepItem per field, all of shape s).
se2conv_status enqueue_sep_items(se2conv_plan_s* p, const se2conv_shape& s, const SepItem* d_items, int nitems,
                                 bool conj, hipStream_t st) {
    const bool d = dbl(p);
    const bool generic_only = (p->flags & SE2CONV_PLAN_GENERIC) != 0;
    const bool two_pass = slab_fits(s, d);
    const bool fast_slab = !d && !generic_only && two_pass && slab_fast_supported(s.nx, s.m);
    const bool fast_pencil = !d && !generic_only && two_pass && pencil_fast_supported(s.nx, s.ny);
    FastSepArgs fa{};
    fa.nitems = nitems;
    fa.nx = s.nx;
    fa.ny = s.ny;
    fa.m = s.m;
    fa.conj_tab = conj ? 1 : 0;
    fa.grid_blocks = p->num_cus * sched_of(p, s).fast_blocks_per_cu;
    fa.cus = p->num_cus;
    fa.axis = 1;
    fa.items = d_items;
    if (!d && !generic_only && !two_pass && three_pass_fast_supported(s.nx, s.ny, s.m))
        return enqueue_three_pass_fast(p, s, fa, st);
    if (fast_slab) {
        fa.tw = reinterpret_cast<const float2*>(tw_of(p, s.nx, false));
        fa.twt = reinterpret_cast<const float2*>(tw_of(p, s.m, false));
        HIPCHK(launch_slab_fast(fa, st));
        HIPCHK(after_pass(0, st));
    } else {
        SlabArgs a{};
        a.items = d_items;
        a.nitems = nitems;
        a.in_mode = 0;
        a.out_mode = 0;
        a.nx = s.nx;
        a.ny = s.ny;
        a.m = s.m;
        a.nslab = s.ny / 2;
        a.fwd = 1;
        a.inv = 1;
        a.mul = 1;
        a.ntab = 0;  // factors come from the items
        a.conj_tab = conj ? 1 : 0;
        a.px = radix_plan_of(p, s.nx, d);
        a.pt = radix_plan_of(p, s.m, d);
        a.twx = stage_tw_of(p, a.px, d);
        a.twt = stage_tw_of(p, a.pt, d);
        if (two_pass) {
            a.rows_per_tile = s.m;
            a.ntile_t = 1;
            a.do_t = 1;
            a.scale = 1.0 / ((double)s.nx * s.m);
        } else {
            a.rows_per_tile = rows_for_xpass(s, d, sched_of(p, s).xrow_points);
            a.ntile_t = (s.m + a.rows_per_tile - 1) / a.rows_per_tile;
            a.do_t = 0;
            a.scale = 1.0 / (double)s.nx;
        }
        HIPCHK(run_slab(p, a, d, st));
    }
    auto pencil = [&](int axis) -> hipError_t {
        PencilArgs b{};
        b.items = d_items;
        b.nitems = nitems;
        b.mode = 0;
        b.axis = axis;
        b.nx = s.nx;
        b.ny = s.ny;
        b.m = s.m;
        b.ncols = s.nx / 2;
        const int L = axis == 1 ? s.ny : s.m;
        b.W = pencil_width(b.ncols, L, d, sched_of(p, s).pencil_w);
        b.fwd = 1;
        b.inv = 1;
        b.mul = 1;
        b.ntab = 0;
        b.conj_tab = conj ? 1 : 0;
        b.scale = 1.0 / (double)L;
        b.p = radix_plan_of(p, L, d);
        b.tw = stage_tw_of(p, b.p, d);
        return run_pencil(p, b, d, st);
    };
    if (fast_pencil) {
        FastSepArgs fb = fa;
        fb.tw = reinterpret_cast<const float2*>(tw_of(p, s.ny, false));
        HIPCHK(launch_pencil_fast(fb, st));
        HIPCHK(after_pass(1, st));
    } else {
        HIPCHK(pencil(1));
    }
    if (!two_pass) HIPCHK(pencil(2));
    return SE2CONV_OK;
}

// Forward (dir = 0) or inverse (dir = 1) transform along x and theta of complex
// plane pairs.  in/out planes per item: (in0 + it*stride, in1 + it*stride).
hipError_t xt_transform(se2conv_plan_s* p, const se2conv_shape& s, bool d, int dir, const void* in0,
                        const void* in1, void* out0, void* out1, const void* lone_in1, void* lone_out1,
                        long long stride_in, long long stride_out, int nitems, hipStream_t st, int cplx = 0) {
    const RadixPlan px = radix_plan_of(p, s.nx, d), pt = radix_plan_of(p, s.m, d);
    SlabArgs a{};
    a.cplx = cplx;
    a.in0 = in0;
    a.in1 = in1;
    a.out0 = out0;
    a.out1 = out1;
    a.lone_in1 = lone_in1;
    a.lone_out1 = lone_out1;
    a.item_stride_in = stride_in;
    a.item_stride_out = stride_out;
    a.nitems = nitems;
    a.in_mode = 1;
    a.out_mode = 1;
    a.nx = s.nx;
    a.ny = s.ny;
    a.m = s.m;
    a.nslab = s.ny;
    a.pad = 0;
    a.fwd = dir == 0;
    a.inv = dir == 1;
    a.mul = 0;
    a.px = px;
    a.pt = pt;
    a.twx = stage_tw_of(p, px, d);
    a.twt = stage_tw_of(p, pt, d);
    if (slab_fits(s, d)) {
        a.rows_per_tile = s.m;
        a.ntile_t = 1;
        a.do_t = 1;
        return run_slab(p, a, d, st);
    }
    // split: x rows and theta pencils (planes mode), in the right order
    a.rows_per_tile = rows_for_xpass(s, d, sched_of(p, s).xrow_points);
    a.ntile_t = (s.m + a.rows_per_tile - 1) / a.rows_per_tile;
    a.do_t = 0;
    PencilArgs b{};
    b.cplx = cplx;
    b.mode = 1;
    b.axis = 2;
    b.nx = s.nx;
    b.ny = s.ny;
    b.m = s.m;
    b.ncols = s.nx;
    b.W = pencil_width(b.ncols, s.m, d, sched_of(p, s).pencil_w);
    b.pad = 0;
    b.fwd = dir == 0;
    b.inv = dir == 1;
    b.mul = 0;
    b.p = pt;
    b.tw = stage_tw_of(p, pt, d);
    b.nitems = nitems;
    hipError_t e;
    if (dir == 0) {
        e = run_slab(p, a, d, st);  // in -> out
        if (e != hipSuccess) return e;
        b.in0 = out0;
        b.in1 = out1;
        b.out0 = out0;
        b.out1 = out1;
        b.lone_in1 = lone_out1;
        b.lone_out1 = lone_out1;
        b.item_stride_in = stride_out;
        b.item_stride_out = stride_out;
        return run_pencil(p, b, d, st);
    }
    b.in0 = in0;
    b.in1 = in1;
    b.out0 = const_cast<void*>(in0);
    b.out1 = const_cast<void*>(in1);
    b.lone_in1 = lone_in1;
    b.lone_out1 = const_cast<void*>(lone_in1);
    b.item_stride_in = stride_in;
    b.item_stride_out = stride_in;
    e = run_pencil(p, b, d, st);  // in place on the input planes
    if (e != hipSuccess) return e;
    return run_slab(p, a, d, st);
}

// y pencils on complex plane pairs: forward, optional product, inverse.
hipError_t y_pass(se2conv_plan_s* p, const se2conv_shape& s, bool d, void* re, void* im, void* lone_im,
                  long long stride, int nitems, int fwd, int inv, int mul, const Chain* ch, bool conj,
                  double scale, hipStream_t st, int cplx = 0) {
    PencilArgs b{};
    b.cplx = cplx;
    b.in0 = re;
    b.in1 = im;
    b.out0 = re;
    b.out1 = im;
    b.lone_in1 = lone_im;
    b.lone_out1 = lone_im;
    b.item_stride_in = stride;
    b.item_stride_out = stride;
    b.nitems = nitems;
    b.mode = 1;
    b.axis = 1;
    b.nx = s.nx;
    b.ny = s.ny;
    b.m = s.m;
    b.ncols = s.nx;
    b.W = pencil_width(b.ncols, s.ny, d, sched_of(p, s).pencil_w);
    b.pad = 0;
    b.fwd = fwd;
    b.inv = inv;
    b.mul = mul;
    b.p = radix_plan_of(p, s.ny, d);
    b.tw = stage_tw_of(p, b.p, d);
    b.conj_tab = conj ? 1 : 0;
    b.scale = scale;
    if (mul && ch) {
        const size_t cb = cplx_bytes(p);
        b.ntab = ch->ntab;
        for (int j = 0; j < ch->ntab; ++j) {
            if (ch->kind[j] == SE2CONV_TABLE_FULL || ch->kind[j] == SE2CONV_TABLE_QUARTER) {
                b.tab3[j] = ch->ptr[j];
                if (ch->kind[j] == SE2CONV_TABLE_QUARTER) b.tab3_quarter |= 1u << j;
            } else {
                b.tab3[j] = nullptr;
                b.sepx[j] = ch->ptr[j];
                b.sepy[j] = (const char*)ch->ptr[j] + cb * s.nx;
                b.sept[j] = (const char*)ch->ptr[j] + cb * (s.nx + s.ny);
            }
        }
    }
    return run_pencil(p, b, d, st);
}

// y pencils on complex plane pairs, input planes -> output planes (may coincide).
hipError_t y_pass_io(se2conv_plan_s* p, const se2conv_shape& s, bool d, const void* in_re, const void* in_im,
                     void* out_re, void* out_im, const void* lone_in, void* lone_out, long long stride, int nitems,
                     int fwd, int inv, int mul, const Chain* ch, bool conj, double scale, hipStream_t st) {
    PencilArgs b{};
    b.in0 = in_re;
    b.in1 = in_im;
    b.out0 = out_re;
    b.out1 = out_im;
    b.lone_in1 = lone_in;
    b.lone_out1 = lone_out;
    b.item_stride_in = stride;
    b.item_stride_out = stride;
    b.nitems = nitems;
    b.mode = 1;
    b.axis = 1;
    b.nx = s.nx;
    b.ny = s.ny;
    b.m = s.m;
    b.ncols = s.nx;
    b.W = pencil_width(b.ncols, s.ny, d, sched_of(p, s).pencil_w);
    b.fwd = fwd;
    b.inv = inv;
    b.mul = mul;
    b.p = radix_plan_of(p, s.ny, d);
    b.tw = stage_tw_of(p, b.p, d);
    b.conj_tab = conj ? 1 : 0;
    b.scale = scale;
    if (mul && ch) {
        const size_t cb = cplx_bytes(p);
        b.ntab = ch->ntab;
        for (int j = 0; j < ch->ntab; ++j) {
            if (ch->kind[j] == SE2CONV_TABLE_FULL || ch->kind[j] == SE2CONV_TABLE_QUARTER) {
                b.tab3[j] = ch->ptr[j];
                if (ch->kind[j] == SE2CONV_TABLE_QUARTER) b.tab3_quarter |= 1u << j;
            } else {
                b.tab3[j] = nullptr;
                b.sepx[j] = ch->ptr[j];
                b.sepy[j] = (const char*)ch->ptr[j] + cb * s.nx;
                b.sept[j] = (const char*)ch->ptr[j] + cb * (s.nx + s.ny);
            }
        }
    }
    return run_pencil(p, b, d, st);
}

// Full (non-separable) chain on pairs of fields.
// FP32 register kernels of the full path (x-theta forward, y product, x-theta inverse).
FullFastArgs full_fast_args(se2conv_plan_s* p, const se2conv_shape& s, int batch) {
    FullFastArgs a{};
    a.n = (long long)s.nx * s.ny * s.m;
    a.batch = batch;
    a.nx = s.nx;
    a.ny = s.ny;
    a.m = s.m;
    a.lone = (batch & 1) ? reinterpret_cast<float*>(p->ws) : nullptr;
    a.twx = reinterpret_cast<const float2*>(tw_of(p, s.nx, false));
    a.twy = reinterpret_cast<const float2*>(tw_of(p, s.ny, false));
    a.twt = reinterpret_cast<const float2*>(tw_of(p, s.m, false));
    a.scale = 1.0f;
    return a;
}

void set_chain(FullFastArgs* a, const Chain& ch, bool conj, double scale) {
    a->ntab = ch.ntab;
    for (int j = 0; j < ch.ntab; ++j) {
        a->tab[j] = ch.ptr[j];
        a->tab_full[j] = ch.kind[j] == SE2CONV_TABLE_FULL ? 1 : ch.kind[j] == SE2CONV_TABLE_QUARTER ? 2 : 0;
    }
    a->conj_tab = conj ? 1 : 0;
    a->scale = (float)scale;
}

bool use_full_fast(const se2conv_plan_s* p, const se2conv_shape& s) {
    return !dbl(p) && !(p->flags & SE2CONV_PLAN_GENERIC) && full_fast_supported(s.nx, s.ny, s.m);
}

se2conv_status enqueue_full(se2conv_plan_s* p, const se2conv_shape& s, const void* f, void* out, int batch,
                            const Chain& ch, bool conj, hipStream_t st) {
    const bool d = dbl(p);
    if (use_full_fast(p, s)) {
        FullFastArgs a = full_fast_args(p, s, batch);
        set_chain(&a, ch, conj, 1.0 / (double)a.n);
        a.in = reinterpret_cast<const float*>(f);
        a.out = reinterpret_cast<float*>(out);
        HIPCHK(launch_xt_full_fwd(a, st));
        HIPCHK(after_pass(0, st));
        a.in = a.out;
        HIPCHK(launch_y_full(a, st));
        HIPCHK(after_pass(1, st));
        HIPCHK(launch_xt_full_inv(a, st));
        HIPCHK(after_pass(0, st));
        return SE2CONV_OK;
    }
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t rb = real_bytes(p);
    const int pairs = (batch + 1) / 2;
    const bool odd = (batch & 1) != 0;
    const void* f1 = (const char*)f + rb * n;
    void* o1 = (char*)out + rb * n;
    // the odd item's imaginary plane: zero on input, plan workspace in between
    void* lone = odd ? p->ws : nullptr;
    if (batch == 1) {
        f1 = nullptr;
        o1 = nullptr;
    }
    HIPCHK(xt_transform(p, s, d, 0, f, batch == 1 ? nullptr : f1, out, batch == 1 ? nullptr : o1,
                        nullptr, odd ? lone : nullptr, 2 * n, 2 * n, pairs, st));
    // With batch == 1 the only item is "lone": xt_transform wrote its imaginary
    // part to lone (because lone_out1 is used for the last odd item).
    HIPCHK(y_pass(p, s, d, out, o1, lone, 2 * n, pairs, 1, 1, 2, &ch, conj, 1.0 / (double)n, st));
    HIPCHK(xt_transform(p, s, d, 1, out, o1, out, o1, lone, nullptr, 2 * n, 2 * n, pairs, st));
    return SE2CONV_OK;
}

constexpr int kChainStreams = 4;

// Auxiliary streams and events of the plan (created once, under the plan mutex).
se2conv_status ensure_aux_streams(se2conv_plan_s* p) {
    std::lock_guard<std::mutex> g(p->mu);
    if (!p->aux.empty()) return SE2CONV_OK;
    std::vector<hipStream_t> st(kChainStreams, nullptr);
    std::vector<hipEvent_t> ev(kChainStreams, nullptr);
    hipEvent_t fork = nullptr;
    bool good = hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; good && i < kChainStreams; ++i)
        good = hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
    if (!good) {
        for (auto x : st)
            if (x) (void)hipStreamDestroy(x);
        for (auto x : ev)
            if (x) (void)hipEventDestroy(x);
        if (fork) (void)hipEventDestroy(fork);
        return fail(SE2CONV_ERR_DEVICE, "could not create the chain streams");
    }
    p->aux = st;
    p->ev_join = ev;
    p->ev_fork = fork;
    return SE2CONV_OK;
}


// Every shape class of a grouped item list in one launch per pass and class kind (the
// multi-class register kernels), when every class has them; *done tells whether it ran.
// Classes go largest first, so that the last workgroups of a grid are the small ones.
// fork_ok: the second kind may run on an auxiliary stream (not under pass timing, not in
// the allocation-free entry point).
se2conv_status enqueue_multi(se2conv_plan_s* p, const SepItem* d_items, const std::vector<std::pair<int, int>>& groups,
                             const std::vector<int>& counts, bool conj, hipStream_t st, bool* done, bool fork_ok) {
    *done = false;
    static const bool enabled = [] {
        const char* e = std::getenv("SE2CONV_CHAIN_MULTI");
        return !(e && std::atoi(e) == 0);
    }();
    const int ng = (int)groups.size();
    if (!enabled || dbl(p) || (p->flags & SE2CONV_PLAN_GENERIC) || ng < 1 || ng > SE2C_MAX_CLASSES) return SE2CONV_OK;
    for (int gi = 0; gi < ng; ++gi) {
        const se2conv_shape& s = p->shapes[groups[gi].first];
        if (!slab_fits(s, false) || !multi_slab_supported(s.nx, s.m) || !multi_pencil_supported(s.nx, s.ny))
            return SE2CONV_OK;
    }
    std::vector<int> order(ng);
    for (int gi = 0; gi < ng; ++gi) order[gi] = gi;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const se2conv_shape& sa = p->shapes[groups[a].first];
        const se2conv_shape& sb = p->shapes[groups[b].first];
        return (long long)sa.nx * sa.ny * sa.m * counts[a] > (long long)sb.nx * sb.ny * sb.m * counts[b];
    });
    MultiArgs m{};
    m.items = d_items;
    m.conj_tab = conj ? 1 : 0;
    m.nclass = ng;
    for (int k = 0; k < ng; ++k) {
        const int gi = order[k];
        const se2conv_shape& s = p->shapes[groups[gi].first];
        MultiClass& c = m.c[k];
        c.nx = s.nx;
        c.ny = s.ny;
        c.m = s.m;
        c.nitems = counts[gi];
        c.item0 = groups[gi].second;
        c.twx = reinterpret_cast<const float2*>(tw_of(p, s.nx, false));
        c.twy = reinterpret_cast<const float2*>(tw_of(p, s.ny, false));
        c.twt = reinterpret_cast<const float2*>(tw_of(p, s.m, false));
    }
    // Classes with NX = 3 * 2^k run their slab kernel at two waves per SIMD, the others at
    // three: two kernels per pass.  With both kinds present they go to two streams (two
    // branches of a captured graph), so that the kinds share the GPU instead of each
    // running alone: 256 uneven problems in 15 classes, 0.396 ms per replay in one slab and one
    // pencil launch, 0.376 ms with the kinds in turn on one stream, 0.349 ms on two.
    MultiArgs part[2] = {m, m};
    part[0].nclass = part[1].nclass = 0;
    for (int k = 0; k < ng; ++k) {
        MultiArgs& q = part[(m.c[k].nx & (m.c[k].nx - 1)) == 0 ? 0 : 1];
        q.c[q.nclass++] = m.c[k];
    }
    if (fork_ok && part[0].nclass && part[1].nclass) {
        se2conv_status r = ensure_aux_streams(p);
        if (r != SE2CONV_OK) return r;
        std::lock_guard<std::mutex> g(p->fork_mu);
        hipStream_t side = p->aux[0];
        HIPCHK(hipEventRecord(p->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(side, p->ev_fork, 0));
        HIPCHK(launch_slab_multi(part[1], side));
        HIPCHK(launch_pencil_multi(part[1], side));
        HIPCHK(launch_slab_multi(part[0], st));
        HIPCHK(launch_pencil_multi(part[0], st));
        HIPCHK(hipEventRecord(p->ev_join[0], side));
        HIPCHK(hipStreamWaitEvent(st, p->ev_join[0], 0));
        *done = true;
        return SE2CONV_OK;
    }
    HIPCHK(launch_slab_multi(m, st));
    HIPCHK(after_pass(0, st));
    HIPCHK(launch_pencil_multi(m, st));
    HIPCHK(after_pass(1, st));
    *done = true;
    return SE2CONV_OK;
}

// x lines only (forward or inverse) on plane pairs, theta chunks as in the x-row pass.
hipError_t x_pass(se2conv_plan_s* p, const se2conv_shape& s, bool d, int dir, const void* in0, const void* in1,
                  void* out0, void* out1, const void* lone_in1, void* lone_out1, long long stride, int nitems,
                  hipStream_t st) {
    SlabArgs a{};
    a.in0 = in0;
    a.in1 = in1;
    a.out0 = out0;
    a.out1 = out1;
    a.lone_in1 = lone_in1;
    a.lone_out1 = lone_out1;
    a.item_stride_in = stride;
    a.item_stride_out = stride;
    a.nitems = nitems;
    a.in_mode = 1;
    a.out_mode = 1;
    a.nx = s.nx;
    a.ny = s.ny;
    a.m = s.m;
    a.nslab = s.ny;
    a.fwd = dir == 0;
    a.inv = dir == 1;
    a.px = radix_plan_of(p, s.nx, d);
    a.pt = radix_plan_of(p, s.m, d);
    a.twx = stage_tw_of(p, a.px, d);
    a.twt = stage_tw_of(p, a.pt, d);
    a.rows_per_tile = rows_for_xpass(s, d, sched_of(p, s).xrow_points);
    a.ntile_t = (s.m + a.rows_per_tile - 1) / a.rows_per_tile;
    a.do_t = 0;
    return run_slab(p, a, d, st);
}

// Sum of SE(2)-shifted radial kernels on pairs of fields (two real fields as one complex
// field: every step is real-linear and maps real fields to real fields).  Five passes over
// plane pairs: x forward, y forward (spatial spectra of every theta-slice), theta lines
// with the shift mix, forward transform, product with the radial kernel's coefficients
// (x 1/n) and inverse, y inverse, x inverse.
se2conv_status enqueue_shifted(se2conv_plan_s* p, const se2conv_shape& s, const void* f, void* out, int batch,
                               const Chain& ch, const void* qtab, const std::vector<int>& rolls, hipStream_t st) {
    const bool d = dbl(p);
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t rb = real_bytes(p);
    const int pairs = (batch + 1) / 2;
    const bool odd = (batch & 1) != 0;
    const void* f1 = batch == 1 ? nullptr : (const char*)f + rb * n;
    void* o1 = batch == 1 ? nullptr : (char*)out + rb * n;
    void* lone = odd ? p->ws : nullptr;  // the odd field's imaginary plane between the passes
    // FP32 register kernels where the full-table path has them: x forward (theta in space),
    // y forward, [shift mix, theta forward, product] in the pencils, y inverse, then the
    // x-theta inverse; else the generic passes with the theta inverse in the pencils
    const bool fast = use_full_fast(p, s);
    if (fast) {
        FullFastArgs a = full_fast_args(p, s, batch);
        a.in = reinterpret_cast<const float*>(f);
        a.out = reinterpret_cast<float*>(out);
        HIPCHK(launch_x_full_fwd(a, st));
        HIPCHK(after_pass(3, st));
        a.in = a.out;
        a.save = a.out;  // the y spectra in place (a lone last field's im plane in lone)
        a.save_lone = a.lone;
        HIPCHK(launch_y_full_spectra(a, st));
        HIPCHK(after_pass(1, st));
    } else {
        HIPCHK(x_pass(p, s, d, 0, f, f1, out, o1, nullptr, lone, 2 * n, pairs, st));
        HIPCHK(y_pass(p, s, d, out, o1, lone, 2 * n, pairs, 1, 0, 0, nullptr, false, 1.0, st));
    }
    PencilArgs b{};
    b.in0 = out;
    b.in1 = o1;
    b.out0 = out;
    b.out1 = o1;
    b.lone_in1 = lone;
    b.lone_out1 = lone;
    b.item_stride_in = 2 * n;
    b.item_stride_out = 2 * n;
    b.nitems = pairs;
    b.mode = 1;
    b.axis = 2;
    b.nx = s.nx;
    b.ny = s.ny;
    b.m = s.m;
    b.ncols = s.nx;
    b.W = pencil_width(b.ncols, s.m, d, sched_of(p, s).pencil_w);
    if (!odd_len(s.m))  // the shift-mix pencils hold SE2C_MAXV_SHIFT values per thread
        while (b.W > 1 && (long long)b.W * s.m > (long long)SE2C_MAXV_SHIFT * 512) b.W /= 2;
    b.fwd = 1;
    b.inv = fast ? 0 : 1;
    b.mul = 3;
    b.p = radix_plan_of(p, s.m, d);
    b.tw = stage_tw_of(p, b.p, d);
    b.scale = 1.0 / (double)n;
    b.qtab = qtab;
    b.nshift = (int)rolls.size();
    for (size_t j = 0; j < rolls.size(); ++j) b.rolls[j] = rolls[j];
    const size_t cb = cplx_bytes(p);
    b.ntab = ch.ntab;
    for (int j = 0; j < ch.ntab; ++j) {
        if (ch.kind[j] == SE2CONV_TABLE_FULL || ch.kind[j] == SE2CONV_TABLE_QUARTER) {
            b.tab3[j] = ch.ptr[j];
            if (ch.kind[j] == SE2CONV_TABLE_QUARTER) b.tab3_quarter |= 1u << j;
        } else {
            b.tab3[j] = nullptr;
            b.sepx[j] = ch.ptr[j];
            b.sepy[j] = (const char*)ch.ptr[j] + cb * s.nx;
            b.sept[j] = (const char*)ch.ptr[j] + cb * (s.nx + s.ny);
        }
    }
    if (fast && t_shift_supported(s.nx, s.m, (int)rolls.size())) {
        // the theta pass on register kernels: the shift-phase tiles in LDS for every pair
        FullFastArgs a = full_fast_args(p, s, batch);
        a.in = reinterpret_cast<const float*>(out);
        a.out = reinterpret_cast<float*>(out);
        set_chain(&a, ch, false, 1.0 / (double)n);
        a.qtab = reinterpret_cast<const float2*>(qtab);
        a.nshift = (int)rolls.size();
        for (size_t j = 0; j < rolls.size(); ++j) a.rolls[j] = rolls[j];
        HIPCHK(launch_t_shift(a, st));
        HIPCHK(after_pass(2, st));
    } else {
        HIPCHK(run_pencil(p, b, d, st));
    }
    if (fast) {
        FullFastArgs a = full_fast_args(p, s, batch);
        a.in = reinterpret_cast<const float*>(out);
        a.out = reinterpret_cast<float*>(out);
        HIPCHK(launch_y_full_inverse(a, st));
        HIPCHK(after_pass(1, st));
        HIPCHK(launch_xt_full_inv(a, st));
        HIPCHK(after_pass(0, st));
        return SE2CONV_OK;
    }
    HIPCHK(y_pass(p, s, d, out, o1, lone, 2 * n, pairs, 0, 1, 0, nullptr, false, 1.0, st));
    HIPCHK(x_pass(p, s, d, 1, out, o1, out, o1, lone, nullptr, 2 * n, pairs, st));
    return SE2CONV_OK;
}

se2conv_status lookup_chain(se2conv_plan_s* p, int shape_idx, const void* const* tables, int ntab, Chain* ch,
                            bool* all_sep) {
    if (ntab < 1 || ntab > SE2C_MAX_TABLES)
        return fail(SE2CONV_ERR_INVALID_ARG, "n_tables must lie in [1, %d]", SE2C_MAX_TABLES);
    ch->ntab = ntab;
    *all_sep = true;
    std::lock_guard<std::mutex> g(p->mu);
    for (int j = 0; j < ntab; ++j) {
        auto it = p->tables.find(reinterpret_cast<uintptr_t>(tables[j]));
        if (tables[j] == nullptr || it == p->tables.end())
            return fail(SE2CONV_ERR_INVALID_ARG, "table %d was not produced by this plan", j);
        if (it->second.shape_idx != shape_idx)
            return fail(SE2CONV_ERR_INVALID_ARG, "table %d belongs to shape %d, not %d", j, it->second.shape_idx,
                        shape_idx);
        if (it->second.kind == SE2CONV_TABLE_SHIFT)
            return fail(SE2CONV_ERR_INVALID_ARG, "table %d is a shift table (use se2conv_apply_shifted)", j);
        ch->kind[j] = it->second.kind;
        ch->ptr[j] = tables[j];
        if (it->second.kind != SE2CONV_TABLE_SEPARABLE) *all_sep = false;
    }
    return SE2CONV_OK;
}

se2conv_status validate_io(se2conv_plan_s* p, int32_t shape_idx, const void* f, void* out, int32_t batch) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (batch < 1) return fail(SE2CONV_ERR_INVALID_ARG, "batch must be >= 1 (got %d)", batch);
    if (!f || !out) return fail(SE2CONV_ERR_INVALID_ARG, "f and out must be non-null");
    if (!aligned16(f) || !aligned16(out)) return fail(SE2CONV_ERR_INVALID_ARG, "f and out must be 16-byte aligned");
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long bytes = (long long)batch * s.nx * s.ny * s.m * (long long)real_bytes(p);
    const char* a = (const char*)f;
    const char* b = (const char*)out;
    if (a != b && a < b + bytes && b < a + bytes)
        return fail(SE2CONV_ERR_INVALID_ARG, "f and out overlap without being equal");
    return SE2CONV_OK;
}

// Separable chain on a grid with an odd side: fields packed in pairs (re/im planes, the
// odd batch's last imaginary plane in the workspace), and the 3-D product regrouped into
// 1-D circular convolutions as on even grids: x and theta in one slab pass when the slab
// fits in LDS, else x rows then theta pencils, and y pencils; each pass forward, product
// with its axis' factor, inverse.  Two or three passes over the batch instead of the
// general path's three or five (forward, 3-D product along y, inverse).  The packing
// holds because every 1-D factor of a separable table is the transform of a real kernel
// along its axis.
se2conv_status enqueue_sep_pairs(se2conv_plan_s* p, const se2conv_shape& s, const void* f, void* out, int batch,
                                 const Chain& ch, bool conj, hipStream_t st) {
    const bool d = dbl(p);
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t rb = real_bytes(p), cb = cplx_bytes(p);
    const int pairs = (batch + 1) / 2;
    const bool odd = (batch & 1) != 0;
    const void* f1 = batch == 1 ? nullptr : (const char*)f + rb * n;
    void* o1 = batch == 1 ? nullptr : (char*)out + rb * n;
    void* lone = odd ? p->ws : nullptr;
    const RadixPlan px = radix_plan_of(p, s.nx, d), py = radix_plan_of(p, s.ny, d), pt = radix_plan_of(p, s.m, d);
    const bool fits = slab_fits(s, d);
    SlabArgs a{};
    a.in0 = f;
    a.in1 = f1;
    a.out0 = out;
    a.out1 = o1;
    a.lone_in1 = nullptr;  // the odd item's imaginary plane is zero on input
    a.lone_out1 = lone;
    a.item_stride_in = 2 * n;
    a.item_stride_out = 2 * n;
    a.nitems = pairs;
    a.in_mode = 1;
    a.out_mode = 1;
    a.nx = s.nx;
    a.ny = s.ny;
    a.m = s.m;
    a.nslab = s.ny;
    a.pad = 0;
    a.fwd = 1;
    a.inv = 1;
    a.mul = 1;
    a.ntab = ch.ntab;
    a.conj_tab = conj ? 1 : 0;
    a.px = px;
    a.pt = pt;
    a.twx = stage_tw_of(p, px, d);
    a.twt = stage_tw_of(p, pt, d);
    for (int j = 0; j < ch.ntab; ++j) {
        a.tx[j] = ch.ptr[j];
        a.tt[j] = (const char*)ch.ptr[j] + cb * (s.nx + s.ny);
    }
    if (fits) {
        a.rows_per_tile = s.m;
        a.ntile_t = 1;
        a.do_t = 1;
        a.scale = 1.0 / ((double)s.nx * s.m);
    } else {
        a.rows_per_tile = rows_for_xpass(s, d, sched_of(p, s).xrow_points);
        a.ntile_t = (s.m + a.rows_per_tile - 1) / a.rows_per_tile;
        a.do_t = 0;
        a.scale = 1.0 / (double)s.nx;
    }
    HIPCHK(run_slab(p, a, d, st));
    auto pencil = [&](int axis) -> hipError_t {
        const int L = axis == 1 ? s.ny : s.m;
        PencilArgs b{};
        b.in0 = out;
        b.in1 = o1;
        b.out0 = out;
        b.out1 = o1;
        b.lone_in1 = lone;
        b.lone_out1 = lone;
        b.item_stride_in = 2 * n;
        b.item_stride_out = 2 * n;
        b.nitems = pairs;
        b.mode = 1;
        b.axis = axis;
        b.nx = s.nx;
        b.ny = s.ny;
        b.m = s.m;
        b.ncols = s.nx;
        b.W = pencil_width(b.ncols, L, d, sched_of(p, s).pencil_w);
        b.pad = 0;
        b.fwd = 1;
        b.inv = 1;
        b.mul = 1;
        b.ntab = ch.ntab;
        for (int j = 0; j < ch.ntab; ++j) b.tab1[j] = (const char*)ch.ptr[j] + cb * (axis == 1 ? s.nx : s.nx + s.ny);
        b.conj_tab = conj ? 1 : 0;
        b.scale = 1.0 / (double)L;
        b.p = axis == 1 ? py : pt;
        b.tw = stage_tw_of(p, b.p, d);
        return run_pencil(p, b, d, st);
    };
    HIPCHK(pencil(1));
    if (!fits) HIPCHK(pencil(2));
    return SE2CONV_OK;
}

se2conv_status enqueue_problem(se2conv_plan_s* p, int shape_idx, const void* f, void* out, int batch,
                               const Chain& ch, bool all_sep, bool conj, hipStream_t st) {
    const se2conv_shape& s = p->shapes[shape_idx];
    if (all_sep && pair_layout(s)) return enqueue_sep(p, s, f, out, batch, ch, conj, st);
    if (all_sep) return enqueue_sep_pairs(p, s, f, out, batch, ch, conj, st);
    return enqueue_full(p, s, f, out, batch, ch, conj, st);
}

// ---- tuning cache: JSON lines {"nx":..,"ny":..,"m":..,"dtype":..,"w":..,"b":..,"x":..}
const char* tune_cache_path() { return std::getenv("SE2CONV_TUNE_CACHE"); }

bool parse_int_field(const std::string& line, const char* key, int* out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t pos = line.find(k);
    if (pos == std::string::npos) return false;
    char* end = nullptr;
    const long v = std::strtol(line.c_str() + pos + k.size(), &end, 10);
    if (end == line.c_str() + pos + k.size()) return false;
    *out = (int)v;
    return true;
}

// Malformed lines are ignored: a corrupt cache only means default schedules.
void load_tune_cache(se2conv_plan_s* p) {
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* fh = std::fopen(path, "r");
    if (!fh) return;
    char buf[512];
    while (std::fgets(buf, sizeof(buf), fh)) {
        const std::string line(buf);
        int nx, ny, m, dt, w, b, x;
        if (!parse_int_field(line, "nx", &nx) || !parse_int_field(line, "ny", &ny) ||
            !parse_int_field(line, "m", &m) || !parse_int_field(line, "dtype", &dt) ||
            !parse_int_field(line, "w", &w) || !parse_int_field(line, "b", &b) || !parse_int_field(line, "x", &x))
            continue;
        if (dt != (int)p->dtype || w < 1 || w > 64 || b < 1 || b > 32 || x < 64 || x > 65536) continue;
        for (size_t i = 0; i < p->shapes.size(); ++i) {
            if (p->shapes[i].nx == nx && p->shapes[i].ny == ny && p->shapes[i].m == m) {
                p->sched[i].pencil_w = w;
                p->sched[i].fast_blocks_per_cu = b;
                p->sched[i].xrow_points = x;
                p->sched[i].tuned = true;
            }
        }
    }
    std::fclose(fh);
}

void append_tune_cache(const se2conv_plan_s* p, int i) {
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* fh = std::fopen(path, "a");
    if (!fh) return;
    const se2conv_shape& s = p->shapes[i];
    const Schedule& sc = p->sched[i];
    std::fprintf(fh, "{\"nx\":%d,\"ny\":%d,\"m\":%d,\"dtype\":%d,\"w\":%d,\"b\":%d,\"x\":%d}\n", s.nx, s.ny, s.m,
                 (int)p->dtype, sc.pencil_w, sc.fast_blocks_per_cu, sc.xrow_points);
    std::fclose(fh);
}

se2conv_status ensure_scratch64(se2conv_plan_s* p, size_t bytes) {
    if (p->scratch64_bytes >= bytes) return SE2CONV_OK;
    if (p->scratch64) {
        hipError_t e = hipFree(p->scratch64);
        p->scratch64 = nullptr;
        p->scratch64_bytes = 0;
        if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "hipFree: %s", hipGetErrorString(e));
    }
    if (hipMalloc(&p->scratch64, bytes) != hipSuccess)
        return fail(SE2CONV_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of FP64 scratch", bytes);
    p->scratch64_bytes = bytes;
    return SE2CONV_OK;
}

}  // namespace

// ===================================================================== C ABI
// Hat basis of a radial-profile geometry (shared by the profile gradient and the table
// builder); rebuilt when the shape, knot count or radius changes.  Caller holds p->mu.
se2conv_status ensure_profile_basis(se2conv_plan_s* p, int shape_idx, int n_knots, double r_max, hipStream_t stream) {
    const se2conv_shape& s = p->shapes[shape_idx];
    if (p->basis_shape == shape_idx && p->basis_knots == n_knots && p->basis_rmax == r_max) return SE2CONV_OK;
    const size_t need = sizeof(double) * (size_t)((long long)s.nx * s.ny * n_knots);
    if (p->basis_bytes < need) {
        if (p->basis) {
            hipError_t e = hipFree(p->basis);
            p->basis = nullptr;
            p->basis_bytes = 0;
            if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "hipFree: %s", hipGetErrorString(e));
        }
        if (hipMalloc(reinterpret_cast<void**>(&p->basis), need) != hipSuccess)
            return fail(SE2CONV_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes for the profile basis", need);
        p->basis_bytes = need;
    }
    p->basis_shape = -1;
    p->bh_shape = -1;  // its spectrum is stale too
    HIPCHK(launch_profile_basis(p->basis, n_knots, r_max, s.nx, s.ny, stream));
    p->basis_shape = shape_idx;
    p->basis_knots = n_knots;
    p->basis_rmax = r_max;
    return SE2CONV_OK;
}

// Real 2-D DFT of that basis on the quadrant (FP64), for building radial-profile tables as
// a contraction over the knots.  tmp: n_knots ny (nx/2+1) double2 of scratch.  Caller
// holds p->mu.
se2conv_status ensure_basis_hat(se2conv_plan_s* p, int shape_idx, int n_knots, double r_max, double2* tmp,
                                hipStream_t stream) {
    se2conv_status r = ensure_profile_basis(p, shape_idx, n_knots, r_max, stream);
    if (r != SE2CONV_OK) return r;
    if (p->bh_shape == shape_idx && p->bh_knots == n_knots && p->bh_rmax == r_max) return SE2CONV_OK;
    const se2conv_shape& s = p->shapes[shape_idx];
    const size_t need = sizeof(double) * (size_t)((long long)(s.nx / 2 + 1) * (s.ny / 2 + 1) * n_knots);
    if (p->basis_hat_bytes < need) {
        if (p->basis_hat) {
            hipError_t e = hipFree(p->basis_hat);
            p->basis_hat = nullptr;
            p->basis_hat_bytes = 0;
            if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "hipFree: %s", hipGetErrorString(e));
        }
        if (hipMalloc(reinterpret_cast<void**>(&p->basis_hat), need) != hipSuccess)
            return fail(SE2CONV_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes for the basis spectrum", need);
        p->basis_hat_bytes = need;
    }
    HIPCHK(launch_basis_dft(p->basis, reinterpret_cast<const double2*>(tw_of(p, s.nx, true)),
                            reinterpret_cast<const double2*>(tw_of(p, s.ny, true)), n_knots, s.nx, s.ny, tmp,
                            p->basis_hat, stream));
    p->bh_shape = shape_idx;
    p->bh_knots = n_knots;
    p->bh_rmax = r_max;
    return SE2CONV_OK;
}

// The knot contraction applies when its per-k3 sums fit the fold kernel.
bool profile_by_basis(const se2conv_shape& s, int n_knots) {
    return s.m <= kProfileFoldMaxM && n_knots <= kProfileFoldMaxM;
}

extern "C" {

se2conv_status se2conv_pass_times(se2conv_plan_t p, float* ms, int32_t* kinds, int32_t cap, int32_t* n) {
    if (!p || !n || cap < 0 || (cap > 0 && (!ms || !kinds))) return fail(SE2CONV_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> g(p->mu);
    *n = (int32_t)p->ev_kind.size();
    if (!p->ev_rec.empty()) {
        HIPCHK(hipEventSynchronize(p->ev_rec.back()));
        // events are grouped per submission: each submission starts with an extra
        // event, so walk the records and pair every pass with the event before it.
        size_t k = 0;
        for (size_t i = 1; i < p->ev_rec.size() && k < p->ev_kind.size(); ++i) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, p->ev_rec[i - 1], p->ev_rec[i]));
            if (p->ev_sub_start.count(i)) continue;
            if ((int32_t)k < cap) {
                ms[k] = t;
                kinds[k] = p->ev_kind[k];
            }
            ++k;
        }
    }
    for (auto ev : p->ev_rec) p->ev_pool.push_back(ev);
    p->ev_rec.clear();
    p->ev_kind.clear();
    p->ev_sub_start.clear();
    return ok();
}

const char* se2conv_status_string(se2conv_status s) {
    switch (s) {
        case SE2CONV_OK: return "ok";
        case SE2CONV_ERR_INVALID_ARG: return "invalid argument";
        case SE2CONV_ERR_UNSUPPORTED_SIZE: return "unsupported size";
        case SE2CONV_ERR_OUT_OF_MEMORY: return "out of device memory";
        case SE2CONV_ERR_DEVICE: return "device error";
        case SE2CONV_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* se2conv_last_error(void) { return g_last_error.c_str(); }

se2conv_status se2conv_plan(const se2conv_shape* shapes, int32_t n_shapes, se2conv_dtype dtype, uint32_t flags,
                            se2conv_plan_t* out) {
    if (!out) return fail(SE2CONV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!shapes || n_shapes < 1 || n_shapes > 4096)
        return fail(SE2CONV_ERR_INVALID_ARG, "need 1..4096 shapes");
    if (dtype != SE2CONV_F32 && dtype != SE2CONV_F64) return fail(SE2CONV_ERR_INVALID_ARG, "bad dtype %d", (int)dtype);
    if (flags & ~(SE2CONV_PLAN_HOST_ONLY | SE2CONV_PLAN_GENERIC))
        return fail(SE2CONV_ERR_INVALID_ARG, "unknown plan flags 0x%x", flags);
    for (int i = 0; i < n_shapes; ++i) {
        std::string why;
        if (!shape_supported(shapes[i], &why))
            return fail(SE2CONV_ERR_UNSUPPORTED_SIZE, "shape %d (%d x %d x %d): %s", i, shapes[i].nx, shapes[i].ny,
                        shapes[i].m, why.c_str());
    }
    auto* p = new se2conv_plan_s();
    p->dtype = dtype;
    p->flags = flags;
    p->shapes.assign(shapes, shapes + n_shapes);
    p->sched.assign(n_shapes, default_schedule(dtype == SE2CONV_F64));
    load_tune_cache(p);
    if (flags & SE2CONV_PLAN_HOST_ONLY) {
        p->host_only = true;
        *out = p;
        return ok();
    }
    auto cleanup = [&](se2conv_status st) {
        se2conv_plan_destroy(p);
        return st;
    };
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return cleanup(fail(SE2CONV_ERR_DEVICE, "no HIP device available"));
    if (hipGetDevice(&p->device) != hipSuccess) return cleanup(fail(SE2CONV_ERR_DEVICE, "hipGetDevice failed"));
    {
        const se2conv_status sr = noalloc_scratch_setup(p->device);
        if (sr != SE2CONV_OK) return cleanup(sr);
    }
    if (hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
        p->num_cus < 1)
        return cleanup(fail(SE2CONV_ERR_DEVICE, "could not query the compute-unit count"));
    // twiddles for every distinct length, generated in FP64
    std::vector<int> lens;
    size_t maxn = 0;
    for (auto& s : p->shapes) {
        lens.push_back(s.nx);
        lens.push_back(s.ny);
        lens.push_back(s.m);
        maxn = std::max(maxn, (size_t)s.nx * s.ny * s.m);
    }
    std::sort(lens.begin(), lens.end());
    lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
    for (int L : lens) {
        void* t64 = nullptr;
        void* t32 = nullptr;
        if (hipMalloc(&t64, sizeof(double2) * L) != hipSuccess)
            return cleanup(fail(SE2CONV_ERR_OUT_OF_MEMORY, "twiddle allocation"));
        p->tw64[L] = t64;
        if (hipMalloc(&t32, sizeof(float2) * L) != hipSuccess)
            return cleanup(fail(SE2CONV_ERR_OUT_OF_MEMORY, "twiddle allocation"));
        p->tw32[L] = t32;
        if (launch_twiddles((double2*)t64, (float2*)t32, L, nullptr) != hipSuccess)
            return cleanup(fail(SE2CONV_ERR_DEVICE, "twiddle generation launch failed"));
        if (make_radix_plan(L).rader) {
            std::vector<unsigned char> h64, h32;
            rader_tables(L, h64, h32);
            void* r64 = nullptr;
            void* r32 = nullptr;
            if (hipMalloc(&r64, h64.size()) != hipSuccess)
                return cleanup(fail(SE2CONV_ERR_OUT_OF_MEMORY, "Rader table allocation"));
            p->rader64[L] = r64;
            if (hipMalloc(&r32, h32.size()) != hipSuccess)
                return cleanup(fail(SE2CONV_ERR_OUT_OF_MEMORY, "Rader table allocation"));
            p->rader32[L] = r32;
            if (hipMemcpy(r64, h64.data(), h64.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(r32, h32.data(), h32.size(), hipMemcpyHostToDevice) != hipSuccess)
                return cleanup(fail(SE2CONV_ERR_DEVICE, "Rader table upload failed"));
        }
    }
    if (prepare_kernels() != hipSuccess) return cleanup(fail(SE2CONV_ERR_DEVICE, "kernel attribute setup failed"));
    p->ws_bytes = maxn * real_bytes(p);
    if (hipMalloc(&p->ws, p->ws_bytes) != hipSuccess)
        return cleanup(fail(SE2CONV_ERR_OUT_OF_MEMORY, "workspace allocation (%zu bytes)", p->ws_bytes));
    if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(SE2CONV_ERR_DEVICE, "plan synchronisation failed"));
    *out = p;
    return ok();
}

se2conv_status se2conv_plan_destroy(se2conv_plan_t p) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (!p->host_only) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (p->device >= 0) (void)hipSetDevice(p->device);
        (void)hipDeviceSynchronize();
        p->subs.clear();
        for (auto ev : p->ev_pool) (void)hipEventDestroy(ev);
        for (auto st : p->aux) (void)hipStreamDestroy(st);
        for (auto ev : p->ev_join) (void)hipEventDestroy(ev);
        if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
        for (auto ev : p->ev_rec) (void)hipEventDestroy(ev);
        for (auto& kv : p->tw32) (void)hipFree(kv.second);
        for (auto& kv : p->tw64) (void)hipFree(kv.second);
        for (auto& kv : p->rader32) (void)hipFree(kv.second);
        for (auto& kv : p->rader64) (void)hipFree(kv.second);
        if (p->ws) (void)hipFree(p->ws);
        if (p->ws2) (void)hipFree(p->ws2);
        if (p->ws4) (void)hipFree(p->ws4);
        if (p->scratch64) (void)hipFree(p->scratch64);
        if (p->sum64) (void)hipFree(p->sum64);
        if (p->qstat) (void)hipFree(p->qstat);
        if (p->basis) (void)hipFree(p->basis);
        if (p->basis_hat) (void)hipFree(p->basis_hat);
        if (p->pad_ws) (void)hipFree(p->pad_ws);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    delete p;
    return SE2CONV_OK;  // keeps the thread's last error (plan creation cleans up through here)
}

namespace {

// Checks a kernel list; *sep tells whether every kernel is GAUSS_VM (a SEPARABLE chain).
se2conv_status validate_kernels(const se2conv_kernel_desc* kernels, int32_t n_kernels, bool* sep_out) {
    bool sep = true;
    for (int j = 0; j < n_kernels; ++j) {
        const se2conv_kernel_desc& k = kernels[j];
        const uint32_t norm = k.flags & 3u;
        if (k.flags & ~3u) return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: unknown flags 0x%x", j, k.flags);
        if (norm == 3u) return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: bad normalisation", j);
        switch (k.kind) {
            case SE2CONV_K_GAUSS_VM:
                if (!(k.sigma > 0.0) || !std::isfinite(k.sigma) || !(k.kappa >= 0.0) || !std::isfinite(k.kappa) ||
                    k.kappa > 700.0 || !std::isfinite(k.theta0))
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: need sigma > 0, 0 <= kappa <= 700", j);
                break;
            case SE2CONV_K_SAMPLES:
                sep = false;
                if (!k.data) return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: samples pointer is null", j);
                if (norm == SE2CONV_KNORM_CONTINUOUS)
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: continuous normalisation needs GAUSS_VM", j);
                break;
            case SE2CONV_K_RADIAL_PROFILE:
                sep = false;
                if (!k.data) return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: profile pointer is null", j);
                if (k.n_knots < 2 || k.n_knots > 4096)
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: n_knots must lie in [2, 4096]", j);
                if (!(k.r_max > 0.0) || !(k.r_max <= 1.0))
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: r_max must lie in (0, 1]", j);
                if (norm == SE2CONV_KNORM_CONTINUOUS)
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: continuous normalisation needs GAUSS_VM", j);
                break;
            case SE2CONV_K_EXP_GAUSS:
                sep = false;
                if (!(k.sigma > 0.0) || !std::isfinite(k.sigma))
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: need finite sigma > 0", j);
                if (norm == SE2CONV_KNORM_CONTINUOUS)
                    return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: continuous normalisation needs GAUSS_VM", j);
                break;
            default:
                return fail(SE2CONV_ERR_INVALID_ARG, "kernel %d: unknown kind %d", j, k.kind);
        }
    }
    *sep_out = sep;
    return SE2CONV_OK;
}

// FP64 scratch of se2conv_coeffs for one shape: separable accumulator | full accumulator
// n | spectrum re n | im n | samples n (re .. samples also serve as the basis-DFT
// temporary of a radial profile).
struct CoeffScratch {
    double2* sepacc;
    double2* full;
    double* re;
    double* im;
    double* samp;
};

se2conv_status coeff_scratch(se2conv_plan_s* p, const se2conv_shape& s, const se2conv_kernel_desc* kernels,
                             int32_t n_kernels, bool sep, CoeffScratch* cs) {
    const long long n = (long long)s.nx * s.ny * s.m;
    const int nsep = s.nx + s.ny + s.m;
    size_t need = sizeof(double2) * nsep + (sep ? 0 : (sizeof(double2) * n + 3 * sizeof(double) * n));
    for (int j = 0; j < n_kernels && !sep; ++j)
        if (kernels[j].kind == SE2CONV_K_RADIAL_PROFILE && profile_by_basis(s, kernels[j].n_knots))
            need = std::max(need, sizeof(double2) * (nsep + (size_t)n) +
                                      sizeof(double2) * (size_t)((long long)kernels[j].n_knots * s.ny * (s.nx / 2 + 1)));
    se2conv_status r = ensure_scratch64(p, need);
    if (r != SE2CONV_OK) return r;
    cs->sepacc = reinterpret_cast<double2*>(p->scratch64);
    cs->full = cs->sepacc + nsep;
    cs->re = reinterpret_cast<double*>(cs->full + n);
    cs->im = cs->re + n;
    cs->samp = cs->im + n;
    return SE2CONV_OK;
}

// Multiplies the FULL FP64 accumulator by the coefficients of one kernel (first: sets it).
se2conv_status fold_kernel_full(se2conv_plan_s* p, int32_t shape_idx, const se2conv_kernel_desc& k,
                                const CoeffScratch& cs, bool first, hipStream_t stream) {
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long n = (long long)s.nx * s.ny * s.m;
    const int norm = (int)(k.flags & 3u);
    if (k.kind == SE2CONV_K_GAUSS_VM) {
        SepKernelParams kp;
        kp.sigma = k.sigma;
        kp.kappa = k.kappa;
        kp.theta0 = k.theta0;
        kp.ive0 = std::cyl_bessel_i(0.0, k.kappa) * std::exp(-k.kappa);
        kp.norm = norm;
        HIPCHK(launch_sep_factor(kp, s.nx, s.ny, s.m, cs.sepacc, 1, stream));
        HIPCHK(launch_full_fold_sep(cs.sepacc, cs.full, n, s.nx, s.ny, first, stream));
    } else if (k.kind == SE2CONV_K_RADIAL_PROFILE && profile_by_basis(s, k.n_knots)) {
        // P^ = sum_q prof^[q] H_q^ with the basis spectrum cached per geometry
        auto* tmp = reinterpret_cast<double2*>(cs.re);
        se2conv_status rb = ensure_basis_hat(p, shape_idx, k.n_knots, k.r_max, tmp, stream);
        if (rb != SE2CONV_OK) return rb;
        HIPCHK(launch_profile_fold(reinterpret_cast<const double*>(k.data),
                                   reinterpret_cast<const double2*>(tw_of(p, s.m, true)), p->basis_hat, k.n_knots,
                                   s.nx, s.ny, s.m, norm == 0 ? 0 : 1, tmp, cs.full, first, stream));
    } else {
        const double* src = reinterpret_cast<const double*>(k.data);
        if (k.kind == SE2CONV_K_RADIAL_PROFILE) {
            HIPCHK(launch_profile_samples(src, k.n_knots, k.r_max, s.nx, s.ny, s.m, cs.samp, stream));
            src = cs.samp;
        } else if (k.kind == SE2CONV_K_EXP_GAUSS) {
            HIPCHK(launch_exp_gauss_samples(k.sigma, s.nx, s.ny, s.m, cs.samp, stream));
            src = cs.samp;
        }
        // FP64 forward 3-D DFT of the real samples into (re, im) planes
        HIPCHK(xt_transform(p, s, true, 0, src, nullptr, cs.re, cs.im, nullptr, nullptr, n, n, 1, stream));
        HIPCHK(y_pass(p, s, true, cs.re, cs.im, nullptr, n, 1, 1, 0, 0, nullptr, false, 1.0, stream));
        HIPCHK(launch_full_fold(cs.re, cs.im, cs.full, n, s.nx, s.ny, norm == 0 ? 0 : 1, first, stream));
    }
    return SE2CONV_OK;
}

}  // namespace

se2conv_status se2conv_coeffs(se2conv_plan_t p, int32_t shape_idx, const se2conv_kernel_desc* kernels,
                              int32_t n_kernels, void* d_table, size_t* table_bytes, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (!kernels || n_kernels < 1 || n_kernels > 64) return fail(SE2CONV_ERR_INVALID_ARG, "need 1..64 kernels");
    if (!table_bytes) return fail(SE2CONV_ERR_INVALID_ARG, "table_bytes is null");
    const se2conv_shape& s = p->shapes[shape_idx];
    bool sep = true;
    se2conv_status vr = validate_kernels(kernels, n_kernels, &sep);
    if (vr != SE2CONV_OK) return vr;
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t cb = cplx_bytes(p);
    const size_t bytes = sep ? cb * (size_t)(s.nx + s.ny + s.m) : cb * (size_t)n;
    if (!d_table) {
        *table_bytes = bytes;
        return ok();
    }
    if (*table_bytes < bytes) return fail(SE2CONV_ERR_INVALID_ARG, "table buffer too small (%zu < %zu)", *table_bytes, bytes);
    if (!aligned16(d_table)) return fail(SE2CONV_ERR_INVALID_ARG, "table must be 16-byte aligned");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");

    std::lock_guard<std::mutex> g(p->mu);
    const int nsep = s.nx + s.ny + s.m;
    CoeffScratch cs;
    se2conv_status r = coeff_scratch(p, s, kernels, n_kernels, sep, &cs);
    if (r != SE2CONV_OK) return r;
    for (int j = 0; j < n_kernels; ++j) {
        const se2conv_kernel_desc& k = kernels[j];
        if (sep) {
            SepKernelParams kp;
            kp.sigma = k.sigma;
            kp.kappa = k.kappa;
            kp.theta0 = k.theta0;
            kp.ive0 = std::cyl_bessel_i(0.0, k.kappa) * std::exp(-k.kappa);
            kp.norm = (int)(k.flags & 3u);
            HIPCHK(launch_sep_factor(kp, s.nx, s.ny, s.m, cs.sepacc, j == 0, stream));
        } else {
            r = fold_kernel_full(p, shape_idx, k, cs, j == 0, stream);
            if (r != SE2CONV_OK) return r;
        }
    }
    HIPCHK(launch_round(sep ? cs.sepacc : cs.full, d_table, sep ? nsep : n, dbl(p) ? 1 : 0, stream));
    TableRec rec;
    rec.shape_idx = shape_idx;
    rec.kind = sep ? SE2CONV_TABLE_SEPARABLE : SE2CONV_TABLE_FULL;
    rec.bytes = bytes;
    register_table(p, d_table, rec);
    return ok();
}

se2conv_status se2conv_coeffs_sum(se2conv_plan_t p, int32_t shape_idx, const se2conv_kernel_desc* kernels,
                                  const double* weights, int32_t n_terms, void* d_table, size_t* table_bytes,
                                  hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (!kernels || !weights || n_terms < 1 || n_terms > 64)
        return fail(SE2CONV_ERR_INVALID_ARG, "need 1..64 kernels and their weights");
    if (!table_bytes) return fail(SE2CONV_ERR_INVALID_ARG, "table_bytes is null");
    for (int j = 0; j < n_terms; ++j)
        if (!std::isfinite(weights[j])) return fail(SE2CONV_ERR_INVALID_ARG, "weight %d is not finite", j);
    const se2conv_shape& s = p->shapes[shape_idx];
    bool sep = true;
    se2conv_status vr = validate_kernels(kernels, n_terms, &sep);
    if (vr != SE2CONV_OK) return vr;
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t bytes = cplx_bytes(p) * (size_t)n;  // a sum of kernels is FULL
    if (!d_table) {
        *table_bytes = bytes;
        return ok();
    }
    if (*table_bytes < bytes) return fail(SE2CONV_ERR_INVALID_ARG, "table buffer too small (%zu < %zu)", *table_bytes, bytes);
    if (!aligned16(d_table)) return fail(SE2CONV_ERR_INVALID_ARG, "table must be 16-byte aligned");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");

    std::lock_guard<std::mutex> g(p->mu);
    CoeffScratch cs;
    se2conv_status r = coeff_scratch(p, s, kernels, n_terms, false, &cs);
    if (r != SE2CONV_OK) return r;
    if (p->sum64_bytes < sizeof(double2) * (size_t)n) {
        if (p->sum64) {
            hipError_t e = hipFree(p->sum64);
            p->sum64 = nullptr;
            p->sum64_bytes = 0;
            if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "hipFree: %s", hipGetErrorString(e));
        }
        if (hipMalloc(&p->sum64, sizeof(double2) * (size_t)n) != hipSuccess)
            return fail(SE2CONV_ERR_OUT_OF_MEMORY, "FP64 sum accumulator (%zu bytes)", sizeof(double2) * (size_t)n);
        p->sum64_bytes = sizeof(double2) * (size_t)n;
    }
    auto* sum = reinterpret_cast<double2*>(p->sum64);
    for (int j = 0; j < n_terms; ++j) {
        r = fold_kernel_full(p, shape_idx, kernels[j], cs, true, stream);
        if (r != SE2CONV_OK) return r;
        HIPCHK(launch_axpy64(cs.full, sum, n, weights[j], j == 0 ? 1 : 0, stream));
    }
    HIPCHK(launch_round(sum, d_table, n, dbl(p) ? 1 : 0, stream));
    TableRec rec;
    rec.shape_idx = shape_idx;
    rec.kind = SE2CONV_TABLE_FULL;
    rec.bytes = bytes;
    register_table(p, d_table, rec);
    return ok();
}

se2conv_status se2conv_field_coeffs(se2conv_plan_t p, int32_t shape_idx, const void* d_f, int32_t batch,
                                    void* d_tables, size_t table_stride, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (batch < 1) return fail(SE2CONV_ERR_INVALID_ARG, "batch must be >= 1");
    if (!d_f || !d_tables || !aligned16(d_f) || !aligned16(d_tables))
        return fail(SE2CONV_ERR_INVALID_ARG, "d_f and d_tables must be non-null and 16-byte aligned");
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t tbytes = cplx_bytes(p) * (size_t)n;
    if (table_stride < tbytes || (table_stride & 15u))
        return fail(SE2CONV_ERR_INVALID_ARG, "table_stride must be >= %zu and a multiple of 16", tbytes);
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const bool d = dbl(p);
    {
        std::lock_guard<std::mutex> g(p->mu);
        if (!p->ws2) {
            if (hipMalloc(&p->ws2, 2 * p->ws_bytes) != hipSuccess)
                return fail(SE2CONV_ERR_OUT_OF_MEMORY, "field-table workspace (%zu bytes)", 2 * p->ws_bytes);
        }
    }
    void* zre = p->ws2;
    void* zim = (char*)p->ws2 + p->ws_bytes;
    const size_t rb = real_bytes(p);
    for (int b = 0; b < batch; b += 2) {
        const void* fa = (const char*)d_f + rb * n * b;
        const void* fb = (b + 1 < batch) ? (const char*)d_f + rb * n * (b + 1) : nullptr;
        // complex 3-D DFT of z = f_a + i f_b into the (re, im) workspace planes
        HIPCHK(xt_transform(p, s, d, 0, fa, fb, zre, zim, nullptr, nullptr, n, n, 1, stream));
        HIPCHK(y_pass(p, s, d, zre, zim, nullptr, n, 1, 1, 0, 0, nullptr, false, 1.0, stream));
        void* ta = (char*)d_tables + table_stride * b;
        void* tb = fb ? (char*)d_tables + table_stride * (b + 1) : nullptr;
        HIPCHK(launch_unpack_tables(zre, zim, ta, tb, s.nx, s.ny, s.m, d, stream));
    }
    std::lock_guard<std::mutex> g(p->mu);
    for (int b = 0; b < batch; ++b) {
        TableRec rec;
        rec.shape_idx = shape_idx;
        rec.kind = SE2CONV_TABLE_FULL;
        rec.bytes = tbytes;
        register_table(p, (char*)d_tables + table_stride * b, rec);
    }
    return ok();
}

se2conv_status se2conv_kernel_grad(se2conv_plan_t p, int32_t shape_idx, const void* d_g, const void* d_ftables,
                                   size_t table_stride, int32_t batch, void* d_grad, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (batch < 1 || !d_g || !d_ftables || !d_grad || !aligned16(d_g) || !aligned16(d_grad))
        return fail(SE2CONV_ERR_INVALID_ARG, "need batch >= 1 and aligned device pointers");
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t tbytes = cplx_bytes(p) * (size_t)n;
    if (table_stride < tbytes || (table_stride & 15u))
        return fail(SE2CONV_ERR_INVALID_ARG, "table_stride must be >= %zu and a multiple of 16", tbytes);
    {
        std::lock_guard<std::mutex> g(p->mu);
        for (int b = 0; b < batch; ++b) {
            auto it = p->tables.find(reinterpret_cast<uintptr_t>((const char*)d_ftables + table_stride * b));
            if (it == p->tables.end() || it->second.shape_idx != shape_idx || it->second.kind != SE2CONV_TABLE_FULL)
                return fail(SE2CONV_ERR_INVALID_ARG, "field table %d was not produced by this plan for this shape", b);
        }
    }
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const bool d = dbl(p);
    {
        std::lock_guard<std::mutex> g(p->mu);
        if (!p->ws4 && hipMalloc(&p->ws4, 4 * p->ws_bytes) != hipSuccess)
            return fail(SE2CONV_ERR_OUT_OF_MEMORY, "kernel-gradient workspace (%zu bytes)", 4 * p->ws_bytes);
    }
    const size_t rb = real_bytes(p);
    void* zre = p->ws4;
    void* zim = (char*)p->ws4 + p->ws_bytes;
    void* are = (char*)p->ws4 + 2 * p->ws_bytes;
    void* aim = (char*)p->ws4 + 3 * p->ws_bytes;
    for (int b = 0; b < batch; b += 2) {
        const void* ga = (const char*)d_g + rb * n * b;
        const void* gb = (b + 1 < batch) ? (const char*)d_g + rb * n * (b + 1) : nullptr;
        HIPCHK(xt_transform(p, s, d, 0, ga, gb, zre, zim, nullptr, nullptr, n, n, 1, stream));
        HIPCHK(y_pass(p, s, d, zre, zim, nullptr, n, 1, 1, 0, 0, nullptr, false, 1.0, stream));
        const void* ta = (const char*)d_ftables + table_stride * b;
        const void* tb = gb ? (const char*)d_ftables + table_stride * (b + 1) : nullptr;
        HIPCHK(launch_accumulate_pair(zre, zim, ta, tb, are, aim, s.nx, s.ny, s.m, 1.0 / (double)n, b == 0, d, stream));
    }
    // inverse of the accumulated (Hermitian) spectrum; the imaginary part is rounding only
    HIPCHK(y_pass(p, s, d, are, aim, nullptr, n, 1, /*fwd=*/0, /*inv=*/1, /*mul=*/0, nullptr, false, 1.0, stream));
    HIPCHK(xt_transform(p, s, d, 1, are, aim, d_grad, nullptr, nullptr, nullptr, n, n, 1, stream));
    return ok();
}

se2conv_status se2conv_profile_grad(se2conv_plan_t p, int32_t shape_idx, const void* d_grad_samples, int32_t batch,
                                    int32_t n_knots, double r_max, double* d_grad_prof, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (batch < 1 || !d_grad_samples || !d_grad_prof)
        return fail(SE2CONV_ERR_INVALID_ARG, "need batch >= 1 and non-null device pointers");
    if (n_knots < 2 || n_knots > 4096 || !(r_max > 0.0) || !(r_max <= 1.0))
        return fail(SE2CONV_ERR_INVALID_ARG, "need 2 <= n_knots <= 4096 and 0 < r_max <= 1");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long npts = (long long)s.nx * s.ny;
    std::lock_guard<std::mutex> g(p->mu);
    {
        se2conv_status rb = ensure_profile_basis(p, shape_idx, n_knots, r_max, stream);
        if (rb != SE2CONV_OK) return rb;
    }
    const long long nsplit = profile_grad_splits(npts);
    se2conv_status r = ensure_scratch64(p, sizeof(double) * (size_t)(npts * s.m + nsplit * n_knots * s.m));
    if (r != SE2CONV_OK) return r;
    double* G = reinterpret_cast<double*>(p->scratch64);
    double* part = G + npts * s.m;
    HIPCHK(launch_profile_grad(d_grad_samples, batch, dbl(p), n_knots, s.nx, s.ny, s.m, p->basis, G, part, d_grad_prof,
                               stream));
    return ok();
}

se2conv_status se2conv_autotune(se2conv_plan_t p, int32_t shape_idx, int32_t batch, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (batch < 1 || batch > 4096) return fail(SE2CONV_ERR_INVALID_ARG, "batch must lie in [1, 4096]");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const se2conv_shape s = p->shapes[shape_idx];
    const size_t bytes = real_bytes(p) * (size_t)batch * s.nx * s.ny * s.m;
    void* f = nullptr;
    void* out = nullptr;
    void* tab = nullptr;
    if (hipMalloc(&f, bytes) != hipSuccess) return fail(SE2CONV_ERR_OUT_OF_MEMORY, "autotune buffers");
    auto release = [&]() {
        (void)hipStreamSynchronize(stream);
        if (f) (void)hipFree(f);
        if (out) (void)hipFree(out);
        if (tab) (void)hipFree(tab);
    };
    if (hipMalloc(&out, bytes) != hipSuccess) {
        release();
        return fail(SE2CONV_ERR_OUT_OF_MEMORY, "autotune buffers");
    }
    se2conv_kernel_desc k{};
    k.kind = SE2CONV_K_GAUSS_VM;
    k.sigma = 0.05;
    k.kappa = 4.0;
    size_t tb = 0;
    se2conv_status r = se2conv_coeffs(p, shape_idx, &k, 1, nullptr, &tb, stream);
    if (r == SE2CONV_OK && hipMalloc(&tab, tb) != hipSuccess) r = fail(SE2CONV_ERR_OUT_OF_MEMORY, "autotune table");
    if (r == SE2CONV_OK) r = se2conv_coeffs(p, shape_idx, &k, 1, tab, &tb, stream);
    if (r == SE2CONV_OK && hipMemsetAsync(f, 0, bytes, stream) != hipSuccess)
        r = fail(SE2CONV_ERR_DEVICE, "autotune fill");
    if (r != SE2CONV_OK) {
        release();
        return r;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release();
        return fail(SE2CONV_ERR_DEVICE, "event creation");
    }
    // only the knobs this shape's schedule uses are varied
    const bool d = dbl(p);
    const bool generic = d || (p->flags & SE2CONV_PLAN_GENERIC) != 0;
    const bool two_pass = slab_fits(s, d);
    // register kernels: persistent pencils (blocks per CU); generic kernels: pencil
    // width and, without the slab, x-row tile size
    const bool fast_lines = !generic && (two_pass ? pencil_fast_supported(s.nx, s.ny)
                                                  : three_pass_fast_supported(s.nx, s.ny, s.m));
    const Schedule dflt = default_schedule(d);
    std::vector<int> widths = {dflt.pencil_w}, blocks = {dflt.fast_blocks_per_cu}, xrows = {dflt.xrow_points};
    if (fast_lines) blocks = {2, 4, 8};
    else widths = {4, 8, 16, 32};
    if (!two_pass && !fast_lines) xrows = {1024, 2048, 4096, 8192};
    Schedule best = p->sched[shape_idx];
    float best_ms = 1e30f;
    for (int w : widths)
        for (int b : blocks)
            for (int x : xrows) {
                Schedule c;
                c.pencil_w = w;
                c.fast_blocks_per_cu = b;
                c.xrow_points = x;
                p->sched[shape_idx] = c;
                float ms = 0.f;
                bool okrun = true;
                for (int rep = 0; rep < 2 && okrun; ++rep) okrun = se2conv_apply(p, shape_idx, f, tab, out, batch, 0, stream) == SE2CONV_OK;
                okrun = okrun && hipEventRecord(e0, stream) == hipSuccess;
                for (int rep = 0; rep < 5 && okrun; ++rep) okrun = se2conv_apply(p, shape_idx, f, tab, out, batch, 0, stream) == SE2CONV_OK;
                okrun = okrun && hipEventRecord(e1, stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                        hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (okrun && ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> g(p->mu);
        purge_subs_naming(p, reinterpret_cast<uintptr_t>(tab));
        p->tables.erase(reinterpret_cast<uintptr_t>(tab));
    }
    release();
    best.tuned = true;
    p->sched[shape_idx] = best;
    append_tune_cache(p, shape_idx);
    return ok();
}

se2conv_status se2conv_sample_bumps(se2conv_plan_t p, int32_t shape_idx, const double* d_params, int32_t n_bumps,
                                    double s, double kappa, void* d_out, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (!d_params || !d_out || n_bumps < 1 || n_bumps > (1 << 20))
        return fail(SE2CONV_ERR_INVALID_ARG, "need device pointers and 1 <= n_bumps <= 2^20");
    if (!(s > 0.0) || !std::isfinite(s) || !(kappa >= 0.0) || kappa > 700.0)
        return fail(SE2CONV_ERR_INVALID_ARG, "need s > 0 and 0 <= kappa <= 700");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const se2conv_shape& sh = p->shapes[shape_idx];
    std::lock_guard<std::mutex> g(p->mu);
    se2conv_status r = ensure_scratch64(p, sizeof(double) * (size_t)n_bumps * (sh.nx + sh.ny + sh.m));
    if (r != SE2CONV_OK) return r;
    HIPCHK(launch_sample_bumps(d_params, n_bumps, s, kappa, sh.nx, sh.ny, sh.m,
                               reinterpret_cast<double*>(p->scratch64), d_out, dbl(p), stream));
    return ok();
}

se2conv_status se2conv_powers(se2conv_plan_t p, int32_t shape_idx, const void* d_f, const void* d_table, int32_t q,
                              void* d_out, int32_t batch, uint32_t flags, hipStream_t stream) {
    if (q < 1 || q > 4096) return fail(SE2CONV_ERR_INVALID_ARG, "q must lie in [1, 4096]");
    se2conv_status r = validate_io(p, shape_idx, d_f, d_out, batch);
    if (r != SE2CONV_OK) return r;
    if (flags & ~SE2CONV_ADJOINT) return fail(SE2CONV_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t rb = real_bytes(p);
    {
        const char* a = (const char*)d_f;
        const char* b = (const char*)d_out;
        const long long fb = (long long)batch * n * (long long)rb, ob = fb * q;
        if (a < b + ob && b < a + fb) return fail(SE2CONV_ERR_INVALID_ARG, "d_out must not overlap d_f");
    }
    Chain ch;
    bool all_sep = true;
    const void* tabs[1] = {d_table};
    r = lookup_chain(p, shape_idx, tabs, 1, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const bool d = dbl(p);
    const bool conj = (flags & SE2CONV_ADJOINT) != 0;
    const bool odd = (batch & 1) != 0;
    if (use_full_fast(p, s) && !odd && (long long)batch * q * s.ny / 2 < (1LL << 31)) {
        // register kernels: x-theta forward into the last slot, one y pass for every power
        // (the spectrum stays in registers), one x-theta inverse over all q slots
        FullFastArgs a = full_fast_args(p, s, batch);
        set_chain(&a, ch, conj, 1.0 / (double)n);
        char* last = (char*)d_out + rb * ((long long)(q - 1) * batch * n);
        a.in = reinterpret_cast<const float*>(d_f);
        a.out = reinterpret_cast<float*>(last);
        HIPCHK(launch_xt_full_fwd(a, stream));
        a.out = reinterpret_cast<float*>(d_out);
        a.q = q;
        a.slot = (long long)batch * n;
        HIPCHK(launch_y_full_powers(a, stream));
        FullFastArgs b = full_fast_args(p, s, batch * q);
        b.in = reinterpret_cast<const float*>(d_out);
        b.out = reinterpret_cast<float*>(d_out);
        HIPCHK(launch_xt_full_inv(b, stream));
        return ok();
    }
    const int pairs = (batch + 1) / 2;
    if (odd) {
        std::lock_guard<std::mutex> g(p->mu);
        if (!p->ws2 && hipMalloc(&p->ws2, 2 * p->ws_bytes) != hipSuccess)
            return fail(SE2CONV_ERR_OUT_OF_MEMORY, "workspace (%zu bytes)", 2 * p->ws_bytes);
    }
    const long long slot = (long long)batch * n;  // elements per output slot
    auto slot_re = [&](int k) { return (char*)d_out + rb * (slot * k); };
    auto slot_im = [&](int k) { return batch == 1 ? nullptr : (char*)d_out + rb * (slot * k + n); };
    const void* f_im = batch == 1 ? nullptr : (const char*)d_f + rb * n;
    void* spec_lone = odd ? p->ws : nullptr;    // imaginary plane of the lone field's spectrum
    void* step_lone = odd ? p->ws2 : nullptr;   // imaginary plane of its per-step inverse
    char* S_re = slot_re(q - 1);
    char* S_im = slot_im(q - 1);
    // forward: H_0 = F^ (pairs of fields packed as re/im), stored in the last slot
    HIPCHK(xt_transform(p, s, d, 0, d_f, f_im, S_re, S_im, nullptr, spec_lone, 2 * n, 2 * n, pairs, stream));
    HIPCHK(y_pass_io(p, s, d, S_re, S_im, S_re, S_im, spec_lone, spec_lone, 2 * n, pairs, 1, 0, 0, nullptr, false,
                     1.0, stream));
    for (int k = 1; k <= q; ++k) {
        // running product H_k = H_{k-1} . rho^  (the iDFT's 1/n is folded in once, at k = 1)
        HIPCHK(y_pass_io(p, s, d, S_re, S_im, S_re, S_im, spec_lone, spec_lone, 2 * n, pairs, 0, 0, 2, &ch, conj,
                         k == 1 ? 1.0 / (double)n : 1.0, stream));
        // inverse into slot k-1 (the last step inverts the running spectrum in place)
        char* O_re = slot_re(k - 1);
        char* O_im = slot_im(k - 1);
        void* o_lone = k == q ? spec_lone : step_lone;
        HIPCHK(y_pass_io(p, s, d, S_re, S_im, O_re, O_im, spec_lone, o_lone, 2 * n, pairs, 0, 1, 0, nullptr, false,
                         1.0, stream));
        HIPCHK(xt_transform(p, s, d, 1, O_re, O_im, O_re, O_im, o_lone, nullptr, 2 * n, 2 * n, pairs, stream));
    }
    return ok();
}

se2conv_status se2conv_table_info(se2conv_plan_t p, const void* d_table, int32_t* kind, int32_t* shape_idx,
                                  size_t* bytes) {
    if (!p || !d_table) return fail(SE2CONV_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->tables.find(reinterpret_cast<uintptr_t>(d_table));
    if (it == p->tables.end()) return fail(SE2CONV_ERR_INVALID_ARG, "table was not produced by this plan");
    if (kind) *kind = it->second.kind;
    if (shape_idx) *shape_idx = it->second.shape_idx;
    if (bytes) *bytes = it->second.bytes;
    return ok();
}

se2conv_status se2conv_table_quarter(se2conv_plan_t p, const void* d_full, void* d_quarter, size_t* quarter_bytes,
                                     hipStream_t stream) {
    if (!p || !d_full || !quarter_bytes) return fail(SE2CONV_ERR_INVALID_ARG, "null argument");
    int shape_idx = -1;
    size_t full_bytes = 0;
    {
        std::lock_guard<std::mutex> g(p->mu);
        auto it = p->tables.find(reinterpret_cast<uintptr_t>(d_full));
        if (it == p->tables.end()) return fail(SE2CONV_ERR_INVALID_ARG, "table was not produced by this plan");
        if (it->second.kind != SE2CONV_TABLE_FULL)
            return fail(SE2CONV_ERR_INVALID_ARG, "only a FULL table can be folded (kind %d)", it->second.kind);
        shape_idx = it->second.shape_idx;
        full_bytes = it->second.bytes;
    }
    const se2conv_shape& s = p->shapes[shape_idx];
    const size_t bytes = cplx_bytes(p) * (size_t)s.m * (size_t)(s.ny / 2 + 1) * (size_t)(s.nx / 2 + 1);
    if (!d_quarter) {
        *quarter_bytes = bytes;
        return ok();
    }
    if (*quarter_bytes < bytes)
        return fail(SE2CONV_ERR_INVALID_ARG, "quarter buffer too small (%zu < %zu)", *quarter_bytes, bytes);
    if (!aligned16(d_quarter)) return fail(SE2CONV_ERR_INVALID_ARG, "quarter table must be 16-byte aligned");
    const uintptr_t f0 = reinterpret_cast<uintptr_t>(d_full), q0 = reinterpret_cast<uintptr_t>(d_quarter);
    if (q0 < f0 + full_bytes && f0 < q0 + bytes)
        return fail(SE2CONV_ERR_INVALID_ARG, "the quarter table must not overlap the FULL table");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    std::lock_guard<std::mutex> g(p->mu);
    if (!p->qstat && hipMalloc(&p->qstat, 2 * sizeof(unsigned long long)) != hipSuccess)
        return fail(SE2CONV_ERR_OUT_OF_MEMORY, "symmetry-check buffer (16 bytes)");
    auto* st = reinterpret_cast<unsigned long long*>(p->qstat);
    HIPCHK(launch_quarter(d_full, d_quarter, s.nx, s.ny, s.m, dbl(p) ? 1 : 0, st, stream));
    unsigned long long h[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    double dev, big;
    std::memcpy(&dev, &h[0], sizeof(double));
    std::memcpy(&big, &h[1], sizeof(double));
    // rounding level of a table generated in FP64 and rounded once to the plan dtype
    const double tol = (dbl(p) ? 1e-12 : 1e-5) * big;
    if (!(dev <= tol))
        return fail(SE2CONV_ERR_INVALID_ARG,
                    "table is not symmetric under k1 -> -k1, k2 -> -k2: max deviation %.3g against %.3g "
                    "(max |T| %.3g); the kernel is not radial in translations",
                    dev, tol, big);
    TableRec rec;
    rec.shape_idx = shape_idx;
    rec.kind = SE2CONV_TABLE_QUARTER;
    rec.bytes = bytes;
    register_table(p, d_quarter, rec);
    return ok();
}

se2conv_status se2conv_table_release(se2conv_plan_t p, const void* d_table) {
    if (!p || !d_table) return fail(SE2CONV_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->tables.find(reinterpret_cast<uintptr_t>(d_table));
    if (it == p->tables.end()) return fail(SE2CONV_ERR_INVALID_ARG, "table was not produced by this plan");
    purge_subs_naming(p, it->first);
    p->tables.erase(it);
    return ok();
}

se2conv_status se2conv_plan_counts(se2conv_plan_t p, int64_t* n_tables, int64_t* n_submissions) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    std::lock_guard<std::mutex> g(p->mu);
    if (n_tables) *n_tables = (int64_t)p->tables.size();
    if (n_submissions) *n_submissions = (int64_t)p->subs.size();
    return ok();
}

se2conv_status se2conv_shift_table(se2conv_plan_t p, int32_t shape_idx, const se2conv_shift* shifts,
                                   int32_t n_shifts, void* d_table, size_t* table_bytes, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (!table_bytes) return fail(SE2CONV_ERR_INVALID_ARG, "table_bytes is null");
    if (!shifts || n_shifts < 1 || n_shifts > SE2C_MAX_SHIFT_TERMS)
        return fail(SE2CONV_ERR_INVALID_ARG, "need 1..%d shifts", SE2C_MAX_SHIFT_TERMS);
    const se2conv_shape& s = p->shapes[shape_idx];
    std::vector<int> rolls;
    for (int k = 0; k < n_shifts; ++k) {
        const se2conv_shift& q = shifts[k];
        if (!std::isfinite(q.tx) || !std::isfinite(q.ty) || !std::isfinite(q.weight) || std::fabs(q.tx) > 1e6 ||
            std::fabs(q.ty) > 1e6)
            return fail(SE2CONV_ERR_INVALID_ARG, "shift %d: translation and weight must be finite (|t| <= 1e6)", k);
        if (q.roll < 0 || q.roll >= s.m)
            return fail(SE2CONV_ERR_INVALID_ARG, "shift %d: roll %d outside [0, M = %d)", k, q.roll, s.m);
        if (std::find(rolls.begin(), rolls.end(), q.roll) == rolls.end()) rolls.push_back(q.roll);
    }
    if ((int)rolls.size() > SE2C_MAX_SHIFT_CLASSES)
        return fail(SE2CONV_ERR_INVALID_ARG, "at most %d distinct rolls per table (got %zu)", SE2C_MAX_SHIFT_CLASSES,
                    rolls.size());
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t bytes = cplx_bytes(p) * (size_t)n * rolls.size();
    if (!d_table) {
        *table_bytes = bytes;
        return ok();
    }
    if (*table_bytes < bytes) return fail(SE2CONV_ERR_INVALID_ARG, "table buffer too small (%zu < %zu)", *table_bytes, bytes);
    if (!aligned16(d_table)) return fail(SE2CONV_ERR_INVALID_ARG, "table must be 16-byte aligned");
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    for (size_t j = 0; j < rolls.size(); ++j) {
        ShiftClassArgs a{};
        a.nx = s.nx;
        a.ny = s.ny;
        a.m = s.m;
        for (int k = 0; k < n_shifts; ++k)
            if (shifts[k].roll == rolls[j]) a.t[a.nterm++] = ShiftTerm{shifts[k].tx, shifts[k].ty, shifts[k].weight};
        HIPCHK(launch_shift_table(a, (char*)d_table + cplx_bytes(p) * (size_t)n * j, dbl(p), stream));
    }
    TableRec rec;
    rec.shape_idx = shape_idx;
    rec.kind = SE2CONV_TABLE_SHIFT;
    rec.bytes = bytes;
    rec.rolls = rolls;
    std::lock_guard<std::mutex> g(p->mu);
    register_table(p, d_table, rec);
    return ok();
}

se2conv_status se2conv_apply_shifted(se2conv_plan_t p, int32_t shape_idx, const void* d_f, const void* d_shift_table,
                                     const void* const* kernel_tables, int32_t n_kernel_tables, void* d_out,
                                     int32_t batch, uint32_t flags, hipStream_t stream) {
    se2conv_status r = validate_io(p, shape_idx, d_f, d_out, batch);
    if (r != SE2CONV_OK) return r;
    if (flags & ~SE2CONV_TIMING) return fail(SE2CONV_ERR_INVALID_ARG, "unknown flags 0x%x (only SE2CONV_TIMING)", flags);
    if (!d_shift_table || !kernel_tables) return fail(SE2CONV_ERR_INVALID_ARG, "null table");
    std::vector<int> rolls;
    {
        std::lock_guard<std::mutex> g(p->mu);
        auto it = p->tables.find(reinterpret_cast<uintptr_t>(d_shift_table));
        if (it == p->tables.end() || it->second.kind != SE2CONV_TABLE_SHIFT)
            return fail(SE2CONV_ERR_INVALID_ARG, "d_shift_table is not a shift table of this plan");
        if (it->second.shape_idx != shape_idx)
            return fail(SE2CONV_ERR_INVALID_ARG, "shift table belongs to shape %d, not %d", it->second.shape_idx,
                        shape_idx);
        rolls = it->second.rolls;
    }
    Chain ch;
    bool all_sep = true;
    r = lookup_chain(p, shape_idx, kernel_tables, n_kernel_tables, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    if (flags & SE2CONV_TIMING) {
        HIPCHK(record_event(p, stream, true));
        g_timing_plan = p;
    }
    r = enqueue_shifted(p, p->shapes[shape_idx], d_f, d_out, batch, ch, d_shift_table, rolls, stream);
    g_timing_plan = nullptr;
    return r == SE2CONV_OK ? ok() : r;
}

se2conv_status se2conv_apply(se2conv_plan_t p, int32_t shape_idx, const void* d_f, const void* d_table, void* d_out,
                             int32_t batch, uint32_t flags, hipStream_t stream) {
    se2conv_status r = validate_io(p, shape_idx, d_f, d_out, batch);
    if (r != SE2CONV_OK) return r;
    if (flags & ~(SE2CONV_ADJOINT | SE2CONV_TIMING))
        return fail(SE2CONV_ERR_INVALID_ARG, "unknown apply flags 0x%x", flags);
    Chain ch;
    bool all_sep = true;
    const void* tabs[1] = {d_table};
    r = lookup_chain(p, shape_idx, tabs, 1, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    if (flags & SE2CONV_TIMING) {
        std::lock_guard<std::mutex> g(p->mu);
        HIPCHK(record_event(p, stream, true));
        g_timing_plan = p;
    }
    r = enqueue_problem(p, shape_idx, d_f, d_out, batch, ch, all_sep, (flags & SE2CONV_ADJOINT) != 0, stream);
    g_timing_plan = nullptr;
    if (r != SE2CONV_OK) return r;
    return ok();
}

// ---- fused differentiation (register kernels of the full path)
se2conv_status se2conv_apply_padded(se2conv_plan_t p, int32_t shape_idx, const void* d_f, const void* d_table,
                                    int32_t out_shape_idx, void* d_out, int32_t batch, uint32_t flags,
                                    hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    const int nsh = (int)p->shapes.size();
    if (shape_idx < 0 || shape_idx >= nsh || out_shape_idx < 0 || out_shape_idx >= nsh)
        return fail(SE2CONV_ERR_INVALID_ARG, "shape index out of range");
    const se2conv_shape& s = p->shapes[shape_idx];
    const se2conv_shape& g = p->shapes[out_shape_idx];
    if (g.nx < s.nx || g.ny < s.ny || g.m < s.m)
        return fail(SE2CONV_ERR_INVALID_ARG, "output grid %d x %d x %d is coarser than the sampling grid %d x %d x %d",
                    g.nx, g.ny, g.m, s.nx, s.ny, s.m);
    if (batch < 1) return fail(SE2CONV_ERR_INVALID_ARG, "batch must be >= 1 (got %d)", batch);
    if (!d_f || !d_out || !aligned16(d_f) || !aligned16(d_out))
        return fail(SE2CONV_ERR_INVALID_ARG, "f and out must be non-null and 16-byte aligned");
    if (flags & ~(SE2CONV_ADJOINT | SE2CONV_TIMING))
        return fail(SE2CONV_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const long long n = (long long)s.nx * s.ny * s.m;
    const long long ng = (long long)g.nx * g.ny * g.m;
    const size_t rb = real_bytes(p);
    {
        const char* a = (const char*)d_f;
        const char* b = (const char*)d_out;
        const long long fb = (long long)batch * n * (long long)rb, ob = (long long)batch * ng * (long long)rb;
        if (a < b + ob && b < a + fb) return fail(SE2CONV_ERR_INVALID_ARG, "d_out must not overlap d_f");
    }
    Chain ch;
    bool all_sep = true;
    const void* tabs[1] = {d_table};
    se2conv_status r = lookup_chain(p, shape_idx, tabs, 1, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const int pairs = (batch + 1) / 2;
    const bool odd = (batch & 1) != 0;
    {
        // the product spectra of every pair on the sampling grid (two planes per pair)
        std::lock_guard<std::mutex> lk(p->mu);
        const size_t need = 2 * (size_t)pairs * (size_t)n * rb;
        if (p->pad_ws_bytes < need) {
            if (p->pad_ws) {
                hipError_t e = hipFree(p->pad_ws);
                p->pad_ws = nullptr;
                p->pad_ws_bytes = 0;
                if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "hipFree: %s", hipGetErrorString(e));
            }
            if (hipMalloc(&p->pad_ws, need) != hipSuccess)
                return fail(SE2CONV_ERR_OUT_OF_MEMORY, "padded-evaluation workspace (%zu bytes)", need);
            p->pad_ws_bytes = need;
        }
    }
    const bool d = dbl(p);
    const bool conj = (flags & SE2CONV_ADJOINT) != 0;
    if (flags & SE2CONV_TIMING) {
        std::lock_guard<std::mutex> lk(p->mu);
        HIPCHK(record_event(p, stream, true));
        g_timing_plan = p;
    }
    if (!d && !(p->flags & SE2CONV_PLAN_GENERIC) && !odd && full_fast_supported(s.nx, s.ny, s.m) &&
        full_fast_supported(g.nx, g.ny, g.m)) {
        // register kernels: x-theta forward and the y spectra on the sampling grid (in the
        // workspace), then one y pass on the evaluation grid that pads, multiplies by the
        // table and inverts, and the x-theta inverse in place in the output
        FullFastArgs a = full_fast_args(p, s, batch);
        a.in = reinterpret_cast<const float*>(d_f);
        a.out = reinterpret_cast<float*>(p->pad_ws);
        a.save = a.out;
        hipError_t e = launch_xt_full_fwd(a, stream);
        if (e == hipSuccess) e = after_pass(0, stream);
        if (e == hipSuccess) e = launch_y_full_spectra(a, stream);
        if (e == hipSuccess) e = after_pass(1, stream);
        FullFastArgs b = full_fast_args(p, g, batch);
        set_chain(&b, ch, conj, 1.0 / (double)n);
        b.zsrc = reinterpret_cast<const float*>(p->pad_ws);
        b.lx = s.nx;
        b.ly = s.ny;
        b.lm = s.m;
        b.nl = n;
        b.in = reinterpret_cast<const float*>(d_out);
        b.out = reinterpret_cast<float*>(d_out);
        if (e == hipSuccess) e = launch_y_full_pad_inv(b, stream);
        if (e == hipSuccess) e = after_pass(1, stream);
        if (e == hipSuccess) e = launch_xt_full_inv(b, stream);
        if (e == hipSuccess) e = after_pass(0, stream);
        g_timing_plan = nullptr;
        if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "padded evaluation: %s", hipGetErrorString(e));
        return ok();
    }
    // sampling grid: pairs of fields packed as re/im (a lone last field pairs with zero);
    // pair i's planes at pad_ws + 2 i n (re) and + n (im)
    char* hre = (char*)p->pad_ws;
    char* him = hre + rb * n;
    const void* f1 = batch == 1 ? nullptr : (const char*)d_f + rb * n;
    void* h_lone = odd ? hre + rb * ((long long)(2 * (pairs - 1) + 1) * n) : nullptr;
    // evaluation grid: the pair's two output fields hold its re / im planes; a lone field's
    // im plane goes to the plan workspace (discarded)
    char* ore = (char*)d_out;
    char* oim = batch == 1 ? nullptr : ore + rb * ng;
    void* o_lone = odd ? p->ws : nullptr;
    hipError_t e = xt_transform(p, s, d, 0, d_f, f1, hre, batch == 1 ? nullptr : him, nullptr, h_lone, 2 * n, 2 * n,
                                pairs, stream);
    if (e == hipSuccess)
        e = y_pass(p, s, d, hre, batch == 1 ? nullptr : him, h_lone, 2 * n, pairs, 1, 0, 2, &ch, conj,
                   1.0 / (double)n, stream);
    if (e == hipSuccess)
        e = launch_pad_spectrum(hre, ore, o_lone, pairs, 2 * n, 2 * ng, s.nx, s.ny, s.m, g.nx, g.ny, g.m, d, stream);
    if (e == hipSuccess) e = y_pass(p, g, d, ore, oim, o_lone, 2 * ng, pairs, 0, 1, 0, nullptr, false, 1.0, stream);
    if (e == hipSuccess)
        e = xt_transform(p, g, d, 1, ore, oim, ore, oim, o_lone, nullptr, 2 * ng, 2 * ng, pairs, stream);
    g_timing_plan = nullptr;
    if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "padded evaluation: %s", hipGetErrorString(e));
    return ok();
}

se2conv_status se2conv_apply_complex(se2conv_plan_t p, int32_t shape_idx, const void* d_f, const void* d_table,
                                     void* d_out, int32_t batch, uint32_t flags, hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (batch < 1) return fail(SE2CONV_ERR_INVALID_ARG, "batch must be >= 1 (got %d)", batch);
    if (!d_f || !d_out || !aligned16(d_f) || !aligned16(d_out))
        return fail(SE2CONV_ERR_INVALID_ARG, "f and out must be non-null and 16-byte aligned");
    if (flags & ~(SE2CONV_ADJOINT | SE2CONV_TIMING))
        return fail(SE2CONV_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const se2conv_shape& s = p->shapes[shape_idx];
    const long long n = (long long)s.nx * s.ny * s.m;
    const size_t rb = real_bytes(p);
    {
        const char* a = (const char*)d_f;
        const char* b = (const char*)d_out;
        const long long bytes = 2LL * batch * n * (long long)rb;
        if (a != b && a < b + bytes && b < a + bytes)
            return fail(SE2CONV_ERR_INVALID_ARG, "f and out overlap without being equal");
    }
    Chain ch;
    bool all_sep = true;
    const void* tabs[1] = {d_table};
    se2conv_status r = lookup_chain(p, shape_idx, tabs, 1, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const bool d = dbl(p);
    if (flags & SE2CONV_TIMING) {
        std::lock_guard<std::mutex> lk(p->mu);
        HIPCHK(record_event(p, stream, true));
        g_timing_plan = p;
    }
    // Re and Im of each field are the two planes of one pair, interleaved: the element
    // stride is 2, the field stride 2n reals.
    const void* f_im = (const char*)d_f + rb;
    void* o_im = (char*)d_out + rb;
    hipError_t e = xt_transform(p, s, d, 0, d_f, f_im, d_out, o_im, nullptr, nullptr, 2 * n, 2 * n, batch, stream, 1);
    if (e == hipSuccess)
        e = y_pass(p, s, d, d_out, o_im, nullptr, 2 * n, batch, 1, 1, 2, &ch, (flags & SE2CONV_ADJOINT) != 0,
                   1.0 / (double)n, stream, 1);
    if (e == hipSuccess)
        e = xt_transform(p, s, d, 1, d_out, o_im, d_out, o_im, nullptr, nullptr, 2 * n, 2 * n, batch, stream, 1);
    g_timing_plan = nullptr;
    if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "complex apply: %s", hipGetErrorString(e));
    return ok();
}

int32_t se2conv_fused_supported(se2conv_plan_t p, int32_t shape_idx) {
    if (!p || p->host_only || shape_idx < 0 || shape_idx >= (int)p->shapes.size()) return 0;
    return use_full_fast(p, p->shapes[shape_idx]) ? 1 : 0;
}

namespace {

se2conv_status check_fused(se2conv_plan_s* p, int32_t shape_idx) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (shape_idx < 0 || shape_idx >= (int)p->shapes.size())
        return fail(SE2CONV_ERR_INVALID_ARG, "shape_idx %d out of range", shape_idx);
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    if (!use_full_fast(p, p->shapes[shape_idx]))
        return fail(SE2CONV_ERR_UNSUPPORTED_SIZE,
                    "fused differentiation needs an FP32 plan without SE2CONV_PLAN_GENERIC and nx in {64,128,256}, "
                    "m in {16,32,64}, ny in {64,128,256,512}");
    return SE2CONV_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

}  // namespace

se2conv_status se2conv_field_spectra(se2conv_plan_t p, int32_t shape_idx, const void* d_f, int32_t batch,
                                     void* d_spectra, hipStream_t stream) {
    se2conv_status r = check_fused(p, shape_idx);
    if (r != SE2CONV_OK) return r;
    if (batch < 1 || !d_f || !d_spectra || !aligned16(d_f) || !aligned16(d_spectra))
        return fail(SE2CONV_ERR_INVALID_ARG, "need batch >= 1 and 16-byte aligned device pointers");
    const se2conv_shape& s = p->shapes[shape_idx];
    FullFastArgs a = full_fast_args(p, s, batch);
    const size_t plane = sizeof(float) * (size_t)a.n;
    if (overlaps(d_f, plane * batch, d_spectra, plane * 2 * ((batch + 1) / 2)))
        return fail(SE2CONV_ERR_INVALID_ARG, "d_spectra overlaps d_f");
    a.in = reinterpret_cast<const float*>(d_f);
    a.out = reinterpret_cast<float*>(d_spectra);
    a.save = a.out;
    a.lone = (batch & 1) ? a.out + (long long)batch * a.n : nullptr;
    HIPCHK(launch_xt_full_fwd(a, stream));
    HIPCHK(launch_y_full_spectra(a, stream));
    return ok();
}

se2conv_status se2conv_apply_save(se2conv_plan_t p, int32_t shape_idx, const void* d_f, const void* d_table,
                                  void* d_out, int32_t batch, void* d_spectra, hipStream_t stream) {
    se2conv_status r = validate_io(p, shape_idx, d_f, d_out, batch);
    if (r != SE2CONV_OK) return r;
    r = check_fused(p, shape_idx);
    if (r != SE2CONV_OK) return r;
    const se2conv_shape& s = p->shapes[shape_idx];
    FullFastArgs a = full_fast_args(p, s, batch);
    const size_t plane = sizeof(float) * (size_t)a.n;
    const size_t sbytes = plane * 2 * ((batch + 1) / 2);
    if (!d_spectra || !aligned16(d_spectra) || overlaps(d_f, plane * batch, d_spectra, sbytes) ||
        overlaps(d_out, plane * batch, d_spectra, sbytes))
        return fail(SE2CONV_ERR_INVALID_ARG, "d_spectra must be 16-byte aligned and not overlap d_f or d_out");
    Chain ch;
    bool all_sep = true;
    const void* tabs[1] = {d_table};
    r = lookup_chain(p, shape_idx, tabs, 1, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    set_chain(&a, ch, false, 1.0 / (double)a.n);
    a.in = reinterpret_cast<const float*>(d_f);
    a.out = reinterpret_cast<float*>(d_out);
    a.save = reinterpret_cast<float*>(d_spectra);
    HIPCHK(launch_xt_full_fwd(a, stream));
    a.in = a.out;
    HIPCHK(launch_y_full(a, stream));
    HIPCHK(launch_xt_full_inv(a, stream));
    return ok();
}

se2conv_status se2conv_backward(se2conv_plan_t p, int32_t shape_idx, const void* d_g, const void* d_table,
                                const void* d_spectra, int32_t batch, void* d_grad_f, void* d_grad_p,
                                hipStream_t stream) {
    se2conv_status r = validate_io(p, shape_idx, d_g, d_grad_f, batch);
    if (r != SE2CONV_OK) return r;
    r = check_fused(p, shape_idx);
    if (r != SE2CONV_OK) return r;
    const se2conv_shape& s = p->shapes[shape_idx];
    FullFastArgs a = full_fast_args(p, s, batch);
    const size_t plane = sizeof(float) * (size_t)a.n;
    const size_t sbytes = plane * 2 * ((batch + 1) / 2);
    if (!d_spectra || !d_grad_p || !aligned16(d_spectra) || !aligned16(d_grad_p))
        return fail(SE2CONV_ERR_INVALID_ARG, "d_spectra and d_grad_p must be 16-byte aligned device pointers");
    if (overlaps(d_grad_f, plane * batch, d_spectra, sbytes) || overlaps(d_grad_f, plane * batch, d_grad_p, plane) ||
        overlaps(d_g, plane * batch, d_grad_p, plane) || overlaps(d_spectra, sbytes, d_grad_p, plane))
        return fail(SE2CONV_ERR_INVALID_ARG, "d_grad_f, d_grad_p and d_spectra must not overlap");
    Chain ch;
    bool all_sep = true;
    const void* tabs[1] = {d_table};
    r = lookup_chain(p, shape_idx, tabs, 1, &ch, &all_sep);
    if (r != SE2CONV_OK) return r;
    {
        std::lock_guard<std::mutex> g(p->mu);
        if (!p->ws2 && hipMalloc(&p->ws2, 2 * p->ws_bytes) != hipSuccess)
            return fail(SE2CONV_ERR_OUT_OF_MEMORY, "backward workspace (%zu bytes)", 2 * p->ws_bytes);
    }
    float* acc = reinterpret_cast<float*>(p->ws2);
    set_chain(&a, ch, true, 1.0 / (double)a.n);
    a.in = reinterpret_cast<const float*>(d_g);
    a.out = reinterpret_cast<float*>(d_grad_f);
    HIPCHK(launch_xt_full_fwd(a, stream));
    a.in = a.out;
    a.zf = reinterpret_cast<const float*>(d_spectra);
    a.acc = acc;
    a.acc_scale = (float)(1.0 / ((double)a.n * (double)a.n));
    HIPCHK(launch_y_full_backward(a, stream));
    HIPCHK(launch_xt_full_inv(a, stream));
    // x-theta inverse of the accumulated spectrum: real part = dL/dP (imaginary part dropped)
    FullFastArgs b = full_fast_args(p, s, 1);
    b.in = acc;
    b.lone = acc + a.n;
    b.out = reinterpret_cast<float*>(d_grad_p);
    HIPCHK(launch_xt_full_inv(b, stream));
    return ok();
}


se2conv_status se2conv_chain(se2conv_plan_t p, const se2conv_problem* probs, int32_t n_probs, uint32_t flags,
                             hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (!probs || n_probs < 1) return fail(SE2CONV_ERR_INVALID_ARG, "need at least one problem");
    if (flags & ~(SE2CONV_ADJOINT | SE2CONV_GRAPH | SE2CONV_TIMING))
        return fail(SE2CONV_ERR_INVALID_ARG, "unknown chain flags 0x%x", flags);
    if ((flags & SE2CONV_GRAPH) && (flags & SE2CONV_TIMING))
        return fail(SE2CONV_ERR_INVALID_ARG, "SE2CONV_TIMING cannot be combined with SE2CONV_GRAPH");
    if ((flags & SE2CONV_GRAPH) && stream == nullptr)
        return fail(SE2CONV_ERR_INVALID_ARG, "SE2CONV_GRAPH needs a created stream (the null stream cannot be captured)");
    std::vector<Chain> chains(n_probs);
    std::vector<char> seps(n_probs);
    std::vector<uint64_t> key;
    key.push_back(flags);
    for (int i = 0; i < n_probs; ++i) {
        const se2conv_problem& q = probs[i];
        se2conv_status r = validate_io(p, q.shape_idx, q.f, q.out, q.batch);
        if (r != SE2CONV_OK) return fail(r, "problem %d: %s", i, g_last_error.c_str());
        if (!q.tables) return fail(SE2CONV_ERR_INVALID_ARG, "problem %d: tables is null", i);
        bool all_sep = true;
        r = lookup_chain(p, q.shape_idx, q.tables, q.n_tables, &chains[i], &all_sep);
        if (r != SE2CONV_OK) return fail(r, "problem %d: %s", i, g_last_error.c_str());
        seps[i] = all_sep && pair_layout(p->shapes[q.shape_idx]);
        key.push_back((uint64_t)q.shape_idx);
        key.push_back((uint64_t)q.batch);
        key.push_back((uint64_t)(uintptr_t)q.f);
        key.push_back((uint64_t)(uintptr_t)q.out);
        key.push_back((uint64_t)q.n_tables);
        for (int j = 0; j < q.n_tables; ++j) {
            key.push_back((uint64_t)(uintptr_t)q.tables[j]);
            key.push_back((uint64_t)chains[i].kind[j]);
        }
    }
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    const bool conj = (flags & SE2CONV_ADJOINT) != 0;

    // find or build the submission record (device item arrays grouped by shape)
    uint64_t key_hash = 1469598103934665603ull;
    for (uint64_t v : key) key_hash = (key_hash ^ v) * 1099511628211ull;
    std::shared_ptr<SubmissionRec> rec;
    {
        std::lock_guard<std::mutex> g(p->mu);
        for (auto& r : p->subs)
            if (r->key_hash == key_hash && r->key == key) rec = r;
    }
    if (!rec) {
        std::map<int, std::vector<SepItem>> by_shape;
        for (int i = 0; i < n_probs; ++i) {
            if (!seps[i]) continue;
            const se2conv_problem& q = probs[i];
            const se2conv_shape& s = p->shapes[q.shape_idx];
            const long long n = (long long)s.nx * s.ny * s.m;
            for (int b = 0; b < q.batch; ++b) {
                SepItem it{};
                it.in = (const char*)q.f + real_bytes(p) * n * b;
                it.out = (char*)q.out + real_bytes(p) * n * b;
                it.ntab = q.n_tables;
                for (int j = 0; j < q.n_tables; ++j) it.tab[j] = q.tables[j];
                by_shape[q.shape_idx].push_back(it);
            }
        }
        auto nr = std::make_shared<SubmissionRec>();
        nr->key = key;
        nr->key_hash = key_hash;
        for (int i = 0; i < n_probs; ++i)
            for (int j = 0; j < probs[i].n_tables; ++j)
                nr->tabs.push_back(reinterpret_cast<uintptr_t>(probs[i].tables[j]));
        std::vector<SepItem> all;
        for (auto& kv : by_shape) {
            nr->groups.push_back({kv.first, (int)all.size()});
            nr->group_counts.push_back((int)kv.second.size());
            all.insert(all.end(), kv.second.begin(), kv.second.end());
        }
        if (hipEventCreateWithFlags(&nr->done, hipEventDisableTiming) != hipSuccess) {
            nr->done = nullptr;
            return fail(SE2CONV_ERR_DEVICE, "could not create the submission event");
        }
        if (!all.empty()) {
            if (hipMalloc(&nr->d_items, sizeof(SepItem) * all.size()) != hipSuccess) {
                nr->d_items = nullptr;
                return fail(SE2CONV_ERR_OUT_OF_MEMORY, "item list (%zu items)", all.size());
            }
            hipError_t e = hipMemcpyAsync(nr->d_items, all.data(), sizeof(SepItem) * all.size(),
                                          hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "item upload failed: %s", hipGetErrorString(e));
        }
        // bounded cache: drop the oldest record that no captured graph of the caller's
        // refers to; its destructor waits for its last enqueued use (on whatever stream)
        std::shared_ptr<SubmissionRec> evicted;
        std::lock_guard<std::mutex> g(p->mu);
        if (p->subs.size() >= 64) {
            for (auto it = p->subs.begin(); it != p->subs.end(); ++it)
                if (!(*it)->pinned) {
                    evicted = *it;
                    p->subs.erase(it);
                    break;
                }
        }
        p->subs.push_back(nr);
        rec = nr;
    }
    // Shape classes are independent: with several of them (and no per-pass timing) they run
    // concurrently on the plan's auxiliary streams, forked from and joined back into the
    // caller's stream (under capture this makes parallel branches of the graph).
    const int ngroups = (int)rec->groups.size();
    // Streams the shape classes are dealt over: one by default.  Measured on MI355X with
    // 256 problems in 15 classes, the caller's stream alone replays in 0.57 ms against
    // 0.70-0.74 ms forked over four streams: the large classes fill the GPU by themselves
    // and the forks only add scheduling gaps.  SE2CONV_CHAIN_STREAMS (1..4) overrides.
    const int chain_streams = [] {
        const char* e = std::getenv("SE2CONV_CHAIN_STREAMS");
        const int v = e ? std::atoi(e) : 1;
        return std::max(1, std::min(v, kChainStreams));
    }();
    const bool fan_out = ngroups > 1 && chain_streams > 1 && !(flags & SE2CONV_TIMING);
    if (fan_out) {
        se2conv_status r = ensure_aux_streams(p);
        if (r != SE2CONV_OK) return r;
    }
    auto submit = [&]() -> se2conv_status {
        // every separable problem: one launch per pass per shape group
        if (fan_out) {
            // largest classes first, dealt round-robin over the streams
            std::vector<int> order(ngroups);
            for (int gi = 0; gi < ngroups; ++gi) order[gi] = gi;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                const se2conv_shape& sa = p->shapes[rec->groups[a].first];
                const se2conv_shape& sb = p->shapes[rec->groups[b].first];
                return (long long)sa.nx * sa.ny * sa.m * rec->group_counts[a] >
                       (long long)sb.nx * sb.ny * sb.m * rec->group_counts[b];
            });
            const int nst = std::min(ngroups, chain_streams);
            std::lock_guard<std::mutex> fg(p->fork_mu);
            HIPCHK(hipEventRecord(p->ev_fork, stream));
            for (int k = 0; k < nst; ++k) HIPCHK(hipStreamWaitEvent(p->aux[k], p->ev_fork, 0));
            for (int oi = 0; oi < ngroups; ++oi) {
                const int gi = order[oi];
                const int sidx = rec->groups[gi].first;
                const SepItem* items = reinterpret_cast<const SepItem*>(rec->d_items) + rec->groups[gi].second;
                se2conv_status r =
                    enqueue_sep_items(p, p->shapes[sidx], items, rec->group_counts[gi], conj, p->aux[oi % nst]);
                if (r != SE2CONV_OK) return r;
            }
            for (int k = 0; k < nst; ++k) {
                HIPCHK(hipEventRecord(p->ev_join[k], p->aux[k]));
                HIPCHK(hipStreamWaitEvent(stream, p->ev_join[k], 0));
            }
        } else {
            bool multi = false;
            se2conv_status r = enqueue_multi(p, reinterpret_cast<const SepItem*>(rec->d_items), rec->groups,
                                             rec->group_counts, conj, stream, &multi, !(flags & SE2CONV_TIMING));
            if (r != SE2CONV_OK) return r;
            for (int gi = 0; !multi && gi < ngroups; ++gi) {
                const int sidx = rec->groups[gi].first;
                const SepItem* items = reinterpret_cast<const SepItem*>(rec->d_items) + rec->groups[gi].second;
                r = enqueue_sep_items(p, p->shapes[sidx], items, rec->group_counts[gi], conj, stream);
                if (r != SE2CONV_OK) return r;
            }
        }
        // problems with full tables: one submission each
        for (int i = 0; i < n_probs; ++i) {
            if (seps[i]) continue;
            se2conv_status r = enqueue_problem(p, probs[i].shape_idx, probs[i].f, probs[i].out, probs[i].batch,
                                               chains[i], false, conj, stream);
            if (r != SE2CONV_OK) return r;
        }
        return SE2CONV_OK;
    };
    // after every enqueue of the record's work: mark where it ends on this stream (or, on
    // a stream that the caller is capturing, keep the record for the plan's lifetime)
    auto mark_done = [&]() -> se2conv_status {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(hipStreamIsCapturing(stream, &cs));
        std::lock_guard<std::mutex> g(p->mu);
        if (cs != hipStreamCaptureStatusNone) {
            rec->pinned = true;
            return SE2CONV_OK;
        }
        HIPCHK(hipEventRecord(rec->done, stream));
        rec->used = true;
        return SE2CONV_OK;
    };
    if (!(flags & SE2CONV_GRAPH)) {
        if (flags & SE2CONV_TIMING) {
            HIPCHK(record_event(p, stream, true));
            g_timing_plan = p;
        }
        se2conv_status r = submit();
        g_timing_plan = nullptr;
        if (r != SE2CONV_OK) return r;
        r = mark_done();
        return r == SE2CONV_OK ? ok() : r;
    }
    hipGraphExec_t cached = nullptr;
    {
        std::lock_guard<std::mutex> g(p->mu);
        cached = rec->exec;
    }
    if (cached) {
        HIPCHK(hipGraphLaunch(cached, stream));
        se2conv_status r = mark_done();
        return r == SE2CONV_OK ? ok() : r;
    }
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    se2conv_status r = submit();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &graph);
    if (r != SE2CONV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess) return fail(SE2CONV_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(SE2CONV_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> g(p->mu);
        if (rec->exec) {  // another call captured the same list meanwhile: keep that one
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
        } else {
            rec->graph = graph;
            rec->exec = exec;
        }
    }
    HIPCHK(hipGraphLaunch(rec->exec, stream));
    r = mark_done();
    return r == SE2CONV_OK ? ok() : r;
}

se2conv_status se2conv_chain_noalloc(se2conv_plan_t p, const se2conv_problem* probs, int32_t n_probs, uint32_t flags,
                                     hipStream_t stream) {
    if (!p) return fail(SE2CONV_ERR_INVALID_ARG, "plan is null");
    if (!probs || n_probs < 1) return fail(SE2CONV_ERR_INVALID_ARG, "need at least one problem");
    if (flags & ~SE2CONV_ADJOINT)
        return fail(SE2CONV_ERR_INVALID_ARG, "se2conv_chain_noalloc takes only SE2CONV_ADJOINT (flags 0x%x)", flags);
    std::map<int, std::vector<SepItem>> by_shape;
    long long total = 0;
    for (int i = 0; i < n_probs; ++i) {
        const se2conv_problem& q = probs[i];
        se2conv_status r = validate_io(p, q.shape_idx, q.f, q.out, q.batch);
        if (r != SE2CONV_OK) return fail(r, "problem %d: %s", i, g_last_error.c_str());
        if (!q.tables) return fail(SE2CONV_ERR_INVALID_ARG, "problem %d: tables is null", i);
        Chain ch;
        bool all_sep = true;
        r = lookup_chain(p, q.shape_idx, q.tables, q.n_tables, &ch, &all_sep);
        if (r != SE2CONV_OK) return fail(r, "problem %d: %s", i, g_last_error.c_str());
        const se2conv_shape& s = p->shapes[q.shape_idx];
        if (!all_sep || !pair_layout(s))
            return fail(SE2CONV_ERR_INVALID_ARG,
                        "problem %d: se2conv_chain_noalloc needs SEPARABLE tables on a shape with even Nx and Ny "
                        "(use se2conv_chain)", i);
        total += q.batch;
        if (total > kNoAllocMaxItems)
            return fail(SE2CONV_ERR_INVALID_ARG,
                        "se2conv_chain_noalloc holds at most %d fields per call (problem %d brings the total to %lld)",
                        kNoAllocMaxItems, i, total);
        const long long n = (long long)s.nx * s.ny * s.m;
        for (int b = 0; b < q.batch; ++b) {
            SepItem it{};
            it.in = (const char*)q.f + real_bytes(p) * n * b;
            it.out = (char*)q.out + real_bytes(p) * n * b;
            it.ntab = q.n_tables;
            for (int j = 0; j < q.n_tables; ++j) it.tab[j] = q.tables[j];
            by_shape[q.shape_idx].push_back(it);
        }
    }
    if (p->host_only) return fail(SE2CONV_ERR_DEVICE, "host-only plan cannot run device work");
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != p->device)
        return fail(SE2CONV_ERR_INVALID_ARG, "the plan's device (%d) must be current (current: %d)", p->device, cur);
    SepItem* sp = noalloc_scratch_of(p->device);
    if (!sp) return fail(SE2CONV_ERR_INTERNAL, "no scratch address for device %d", p->device);
    const bool conj = (flags & SE2CONV_ADJOINT) != 0;
    // write every group's items into the scratch, then run each group's passes on them
    int first = 0;
    for (auto& kv : by_shape) {
        const std::vector<SepItem>& v = kv.second;
        for (int k = 0; k < (int)v.size(); k += kFillBatch) {
            ItemBatch b{};
            b.first = first + k;
            b.n = std::min(kFillBatch, (int)v.size() - k);
            for (int j = 0; j < b.n; ++j) b.it[j] = v[k + j];
            hipLaunchKernelGGL(fill_items_kernel, dim3(1), dim3(kFillBatch), 0, stream, sp, b);
            HIPCHK(hipGetLastError());
        }
        first += (int)v.size();
    }
    std::vector<std::pair<int, int>> groups;
    std::vector<int> counts;
    first = 0;
    for (auto& kv : by_shape) {
        groups.push_back({kv.first, first});
        counts.push_back((int)kv.second.size());
        first += (int)kv.second.size();
    }
    bool multi = false;
    se2conv_status mr = enqueue_multi(p, sp, groups, counts, conj, stream, &multi, false);
    if (mr != SE2CONV_OK) return mr;
    for (size_t gi = 0; !multi && gi < groups.size(); ++gi) {
        se2conv_status r = enqueue_sep_items(p, p->shapes[groups[gi].first], sp + groups[gi].second, counts[gi], conj,
                                             stream);
        if (r != SE2CONV_OK) return r;
    }
    return ok();
}

}  // extern "C"
