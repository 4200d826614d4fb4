"""FP64 CPU oracle for the convolutional finite Fourier series on Z^2\\SE(2).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything under this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

Everything here is plain and slow on purpose:

* ``transforms``   the 3-D DFT and inverse DFT of paper Sec. 2.3, eqs. (3DFT) and
                   (3iDFT), as explicit FP64 DFT matrices applied one axis at a
                   time, with twiddles taken from the reduced integer products
                   (k*i mod L).
* ``ffc``          finite Fourier coefficients (Sec. 3.2, eq. (fkLvMain); matrix form
                   eq. (FkLv)) and the finite Fourier series on the grid.
* ``conv``         the convolutional finite Fourier series S_K[f, rho] (Sec. 5.2,
                   eq. (SKfg)), chains of kernels, the power form of Algorithm 4
                   (eq. (MatSqKfgG)), the all-powers loop of Algorithm 7 and the
                   sampled-point evaluation used at sizes where a full inverse is
                   too slow.
* ``quadrature``   direct rectangle-rule quadrature of the coset convolution
                   (Sec. 5.1, eqs. (oslash), (f*g)) with the explicit rotation
                   R_{-alpha} and lattice images; the heavy sum runs in plain C
                   (csrc/quad.c).
* ``kernels``      samplers for the kernels rho used in tests (Gaussian x von Mises,
                   anisotropic control, radial profile).
* ``closed_form``  continuous closed forms for Gaussian x von Mises bumps convolved
                   with Gaussian x von Mises kernels.
* ``adjoint``      gradients of the convolution with respect to the field samples
                   and the kernel samples.
* ``shifted``      kernels that are sums of SE(2)-shifts of one radial kernel (the
                   outlook of Sec. 1): each shift moved onto the field as a per-slice
                   translation phase and a theta shift, then the radial product.

Array layout everywhere: [theta][y][x] (x fastest), sizes (M, Ny, Nx).
"""
