"""MI355X (gfx950) implementation of the convolutional finite Fourier series on
Z^2\\SE(2) (fast SE(2) convolutions with kernels radial in translations).

The compute path is libse2conv.so (hand-written HIP kernels behind a C ABI,
include/se2conv.h); this package is its Python binding.
"""
from ._lib import LIB_PATH, Se2convError  # noqa: F401
from .api import ExpGauss, GaussVM, Plan, RadialProfile, Samples, Table  # noqa: F401
