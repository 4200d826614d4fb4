"""Helpers shared by the GPU parity tests (oracle side and HIP side kept apart)."""
import numpy as np

from inputs import rel_l2
from oracle import conv as oc
from oracle import kernels as ok


def tol32(n_points: int) -> float:
    """FP32 bound on the relative L2 error against the FP64 oracle: 2e-6 log2(N^2 M)."""
    return 2e-6 * np.log2(n_points)


TOL64 = 1e-12


def parity_err(a, b) -> float:
    """Parity error of a HIP result a against a reference b.

    The larger of ||a - b||_2 / ||b||_2 and max|a - b| / (10 max|b|).  A test that
    asserts parity_err <= tol therefore bounds the relative L2 error by tol and every
    element by 10 tol max|b|, so a local fault (one wrong tile of a few hundred points)
    cannot hide inside the norm.
    """
    a = np.asarray(a)
    b = np.asarray(b)
    scale = float(np.max(np.abs(b))) if b.size else 0.0
    elem = float(np.max(np.abs(a - b))) / (10.0 * scale) if scale > 0 else float(np.max(np.abs(a - b), initial=0.0))
    return max(rel_l2(a, b), elem)


def case(msg: str) -> None:
    print(f"[case] {msg}", flush=True)


def oracle_table_gauss(nx, ny, m, chain, norm="discrete"):
    """Oracle coefficient table prod_j rho_j^[k; L] for Gauss x vM kernels (route 1 step 1)."""
    ps = [ok.gauss_vm(nx, ny, m, k[0], k[1], k[2] if len(k) > 2 else 0.0, normalize=norm) for k in chain]
    return oc.coeff_product(ps)


def oracle_conv(f, table):
    return oc.conv_with_coeffs(f, table)
