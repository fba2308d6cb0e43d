"""Low eigenpairs of K on the GPU for the deflation term of Sec. 2, eq. 3.

The paper precomputes the lowest eigenpairs of K once per gauge field with a polynomial-
preconditioned implicitly restarted Lanczos method, at negligible cost compared with the sign
function (Sec. 2).  ``low_modes`` plays that role: argument marshalling for ``ovl_low_modes``
(Chebyshev-filtered subspace iteration in the library: fused stencil launches with the whole block
as right-hand sides, FP64 Gram, rotation and residual kernels, host Hermitian eigen-problems of the
block size).  It is not part of the timed operator.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from .api import M_W, GaugeField, _dims_arr, _ptr, _stream  # noqa: F401
from ._lib import call


def low_modes(g: GaugeField, n_ev: int, lmax: float, block: int = None, degree: int = 60,
              iters: int = 40, tol: float = 1e-10, seed: int = 0, cut: float = 1.0,
              m_w: float = M_W, strict: bool = False):
    """The n_ev eigenpairs of K with the smallest |lambda| (FP64 gauge handle required).

    ``block`` must exceed the number of eigenvalues in any near-degenerate cluster that straddles
    the n_ev-th one (default max(2 n_ev + 8, n_ev + 16)).  Returns (lam: np.ndarray[n_ev], phi:
    complex128 tensor [n_ev, 4, 3, T, Z, Y, X], residuals: np.ndarray[n_ev] = ||K phi - lambda
    phi||, eps_next = |lambda| of the first undeflated Ritz value / lmax).  With strict, a
    residual above tol after ``iters`` iterations raises OvlError (OVL_EDIVERGED); otherwise the
    last iterate is returned and the residuals tell.  The filter's K launches on the block take the
    configuration ``autotune`` keeps for (this lattice, FP64, ``block`` right-hand sides); without
    one, the first call measures the candidates on its start block (about a second at 16^3 x 32).
    """
    if g.store != "f64":
        raise ValueError("the eigen-solve needs an FP64 gauge handle")
    lx, ly, lz, lt = g.dims
    m = block or max(2 * n_ev + 8, n_ev + 16)
    phi = torch.empty((n_ev, 4, 3, lt, lz, ly, lx), dtype=torch.complex128, device=g.device)
    lam = (ctypes.c_double * n_ev)()
    res = (ctypes.c_double * n_ev)()
    eps = ctypes.c_double(0.0)
    its = ctypes.c_int(0)
    lib = _lib.load()
    rc = lib.ovl_low_modes(g.handle, int(n_ev), int(m), float(lmax), float(cut), int(degree),
                           int(iters), float(tol), ctypes.c_uint64(int(seed)), float(m_w),
                           _ptr(phi), lam, res, ctypes.byref(eps), ctypes.byref(its), _stream())
    if rc != 0 and (strict or rc != -8):
        raise _lib.OvlError("ovl_low_modes", rc, lib.ovl_last_error().decode(errors="replace"))
    return np.array(lam[:]), phi, np.array(res[:]), float(eps.value)
