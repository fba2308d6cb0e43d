"""Pins of the oracle's overlap inversion (CG on the normal equations)."""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import overlap as oov
from oracle import solver as osol
from tests.conftest import rel_err

LMAX = 6.5


def test_cgnr_matches_dense_solve_2x2x2x2():
    """On 2^4 the 192 x 192 matrix of D[mu] is assembled and solved by LAPACK."""
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 501)
    b = latgen.gaussian_spinor(dims, 502)
    alpha = och.coeffs_sign_interp(21, 0.1)
    mat = osol.dense_overlap(u, 0.1, alpha, LMAX)
    ref = np.linalg.solve(mat, b.reshape(-1)).reshape(b.shape)
    x, it = osol.overlap_cgnr(u, b, 0.1, alpha, LMAX, tol=1e-14, max_iter=400)
    assert rel_err(x, ref) < 1e-10
    assert it <= 192 + 20          # CG on a Hermitian positive matrix of order 192


def test_cgnr_mu_one_is_identity():
    """D[1] = 1: the solution is b, found in one iteration."""
    dims = (2, 2, 2, 4)
    u = latgen.random_su3_field(dims, 503)
    b = latgen.gaussian_spinor(dims, 504)
    alpha = och.coeffs_sign_interp(15, 0.1)
    x, it = osol.overlap_cgnr(u, b, 1.0, alpha, LMAX, tol=1e-14)
    assert rel_err(x, b) < 1e-14
    assert it == 1


@pytest.mark.slow
def test_cgnr_residual_deflated_4x4x4x4():
    """With a deflated sign function the true residual ||b - D x|| follows the normal-equation
    residual to within the condition number of D."""
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 505, steps=1)
    b = latgen.gaussian_spinor(dims, 506)
    from oracle.eigen import low_modes
    lam, phi, _ = low_modes(u, 4, LMAX, filter_degree=16)
    alpha = och.coeffs_sign_interp(31, 0.07)
    x, it = osol.overlap_cgnr(u, b, 0.05, alpha, LMAX, phi, lam, tol=1e-12)
    res = b - oov.overlap_apply(u, x, 0.05, alpha, LMAX, phi, lam)
    assert np.linalg.norm(res) / np.linalg.norm(b) < 1e-9
    assert it < 300
