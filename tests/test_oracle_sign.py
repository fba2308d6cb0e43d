"""Pins of the oracle's Chebyshev sign function, deflation and overlap operator.

Sec. 2, eq. 3 (deflated Chebyshev sign function) and eq. 1 (overlap operator).  Checks come from
closed forms (the Chebyshev series of sign(x), free-field plane waves), dense diagonalisation by
LAPACK on a 2^4 lattice, structural identities (the Ginsparg-Wilson residual identity, gauge
covariance, hermiticity) and a library routine (NumPy's Chebyshev series evaluation).
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import latgen
from oracle import chebyshev as ch
from oracle import deflation, overlap, wilson
from oracle.eigen import dense_eigs, dense_kop
from oracle.gamma import GAMMA, GAMMA5
from tests.conftest import rel_err
from tests.test_oracle_wilson import plane_wave, unit_field

LMAX = 6.5


def test_degree_reading():
    assert ch.top_odd_degree(64) == 63
    assert ch.top_odd_degree(200) == 199
    assert ch.top_odd_degree(299) == 299
    assert len(ch.coeffs_sign_interp(64, 0.1)) == 64


def test_series_rule_closed_form():
    """Rule A: p(cos th) = (4/pi) sum_k (-1)^k cos((2k+1) th)/(2k+1) (Fourier series of sign)."""
    alpha = ch.coeffs_sign_series(31)
    th = np.linspace(0.01, np.pi - 0.01, 97)
    trig = (4 / np.pi) * sum((-1) ** k * np.cos((2 * k + 1) * th) / (2 * k + 1)
                             for k in range(16))
    assert np.allclose(ch.cheb_eval_scalar(alpha, np.cos(th)), trig, atol=1e-13)


def test_scalar_recurrence_matches_library():
    alpha = ch.coeffs_sign_interp(63, 0.08)
    x = np.linspace(-1, 1, 301)
    assert np.allclose(ch.cheb_eval_scalar(alpha, x), npcheb.chebval(x, alpha), atol=1e-13)


@pytest.mark.parametrize("deg,eps,tol", [(63, 0.077, 6e-3), (199, 0.03, 6e-3), (399, 0.01, 2e-2)])
def test_interp_rule_quality(deg, eps, tol):
    alpha = ch.coeffs_sign_interp(deg, eps)
    assert np.all(alpha[0::2] == 0.0)
    x = np.linspace(eps, 1.0, 4001)
    p = ch.cheb_eval_scalar(alpha, x)
    assert np.max(np.abs(p - 1.0)) < tol
    assert np.allclose(ch.cheb_eval_scalar(alpha, -x), -p, atol=1e-14)   # odd
    xall = np.linspace(-1, 1, 8001)
    assert np.max(np.abs(ch.cheb_eval_scalar(alpha, xall))) < 1.02


def test_free_field_polynomial_closed_form():
    """U = 1: on a plane wave, p(X) psi = (p(E/lmax)/E) K(p) psi (K(p)^2 = E^2, p odd)."""
    dims = (4, 4, 4, 4)
    u = unit_field(dims)
    alpha = ch.coeffs_sign_interp(33, 0.07)
    rng = np.random.default_rng(3)
    for n in [(1, 0, 0, 0), (1, 2, 3, 1), (0, 0, 0, 0), (2, 0, 0, 0)]:
        sc = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, p = plane_wave(dims, n, sc)
        m = sum(1 - np.cos(q) for q in p)
        kp = GAMMA5 @ ((m - 1.5) * np.eye(4) + 1j * sum(np.sin(p[i]) * GAMMA[i] for i in range(4)))
        e = np.sqrt((m - 1.5) ** 2 + sum(np.sin(q) ** 2 for q in p))
        scale = ch.cheb_eval_scalar(alpha, e / LMAX) / e
        expect = scale * np.einsum("st,tc...->sc...", kp, psi)
        assert rel_err(ch.poly_apply(u, psi, alpha, LMAX), expect) < 1e-13


@pytest.fixture(scope="module")
def dense2():
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 51, noise=0.6)
    lam, vecs = dense_eigs(u)
    return dims, u, lam, vecs


def test_dense_polynomial(dense2):
    dims, u, lam, vecs = dense2
    alpha = ch.coeffs_sign_interp(45, 0.05)
    psi = latgen.gaussian_spinor(dims, 52)
    v = vecs.reshape(len(lam), -1).T
    expect = v @ (ch.cheb_eval_scalar(alpha, lam / LMAX) * (v.conj().T @ psi.ravel()))
    assert rel_err(ch.poly_apply(u, psi, alpha, LMAX).ravel(), expect) < 1e-13


def test_chebyshev_vectors_spectral_closed_form(dense2):
    """T_m(X) psi from the forward recurrence equals V cos(m arccos(Lambda/lmax)) V^+ psi, the
    first-kind Chebyshev polynomial in its trigonometric closed form applied on the exact
    eigenbasis (LAPACK); a dropped factor 2 or a shifted index fails from m = 2 on.  The norm
    bound ||T_m(X) psi|| <= ||psi|| for lmax >= ||K|| follows and is checked too."""
    dims, u, lam, vecs = dense2
    assert np.abs(lam).max() < LMAX
    psi = latgen.gaussian_spinor(dims, 53)
    nrm = np.linalg.norm(psi)
    v = vecs.reshape(len(lam), -1).T
    coef = v.conj().T @ psi.ravel()
    theta = np.arccos(lam / LMAX)
    ts = ch.chebyshev_vectors(u, psi, 60, LMAX)
    assert len(ts) == 61
    for m, t in enumerate(ts):
        expect = v @ (np.cos(m * theta) * coef)
        assert rel_err(t.ravel(), expect) < 1e-12, m
        assert np.linalg.norm(t) <= nrm * (1 + 1e-12)
    # the weighted sum of the vectors is the polynomial
    alpha = ch.coeffs_sign_interp(59, 0.06)
    total = sum(a * t for a, t in zip(alpha, ts))
    assert rel_err(total, ch.poly_apply(u, psi, alpha, LMAX)) < 1e-13


def test_deflation_exact_on_span_and_square_bound(dense2):
    dims, u, lam, vecs = dense2
    n_ev = 8
    alpha = ch.coeffs_sign_interp(31, np.abs(lam[n_ev]) / LMAX)
    phi, lam_d = vecs[:n_ev], lam[:n_ev]
    for i in range(n_ev):
        s = ch.sign_apply(u, phi[i], alpha, LMAX, phi, lam_d)
        assert rel_err(s, np.sign(lam_d[i]) * phi[i]) < 1e-13
    psi = latgen.gaussian_spinor(dims, 54)
    s = ch.sign_apply(u, psi, alpha, LMAX, phi, lam_d)
    s2 = ch.sign_apply(u, s, alpha, LMAX, phi, lam_d)
    undeflated = lam[n_ev:] / LMAX
    bound = np.max(np.abs(ch.cheb_eval_scalar(alpha, undeflated) ** 2 - 1.0))
    assert np.linalg.norm(s2 - psi) <= bound * np.linalg.norm(psi) * (1 + 1e-10)
    # and the exact spectral form: (S^2 - 1) = (p^2 - 1)(1 - P)
    v = vecs.reshape(len(lam), -1).T
    pv = ch.cheb_eval_scalar(alpha, lam / LMAX)
    sv = np.where(np.arange(len(lam)) < n_ev, np.sign(lam), pv)
    expect = v @ (sv * sv * (v.conj().T @ psi.ravel()))
    assert rel_err(s2.ravel(), expect) < 1e-12


def test_weights():
    alpha = ch.coeffs_sign_interp(31, 0.1)
    lam = np.array([-0.3, 0.2, 0.0, 1.1])
    w = ch.deflation_weights(alpha, lam, LMAX)
    assert np.allclose(w, np.sign(lam) - npcheb.chebval(lam / LMAX, alpha), atol=1e-15)
    assert w[2] == 0.0


def test_cgs2_and_projection_adjoint():
    dims = (2, 2, 2, 4)
    raw = latgen.gaussian_spinor(dims, 61, nrhs=6)
    q = deflation.cgs2(raw)
    g = q.reshape(6, -1).conj() @ q.reshape(6, -1).T
    assert np.abs(g - np.eye(6)).max() < 1e-14
    # same span as LAPACK's QR: identical projectors
    qr, _ = np.linalg.qr(raw.reshape(6, -1).T)
    p1 = q.reshape(6, -1).T @ q.reshape(6, -1).conj()
    p2 = qr @ qr.conj().T
    assert np.abs(p1 - p2).max() < 1e-13
    # <c, Phi^+ psi> = <Phi c, psi>
    psi = latgen.gaussian_spinor(dims, 62)
    c = np.random.default_rng(1).standard_normal(6) + 0j
    lhs = np.vdot(c, deflation.project(q, psi))
    rhs = np.vdot(deflation.correct(q, np.zeros_like(psi), c, np.ones(6)), psi)
    assert abs(lhs - rhs) < 1e-13


def test_sign_and_overlap_gauge_covariance():
    dims = (2, 2, 4, 2)
    u = latgen.random_su3_field(dims, 71, noise=0.5)
    lam, vecs = dense_eigs(u)
    n_ev = 4
    alpha = ch.coeffs_sign_interp(41, abs(lam[n_ev]) / LMAX)
    psi = latgen.gaussian_spinor(dims, 72)
    om = latgen.random_gauge_transform(dims, 73)
    u2 = latgen.gauge_transform_links(u, om)
    phi2 = latgen.gauge_transform_spinor(vecs[:n_ev], om)
    psi2 = latgen.gauge_transform_spinor(psi, om)
    for mu in (0.0, 0.05):
        a = overlap.overlap_apply(u2, psi2, mu, alpha, LMAX, phi2, lam[:n_ev])
        b = latgen.gauge_transform_spinor(
            overlap.overlap_apply(u, psi, mu, alpha, LMAX, vecs[:n_ev], lam[:n_ev]), om)
        assert rel_err(a, b) < 1e-13


def test_overlap_adjoint_and_gw_identity(dense2):
    dims, u, lam, vecs = dense2
    n_ev = 6
    alpha = ch.coeffs_sign_interp(31, abs(lam[n_ev]) / LMAX)
    phi, lam_d = vecs[:n_ev], lam[:n_ev]
    chi = latgen.gaussian_spinor(dims, 81)
    psi = latgen.gaussian_spinor(dims, 82)
    mu = 0.05
    lhs = np.vdot(chi, overlap.overlap_dagger_apply(u, psi, mu, alpha, LMAX, phi, lam_d))
    rhs = np.vdot(overlap.overlap_apply(u, chi, mu, alpha, LMAX, phi, lam_d), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13

    def d(v):
        return overlap.overlap_apply(u, v, 0.0, alpha, LMAX, phi, lam_d)

    def s(v):
        return ch.sign_apply(u, v, alpha, LMAX, phi, lam_d)

    g5 = wilson.gamma5
    gw = g5(d(psi)) + d(g5(psi)) - 2.0 * d(g5(d(psi)))
    rhs = -0.5 * g5(s(s(psi)) - psi)
    assert np.linalg.norm(gw - rhs) < 1e-13 * np.linalg.norm(psi)
    # at this degree the GW residual is small but not zero; it is bounded by the sign error
    undeflated = lam[n_ev:] / LMAX
    bound = 0.5 * np.max(np.abs(ch.cheb_eval_scalar(alpha, undeflated) ** 2 - 1.0))
    assert np.linalg.norm(gw) <= bound * np.linalg.norm(psi) * (1 + 1e-10)


def test_overlap_free_field_zero_mode():
    """U = 1, p = 0: K = -1.5 gamma5, exact sign gives D[mu] = mu; the polynomial deviates by at
    most (1 - mu)/2 |1 - p(1.5/lmax)|."""
    dims = (4, 4, 4, 4)
    u = unit_field(dims)
    alpha = ch.coeffs_sign_interp(63, 0.07)
    sc = np.random.default_rng(5).standard_normal((4, 3)) + 0j
    psi, _ = plane_wave(dims, (0, 0, 0, 0), sc)
    mu = 0.1
    out = overlap.overlap_apply(u, psi, mu, alpha, LMAX)
    pv = ch.cheb_eval_scalar(alpha, 1.5 / LMAX)
    expect = (mu + 0.5 * (1 - mu) * (1 - pv)) * psi
    assert rel_err(out, expect) < 1e-13
    assert abs(1 - pv) < 5e-3
