"""Pins of the oracle's gauge-link derivatives against finite differences and exact identities.

The force G = d Re<chi, p(K/lmax) psi>/dU is not printed in the paper (HMC context, Sec. 1); it is
pinned by central finite differences in FP64 (which share nothing with the reverse sweep), by the
exact affine dependence of D_W on U (Sec. 2, eq. 2), by gauge covariance, and by the degree-1 case.
"""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as ch
from oracle import force, wilson
from tests.conftest import rel_err

LMAX = 6.5


def _loss(u, chi, psi, alpha):
    return float(np.real(np.vdot(chi, ch.poly_apply(u, psi, alpha, LMAX))))


def test_wilson_vjp_affine_exact():
    """L(U) = Re<a, D_W(U) t> is affine in U: L(U) - L(0) = Re sum tr(G^+ U) exactly."""
    dims = (3, 2, 2, 4)
    u = latgen.random_su3_field(dims, 91, noise=0.9)
    a = latgen.gaussian_spinor(dims, 92)
    t = latgen.gaussian_spinor(dims, 93)
    g = force.wilson_link_vjp(a, t)
    l_u = np.real(np.vdot(a, wilson.dw(u, t)))
    l_0 = np.real(np.vdot(a, wilson.dw(np.zeros_like(u), t)))
    assert abs((l_u - l_0) - np.real(np.vdot(g, u))) < 1e-12 * abs(l_u - l_0)


def test_degree_one_reduces_to_vjp():
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 94)
    chi = latgen.gaussian_spinor(dims, 95)
    psi = latgen.gaussian_spinor(dims, 96)
    g = force.sign_force(u, chi, psi, np.array([0.0, 1.0]), LMAX)
    assert rel_err(g, force.wilson_link_vjp(wilson.gamma5(chi), psi) / LMAX) < 1e-15


@pytest.mark.parametrize("deg", [9, 63])
def test_force_central_fd(deg):
    dims = (2, 2, 2, 4)
    u = latgen.random_su3_field(dims, 101, noise=0.5)
    chi = latgen.gaussian_spinor(dims, 102)
    psi = latgen.gaussian_spinor(dims, 103)
    alpha = ch.coeffs_sign_interp(deg, 0.1)
    g = force.sign_force(u, chi, psi, alpha, LMAX)
    rng = np.random.Generator(np.random.PCG64(latgen.seed_for("direction", 0)))
    # one whole-field direction (arbitrary complex perturbation, not restricted to SU(3))
    d = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    errs = []
    for eps in (1e-5, 1e-6):
        fd = (_loss(u + eps * d, chi, psi, alpha) - _loss(u - eps * d, chi, psi, alpha)) / (2 * eps)
        an = np.real(np.vdot(g, d))
        errs.append(abs(fd - an) / abs(an))
    assert errs[1] < 1e-7
    # sampled single entries (real and imaginary parts)
    for _ in range(8):
        idx = tuple(int(rng.integers(0, n)) for n in u.shape)
        for part in (1.0, 1j):
            e = np.zeros_like(u)
            e[idx] = part
            h = 1e-6
            fd = (_loss(u + h * e, chi, psi, alpha) - _loss(u - h * e, chi, psi, alpha)) / (2 * h)
            an = g[idx].real if part == 1.0 else g[idx].imag
            assert abs(fd - an) < 1e-7 * max(1.0, np.abs(g).max())


@pytest.mark.slow
def test_force_central_fd_degree_299_4x4x4x4():
    """The force workload's degree (299) on a 4^4 lattice, one whole-field direction."""
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 10500 + 1)
    chi = latgen.gaussian_spinor(dims, 20501)
    psi = latgen.gaussian_spinor(dims, 20500)
    alpha = ch.coeffs_sign_interp(299, 0.05)
    g = force.sign_force(u, chi, psi, alpha, LMAX)
    rng = np.random.Generator(np.random.PCG64(latgen.seed_for("direction", 0)))
    d = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    eps = 1e-6
    fd = (_loss(u + eps * d, chi, psi, alpha) - _loss(u - eps * d, chi, psi, alpha)) / (2 * eps)
    an = np.real(np.vdot(g, d))
    assert abs(fd - an) / abs(an) < 1e-7


def test_force_gauge_covariance():
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 111, noise=0.6)
    chi = latgen.gaussian_spinor(dims, 112)
    psi = latgen.gaussian_spinor(dims, 113)
    om = latgen.random_gauge_transform(dims, 114)
    alpha = ch.coeffs_sign_interp(15, 0.1)
    g = force.sign_force(u, chi, psi, alpha, LMAX)
    g2 = force.sign_force(latgen.gauge_transform_links(u, om),
                          latgen.gauge_transform_spinor(chi, om),
                          latgen.gauge_transform_spinor(psi, om), alpha, LMAX)
    # G transforms like a link: G'_mu(x) = Omega(x) G_mu(x) Omega(x+mu)^+
    assert rel_err(g2, latgen.gauge_transform_links(g, om)) < 1e-13


def test_hmc_force_direction_derivative():
    """dL/d eps along U -> exp(eps Y) U equals Re tr(F^+ Y) with F = -TA(U G^+)."""
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 121, noise=0.6)
    chi = latgen.gaussian_spinor(dims, 122)
    psi = latgen.gaussian_spinor(dims, 123)
    alpha = ch.coeffs_sign_interp(15, 0.1)
    g = force.sign_force(u, chi, psi, alpha, LMAX)
    f = force.hmc_force(u, g)
    # random su(3) direction at every link: Y = i H, H traceless Hermitian
    rng = np.random.default_rng(5)
    h = np.einsum("...a,aij->...ij", rng.standard_normal(latgen.site_shape(dims) + (4, 8)),
                  latgen.gell_mann())
    y = 1j * np.moveaxis(h, (4, 5, 6), (0, 1, 2))

    def moved(eps):
        w, v = np.linalg.eigh(np.moveaxis(-1j * eps * y, (0, 1, 2), (4, 5, 6)))
        ex = np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())
        ex = np.moveaxis(ex, (4, 5, 6), (0, 1, 2))
        return np.einsum("mabTZYX,mbcTZYX->macTZYX", ex, u)

    h_ = 1e-6
    fd = (_loss(moved(h_), chi, psi, alpha) - _loss(moved(-h_), chi, psi, alpha)) / (2 * h_)
    an = np.real(np.vdot(f, y))
    assert abs(fd - an) / abs(an) < 1e-7


@pytest.mark.parametrize("deg", [1, 2, 9, 64])
def test_directional_derivative_fd_and_reverse_mode(deg):
    """The forward-mode directional derivative against central finite differences of the
    polynomial (independent of any derivative code) and against the reverse sweep's G
    contracted with the same direction, Re sum tr(G^+ Y)."""
    dims = (2, 3, 2, 4)
    u = latgen.smeared_field(dims, 111, steps=1)
    chi = latgen.gaussian_spinor(dims, 112)
    psi = latgen.gaussian_spinor(dims, 113)
    alpha = ch.coeffs_sign_interp(max(deg, 1), 0.1) if deg > 2 else np.array([0.3, -0.7, 0.4][:deg + 1])
    rng = np.random.Generator(np.random.PCG64(latgen.seed_for("direction", 3)))
    y = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    dl = force.sign_force_directional(u, chi, psi, alpha, LMAX, y)
    h = 1e-6
    fd = (_loss(u + h * y, chi, psi, alpha) - _loss(u - h * y, chi, psi, alpha)) / (2 * h)
    assert abs(dl - fd) < 1e-7 * max(1.0, abs(fd))
    g = force.sign_force(u, chi, psi, alpha, LMAX)
    assert abs(dl - np.real(np.vdot(g, y))) < 1e-12 * max(1.0, abs(dl))
