"""Pins of the oracle's stout smearing (Sec. 2: 3 steps of over-improved stout smearing, rho = 0.1,
eps = -0.25) and of its chain-rule derivative.

* The staple sum is rho times the gradient of the over-improved action: checked against the
  action computed by explicit loop products (it is linear in every single link, so a central
  difference with a unit step is exact up to rounding).
* eps = 1 reduces to plain stout smearing, implemented independently in latgen.
* Smeared links are SU(3); smearing is gauge covariant; the unit field is a fixed point.
* The derivative through the smearing against central finite differences, alone and composed
  with the force of the Chebyshev sign function.
"""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as ch
from oracle import force, stout
from tests.conftest import rel_err

LMAX = 6.5


def test_staples_are_the_action_gradient():
    dims = (3, 4, 3, 3)
    u = latgen.random_su3_field(dims, 301, noise=0.7)
    eps = -0.25
    c = stout.staples(u, 1.0, eps)
    rng = np.random.default_rng(302)
    for _ in range(12):
        idx = tuple(int(rng.integers(0, n)) for n in u.shape)
        for part in (1.0, 1j):
            e = np.zeros_like(u)
            e[idx] = part
            d = (stout.action(u + e, eps) - stout.action(u - e, eps)) / 2.0
            want = c[idx].real if part == 1.0 else c[idx].imag
            assert abs(d - want) < 1e-11 * max(1.0, np.abs(c).max())


def test_plain_stout_limit_matches_latgen():
    dims = (4, 3, 4, 4)
    u = latgen.random_su3_field(dims, 303, noise=0.5)
    a = stout.smear(u, 0.1, 1.0, 3)
    b = latgen.stout_smear(u, 0.1, 3)
    assert np.abs(a - b).max() < 1e-13


def test_smeared_links_su3_and_gauge_covariant():
    dims = (4, 4, 3, 4)
    u = latgen.random_su3_field(dims, 304, noise=0.6)
    s = stout.smear(u, 0.1, -0.25, 2)
    m = np.moveaxis(s.reshape(4, 3, 3, -1), -1, 1)        # [mu, site, a, b]
    assert np.abs(m @ np.conj(np.swapaxes(m, -1, -2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(m) - 1.0).max() < 1e-13
    om = latgen.random_gauge_transform(dims, 305)
    a = stout.smear(latgen.gauge_transform_links(u, om), 0.1, -0.25, 2)
    b = latgen.gauge_transform_links(s, om)
    assert np.abs(a - b).max() < 1e-12
    one = np.zeros_like(u)
    for mu in range(4):
        for i in range(3):
            one[mu, i, i] = 1.0
    assert np.abs(stout.smear(one, 0.1, -0.25, 3) - one).max() < 1e-15


@pytest.mark.parametrize("eps,steps", [(1.0, 1), (-0.25, 1), (-0.25, 3)])
def test_smear_backward_central_fd(eps, steps):
    """L(U) = Re sum tr(W^+ U'(U)) for a fixed random W: the reverse sweep against central
    differences along a random direction and on single link entries."""
    dims = (3, 3, 3, 4)
    u = latgen.random_su3_field(dims, 306, noise=0.5)
    rng = np.random.default_rng(307)
    w = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)

    def loss(x):
        return float(np.real(np.vdot(w, stout.smear(x, 0.1, eps, steps))))

    g = stout.smear_backward(u, 0.1, eps, steps, w)
    d = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    h = 1e-5
    fd = (loss(u + h * d) - loss(u - h * d)) / (2 * h)
    assert abs(fd - np.real(np.vdot(g, d))) < 1e-8 * abs(fd)
    for _ in range(4):
        idx = tuple(int(rng.integers(0, n)) for n in u.shape)
        for part in (1.0, 1j):
            e = np.zeros_like(u)
            e[idx] = part
            fd = (loss(u + h * e) - loss(u - h * e)) / (2 * h)
            an = g[idx].real if part == 1.0 else g[idx].imag
            assert abs(fd - an) < 1e-8 * max(1.0, np.abs(g).max())


def test_smeared_sign_force_central_fd():
    """L(U) = Re<chi, p(K[U'(U)]/lmax) psi> with U' three over-improved stout steps: the sign
    function's force on the smeared links carried back to the thin links."""
    dims = (2, 2, 3, 4)
    u = latgen.random_su3_field(dims, 308, noise=0.4)
    chi = latgen.gaussian_spinor(dims, 309)
    psi = latgen.gaussian_spinor(dims, 310)
    alpha = ch.coeffs_sign_interp(15, 0.1)

    def loss(x):
        us = stout.smear(x, 0.1, -0.25, 3)
        return float(np.real(np.vdot(chi, ch.poly_apply(us, psi, alpha, LMAX))))

    us = stout.smear(u, 0.1, -0.25, 3)
    g = stout.smear_backward(u, 0.1, -0.25, 3, force.sign_force(us, chi, psi, alpha, LMAX))
    rng = np.random.default_rng(311)
    d = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    h = 1e-5
    fd = (loss(u + h * d) - loss(u - h * d)) / (2 * h)
    assert abs(fd - np.real(np.vdot(g, d))) < 1e-8 * abs(fd)


@pytest.mark.parametrize("eps", [1.0, 0.0, -0.25, 0.5])
def test_action_normalisation_and_limits(eps):
    """The weights of the reading: eps = 1 is the plain (Wilson) staple, eps = 0 the tree-level
    Symanzik weights 5/3 and -1/12, and for every eps c_p + 8 c_r = 1, so a smooth field has the
    Wilson action to leading order: a constant abelian flux f through the (x, y) planes gives
    3 cos f per plaquette and 3 cos 2f per rectangle, S - S(f = 0) = -3/2 f^2 V (c_p + 8 c_r)
    + O(f^4)."""
    cp, cr = stout.coefficients(eps)
    if eps == 1.0:
        assert (cp, cr) == (1.0, 0.0)
    if eps == 0.0:
        assert abs(cp - 5.0 / 3.0) < 1e-15 and abs(cr + 1.0 / 12.0) < 1e-15
    assert abs(cp + 8.0 * cr - 1.0) < 1e-15
    dims = (4, 64, 1, 1)
    lx, ly = dims[0], dims[1]
    f = 2 * np.pi / (lx * ly) * 1   # one flux quantum over the (x, y) torus
    u = np.zeros((4, 3, 3, 1, 1, ly, lx), dtype=np.complex128)
    for mu in range(4):
        for i in range(3):
            u[mu, i, i] = 1.0
    y = np.arange(ly)[:, None] * np.ones((1, lx))
    x = np.arange(lx)[None, :] * np.ones((ly, 1))
    # U_y(x, y) = exp(i f x); U_x = 1 except U_x(lx - 1, y) = exp(-i f lx y): every (x, y)
    # plaquette, also across the periodic boundaries, carries the phase exp(i f)
    ph_y = np.exp(1j * f * x)
    ph_x = np.where(x == lx - 1, np.exp(-1j * f * lx * y), 1.0)
    for i in range(3):
        u[0, i, i, 0, 0] = ph_x
        u[1, i, i, 0, 0] = ph_y
    one = np.zeros_like(u)
    for mu in range(4):
        for i in range(3):
            one[mu, i, i] = 1.0
    vol = lx * ly
    ds = stout.action(u, eps) - stout.action(one, eps)
    want = 3 * vol * (cp * (np.cos(f) - 1) + cr * 2 * (np.cos(2 * f) - 1))
    assert abs(ds - want) < 1e-9 * abs(want)
    assert abs(ds / vol + 1.5 * f * f) < 0.1 * 1.5 * f * f
