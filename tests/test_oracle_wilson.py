"""Pins of the oracle's Wilson operator and kernel K against closed forms and identities.

Sec. 2, eq. 2 defines D_W; K = gamma5 (D_W - m_W), m_W = 1.5 (Sec. 2).  None of these checks
re-types the oracle's formula: free-field plane waves have a closed-form symbol, gamma5-hermiticity
and gauge covariance are structural identities, and the free 2^4 spectrum is known exactly.
"""
import itertools
import json
import os

import numpy as np
import pytest

import latgen
from oracle import wilson
from oracle.gamma import GAMMA, GAMMA5
from tests.conftest import rel_err

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def unit_field(dims):
    shp = latgen.site_shape(dims)
    u = np.zeros((4, 3, 3) + shp, dtype=np.complex128)
    for a in range(3):
        u[:, a, a] = 1.0
    return u


def plane_wave(dims, n, spin_colour):
    """exp(i p.x) u with p_mu = 2 pi n_mu / L_mu, u a constant [4, 3] spin-colour vector."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    p = [2 * np.pi * n[i] / dims[i] for i in range(4)]
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return spin_colour[:, :, None, None, None, None] * phase[None, None], p


def test_paper_parameters_golden():
    with open(os.path.join(GOLDEN, "paper_parameters.json")) as f:
        g = json.load(f)
    assert wilson.M_W == g["m_W"]["value"]
    # the diagonal of D_W is 4: D_W applied to a constant spinor on the unit field is 0 ...
    dims = (2, 2, 2, 2)
    const = np.ones((4, 3) + latgen.site_shape(dims), dtype=np.complex128)
    assert np.abs(wilson.dw(unit_field(dims), const)).max() < 1e-14
    # ... and on a zero gauge field D_W = 4 exactly
    psi = latgen.gaussian_spinor(dims, 1)
    zero = np.zeros((4, 3, 3) + latgen.site_shape(dims), dtype=np.complex128)
    assert np.allclose(wilson.dw(zero, psi), g["wilson_diagonal"]["value"] * psi, atol=0)


def test_gamma_basis():
    for a in range(4):
        assert np.allclose(GAMMA[a], GAMMA[a].conj().T)
        for b in range(4):
            ac = GAMMA[a] @ GAMMA[b] + GAMMA[b] @ GAMMA[a]
            assert np.allclose(ac, 2.0 * np.eye(4) * (a == b), atol=1e-15)
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]), atol=1e-15)


@pytest.mark.parametrize("dims", [(4, 6, 2, 8), (3, 5, 4, 2)])
def test_free_field_plane_waves(dims):
    rng = np.random.default_rng(7)
    u = unit_field(dims)
    for _ in range(6):
        n = [int(rng.integers(0, dims[i])) for i in range(4)]
        sc = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, p = plane_wave(dims, n, sc)
        symbol = sum((1 - np.cos(p[m])) * np.eye(4) + 1j * np.sin(p[m]) * GAMMA[m]
                     for m in range(4))
        expect = np.einsum("st,tc...->sc...", symbol, psi)
        assert rel_err(wilson.dw(u, psi), expect) < 1e-14


def test_free_kernel_spectrum_2x2x2x2():
    """U = 1 on 2^4: K has eigenvalues +-|M - 1.5|, M = 2 * (number of momenta equal to pi)."""
    from oracle.eigen import dense_kop
    dims = (2, 2, 2, 2)
    mat = dense_kop(unit_field(dims))
    assert np.allclose(mat, mat.conj().T, atol=1e-15)
    got = np.sort(np.linalg.eigvalsh(mat))
    expect = []
    for k in range(5):
        mult = 12 * len(list(itertools.combinations(range(4), k)))
        e = abs(2 * k - 1.5)
        # gamma5 (M - 1.5) with zero sines: half the spin components +, half -
        expect += [e] * (mult // 2) + [-e] * (mult // 2)
    assert np.allclose(got, np.sort(expect), atol=1e-13)


def test_free_kernel_extremes_4x4x4x4():
    """|lambda(K)| over free momenta on 4^4 spans [0.5, 6.5] (closed form, sampled momenta)."""
    dims = (4, 4, 4, 4)
    u = unit_field(dims)
    sc = np.zeros((4, 3), dtype=np.complex128)
    vals = []
    for n in [(0, 0, 0, 0), (2, 0, 0, 0), (2, 2, 2, 2), (1, 3, 0, 2)]:
        best = []
        for s in range(4):
            sc[:] = 0
            sc[s, 0] = 1
            psi, p = plane_wave(dims, n, sc)
            kpsi = wilson.kop(u, psi)
            m = sum(1 - np.cos(q) for q in p)
            ssq = sum(np.sin(q) ** 2 for q in p)
            e = np.sqrt((m - 1.5) ** 2 + ssq)
            # K^2 = E^2 on the plane-wave subspace
            k2 = wilson.kop(u, kpsi)
            assert rel_err(k2, e * e * psi) < 1e-13
            best.append(e)
        vals.append(best[0])
    assert np.isclose(min(vals), 0.5) and np.isclose(max(vals), 6.5)


def test_gamma5_hermiticity():
    dims = (3, 2, 4, 5)
    u = latgen.random_su3_field(dims, 11)
    chi = latgen.gaussian_spinor(dims, 12)
    psi = latgen.gaussian_spinor(dims, 13)
    lhs = np.vdot(chi, wilson.dw_dagger(u, psi))
    rhs = np.vdot(wilson.dw(u, chi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-14
    # K is Hermitian
    lhs = np.vdot(chi, wilson.kop(u, psi))
    rhs = np.vdot(wilson.kop(u, chi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-14


def test_gauge_covariance():
    dims = (4, 2, 3, 4)
    u = latgen.random_su3_field(dims, 21, noise=0.7)
    psi = latgen.gaussian_spinor(dims, 22)
    om = latgen.random_gauge_transform(dims, 23)
    u2 = latgen.gauge_transform_links(u, om)
    psi2 = latgen.gauge_transform_spinor(psi, om)
    lhs = wilson.dw(u2, psi2)
    rhs = latgen.gauge_transform_spinor(wilson.dw(u, psi), om)
    assert rel_err(lhs, rhs) < 1e-14
    lhs = wilson.kop(u2, psi2)
    rhs = latgen.gauge_transform_spinor(wilson.kop(u, psi), om)
    assert rel_err(lhs, rhs) < 1e-14


def test_kernel_norm_bound():
    """||D_W - m_W|| <= |4 - m_W| + 4 = 6.5 for unitary links (each hop term is unitary)."""
    from oracle.eigen import dense_kop
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 31, noise=1.0)
    lam = np.linalg.eigvalsh(dense_kop(u))
    assert np.abs(lam).max() <= 6.5 + 1e-12


def test_brute_force_site_loop():
    """Eq. 2 evaluated site by site with explicit modular neighbour indices (extent-2 directions
    included, where x+mu and x-mu are the same site and both hops still contribute)."""
    dims = (2, 3, 2, 3)
    lx, ly, lz, lt = dims
    u = latgen.random_su3_field(dims, 41, noise=0.8)
    psi = latgen.gaussian_spinor(dims, 42)
    one = np.eye(4)
    out = np.zeros_like(psi)
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    acc = 4.0 * psi[:, :, t, z, y, x]
                    for mu in range(4):
                        c = [x, y, z, t]
                        f = list(c)
                        b = list(c)
                        f[mu] = (c[mu] + 1) % dims[mu]
                        b[mu] = (c[mu] - 1) % dims[mu]
                        pf = psi[:, :, f[3], f[2], f[1], f[0]]
                        pb = psi[:, :, b[3], b[2], b[1], b[0]]
                        uf = u[mu, :, :, t, z, y, x]
                        ub = u[mu, :, :, b[3], b[2], b[1], b[0]].conj().T
                        acc = acc - 0.5 * ((one - GAMMA[mu]) @ (pf @ uf.T)
                                           + (one + GAMMA[mu]) @ (pb @ ub.T))
                    out[:, :, t, z, y, x] = acc
    assert rel_err(wilson.dw(u, psi), out) < 1e-15
