"""GPU parity of the stout smearing and its chain rule (Sec. 2: the links entering K are smoothed by
3 steps of over-improved stout smearing, rho = 0.1, eps = -0.25; Sec. 1: HMC needs the force on
the thin links) against the FP64 oracle (oracle/stout.py, pinned by the action gradient, the
plain-stout limit, SU(3), gauge covariance and finite differences).

The device evaluates exp by a scaled Taylor series and its derivative by the Frechet series; the
oracle by eigen-decomposition and divided differences.  Both are FP64, so the tolerance is 1e-12
relative for the links and the derivatives.
"""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import force as oforce
from oracle import stout as ostout
from tests.conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LMAX = 6.5


@pytest.fixture(scope="module")
def ovl():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1510_06897_amd as m
    m.load()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.complex128)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gauss(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# extent-1, extent-2 and odd extents pin the periodic wrap of the five-link paths (offsets up to
# two sites along a direction of extent 1 or 2)
DIMS = [(4, 4, 4, 4), (3, 2, 5, 4), (2, 3, 2, 3), (2, 1, 3, 2)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("eps", [-0.25, 1.0, 0.0])
@pytest.mark.parametrize("steps", [1, 3])
def test_smear_matches_oracle(ovl, dims, eps, steps):
    print(f"stout smear dims={dims} eps={eps} steps={steps}", flush=True)
    u = latgen.random_su3_field(dims, 10600, noise=0.6)
    got = host(ovl.stout_smear(dev(u), 0.1, eps, steps))
    ref = ostout.smear(u, 0.1, eps, steps)
    assert rel_err(got, ref) < 1e-13
    assert np.abs(got - ref).max() < 1e-13


def test_smear_zero_steps_copies_and_large_rho(ovl):
    dims = (3, 2, 4, 2)
    u = latgen.random_su3_field(dims, 10601, noise=1.0)
    assert np.array_equal(host(ovl.stout_smear(dev(u), 0.1, -0.25, 0)), u)
    # rho = 0.7 and rough links: ||M|| above 1/2, so the exponential is scaled and squared
    got = host(ovl.stout_smear(dev(u), 0.7, -0.25, 2))
    assert rel_err(got, ostout.smear(u, 0.7, -0.25, 2)) < 1e-12


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("eps,steps", [(-0.25, 3), (1.0, 1), (-0.25, 2)])
def test_backward_matches_oracle(ovl, dims, eps, steps):
    print(f"stout backward dims={dims} eps={eps} steps={steps}", flush=True)
    u = latgen.random_su3_field(dims, 10602, noise=0.6)
    g_s = gauss(u.shape, 40600)
    got = host(ovl.stout_backward(dev(u), dev(g_s), 0.1, eps, steps))
    ref = ostout.smear_backward(u, 0.1, eps, steps, g_s)
    assert rel_err(got, ref) < 1e-12


def test_backward_is_the_adjoint_of_the_linearisation(ovl):
    """Re tr(G_thin^+ Y) equals the central difference of Re tr(G_s^+ stout(U + h Y)) (a property
    of the device pair alone, at any size)."""
    dims = (4, 3, 2, 4)
    u = latgen.random_su3_field(dims, 10603, noise=0.5)
    g_s = gauss(u.shape, 40601)
    y = gauss(u.shape, 40602)
    gt = host(ovl.stout_backward(dev(u), dev(g_s), 0.1, -0.25, 3))
    h = 1e-5

    def lval(v):
        return float(np.real(np.vdot(g_s, host(ovl.stout_smear(dev(v), 0.1, -0.25, 3)))))

    fd = (lval(u + h * y) - lval(u - h * y)) / (2 * h)
    an = float(np.real(np.vdot(gt, y)))
    assert abs(fd - an) < 1e-7 * abs(an)


def test_smeared_force_composes_with_the_sign_function(ovl):
    """autograd through StoutFunction and SignFunction: d Re<chi, p(X[stout(U)]) psi>/dU against
    the oracle's sign force on the smeared links carried back by its smearing derivative."""
    dims = (4, 4, 4, 4)
    u = latgen.random_su3_field(dims, 10604, noise=0.3)
    psi = latgen.gaussian_spinor(dims, 20604)
    chi = latgen.gaussian_spinor(dims, 20605)
    alpha = och.coeffs_sign_interp(31, 0.1)
    poly = ovl.Polynomial(alpha, LMAX)
    du = dev(u).requires_grad_(True)
    us = ovl.StoutFunction.apply(du, 0.1, -0.25, 3)
    y = ovl.SignFunction.apply(us, dev(psi), poly, "f64")
    loss = torch.real(torch.sum(torch.conj(dev(chi)) * y))
    loss.backward()
    got = host(du.grad)
    us_ref = ostout.smear(u, 0.1, -0.25, 3)
    g_s = oforce.sign_force(us_ref, chi, psi, alpha, LMAX)
    ref = ostout.smear_backward(u, 0.1, -0.25, 3, g_s)
    assert rel_err(got, ref) < 1e-11


def test_stout_rejects_bad_arguments(ovl):
    from paper_1510_06897_amd import _lib
    u = dev(latgen.random_su3_field((2, 2, 2, 2), 1, noise=0.3))
    with pytest.raises(_lib.OvlError) as e:
        ovl.stout_smear(u, 0.1, -0.25, 3, out=u)
    assert e.value.code == -4
    with pytest.raises(_lib.OvlError) as e:
        ovl.stout_smear(u, float("nan"), -0.25, 3)
    assert e.value.code == -7
    with pytest.raises(_lib.OvlError) as e:
        ovl.stout_backward(u, u.clone(), 0.1, -0.25, 3, out=u)
    assert e.value.code == -4
