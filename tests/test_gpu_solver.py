"""Overlap inversion on the GPU (FP64 defect correction around CG on the normal equations)
against the oracle's CG and a dense LAPACK solve."""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import overlap as oov
from oracle import solver as osol
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


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def problem():
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 10500, steps=1)
    b = latgen.gaussian_spinor(dims, 20500)
    from oracle.eigen import low_modes
    lam, phi, _ = low_modes(u, 4, LMAX, filter_degree=16)
    alpha = och.coeffs_sign_interp(31, 0.07)
    x_ref, _ = osol.overlap_cgnr(u, b, 0.05, alpha, LMAX, phi, lam, tol=1e-13, max_iter=2000)
    return dims, u, b, phi, lam, alpha, x_ref


@pytest.mark.parametrize("inner", [None, "f32", "bf16"])
def test_solve_against_oracle(ovl, problem, inner):
    dims, u, b, phi, lam, alpha, x_ref = problem
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    gi = ovl.GaugeField(dev(u), inner) if inner else None
    di = ovl.Deflation(dev(phi), lam, "f32") if inner else None
    x, its, res = ovl.overlap_solve(g, p, dev(b), 0.05, defl=d, g_inner=gi, defl_inner=di,
                                    tol=1e-11)
    got = x.cpu().numpy()
    assert res <= 1e-11 and its > 0
    # the residual with the oracle's operator, and the distance to the oracle's solution
    r = b - oov.overlap_apply(u, got, 0.05, alpha, LMAX, phi, lam)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-11
    assert rel_err(got, x_ref) < 1e-9
    assert g.flags() == 0


def test_solve_dense_2x2x2x2(ovl):
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 10501)
    b = latgen.gaussian_spinor(dims, 20501)
    alpha = och.coeffs_sign_interp(21, 0.1)
    ref = np.linalg.solve(osol.dense_overlap(u, 0.1, alpha, LMAX), b.reshape(-1)).reshape(b.shape)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    x, _, res = ovl.overlap_solve(g, p, dev(b), 0.1, tol=1e-13)
    assert rel_err(x.cpu().numpy(), ref) < 1e-11


def test_solve_errors(ovl):
    dims = (2, 2, 2, 4)
    u = latgen.random_su3_field(dims, 10502)
    b = dev(latgen.gaussian_spinor(dims, 20502))
    alpha = och.coeffs_sign_interp(15, 0.1)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve(g, p, b, 0.05, out=b)
    assert e.value.status == "OVL_EALIAS"
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve(g, p, b, 0.05, g_inner=ovl.GaugeField(dev(u), "f64"))
    assert e.value.status == "OVL_EDTYPE"
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve(g, p, b, 0.01, tol=1e-14, max_iter=2)
    assert e.value.status == "OVL_EDIVERGED"
    g32 = ovl.GaugeField(dev(u), "f32")
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve(g32, p, b, 0.05)
    assert e.value.status == "OVL_EDTYPE"


@pytest.mark.parametrize("inner,relax", [("f32", True), ("bf16", True), (None, False)])
def test_gmresr_to_1e13_against_oracle(ovl, problem, inner, relax):
    """GMRESR with inner CG in FP32 (FP32 or BF16 links) on a truncated polynomial and relaxed
    FP64 outer products, to the paper's overlap accuracy 1e-13 (Sec. 3); the residual with the
    oracle's operator and the distance to the oracle's CG solution."""
    dims, u, b, phi, lam, alpha, x_ref = problem
    print(f"gmresr inner={inner} relax={relax}", flush=True)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    gi = ovl.GaugeField(dev(u), inner) if inner else None
    di = ovl.Deflation(dev(phi), lam, "f32") if inner else None
    x, n_out, n_in, res = ovl.overlap_solve_gmresr(g, p, dev(b), 0.05, defl=d, g_inner=gi,
                                                   defl_inner=di, tol=1e-13, relax=relax)
    got = x.cpu().numpy()
    assert res <= 1e-13 and n_out > 0 and n_in > 0
    r = b - oov.overlap_apply(u, got, 0.05, alpha, LMAX, phi, lam)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 3e-13
    assert rel_err(got, x_ref) < 1e-10
    assert g.flags() == 0


def test_gmresr_dense_2x2x2x2(ovl):
    dims = (2, 2, 2, 2)
    u = latgen.random_su3_field(dims, 10503)
    b = latgen.gaussian_spinor(dims, 20503)
    alpha = och.coeffs_sign_interp(21, 0.1)
    ref = np.linalg.solve(osol.dense_overlap(u, 0.1, alpha, LMAX), b.reshape(-1)).reshape(b.shape)
    g = ovl.GaugeField(dev(u), "f64")
    gi = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    x, n_out, _, res = ovl.overlap_solve_gmresr(g, p, dev(b), 0.1, g_inner=gi, tol=1e-13,
                                                inner_poly_tol=1e-2)
    assert res <= 1e-13
    assert rel_err(x.cpu().numpy(), ref) < 1e-11


def test_gmresr_errors(ovl):
    dims = (2, 2, 2, 4)
    u = latgen.random_su3_field(dims, 10504)
    b = dev(latgen.gaussian_spinor(dims, 20504))
    alpha = och.coeffs_sign_interp(15, 0.1)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve_gmresr(g, p, b, 0.05, out=b)
    assert e.value.status == "OVL_EALIAS"
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve_gmresr(g, p, b, 0.05, inner_tol=1.5)
    assert e.value.status == "OVL_EINVAL"
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve_gmresr(g, p, b, 0.01, tol=1e-15, max_outer=1, max_inner=3)
    assert e.value.status == "OVL_EDIVERGED"
