"""ovl_overlap_apply_noalloc (the overlap operator of Sec. 2, eq. 1, for callers that cannot
allocate) against ovl_overlap_apply through the C ABI: same handles, same inputs, results within
the FP64 bar (1e-12) and the FP32 bar (1e-6) -- in fact bitwise, since both run the same kernels in
the same launch configuration.  Two calls in a row, the second on a smaller input, so the shared
static work space is reused with a different layout; an evaluation that needs more than the
static work space is rejected with EINVAL.
"""
import ctypes

import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
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


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.complex128).numpy()


def noalloc(ovl, g, poly, defl, mu, dagger, out, psi):
    from paper_1510_06897_amd import _lib
    from paper_1510_06897_amd.api import _ptr, _spin_dtype, _stream
    nrhs = 1 if psi.dim() == 6 else int(psi.shape[0])
    lib = _lib.load()
    return lib.ovl_overlap_apply_noalloc(g.handle, poly._h, defl._h if defl is not None else None,
                                         float(mu), int(dagger), _ptr(out), _ptr(psi), nrhs,
                                         _spin_dtype(psi), _stream())


def problem(ovl, dims, store, nrhs, n_ev, seed):
    u = latgen.random_su3_field(dims, seed, noise=0.4)
    psi = latgen.gaussian_spinor(dims, seed + 1, nrhs=nrhs)
    phi = latgen.gaussian_spinor(dims, seed + 2, nrhs=n_ev) if n_ev else None
    g = ovl.GaugeField(dev(u), store)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    d = ovl.Deflation(dev(phi), np.linspace(-0.6, 0.6, n_ev) + 0.01,
                      "f64" if store == "f64" else "f32") if n_ev else None
    x = dev(psi, cdt)
    if nrhs == 1:
        x = x.reshape(x.shape[1:]) if x.dim() == 7 else x
    return g, d, x


@pytest.mark.parametrize("store,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_noalloc_matches_overlap_apply_twice_second_smaller(ovl, store, tol):
    alpha = och.coeffs_sign_interp(64, 0.08)
    poly = ovl.Polynomial(alpha, LMAX)
    cases = [((8, 8, 8, 16), 2, 6, 0.05, 0), ((4, 4, 4, 4), 1, 3, 0.1, 1)]
    for dims, nrhs, n_ev, mu, dagger in cases:
        print(f"noalloc {store} dims={dims} nrhs={nrhs} n_ev={n_ev} dagger={dagger}", flush=True)
        g, d, x = problem(ovl, dims, store, nrhs, n_ev, 10900 + dims[0])
        ref = ovl.overlap_apply(g, poly, x, mu, defl=d, dagger=bool(dagger))
        out = torch.empty_like(x)
        assert noalloc(ovl, g, poly, d, mu, dagger, out, x) == 0
        got, want = host(out), host(ref)
        assert rel_err(got, want) < tol
        assert np.array_equal(got, want)
        assert g.flags() == 0


def test_noalloc_rejects_work_space_above_the_static_size(ovl):
    from paper_1510_06897_amd import _lib
    dims = (8, 8, 8, 16)
    poly = ovl.Polynomial(och.coeffs_sign_interp(8, 0.2), LMAX)
    g, _, _ = problem(ovl, dims, "f64", 1, 0, 10950)
    # 44 FP64 right-hand sides of 8192 sites: a 66 MB recurrence vector
    x = torch.zeros((44, 4, 3, 16, 8, 8, 8), dtype=torch.complex128, device="cuda")
    x[:, 0, 0, 0, 0, 0, 0] = 1.0
    out = torch.empty_like(x)
    rc = noalloc(ovl, g, poly, None, 0.1, 0, out, x)
    assert rc == -1
    assert b"fixed buffer" in _lib.load().ovl_last_error()
    # the same call still works through the allocating entry point
    ovl.overlap_apply(g, poly, x, 0.1, out=out)
    torch.cuda.synchronize()
