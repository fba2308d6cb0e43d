"""Step graphs: repeated small sign and overlap evaluations replay their plain recurrence steps
from a captured HIP graph.  Every replay, with eager work and synchronisations between the
replays, must equal bitwise the result of the same call made with graphs off, and the oracle."""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import deflation as odefl
from oracle import overlap as oov
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
    yield m
    m.graph_enable(True)


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_graph_replays_equal_direct_launches(ovl, store):
    dims = (4, 6, 4, 8)
    u = latgen.smeared_field(dims, 10190, steps=1)
    psi = latgen.gaussian_spinor(dims, 20190)
    phi = odefl.cgs2(latgen.gaussian_spinor(dims, 20191, nrhs=3))
    lam = np.array([-0.3, 0.2, 0.45])
    alpha = och.coeffs_sign_interp(41, 0.08)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    tol = 1e-12 if store == "f64" else 1e-6
    g = ovl.GaugeField(dev(u), store)
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, store)
    x = dev(psi, cdt)
    out = torch.empty_like(x)
    ovl.graph_enable(False)
    direct = {mu: ovl.overlap_apply(g, p, x, mu, defl=d).clone() for mu in (0.01, 0.05)}
    ref = oov.overlap_apply(u, psi, 0.05, alpha, LMAX, phi, lam)
    ovl.graph_enable(True)
    scratch = torch.randn(1 << 16, device="cuda")
    for i in range(6):                      # 1st direct, 2nd captured, then replays
        mu = (0.01, 0.05)[i % 2]
        ovl.overlap_apply(g, p, x, mu, defl=d, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, direct[mu]), (i, mu)
        scratch.mul_(1.0001).add_(1.0)      # eager work between the replays
        torch.cuda.synchronize()
    got = out.detach().to("cpu", torch.complex128).numpy()
    assert rel_err(got, ref) < tol
    assert g.flags() == 0


def test_graph_keys_follow_buffers_and_polynomials(ovl):
    """A new output buffer or polynomial is a different graph; results stay exact."""
    dims = (4, 4, 4, 4)
    u = latgen.random_su3_field(dims, 10192)
    psi = latgen.gaussian_spinor(dims, 20192)
    g = ovl.GaugeField(dev(u), "f64")
    x = dev(psi)
    for degree in (21, 33):
        alpha = och.coeffs_sign_interp(degree, 0.1)
        p = ovl.Polynomial(alpha, LMAX)
        ref = och.sign_apply(u, psi, alpha, LMAX)
        outs = [torch.empty_like(x) for _ in range(2)]
        for rep in range(3):
            for o in outs:
                ovl.sign_apply(g, p, x, out=o)
                got = o.detach().cpu().numpy()
                assert rel_err(got, ref) < 1e-12, (degree, rep)
