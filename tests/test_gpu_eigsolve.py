"""GPU set-up eigen-solve (the low modes of K that Sec. 2 precomputes once per gauge field):
eigenvalues against the oracle's dense LAPACK diagonalisation, residuals through the library's K."""
import numpy as np
import pytest

import latgen
from oracle.eigen import dense_eigs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_low_modes_match_dense_4x4x4x4():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1510_06897_amd as ovl
    from paper_1510_06897_amd.eigsolve import low_modes
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 5)
    lam_ref, _ = dense_eigs(u)
    g = ovl.GaugeField(torch.from_numpy(u).cuda(), "f64")
    lam, phi, res, eps = low_modes(g, 8, 6.5, block=64, cut=1.0, degree=20, iters=30)
    assert res.max() < 1e-10
    assert np.allclose(np.sort(np.abs(lam)), np.sort(np.abs(lam_ref[:8])), atol=1e-10)
    assert abs(eps * 6.5 - abs(lam_ref[8])) < 1e-6
    # residual recomputed through the library operator, and orthonormality
    k = ovl.kernel_apply(g, phi)
    r = torch.linalg.vector_norm((k - torch.from_numpy(lam).cuda()[:, None, None, None, None, None, None] * phi).reshape(8, -1), dim=1)
    assert float(r.max()) < 1e-10
    gram = phi.reshape(8, -1).conj() @ phi.reshape(8, -1).T
    assert float((gram - torch.eye(8, device=gram.device)).abs().max()) < 1e-12
