"""Pin of the oracle's ARPACK low-mode solver against LAPACK on the dense matrix of K."""
import numpy as np

import latgen
from oracle.eigen import dense_eigs, low_modes


def test_low_modes_match_dense():
    dims = (2, 2, 4, 4)
    u = latgen.smeared_field(dims, 131)
    lam_d, vec_d = dense_eigs(u)
    n_ev = 6
    lam, phi, res = low_modes(u, n_ev, 6.5, filter_degree=16)
    assert np.allclose(np.sort(np.abs(lam)), np.sort(np.abs(lam_d[:n_ev])), atol=1e-10)
    assert res.max() < 1e-9
    g = phi.reshape(n_ev, -1).conj() @ phi.reshape(n_ev, -1).T
    assert np.abs(g - np.eye(n_ev)).max() < 1e-12
