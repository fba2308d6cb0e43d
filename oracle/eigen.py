"""Low eigenpairs (phi_i, lambda_i) of K, the inputs of the deflation term in Sec. 2, eq. 3.

The paper computes them once per gauge field with a polynomial-preconditioned implicitly
restarted Lanczos method (Sec. 2).  The oracle does the same with ARPACK (SciPy ``eigsh``, an
implicitly restarted Lanczos code) applied to a Chebyshev filter of K^2 that maps the low end of
the spectrum of K^2 to the top, followed by a Rayleigh-Ritz step with K itself inside the found
subspace so that +lambda and -lambda are separated.  For lattices of a few hundred sites the
dense matrix of K is assembled from unit vectors and diagonalised with LAPACK instead.
"""
import numpy as np
import scipy.sparse.linalg as spla

from .wilson import kop, M_W


def dense_kop(u, m_w=M_W):
    """The full (12V x 12V) matrix of K, built column by column from unit vectors."""
    shp = (4, 3) + u.shape[-4:]
    n = int(np.prod(shp))
    mat = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        mat[:, j] = kop(u, e.reshape(shp), m_w).reshape(n)
        e[j] = 0.0
    return mat


def dense_eigs(u, m_w=M_W):
    """All eigenpairs of K, ascending in |lambda|: (lam[n], vecs[n, 4, 3, T, Z, Y, X])."""
    mat = dense_kop(u, m_w)
    lam, v = np.linalg.eigh(mat)
    order = np.argsort(np.abs(lam), kind="stable")
    shp = (4, 3) + u.shape[-4:]
    vecs = np.stack([v[:, j].reshape(shp) for j in order])
    return lam[order], vecs


def low_modes(u, n_ev, lmax, filter_degree=24, tol=1e-11, seed=0, m_w=M_W):
    """The n_ev eigenpairs of K with smallest |lambda| (ascending |lambda|).

    Returns (lam, phi, residuals) with residuals ||K phi_i - lambda_i phi_i||.
    """
    shp = (4, 3) + u.shape[-4:]
    n = int(np.prod(shp))

    def k_apply(v):
        return kop(u, v.reshape(shp), m_w).reshape(n)

    # filter polynomial T_d(z), z = (2 K^2 - (a + b)) / (b - a): bounded on [a, b] = [cut, lmax^2],
    # growing fastest at K^2 = 0, so the low modes of K become the largest eigenvalues.
    b = lmax * lmax
    cut = 0.06 * b

    def filt(v):
        v = v.reshape(n)

        def zop(x):
            return (2.0 * k_apply(k_apply(x)) - (cut + b) * x) / (b - cut)

        t_prev = v
        t_cur = zop(v)
        for _ in range(2, filter_degree + 1):
            t_prev, t_cur = t_cur, 2.0 * zop(t_cur) - t_prev
        return t_cur

    op = spla.LinearOperator((n, n), matvec=filt, dtype=np.complex128)
    rng = np.random.Generator(np.random.PCG64(seed))
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    nwant = min(n_ev + 4, n - 2)
    _, vecs = spla.eigsh(op, k=nwant, which="LA", v0=v0, tol=tol * 1e-2,
                         ncv=min(n - 1, max(2 * nwant + 1, 20)))
    q, _ = np.linalg.qr(vecs)
    kq = np.stack([k_apply(q[:, j]) for j in range(q.shape[1])], axis=1)
    h = q.conj().T @ kq
    h = 0.5 * (h + h.conj().T)
    lam, y = np.linalg.eigh(h)
    phi_all = q @ y
    order = np.argsort(np.abs(lam), kind="stable")[:n_ev]
    lam = lam[order]
    phi = np.stack([phi_all[:, j].reshape(shp) for j in order])
    res = np.array([np.linalg.norm(k_apply(phi[i]) - lam[i] * phi[i].reshape(n))
                    for i in range(n_ev)])
    return lam, phi, res
