"""Overlap inversion: D[mu] x = b by conjugate gradients on the normal equations
D[mu]^+ D[mu] x = D[mu]^+ b.  Solving with the overlap operator is what it is built for (Sec. 2;
the paper's solver timings are Table 5).  The paper's own outer solver (GMRESR with nested
relaxed-precision sign functions) is not reproduced; CG on the normal equations is the textbook
method for a non-Hermitian operator whose normal matrix is Hermitian positive definite
(mu > 0).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from .overlap import overlap_apply, overlap_dagger_apply


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def overlap_cgnr(u, b, mu, alpha, lmax, phi=None, lam=None, tol=1e-12, max_iter=1000):
    """x with ||D^+ (b - D x)|| <= tol ||D^+ b|| (or max_iter iterations); returns (x, iterations).

    Standard CG on A = D^+ D, c = D^+ b, x_0 = 0:
      q = A p,  a = <r, r> / <p, q>,  x += a p,  r -= a q,  p = r + (<r', r'> / <r, r>) p.
    """
    def op(v):
        return overlap_dagger_apply(u, overlap_apply(u, v, mu, alpha, lmax, phi, lam),
                                    mu, alpha, lmax, phi, lam)

    c = overlap_dagger_apply(u, b.astype(np.complex128), mu, alpha, lmax, phi, lam)
    x = np.zeros_like(c)
    r = c.copy()
    p = r.copy()
    rr = _dot(r, r).real
    stop = tol * tol * rr
    it = 0
    while rr > stop and it < max_iter:
        q = op(p)
        a = rr / _dot(p, q).real
        x = x + a * p
        r = r - a * q
        rr_new = _dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def dense_overlap(u, mu, alpha, lmax, phi=None, lam=None):
    """The full (12V x 12V) matrix of D[mu], column by column from unit vectors."""
    shp = (4, 3) + u.shape[-4:]
    n = int(np.prod(shp))
    mat = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        mat[:, j] = overlap_apply(u, e.reshape(shp), mu, alpha, lmax, phi, lam).reshape(n)
        e[j] = 0.0
    return mat
