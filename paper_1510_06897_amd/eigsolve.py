"""Low eigenpairs of K on the GPU for the deflation term of Sec. 2, eq. 3.

The paper precomputes the lowest eigenpairs of K once per gauge field with a polynomial-
preconditioned implicitly restarted Lanczos method, at negligible cost compared with the sign
function (Sec. 2).  This set-up routine plays that role on the device: Chebyshev-filtered
subspace iteration (filter polynomial of K^2, block Rayleigh-Ritz with K itself so that +lambda
and -lambda separate).  Every K application runs in the library's multi-right-hand-side kernel;
the small dense steps of the set-up (block QR, the Rayleigh-Ritz eigenproblem) use torch's linear
algebra on the device.  It is not part of the timed operator.
"""
import numpy as np
import torch

from .api import M_W, GaugeField, kernel_apply


def _kop(g, v, m_w):
    return kernel_apply(g, v, m_w=m_w)


def low_modes(g: GaugeField, n_ev: int, lmax: float, block: int = None, degree: int = 60,
              iters: int = 40, tol: float = 1e-10, seed: int = 0, cut: float = 1.0,
              m_w: float = M_W):
    """The n_ev eigenpairs of K with the smallest |lambda| (FP64 gauge handle required).

    The filter T_degree((2 K^2 - (cut^2 + lmax^2)) / (lmax^2 - cut^2)) is bounded by 1 for
    |lambda| in [cut, lmax] and grows fastest towards lambda = 0, so the block converges to the
    lowest modes; `block` must exceed the number of eigenvalues in any near-degenerate cluster
    that straddles the n_ev-th one.

    Returns (lam: np.ndarray[n_ev], phi: complex128 tensor [n_ev, 4, 3, T, Z, Y, X],
    residuals: np.ndarray[n_ev] = ||K phi - lambda phi||, eps_next = |lambda| of the first
    undeflated Ritz value / lmax).
    """
    if g.store != "f64":
        raise ValueError("the eigen-solve needs an FP64 gauge handle")
    lx, ly, lz, lt = g.dims
    shape = (4, 3, lt, lz, ly, lx)
    n = int(np.prod(shape))
    m = block or max(2 * n_ev + 8, n_ev + 16)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.complex(torch.randn((m, n), generator=gen, dtype=torch.float64),
                      torch.randn((m, n), generator=gen, dtype=torch.float64)).to(g.device)
    b = lmax * lmax
    a = cut * cut
    lam = res = None
    for it in range(iters):
        # block orthonormalisation (columns of v^T)
        q, _ = torch.linalg.qr(v.T)
        v = q.T.contiguous()
        # Rayleigh-Ritz with K
        kv = _kop(g, v.reshape((m,) + shape), m_w).reshape(m, n)
        h = v.conj() @ kv.T
        h = 0.5 * (h + h.conj().T)
        w, y = torch.linalg.eigh(h)
        v = (y.T @ v).contiguous()
        kv = (y.T @ kv).contiguous()
        # order by ||K v|| (= sqrt(w^2 + residual^2)), not by |w|: directions of the block that
        # have not converged mix +lambda and -lambda and have Rayleigh quotients near zero
        order = torch.argsort(torch.linalg.vector_norm(kv, dim=1))
        w, v, kv = w[order], v[order].contiguous(), kv[order].contiguous()
        r = torch.linalg.vector_norm(kv - w[:, None] * v, dim=1)
        lam = w.cpu().numpy()
        res = r.cpu().numpy()
        if res[:n_ev].max() < tol or it == iters - 1:
            break
        vs = v.reshape((m,) + shape)

        def zop(x):
            kx = _kop(g, x, m_w)
            return (2.0 * _kop(g, kx, m_w) - (a + b) * x) / (b - a)

        t_prev, t_cur = vs, zop(vs)
        for _ in range(2, degree + 1):
            t_prev, t_cur = t_cur, 2.0 * zop(t_cur) - t_prev
        # rescale so the block stays representable
        nrm = torch.linalg.vector_norm(t_cur.reshape(m, n), dim=1, keepdim=True)
        v = (t_cur.reshape(m, n) / nrm).contiguous()
    phi = v[:n_ev].reshape((n_ev,) + shape).contiguous()
    eps_next = abs(lam[n_ev]) / lmax if m > n_ev else None
    return lam[:n_ev], phi, res[:n_ev], eps_next
