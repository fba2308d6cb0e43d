"""Low eigenpairs of K on the GPU for the deflation term of Sec. 2, eq. 3.

The paper precomputes the lowest eigenpairs of K once per gauge field with a polynomial-
preconditioned implicitly restarted Lanczos method, at negligible cost compared with the sign
function (Sec. 2).  This set-up routine plays that role on the device: Chebyshev-filtered
subspace iteration (filter polynomial of K^2, block Rayleigh-Ritz with K itself so that +lambda
and -lambda separate).  Every K application runs in the library's multi-right-hand-side kernel,
each filter step as one plain and one fused K launch (``kernel_axpby``); the small dense steps of
the set-up (Gram-matrix orthonormalisation, the Rayleigh-Ritz eigenproblem) use torch's linear
algebra on the device.  It is not part of the timed operator.
"""
import numpy as np
import torch

from .api import M_W, GaugeField, kernel_apply, kernel_axpby


def _kop(g, v, m_w, out=None):
    return kernel_apply(g, v, m_w=m_w, out=out)


def _inner(a, b):
    """a^* b^T for row blocks a, b (m x n, n = 12 V): the long inner dimension is split into
    chunks summed after one batched product (a single product with n ~ 10^6 inner length runs
    ~40x slower on the device's BLAS)."""
    m, n = a.shape
    chunks = next(c for c in (128, 96, 64, 48, 32, 24, 16, 12, 8, 4, 2, 1) if n % c == 0)
    x = a.conj().resolve_conj().reshape(m, chunks, n // chunks).transpose(0, 1).contiguous()
    y = b.reshape(b.shape[0], chunks, n // chunks).permute(1, 2, 0).contiguous()
    return torch.bmm(x, y).sum(0)


def _small_eigh(h):
    """Eigenpairs of the Hermitian part of a small (block x block) device matrix, computed on the
    host (a few hundred microseconds there, against many small device launches)."""
    hc = h.cpu()
    lam, q = torch.linalg.eigh(0.5 * (hc + hc.conj().T))
    return lam.to(h.device), q.to(h.device)


def _orthonormalize(v, gen, passes=2):
    """Rows of v (m x n) made orthonormal from their Gram matrix G = Q diag(l) Q^+ (singular
    value QB, two passes): v <- diag(l)^(-1/2) Q^T v.  Rows in directions with a negligible Gram
    eigenvalue (numerically dependent after the filter) are replaced by random rows first."""
    done = 0
    for _ in range(passes + 3):
        gram = _inner(v, v)
        lam, q = _small_eigh(gram)
        weak = lam <= 1e-12 * lam[-1]
        if bool(weak.any()):
            k = int(weak.sum())
            fresh = torch.complex(
                torch.randn((k, v.shape[1]), generator=gen, dtype=torch.float64, device=v.device),
                torch.randn((k, v.shape[1]), generator=gen, dtype=torch.float64, device=v.device))
            v = torch.cat([q[:, k:].T @ v, fresh], dim=0)
            continue
        v = (q.T @ v) / torch.sqrt(lam)[:, None]
        done += 1
        if done == passes:
            break
    return v.contiguous()


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
    gen_dev = torch.Generator(device=g.device).manual_seed(seed + 1)
    b = lmax * lmax
    a = cut * cut
    lam = res = None
    for it in range(iters):
        v = _orthonormalize(v, gen_dev)
        # Rayleigh-Ritz with K
        kv = _kop(g, v.reshape((m,) + shape), m_w).reshape(m, n)
        h = _inner(v, kv)
        w, y = _small_eigh(h)
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
        # T_j of Z = (2 K^2 - (a + b)) / (b - a): Z x = c1 K (K x) + c0 x, one plain and one
        # fused K launch per step, t_{j+1} = 2 Z t_j - t_{j-1} written over t_{j-1}
        c1, c0 = 2.0 / (b - a), -(a + b) / (b - a)
        vs = v.reshape((m,) + shape)
        y = _kop(g, vs, m_w)
        t_prev = vs
        t_cur = kernel_axpby(g, y, c1, src=vs, a=c0, m_w=m_w)
        for _ in range(2, degree + 1):
            _kop(g, t_cur, m_w, out=y)
            kernel_axpby(g, y, 2.0 * c1, src=t_cur, a=2.0 * c0, w=t_prev, b=-1.0, m_w=m_w,
                         out=t_prev)
            t_prev, t_cur = t_cur, t_prev
        del y, t_prev
        # rescale so the block stays representable
        nrm = torch.linalg.vector_norm(t_cur.reshape(m, n), dim=1, keepdim=True)
        v = (t_cur.reshape(m, n) / nrm).contiguous()
    phi = v[:n_ev].reshape((n_ev,) + shape).contiguous()
    eps_next = abs(lam[n_ev]) / lmax if m > n_ev else None
    return lam[:n_ev], phi, res[:n_ev], eps_next
