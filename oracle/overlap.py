"""The overlap operator of Sec. 2, eq. 1: D[mu] = 1/2 (1 + mu + (1 - mu) gamma5 sign(K)).

sign(K) is the deflated Chebyshev approximation of eq. 3 (``chebyshev.sign_apply``).  The
adjoint is D[mu]^+ = gamma5 D[mu] gamma5 (sign(K) is Hermitian for real alpha and w).
"""
from .chebyshev import sign_apply
from .wilson import gamma5, M_W


def overlap_apply(u, psi, mu, alpha, lmax, phi=None, lam=None, m_w=M_W):
    s = sign_apply(u, psi, alpha, lmax, phi, lam, m_w)
    return 0.5 * ((1.0 + mu) * psi + (1.0 - mu) * gamma5(s))


def overlap_dagger_apply(u, psi, mu, alpha, lmax, phi=None, lam=None, m_w=M_W):
    return gamma5(overlap_apply(u, gamma5(psi), mu, alpha, lmax, phi, lam, m_w))
