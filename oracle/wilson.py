"""Wilson-Dirac operator and the sign-function kernel (Sec. 2, eq. 2 and the line after eq. 1).

(D_W psi)(x) = 4 psi(x) - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                       + (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu) ]

The printed equation omits psi(x) after the leading 4; the diagonal term is 4 psi(x).  Lattice
spacing a = 1, periodic boundaries in every direction.  K = gamma5 (D_W - m_W) with m_W = 1.5.
"""
import numpy as np

from .gamma import GAMMA, GAMMA5

M_W = 1.5

# mu -> axis of a [..., T, Z, Y, X] array counted from the end
_AXIS = {0: -1, 1: -2, 2: -3, 3: -4}


def shift_fwd(f, mu):
    """f(x + mu) with periodic wrap."""
    return np.roll(f, -1, axis=_AXIS[mu])


def shift_bwd(f, mu):
    """f(x - mu) with periodic wrap."""
    return np.roll(f, 1, axis=_AXIS[mu])


def spin_mul(g, psi):
    """(g psi) for a 4x4 spin matrix g and psi[..., s, c, T, Z, Y, X]."""
    return np.einsum("st,...tcTZYX->...scTZYX", g, psi)


def colour_mul(u, psi):
    """(u psi) for a colour-matrix field u[a, b, T, Z, Y, X] and psi[..., s, b, T, Z, Y, X]."""
    return np.einsum("abTZYX,...sbTZYX->...saTZYX", u, psi)


def colour_mul_dag(u, psi):
    """(u^+ psi) for u[a, b, T, Z, Y, X]."""
    return np.einsum("baTZYX,...sbTZYX->...saTZYX", u.conj(), psi)


def gamma5(psi):
    return spin_mul(GAMMA5, psi)


def hopping(u, psi):
    """sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)]."""
    one = np.eye(4, dtype=np.complex128)
    out = np.zeros_like(psi, dtype=np.complex128)
    for mu in range(4):
        fwd = colour_mul(u[mu], shift_fwd(psi, mu))
        bwd = shift_bwd(colour_mul_dag(u[mu], psi), mu)  # U_mu(x-mu)^+ psi(x-mu)
        out += spin_mul(one - GAMMA[mu], fwd) + spin_mul(one + GAMMA[mu], bwd)
    return out


def dw(u, psi):
    """D_W psi (Sec. 2, eq. 2)."""
    return 4.0 * psi - 0.5 * hopping(u, psi)


def dw_dagger(u, psi):
    """D_W^+ psi = gamma5 D_W gamma5 psi (gamma5-hermiticity of the Wilson operator)."""
    return gamma5(dw(u, gamma5(psi)))


def dw_minus_mass(u, psi, m_w=M_W):
    """(D_W - m_W) psi."""
    return dw(u, psi) - m_w * psi


def kop(u, psi, m_w=M_W):
    """K psi = gamma5 (D_W - m_W) psi, the Hermitian sign-function kernel (Sec. 2)."""
    return gamma5(dw_minus_mass(u, psi, m_w))
