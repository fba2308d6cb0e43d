"""Gauge-link derivatives of the Chebyshev sign function (the HMC fermion-force building block).

The paper uses the overlap operator inside HMC (Sec. 1) but prints no force; this module states
the plain definition and differentiates it directly.

For a real function L of the complex links, the derivative is reported as one complex 3x3 matrix
per link, G_mu(x) = dL/dRe U_mu(x) + i dL/dIm U_mu(x), so that to first order
dL = Re sum_{x, mu} tr(G_mu(x)^+ dU_mu(x)).

* ``wilson_link_vjp(a, t)``: L = Re<a, D_W t>.  D_W (Sec. 2, eq. 2) is affine in U, so
  G_mu(x) = -1/2 sum_s [ ((1 - gamma_mu) a(x))_s (x) conj(t(x + mu))_s
                         + t(x)_s (x) conj(((1 + gamma_mu) a(x + mu))_s) ]
  with (x) the colour outer product v_i conj(w_j).
* ``sign_force(...)``: L = Re<chi, p(X) psi>, p(X) = sum_m alpha_m T_m(X), X = K/lmax, lmax fixed,
  no deflation term.  Reverse mode through the forward recurrence of ``chebyshev.poly_apply``:
  with adjoint vectors tb_m (tb_m = alpha_m chi initially, swept from m = N down to 1),
  t_m = 2 X t_{m-1} - t_{m-2} contributes Re<tb_m, 2 dX t_{m-1}> and t_1 = X t_0 contributes
  Re<tb_1, dX t_0>; dX = gamma5 dD_W / lmax, so every term is a D_W link VJP with a = gamma5 tb.
* ``hmc_force(u, g)``: F_mu(x) = -TA(U_mu(x) G_mu(x)^+), TA the traceless anti-Hermitian part,
  which satisfies dL/d eps along U -> exp(eps Y) U = Re tr(F^+ Y) for Y in su(3).
* ``sign_force_directional(u, chi, psi, alpha, lmax, y)``: the same derivative along one
  direction, dL/d eps of L(U + eps Y) at eps = 0, by forward mode through the forward recurrence
  (t'_0 = 0, t'_1 = X' psi, t'_{m+1} = 2 X t'_m + 2 X' t_m - t'_{m-1}, dL = Re<chi, sum_m alpha_m
  t'_m>, with X' = gamma5 (-1/2 hopping with the links Y) / lmax).  It keeps four vectors, so it
  runs on lattices where the reverse sweep's N stored vectors do not fit; Re tr(G^+ Y) summed
  over the links equals it.
"""
import numpy as np

from .gamma import GAMMA
from .wilson import shift_fwd, spin_mul, gamma5, hopping, kop, M_W


def _outer_spin_summed(v, w):
    """sum_s v[s, i] conj(w[s, j]) per site -> [i, j, T, Z, Y, X]."""
    return np.einsum("siTZYX,sjTZYX->ijTZYX", v, w.conj())


def wilson_link_vjp(a, t):
    """G for L = Re<a, D_W t>; a and t are single spinors [4, 3, T, Z, Y, X]."""
    one = np.eye(4, dtype=np.complex128)
    lt, lz, ly, lx = a.shape[-4:]
    g = np.zeros((4, 3, 3, lt, lz, ly, lx), dtype=np.complex128)
    for mu in range(4):
        term_f = _outer_spin_summed(spin_mul(one - GAMMA[mu], a), shift_fwd(t, mu))
        term_b = _outer_spin_summed(t, spin_mul(one + GAMMA[mu], shift_fwd(a, mu)))
        g[mu] = -0.5 * (term_f + term_b)
    return g


def sign_force(u, chi, psi, alpha, lmax, m_w=M_W):
    """G = d Re<chi, p(K/lmax) psi> / dU (reverse mode through the forward recurrence)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    n = len(alpha) - 1

    def xop(v):
        return kop(u, v, m_w) / lmax

    # forward sweep, every vector kept
    t = [psi.astype(np.complex128)]
    if n >= 1:
        t.append(xop(t[0]))
    for m in range(2, n + 1):
        t.append(2.0 * xop(t[m - 1]) - t[m - 2])

    tb = [alpha[m] * chi.astype(np.complex128) for m in range(n + 1)]
    g = np.zeros((4, 3, 3) + psi.shape[-4:], dtype=np.complex128)
    for m in range(n, 1, -1):
        g += (2.0 / lmax) * wilson_link_vjp(gamma5(tb[m]), t[m - 1])
        tb[m - 1] = tb[m - 1] + 2.0 * xop(tb[m])
        tb[m - 2] = tb[m - 2] - tb[m]
    if n >= 1:
        g += (1.0 / lmax) * wilson_link_vjp(gamma5(tb[1]), t[0])
    return g


def hmc_force(u, g):
    """F_mu(x) = -TA(U_mu(x) G_mu(x)^+) in the [mu, a, b, T, Z, Y, X] layout."""
    a = np.einsum("mikTZYX,mjkTZYX->mijTZYX", u, g.conj())
    ah = a - np.conj(np.swapaxes(a, 1, 2))
    tr = np.einsum("miiTZYX->mTZYX", ah)
    ta = 0.5 * ah - (tr / 6.0)[:, None, None] * np.eye(3)[None, :, :, None, None, None, None]
    return -ta


def sign_force_directional(u, chi, psi, alpha, lmax, y, m_w=M_W):
    """d/d eps Re<chi, p(X[U + eps Y]) psi> at eps = 0 (forward mode through the recurrence)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    n = len(alpha) - 1

    def xop(v):
        return kop(u, v, m_w) / lmax

    def dxop(v):
        # D_W = 4 - 1/2 hopping(U) is real-linear in U (U and U^+ both enter), so its derivative
        # along Y is -1/2 hopping(Y); the mass term does not depend on U
        return gamma5(-0.5 * hopping(y, v)) / lmax

    t_prev = psi.astype(np.complex128)
    dt_prev = np.zeros_like(t_prev)
    dsum = np.zeros_like(t_prev)
    if n >= 1:
        t_cur = xop(t_prev)
        dt_cur = dxop(t_prev)
        dsum = dsum + alpha[1] * dt_cur
        for m in range(2, n + 1):
            t_next = 2.0 * xop(t_cur) - t_prev
            dt_next = 2.0 * xop(dt_cur) + 2.0 * dxop(t_cur) - dt_prev
            dsum = dsum + alpha[m] * dt_next
            t_prev, t_cur = t_cur, t_next
            dt_prev, dt_cur = dt_cur, dt_next
    return float(np.real(np.vdot(chi, dsum)))
