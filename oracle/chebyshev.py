"""Chebyshev approximation of the matrix sign function (Sec. 2, eq. 3).

sign(K) = sum_m alpha_m T_m(K) + sum_i phi_i phi_i^+ [sign(lambda_i) - sum_m alpha_m T_m(lambda_i)]

T_m are first-kind Chebyshev polynomials.  The paper leaves the coefficients alpha_m and the
argument scaling unspecified ("appropriate coefficients"); this oracle reads them as follows:

* the polynomial acts on X = K / lmax with lmax an explicit input (an upper bound on ||K||), so
  the Chebyshev argument lies in [-1, 1]; the eigenvalue correction uses T_m(lambda_i / lmax);
* "degree N" means alpha_0 .. alpha_N with N odd and alpha_m = 0 for every even m (sign is odd);
* ``coeffs_sign_interp`` (rule S): interpolate q(y) ~ y^{-1/2} on [eps^2, 1] at the first-kind
  Chebyshev nodes with a polynomial of degree (N-1)/2, set p(x) = x q(x^2) and re-expand p exactly
  in T_m(x); the even coefficients (zero up to rounding) are set to zero exactly;
* ``coeffs_sign_series`` (rule A): the truncated Chebyshev series of sign(x),
  alpha_{2k+1} = (4/pi) (-1)^k / (2k+1); used by the tests for its closed form.

The matrix polynomial is applied with the forward three-term recurrence the paper describes:
t_0 = psi, t_1 = X psi, t_{m+1} = 2 X t_m - t_{m-1}, result sum_m alpha_m t_m.
"""
import numpy as np

from .wilson import kop, M_W


def top_odd_degree(stated_degree: int) -> int:
    """Largest odd index N <= the stated degree (number of K applications of the recurrence)."""
    n = int(stated_degree)
    if n < 1:
        raise ValueError("degree must be >= 1")
    return n if n % 2 == 1 else n - 1


def _cheb_nodes(n_points: int) -> np.ndarray:
    j = np.arange(n_points)
    return np.cos(np.pi * (j + 0.5) / n_points)


def _cheb_coeffs_from_samples(values: np.ndarray) -> np.ndarray:
    """Interpolating Chebyshev coefficients c_0..c_{n-1} from samples at the n first-kind nodes."""
    n = values.shape[0]
    j = np.arange(n)
    k = np.arange(n)[:, None]
    c = (2.0 / n) * (np.cos(np.pi * k * (j + 0.5) / n) @ values)
    c[0] *= 0.5
    return c


def cheb_eval_scalar(coeffs, x):
    """sum_m c_m T_m(x) for scalar or array x, by the forward recurrence T_{m+1} = 2xT_m - T_{m-1}."""
    x = np.asarray(x, dtype=np.float64)
    t_prev = np.ones_like(x)
    total = coeffs[0] * t_prev
    if len(coeffs) == 1:
        return total
    t_cur = x.copy()
    total = total + coeffs[1] * t_cur
    for m in range(2, len(coeffs)):
        t_next = 2.0 * x * t_cur - t_prev
        total = total + coeffs[m] * t_next
        t_prev, t_cur = t_cur, t_next
    return total


def coeffs_sign_interp(degree: int, eps: float) -> np.ndarray:
    """Rule S: alpha_0..alpha_N for p(x) = x q(x^2), q interpolating y^{-1/2} on [eps^2, 1]."""
    n_top = top_odd_degree(degree)
    if not (0.0 < eps < 1.0):
        raise ValueError("eps must lie in (0, 1)")
    nq = (n_top - 1) // 2 + 1                    # number of nodes of q (degree (N-1)/2)
    a, b = eps * eps, 1.0
    z = _cheb_nodes(nq)
    y = 0.5 * (a + b) + 0.5 * (b - a) * z
    cq = _cheb_coeffs_from_samples(1.0 / np.sqrt(y))

    def p_of_x(x):
        zz = (2.0 * x * x - (a + b)) / (b - a)
        return x * cheb_eval_scalar(cq, zz)

    xs = _cheb_nodes(n_top + 1)
    alpha = _cheb_coeffs_from_samples(p_of_x(xs))
    alpha[0::2] = 0.0
    return alpha


def coeffs_sign_series(degree: int) -> np.ndarray:
    """Rule A: truncated Chebyshev series of sign(x), alpha_{2k+1} = (4/pi)(-1)^k/(2k+1)."""
    n_top = top_odd_degree(degree)
    alpha = np.zeros(n_top + 1)
    for m in range(1, n_top + 1, 2):
        k = (m - 1) // 2
        alpha[m] = (4.0 / np.pi) * (-1) ** k / m
    return alpha


def poly_apply(u, psi, alpha, lmax, m_w=M_W):
    """p(X) psi = sum_m alpha_m T_m(X) psi with X = K/lmax, by the forward recurrence."""
    alpha = np.asarray(alpha, dtype=np.float64)

    def xop(v):
        return kop(u, v, m_w) / lmax

    t_prev = psi.astype(np.complex128)
    out = alpha[0] * t_prev
    if len(alpha) == 1:
        return out
    t_cur = xop(t_prev)
    out = out + alpha[1] * t_cur
    for m in range(2, len(alpha)):
        t_next = 2.0 * xop(t_cur) - t_prev
        out = out + alpha[m] * t_next
        t_prev, t_cur = t_cur, t_next
    return out


def chebyshev_vectors(u, psi, n, lmax, m_w=M_W):
    """[T_0(X) psi, ..., T_n(X) psi] by the forward recurrence (used by the tests)."""
    out = [psi.astype(np.complex128)]
    if n >= 1:
        out.append(kop(u, out[0], m_w) / lmax)
    for _ in range(2, n + 1):
        out.append(2.0 * kop(u, out[-1], m_w) / lmax - out[-2])
    return out


def deflation_weights(alpha, lam, lmax):
    """w_i = sign(lambda_i) - sum_m alpha_m T_m(lambda_i / lmax), with sign(0) = 0 (eq. 3)."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.sign(lam) - cheb_eval_scalar(np.asarray(alpha, dtype=np.float64), lam / lmax)


def sign_apply(u, psi, alpha, lmax, phi=None, lam=None, m_w=M_W):
    """Approximate sign(K) psi of eq. 3: p(X) psi + sum_i phi_i w_i (phi_i^+ psi).

    ``phi`` has shape (n_ev, 4, 3, T, Z, Y, X) (orthonormal columns), ``lam`` the n_ev real
    eigenvalues of K (unscaled).  ``psi`` is a single right-hand side.
    """
    out = poly_apply(u, psi, alpha, lmax, m_w)
    if phi is not None and len(phi) > 0:
        w = deflation_weights(alpha, lam, lmax)
        for i in range(len(phi)):
            c = np.vdot(phi[i], psi)
            out = out + phi[i] * (w[i] * c)
    return out
