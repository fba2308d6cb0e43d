"""Stout smearing of the gauge links and its chain-rule derivative (Sec. 2: the links entering K
are smoothed by 3 steps of over-improved stout smearing with rho = 0.1, eps = -0.25; Sec. 1: the
overlap operator is used inside HMC, whose fermion force must then be carried back through the
smearing).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One stout step replaces every link at once by
    U'_mu(x) = exp(i Q_mu(x)) U_mu(x),
    Q = (i/2)(Omega^+ - Omega) - (i/6) tr(Omega^+ - Omega),   Omega = C_mu(x) U_mu(x)^+,
where the staple sum C_mu(x) is rho times the derivative of the over-improved gauge action
    S = sum_x [ c_p sum_{mu<nu} Re tr P_munu(x) + c_r sum_{mu != nu} Re tr R_munu(x) ],
    c_p = (5 - 2 eps) / 3,  c_r = -(1 - eps) / 12,
with P the 1x1 plaquette and R_munu the 2x1 rectangle (two links along mu, one along nu).
eps = 1 is plain stout smearing (c_p = 1, c_r = 0); eps = 0 the tree-level Symanzik weights.
The paper gives only rho, eps and the step count; this reading of the over-improved staple is
stated here and checked below against the action it differentiates.

The staple of link (x, mu) is a sum over paths from x to x + mu: each path is a list of signed
steps; a step +d from site z contributes the factor U_d(z), a step -d the factor U_d(z - d)^+.

Functions (links in the [mu, a, b, T, Z, Y, X] layout of latgen):
* ``action(u, eps)``            S above, by explicit products around every loop;
* ``staples(u, rho, eps)``      C_mu(x) for every link, from the path lists;
* ``smear(u, rho, eps, steps)``  the smeared links;
* ``smear_backward(u, rho, eps, steps, g)``  the derivative through the smearing: given
  G' = dL/dRe U' + i dL/dIm U' of a real function L of the smeared links, the same for the thin
  links U (reverse mode through every step; the matrix exponential is differentiated on the
  eigenbasis of Q, where its derivative is the matrix of divided differences of exp).
"""
import numpy as np

_AX = {0: 3, 1: 2, 2: 1, 3: 0}   # mu -> axis of a [T, Z, Y, X, ...] array


def _sites(u):
    """[mu, a, b, T, Z, Y, X] -> list over mu of [T, Z, Y, X, a, b]."""
    return [np.ascontiguousarray(np.moveaxis(u[m], (0, 1), (4, 5))) for m in range(4)]


def _field(links):
    return np.ascontiguousarray(np.stack([np.moveaxis(l, (4, 5), (0, 1)) for l in links]))


def _shift(f, off):
    """f(x + off) for a site-major array, off a length-4 integer vector over (x, y, z, t)."""
    for d in range(4):
        if off[d]:
            f = np.roll(f, -off[d], axis=_AX[d])
    return f


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def coefficients(eps):
    return (5.0 - 2.0 * eps) / 3.0, -(1.0 - eps) / 12.0


def staple_paths(mu):
    """[(weight kind, steps)] of the staple of a mu link: steps are (direction, +1 or -1)."""
    out = []
    for nu in range(4):
        if nu == mu:
            continue
        M, N = (mu, 1), (nu, 1)
        Mb, Nb = (mu, -1), (nu, -1)
        out += [("p", [N, M, Nb]), ("p", [Nb, M, N])]
        # 1 x 2 (the link on the short side), 2 x 1 with the link first or second
        out += [("r", [N, N, M, Nb, Nb]), ("r", [Nb, Nb, M, N, N]),
                ("r", [N, M, M, Nb, Mb]), ("r", [Nb, M, M, N, Mb]),
                ("r", [Mb, N, M, M, Nb]), ("r", [Mb, Nb, M, M, N])]
    return out


def _factors(links, steps):
    """[(link field shifted to the path position, daggered?, link direction, site offset)]."""
    pos = np.zeros(4, dtype=int)
    out = []
    for d, sgn in steps:
        if sgn > 0:
            out.append((_shift(links[d], pos), False, d, pos.copy()))
            pos[d] += 1
        else:
            pos[d] -= 1
            out.append((_dag(_shift(links[d], pos)), True, d, pos.copy()))
    return out


def _chain(mats, n_sites_shape):
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), n_sites_shape + (3, 3))
    acc = eye.copy()
    for m in mats:
        acc = acc @ m
    return acc


def staples(u, rho, eps):
    links = _sites(u)
    cp, cr = coefficients(eps)
    out = []
    for mu in range(4):
        c = np.zeros_like(links[mu])
        for kind, steps in staple_paths(mu):
            w = cp if kind == "p" else cr
            if w == 0.0:
                continue
            c = c + w * _chain([f[0] for f in _factors(links, steps)], links[mu].shape[:4])
        out.append(rho * c)
    return _field(out)


def action(u, eps):
    """S = sum_x [c_p sum_{mu<nu} Re tr P_munu + c_r sum_{mu!=nu} Re tr R_munu], loops written out."""
    links = _sites(u)
    cp, cr = coefficients(eps)
    e = [np.eye(4, dtype=int)[d] for d in range(4)]
    s = 0.0
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            um, un = links[mu], links[nu]
            if mu < nu:
                p = um @ _shift(un, e[mu]) @ _dag(_shift(um, e[nu])) @ _dag(un)
                s += cp * float(np.real(np.trace(p, axis1=-2, axis2=-1)).sum())
            r = (um @ _shift(um, e[mu]) @ _shift(un, 2 * e[mu]) @ _dag(_shift(um, e[mu] + e[nu]))
                 @ _dag(_shift(um, e[nu])) @ _dag(un))
            s += cr * float(np.real(np.trace(r, axis1=-2, axis2=-1)).sum())
    return s


def _expi_herm(q):
    """exp(i q) for Hermitian q, with the eigen-decomposition (w, v)."""
    w, v = np.linalg.eigh(q)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj()), w, v


def _q_of(c, u):
    om = c @ _dag(u)
    a = _dag(om) - om
    tr = np.trace(a, axis1=-2, axis2=-1)[..., None, None]
    return 0.5j * a - (1j / 6.0) * tr * np.eye(3)


def smear(u, rho, eps, steps):
    for _ in range(steps):
        c = _sites(staples(u, rho, eps))
        links = _sites(u)
        u = _field([_expi_herm(_q_of(c[m], links[m]))[0] @ links[m] for m in range(4)])
    return u


def _step_backward(u, rho, eps, gbar_out):
    """Thin-link derivative of one step, given the derivative with respect to its output."""
    links = _sites(u)
    c = _sites(staples(u, rho, eps))
    gout = _sites(gbar_out)
    gu = [np.zeros_like(l) for l in links]
    gamma = []
    for m in range(4):
        q = _q_of(c[m], links[m])
        ex, w, v = _expi_herm(q)
        gu[m] = gu[m] + _dag(ex) @ gout[m]                      # U' = E U: dL/dU via U
        g_e = gout[m] @ _dag(links[m])                           # dL/dE
        # E = exp(M), M = i Q: the adjoint of the derivative of exp at M is the derivative at
        # M^+, i.e. V (conj(F) o (V^+ g_e V)) V^+ with F the divided differences of exp(i w)
        ew = np.exp(1j * w)
        dw = w[..., :, None] - w[..., None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            f = (ew[..., :, None] - ew[..., None, :]) / (1j * dw)
        same = np.abs(dw) < 1e-12
        f = np.where(same, np.broadcast_to(ew[..., :, None], f.shape), f)
        h = _dag(v) @ g_e @ v
        g_m = v @ (np.conj(f) * h) @ _dag(v)
        z = -1j * g_m                                            # dL/dQ  (M = i Q)
        trz = np.real(np.trace(z, axis1=-2, axis2=-1))[..., None, None]
        g_om = 0.5j * (z + _dag(z)) - (1j / 3.0) * trz * np.eye(3)   # dL/dOmega
        gamma.append(g_om @ links[m])                            # dL/dC   (Omega = C U^+)
        gu[m] = gu[m] + _dag(g_om) @ c[m]                        # dL/dU via U^+ in Omega
    # C_mu(x) = rho sum_paths w prod(factors): every factor receives prefix^+ Gamma suffix^+
    cp, cr = coefficients(eps)
    shape = links[0].shape[:4]
    for mu in range(4):
        for kind, steps in staple_paths(mu):
            wgt = rho * (cp if kind == "p" else cr)
            if wgt == 0.0:
                continue
            fac = _factors(links, steps)
            mats = [f[0] for f in fac]
            for k, (_, dag, d, off) in enumerate(fac):
                pre = _chain(mats[:k], shape)
                suf = _chain(mats[k + 1:], shape)
                contrib = wgt * (_dag(pre) @ gamma[mu] @ _dag(suf))   # at path start x
                if dag:
                    contrib = _dag(contrib)
                # the factor is link d at x + off: move the contribution there
                gu[d] = gu[d] + _shift(contrib, -off)
    return _field(gu)


def smear_backward(u, rho, eps, steps, g):
    """dL/dRe U + i dL/dIm U of the thin links from that of the smeared links (g)."""
    levels = [u]
    for _ in range(steps):
        levels.append(smear(levels[-1], rho, eps, 1))
    for s in range(steps - 1, -1, -1):
        g = _step_backward(levels[s], rho, eps, g)
    return g
