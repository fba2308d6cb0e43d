"""Seeded synthetic lattice inputs shared by the tests, the benchmark and the oracle's checks.

This module produces *inputs only*: gauge fields, smeared gauge fields, spinors, point sources,
gauge transformations and storage-precision roundings.  It contains none of the arithmetic of the
overlap method itself (no Wilson stencil, no Chebyshev recurrence, no deflation, no overlap
combination, no derivative).  Both the FP64 oracle and the HIP library consume its arrays.

The paper's gauge ensembles (Table 2: an 8^3x32 overlap ensemble and 20^3x64 MILC Asqtad
ensembles) are not available, so seeded synthetic SU(3) fields stand in for them:

* near-unit links U = exp(i * noise * H) with H = sum_a h_a lambda_a / 2, h_a ~ N(0, 1) and
  lambda_a the Gell-Mann matrices (noise 0.3 by default);
* optionally followed by plain stout smearing (rho = 0.1, 3 steps).  The paper smooths its links
  with 3 steps of over-improved stout smearing before building the sign-function kernel (Sec. 2);
  plain stout at the same rho and step count reproduces the smoothing for synthetic inputs.

Array conventions (NumPy, complex128):

* gauge field ``U[mu, a, b, t, z, y, x]``; mu = 0, 1, 2, 3 is the x, y, z, t direction and
  (a, b) are the colour row and column of U_mu(x);
* spinor ``psi[s, c, t, z, y, x]`` (spin s, colour c), or ``psi[r, s, c, t, z, y, x]`` for r
  right-hand sides.  The site index runs fastest, x fastest of all.
* ``dims = (Lx, Ly, Lz, Lt)``.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``; the draw order is canonical
``[t][z][y][x][mu]`` so that a field depends only on its seed and shape.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "site_shape", "volume", "gell_mann", "random_su3_field", "stout_smear", "gaussian_spinor",
    "point_source", "random_gauge_transform", "gauge_transform_links", "gauge_transform_spinor",
    "round_to_f32", "round_to_bf16", "seed_for", "smeared_field",
]


def site_shape(dims):
    """(T, Z, Y, X) array shape of one field component for dims = (Lx, Ly, Lz, Lt)."""
    lx, ly, lz, lt = (int(v) for v in dims)
    return (lt, lz, ly, lx)


def volume(dims) -> int:
    return int(np.prod([int(v) for v in dims]))


def seed_for(kind: str, cfg: int, index: int = 0) -> int:
    """Seed convention: gauge 10000+100*cfg+i, spinor 20000+100*cfg+i, transform 30000+cfg."""
    base = {"gauge": 10000, "spinor": 20000, "transform": 30000, "direction": 40000}[kind]
    if kind == "direction":
        return base + index
    if kind == "transform":
        return base + cfg
    return base + 100 * cfg + index


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1], l[1, 1, 0] = -1j, 1j
    l[2, 0, 0], l[2, 1, 1] = 1, -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2], l[4, 2, 0] = -1j, 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2], l[6, 2, 1] = -1j, 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a stack of Hermitian 3x3 matrices, exact through an eigendecomposition."""
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def _to_field_layout(sm: np.ndarray) -> np.ndarray:
    """[T, Z, Y, X, mu, a, b] -> [mu, a, b, T, Z, Y, X]."""
    return np.ascontiguousarray(np.moveaxis(sm, (4, 5, 6), (0, 1, 2)))


def _to_site_layout(u: np.ndarray) -> np.ndarray:
    """[mu, a, b, T, Z, Y, X] -> [T, Z, Y, X, mu, a, b]."""
    return np.ascontiguousarray(np.moveaxis(u, (0, 1, 2), (4, 5, 6)))


def random_su3_field(dims, seed: int, noise: float = 0.3) -> np.ndarray:
    """Near-unit SU(3) field U_mu(x) = exp(i noise H_mu(x)), H traceless Hermitian Gaussian."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = site_shape(dims)
    h = rng.standard_normal(shp + (4, 8))
    herm = np.einsum("...a,aij->...ij", h, gell_mann()) * 0.5
    u = _expi_hermitian(noise * herm)
    return _to_field_layout(u)


_SITE_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # mu -> axis of a [T, Z, Y, X, ...] array


def _fwd(a: np.ndarray, mu: int) -> np.ndarray:
    """f(x + mu) for a site-major array [T, Z, Y, X, ...] (periodic)."""
    return np.roll(a, -1, axis=_SITE_AXIS[mu])


def _bwd(a: np.ndarray, mu: int) -> np.ndarray:
    """f(x - mu) for a site-major array [T, Z, Y, X, ...] (periodic)."""
    return np.roll(a, 1, axis=_SITE_AXIS[mu])


def _dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def stout_smear(u: np.ndarray, rho: float = 0.1, steps: int = 3) -> np.ndarray:
    """Plain (isotropic) stout smearing of Morningstar and Peardon, all links updated at once.

    C_mu(x) = rho sum_{nu != mu} [U_nu(x) U_mu(x+nu) U_nu(x+mu)^+ +
                                   U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu)],
    Omega = C U^+,  Q = (i/2)(Omega^+ - Omega) - (i/6) tr(Omega^+ - Omega),
    U' = exp(i Q) U.
    """
    w = _to_site_layout(u)
    links = [w[..., m, :, :] for m in range(4)]
    for _ in range(steps):
        new = []
        for mu in range(4):
            c = np.zeros_like(links[mu])
            for nu in range(4):
                if nu == mu:
                    continue
                up = links[nu] @ _fwd(links[mu], nu) @ _dag(_fwd(links[nu], mu))
                un = _bwd(links[nu], nu)
                dn = _dag(un) @ _bwd(links[mu], nu) @ _fwd(un, mu)
                c = c + up + dn
            om = rho * c @ _dag(links[mu])
            a = _dag(om) - om
            tr = np.trace(a, axis1=-2, axis2=-1)[..., None, None]
            q = 0.5j * a - (1j / 6.0) * tr * np.eye(3)
            new.append(_expi_hermitian(q) @ links[mu])
        links = new
    return _to_field_layout(np.stack(links, axis=-3))


def smeared_field(dims, seed: int, noise: float = 0.3, rho: float = 0.1, steps: int = 3):
    """Near-unit field followed by ``steps`` plain stout steps (the smeared workloads)."""
    return stout_smear(random_su3_field(dims, seed, noise), rho, steps)


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor(s): components (a + i b)/sqrt(2), a, b ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = ((nrhs,) if nrhs is not None else ()) + (4, 3) + site_shape(dims)
    re = rng.standard_normal(shp)
    im = rng.standard_normal(shp)
    return (re + 1j * im) / np.sqrt(2.0)


def point_source(dims, s0: int, c0: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """delta_{x, site} delta_{s, s0} delta_{c, c0}; site given as (x, y, z, t)."""
    psi = np.zeros((4, 3) + site_shape(dims), dtype=np.complex128)
    x, y, z, t = site
    psi[s0, c0, t, z, y, x] = 1.0
    return psi


def random_gauge_transform(dims, seed: int, noise: float = 1.0) -> np.ndarray:
    """Omega(x) = exp(i noise H(x)), returned in site layout [T, Z, Y, X, 3, 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal(site_shape(dims) + (8,))
    herm = np.einsum("...a,aij->...ij", h, gell_mann()) * 0.5
    return _expi_hermitian(noise * herm)


def gauge_transform_links(u: np.ndarray, om: np.ndarray) -> np.ndarray:
    """U'_mu(x) = Omega(x) U_mu(x) Omega(x + mu)^+."""
    w = _to_site_layout(u)
    out = np.empty_like(w)
    for mu in range(4):
        out[..., mu, :, :] = om @ w[..., mu, :, :] @ _dag(_fwd(om, mu))
    return _to_field_layout(out)


def gauge_transform_spinor(psi: np.ndarray, om: np.ndarray) -> np.ndarray:
    """psi'(x) = Omega(x) psi(x) for psi[..., s, c, T, Z, Y, X]."""
    return np.einsum("tzyxab,...sbtzyx->...satzyx", om, psi)


def round_to_f32(a: np.ndarray) -> np.ndarray:
    """Round complex128 to complex64 (round to nearest even) and return it as complex128."""
    return a.astype(np.complex64).astype(np.complex128)


def _bf16_rne(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32; finite inputs only."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def round_to_bf16(a: np.ndarray) -> np.ndarray:
    """Round complex128 -> float32 (nearest even) -> bfloat16 (nearest even), back to complex128.

    This is the exact conversion the BF16 link storage performs, so the oracle can be run on the
    same rounded links.
    """
    c = a.astype(np.complex64)
    re = _bf16_rne(c.real)
    im = _bf16_rne(c.imag)
    return re.astype(np.float64) + 1j * im.astype(np.float64)
