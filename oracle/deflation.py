"""Low-mode deflation pieces of Sec. 2, eq. 3, written out on whole vectors.

project:  c_i = phi_i^+ psi                         (one complex number per eigenvector)
correct:  psi <- psi + sum_i phi_i w_i c_i
cgs2:     classical Gram-Schmidt applied twice per vector, then normalisation, which turns a set of
          (approximate) eigenvectors into an exactly orthonormal basis of the same span.
"""
import numpy as np


def project(phi, psi):
    """c_i = <phi_i, psi> for phi[i, ...] and one right-hand side psi[...]."""
    return np.array([np.vdot(phi[i], psi) for i in range(len(phi))], dtype=np.complex128)


def correct(phi, psi, c, w):
    """psi + sum_i phi_i w_i c_i."""
    out = psi.astype(np.complex128).copy()
    for i in range(len(phi)):
        out = out + phi[i] * (w[i] * c[i])
    return out


def cgs2(phi):
    """Orthonormalise the rows phi[i] in order: two classical Gram-Schmidt passes, then scale."""
    q = []
    for i in range(len(phi)):
        v = phi[i].astype(np.complex128).copy()
        for _ in range(2):
            coeffs = [np.vdot(qj, v) for qj in q]
            for qj, cj in zip(q, coeffs):
                v = v - cj * qj
        v = v / np.sqrt(np.vdot(v, v).real)
        q.append(v)
    return np.stack(q) if q else np.zeros_like(phi)
