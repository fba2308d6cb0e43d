"""Euclidean Dirac matrices in the chiral basis (the paper names no basis; Sec. 2).

gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = 1, 2, 3, gamma_4 = [[0, 1], [1, 0]],
gamma5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).  All are Hermitian and satisfy
{gamma_mu, gamma_nu} = 2 delta_{mu nu}; the oracle tests check both facts.
"""
import numpy as np

_S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_Z = np.zeros((2, 2), dtype=np.complex128)
_I = np.eye(2, dtype=np.complex128)


def _block(a, b, c, d):
    return np.block([[a, b], [c, d]])


GAMMA = np.stack([_block(_Z, -1j * s, 1j * s, _Z) for s in (_S1, _S2, _S3)]
                 + [_block(_Z, _I, _I, _Z)])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
