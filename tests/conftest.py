import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: test that takes more than a few seconds")


def rel_err(a, b):
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def complete_third_row(u):
    """Links [4][3][3][...] with row 2 replaced by conj(row0 x row1) in FP64: the matrices a
    two-row link read sees (equal to u for SU(3) links)."""
    import numpy as np
    u = np.array(u, dtype=np.complex128, copy=True)
    r0, r1 = u[:, 0], u[:, 1]
    for b in range(3):
        c, d = (b + 1) % 3, (b + 2) % 3
        u[:, 2, b] = np.conj(r0[:, c] * r1[:, d] - r0[:, d] * r1[:, c])
    return u
