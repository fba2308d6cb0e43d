"""Host-side checks of libovl.so that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before any HIP call, and its coefficient rule agrees with
the oracle's (Sec. 2, eq. 3 leaves the coefficients open; both sides implement the same rule
independently)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import chebyshev as och
from paper_1510_06897_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libovl.so is not built (python -m paper_1510_06897_amd.build)")
    return _lib.load()


def header_symbols():
    text = open(os.path.join(ROOT, "include", "ovl.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(ovl_\w+)\(", text, re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = header_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_version(lib):
    assert b"gfx950" in lib.ovl_version()


@pytest.mark.parametrize("deg,eps", [(64, 0.077), (200, 0.0772), (400, 0.03), (299, 0.05), (1, 0.5)])
def test_coefficients_match_oracle_rule(lib, deg, eps):
    buf = (ctypes.c_double * (deg + 1))()
    n = ctypes.c_int()
    assert lib.ovl_cheb_sign_coeffs(deg, eps, buf, ctypes.byref(n)) == 0
    ours = np.array(buf[: n.value])
    ref = och.coeffs_sign_interp(deg, eps)
    assert len(ours) == len(ref)
    # both sides sum O(N) cosine terms of values up to 1/eps in different orders
    assert np.abs(ours - ref).max() < 2e-15 * (len(ref) + 1) / eps
    assert np.all(ours[0::2] == 0.0)


def test_coefficients_reject_bad_args(lib):
    buf = (ctypes.c_double * 8)()
    n = ctypes.c_int()
    assert lib.ovl_cheb_sign_coeffs(0, 0.1, buf, ctypes.byref(n)) == -1
    assert lib.ovl_cheb_sign_coeffs(7, 1.5, buf, ctypes.byref(n)) == -1
    assert lib.ovl_cheb_sign_coeffs(7, 0.1, None, ctypes.byref(n)) == -1
    assert b"eps" in lib.ovl_last_error() or b"NULL" in lib.ovl_last_error()


def test_poly_handle_and_eval(lib):
    alpha = och.coeffs_sign_interp(31, 0.1)
    h = ctypes.c_void_p()
    a = alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ovl_poly_create(ctypes.byref(h), a, len(alpha), 6.5, 1.5) == 0
    v = ctypes.c_double()
    for lam in (-3.0, 0.4, 2.2, 6.4):
        assert lib.ovl_poly_eval(h, lam, ctypes.byref(v)) == 0
        assert abs(v.value - och.cheb_eval_scalar(alpha, lam / 6.5)) < 1e-14
    assert lib.ovl_poly_destroy(h) == 0


def test_poly_validation(lib):
    h = ctypes.c_void_p()
    good = np.array([0.0, 1.0, 0.0, 0.2])
    bad = np.array([0.0, np.nan, 0.0])
    p = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    assert lib.ovl_poly_create(ctypes.byref(h), p(bad), 3, 6.5, 1.5) == -7        # ENONFINITE
    assert lib.ovl_poly_create(ctypes.byref(h), p(good), 1, 6.5, 1.5) == -1        # too short
    assert lib.ovl_poly_create(ctypes.byref(h), p(good), 4, -1.0, 1.5) == -1       # lmax <= 0
    assert lib.ovl_poly_create(ctypes.byref(h), p(good), 4, float("inf"), 1.5) == -7
    assert lib.ovl_poly_create(None, p(good), 4, 6.5, 1.5) == -1


def test_gauge_create_validation_before_hip(lib):
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    dims = (ctypes.c_int32 * 4)(4, 4, 0, 4)
    assert lib.ovl_gauge_create(ctypes.byref(h), dims, dummy, 0, 0, None) == -2    # EDIMS
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    assert lib.ovl_gauge_create(ctypes.byref(h), dims, dummy, 0, 7, None) == -3    # EDTYPE
    assert lib.ovl_gauge_create(ctypes.byref(h), dims, dummy, 2, 0, None) == -3    # BF16 input
    assert lib.ovl_gauge_create(ctypes.byref(h), dims, None, 0, 0, None) == -1
    big = (ctypes.c_int32 * 4)(2048, 2048, 1024, 2)
    assert lib.ovl_gauge_create(ctypes.byref(h), big, dummy, 0, 0, None) == -2      # V > 2^31


def test_operator_validation_before_hip(lib):
    dummy = ctypes.c_void_p(0x1000)
    assert lib.ovl_wilson_apply(None, dummy, dummy, 1, 0, 0.0, 0, None) == -1
    assert lib.ovl_kernel_apply(None, dummy, dummy, 1, 0, 1.5, None) == -1
    assert lib.ovl_sign_apply(None, None, None, dummy, dummy, 1, 0, None) == -1
    assert lib.ovl_overlap_apply(None, None, None, 0.1, 0, dummy, dummy, 1, 0, None) == -1
    assert lib.ovl_defl_project(None, None, dummy, 1, 0, None) == -1
    assert lib.ovl_defl_correct(None, dummy, None, None, 1, 0, None) == -1
    assert lib.ovl_sign_force(None, None, None, dummy, dummy, 0, 0, None) == -1
    assert lib.ovl_status_flags(None, None, 0) == -1
    assert lib.ovl_kernel_axpby(None, dummy, dummy, 1.0, None, 0.0, None, 0.0, 1, 0, 1.5, None) == -1
    assert lib.ovl_wilson_link_vjp(None, dummy, dummy, dummy, 0, 0, None) == -1
    assert lib.ovl_overlap_solve(None, None, None, 0.1, dummy, dummy, None, None, 1e-10, 10, None,
                                 None, None) == -1
    assert lib.ovl_batch_sign_apply(None, 0, None, 0, None, None) == -1
    assert lib.ovl_autotune(None, 1, None, 0, None, None, None) == -1
    cfg = (ctypes.c_int * 4)()
    assert lib.ovl_batch_launch_config(None, 1, 0, cfg) == -1
    r = (ctypes.c_double * 1)()
    assert lib.ovl_sign_residual(None, None, None, dummy, 1, 0, r, None) == -1
    assert lib.ovl_sign_residual(None, None, None, dummy, 1, 0, None, None) == -1
    h = ctypes.c_void_p()
    lam = (ctypes.c_double * 1)(0.5)
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    assert lib.ovl_defl_create(ctypes.byref(h), dims, dummy, 0, lam, 0, 0, None) == -1
    lam_bad = (ctypes.c_double * 1)(float("nan"))
    assert lib.ovl_defl_create(ctypes.byref(h), dims, dummy, 0, lam_bad, 1, 0, None) == -7
    assert lib.ovl_defl_create(ctypes.byref(h), dims, dummy, 2, lam, 1, 0, None) == -3


def test_destroy_null_is_ok(lib):
    assert lib.ovl_gauge_destroy(None) == 0
    assert lib.ovl_poly_destroy(None) == 0
    assert lib.ovl_defl_destroy(None) == 0


def test_python_binding_raises_with_status(lib):
    from paper_1510_06897_amd import cheb_sign_coeffs, OvlError
    with pytest.raises(OvlError) as e:
        cheb_sign_coeffs(10, 2.0)
    assert e.value.status == "OVL_EINVAL"


def test_autotune_cache_file(lib, tmp_path):
    missing = str(tmp_path / "none.txt").encode()
    assert lib.ovl_autotune_load(missing) == -1
    f = tmp_path / "tune.txt"
    f.write_text("16 16 16 32 1 1 64 1 1 17.5\n8 8 8 16 0 1 16 0 1 9.0\nbad line\n"
                 # batch entries: two items; a right-hand-side block of 4 at 16 sites per
                 # workgroup; rejected: a block with the two-sites-per-lane form, a bad item count
                 "B 1 0 2 16 16 16 32 12 8 8 8 16 1 64 1 1 2 210.5\n"
                 "B 0 1 1 8 8 8 16 4 16 0 1 4 12.0\n"
                 "B 1 0 1 8 8 8 16 4 128 1 1 2 12.0\n"
                 "B 1 0 3 8 8 8 16 4 64 1 1 1 12.0\n")
    assert lib.ovl_autotune_load(str(f).encode()) == 4


def test_two_row_reference_helper():
    """The reference the two-row GPU tests use: SU(3) links come back unchanged, a link that is
    not SU(3) does not, and the completed third row is orthonormal to the first two."""
    import numpy as np
    import latgen
    from tests.conftest import complete_third_row
    u = latgen.random_su3_field((2, 3, 2, 2), 5, noise=0.8)
    assert np.abs(complete_third_row(u) - u).max() < 1e-14
    bad = u.copy()
    bad[:, 2] *= 1.5
    assert np.abs(complete_third_row(bad) - bad).max() > 0.1
    w = complete_third_row(bad * 1.0)
    m = np.moveaxis(w[0].reshape(3, 3, -1), -1, 0)
    assert np.abs(m @ np.conj(np.swapaxes(m, 1, 2)) - np.eye(3)).max() < 1e-14


@pytest.mark.parametrize("n,kind", [(1, "random"), (2, "random"), (7, "random"), (64, "random"),
                                    (128, "random"), (40, "degenerate"), (16, "diagonal"),
                                    (30, "real")])
def test_hermitian_eigh_host(lib, n, kind):
    """The eigen-solve's host Hermitian eigen-decomposition against LAPACK (NumPy): eigenvalues,
    A Q = Q diag(w) and Q^+ Q = 1 to rounding, also for repeated eigenvalues and inputs that are
    already diagonal or real."""
    import numpy as np
    rng = np.random.default_rng(n)
    if kind == "diagonal":
        a = np.diag(rng.standard_normal(n)).astype(np.complex128)
    else:
        x = rng.standard_normal((n, n)) + (0 if kind == "real" else 1j) * rng.standard_normal((n, n))
        a = x + x.conj().T
        if kind == "degenerate":   # eigenvalues 0, 1, 2 each with multiplicity > 1
            q, _ = np.linalg.qr(x)
            a = q @ np.diag(np.arange(n) % 3).astype(np.complex128) @ q.conj().T
            a = 0.5 * (a + a.conj().T)
    a = np.ascontiguousarray(a.astype(np.complex128))
    w = np.zeros(n)
    q = np.zeros((n, n), dtype=np.complex128)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.ovl_hermitian_eigh(n, a.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                  q.ctypes.data_as(dp)) == 0
    scale = max(1.0, np.abs(a).max())
    assert np.abs(w - np.linalg.eigvalsh(a)).max() < 1e-13 * scale * n
    assert np.abs(a @ q - q * w[None, :]).max() < 1e-13 * scale * n
    assert np.abs(q.conj().T @ q - np.eye(n)).max() < 1e-13 * n
    bad = a.copy()
    if n > 1:
        bad[0, 1] += 1.0
        assert lib.ovl_hermitian_eigh(n, bad.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                      q.ctypes.data_as(dp)) == -1


def test_stout_validation_before_hip(lib):
    """ovl_stout_smear / ovl_stout_backward reject bad arguments on the host (fake device
    addresses: nothing reaches the GPU)."""
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    fb = 36 * 256 * 16                                       # one FP64 link field of 4^4
    a, b, c = ctypes.c_void_p(1 << 40), ctypes.c_void_p((1 << 40) + 2 * fb), ctypes.c_void_p((1 << 40) + 4 * fb)
    assert lib.ovl_stout_smear(dims, None, a, 0.1, -0.25, 3, None) == -1
    assert lib.ovl_stout_smear(dims, b, a, 0.1, -0.25, 65, None) == -1
    assert lib.ovl_stout_smear(dims, b, a, 0.1, -0.25, -1, None) == -1
    assert lib.ovl_stout_smear(dims, b, a, float("inf"), -0.25, 3, None) == -7
    assert lib.ovl_stout_smear(dims, b, a, 0.1, float("nan"), 3, None) == -7
    assert lib.ovl_stout_smear(dims, ctypes.c_void_p((1 << 40) + fb // 2), a, 0.1, -0.25, 3, None) == -4
    bad = (ctypes.c_int32 * 4)(4, 0, 4, 4)
    assert lib.ovl_stout_smear(bad, b, a, 0.1, -0.25, 3, None) == -2
    # a link field of 4 GiB or more (the path kernels use 32-bit buffer offsets): 64^3 x 32
    huge = (ctypes.c_int32 * 4)(64, 64, 64, 32)
    far = ctypes.c_void_p(1 << 44)
    assert lib.ovl_stout_smear(huge, far, a, 0.1, -0.25, 3, None) == -2
    assert lib.ovl_stout_backward(huge, far, ctypes.c_void_p(2 << 44), ctypes.c_void_p(3 << 44),
                                  0.1, -0.25, 3, None) == -2
    assert lib.ovl_stout_backward(dims, c, b, None, 0.1, -0.25, 3, None) == -1
    assert lib.ovl_stout_backward(dims, c, b, c, 0.1, -0.25, 3, None) == -4
    assert lib.ovl_stout_backward(dims, c, c, a, 0.1, -0.25, 3, None) == -4
    assert lib.ovl_stout_backward(dims, c, b, a, 0.1, -0.25, 99, None) == -1
    assert b"steps" in lib.ovl_last_error()
