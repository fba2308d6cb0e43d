"""PyTorch-facing binding of libovl.so: argument marshalling only.

Every operator runs in the library's HIP kernels on the tensors' device and on the current torch
stream; PyTorch provides device memory and streams.  Tensors are complex and contiguous:

* gauge field  U[mu, a, b, t, z, y, x]              complex128 or complex64
* spinor       psi[s, c, t, z, y, x]  or  psi[r, s, c, t, z, y, x]  complex128 (FP64 operator)
               or complex64 (FP32 operator, with FP32 or BF16 link storage)

Operators (method of Cundy & Lee, Sec. 2): D_W (eq. 2), K = gamma5 (D_W - m_W), the Chebyshev
sign function with deflation (eq. 3), the overlap operator (eq. 1), the deflation projection and
correction, and the link derivatives of D_W and of the Chebyshev polynomial.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import OVL_BF16, OVL_F32, OVL_F64, call

M_W = 1.5
_STORE = {"f64": OVL_F64, "f32": OVL_F32, "bf16": OVL_BF16}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _spin_dtype(t):
    if t.dtype == torch.complex128:
        return OVL_F64
    if t.dtype == torch.complex64:
        return OVL_F32
    raise TypeError(f"spinor dtype {t.dtype} (complex128 or complex64 expected)")


def _check_spinor(t, dims):
    if not t.is_cuda:
        raise ValueError("spinor must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("spinor must be contiguous")
    lx, ly, lz, lt = dims
    site = (lt, lz, ly, lx)
    if t.dim() == 6 and tuple(t.shape) == (4, 3) + site:
        return 1
    if t.dim() == 7 and tuple(t.shape[1:]) == (4, 3) + site:
        return int(t.shape[0])
    raise ValueError(f"spinor shape {tuple(t.shape)} does not match lattice {dims}")


def _dims_arr(dims):
    return (ctypes.c_int32 * 4)(*[int(v) for v in dims])


def cheb_sign_coeffs(degree: int, eps: float) -> np.ndarray:
    """Library coefficient rule for sign(x) on eps <= |x| <= 1 (N+1 values, N odd <= degree)."""
    n_max = int(degree) + 1
    buf = (ctypes.c_double * n_max)()
    n = ctypes.c_int(0)
    call("ovl_cheb_sign_coeffs", int(degree), float(eps), buf, ctypes.byref(n))
    return np.array(buf[: n.value])


class GaugeField:
    """Links U packed into the library layout and storage dtype ('f64', 'f32', 'bf16')."""

    def __init__(self, u: torch.Tensor, store: str = "f64"):
        if not u.is_cuda or u.dim() != 7 or tuple(u.shape[:3]) != (4, 3, 3):
            raise ValueError("U must be a CUDA tensor of shape (4, 3, 3, T, Z, Y, X)")
        u = u.contiguous()
        in_dt = _spin_dtype(u)
        self.dims = (int(u.shape[6]), int(u.shape[5]), int(u.shape[4]), int(u.shape[3]))
        self.store = store
        self.device = u.device
        h = ctypes.c_void_p()
        with torch.cuda.device(u.device):
            call("ovl_gauge_create", ctypes.byref(h), _dims_arr(self.dims), _ptr(u), in_dt,
                 _STORE[store], _stream())
            torch.cuda.current_stream().synchronize()
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def spin_dtype(self):
        return torch.complex128 if self.store == "f64" else torch.complex64

    # largest stored-vs-completed third-row deviation accepted by default, per storage dtype
    _R12_TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 5e-2}

    def reconstruct(self, on: bool = True, tol: float = None) -> float:
        """Read links as two rows and complete the third (SU(3) fields only): checks the field on
        the device and returns the largest third-row deviation; raises OvlError if above tol."""
        dev = ctypes.c_double(0.0)
        call("ovl_gauge_reconstruct", self._h, 1 if on else 0,
             float(self._R12_TOL[self.store] if tol is None else tol), ctypes.byref(dev), _stream())
        return float(dev.value)

    def flags(self, clear: bool = True) -> int:
        f = ctypes.c_uint32(0)
        call("ovl_status_flags", self._h, ctypes.byref(f), 1 if clear else 0)
        return int(f.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().ovl_gauge_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Polynomial:
    """Chebyshev coefficients alpha_0..alpha_N of p(X), X = gamma5 (D_W - m_W) / lmax."""

    def __init__(self, alpha, lmax: float, m_w: float = M_W):
        a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
        self.alpha = a
        self.lmax = float(lmax)
        self.m_w = float(m_w)
        h = ctypes.c_void_p()
        call("ovl_poly_create", ctypes.byref(h), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             len(a), self.lmax, self.m_w)
        self._h = h

    @property
    def degree(self):
        return len(self.alpha) - 1

    def eval(self, lam: float) -> float:
        v = ctypes.c_double(0)
        call("ovl_poly_eval", self._h, float(lam), ctypes.byref(v))
        return v.value

    def __del__(self):
        try:
            if self._h.value:
                _lib.load().ovl_poly_destroy(self._h)
        except Exception:
            pass


class Deflation:
    """Low eigenpairs (phi_i, lambda_i) of K, orthonormalised on the device by CGS2 (FP64)."""

    def __init__(self, phi: torch.Tensor, lam, store: str = "f64"):
        if not phi.is_cuda or phi.dim() != 7 or tuple(phi.shape[1:3]) != (4, 3):
            raise ValueError("phi must be a CUDA tensor of shape (n_ev, 4, 3, T, Z, Y, X)")
        phi = phi.contiguous()
        self.n_ev = int(phi.shape[0])
        self.dims = (int(phi.shape[6]), int(phi.shape[5]), int(phi.shape[4]), int(phi.shape[3]))
        self.lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
        if self.lam.shape != (self.n_ev,):
            raise ValueError("need one eigenvalue per eigenvector")
        self.store = store
        h = ctypes.c_void_p()
        with torch.cuda.device(phi.device):
            call("ovl_defl_create", ctypes.byref(h), _dims_arr(self.dims), _ptr(phi),
                 _spin_dtype(phi), self.lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 self.n_ev, _STORE[store], _stream())
        self._h = h
        self.device = phi.device

    def basis(self) -> torch.Tensor:
        lx, ly, lz, lt = self.dims
        out = torch.empty((self.n_ev, 4, 3, lt, lz, ly, lx), dtype=torch.complex128,
                          device=self.device)
        call("ovl_defl_basis", self._h, _ptr(out), _stream())
        return out

    def __del__(self):
        try:
            if self._h.value:
                _lib.load().ovl_defl_destroy(self._h)
        except Exception:
            pass


def _out_like(psi, out):
    if out is None:
        return torch.empty_like(psi)
    if out.shape != psi.shape or out.dtype != psi.dtype or not out.is_contiguous():
        raise ValueError("out must match the input's shape and dtype and be contiguous")
    return out


def wilson_apply(g: GaugeField, psi, m_w: float = 0.0, dagger: bool = False, out=None):
    """(D_W - m_W) psi, or gamma5 (D_W - m_W) gamma5 psi when dagger (Sec. 2, eq. 2)."""
    nrhs = _check_spinor(psi, g.dims)
    out = _out_like(psi, out)
    call("ovl_wilson_apply", g.handle, _ptr(out), _ptr(psi), nrhs, _spin_dtype(psi), float(m_w),
         1 if dagger else 0, _stream())
    return out


def kernel_apply(g: GaugeField, psi, m_w: float = M_W, out=None):
    """K psi = gamma5 (D_W - m_W) psi."""
    nrhs = _check_spinor(psi, g.dims)
    out = _out_like(psi, out)
    call("ovl_kernel_apply", g.handle, _ptr(out), _ptr(psi), nrhs, _spin_dtype(psi), float(m_w),
         _stream())
    return out


def kernel_axpby(g: GaugeField, psi, c: float, src=None, a: float = 0.0, w=None, b: float = 0.0,
                 m_w: float = M_W, out=None):
    """out = c K psi + a src + b w in one fused launch (src, w optional; out may be src or w)."""
    nrhs = _check_spinor(psi, g.dims)
    for t in (src, w):
        if t is not None and (t.shape != psi.shape or t.dtype != psi.dtype or not t.is_contiguous()):
            raise ValueError("src and w must match psi in shape and dtype and be contiguous")
    out = _out_like(psi, out)
    call("ovl_kernel_axpby", g.handle, _ptr(out), _ptr(psi), float(c),
         _ptr(src) if src is not None else None, float(a), _ptr(w) if w is not None else None,
         float(b), nrhs, _spin_dtype(psi), float(m_w), _stream())
    return out


def sign_apply(g: GaugeField, poly: Polynomial, psi, defl: Deflation = None, out=None):
    """sum_m alpha_m T_m(X) psi + sum_i phi_i w_i phi_i^+ psi (Sec. 2, eq. 3)."""
    nrhs = _check_spinor(psi, g.dims)
    out = _out_like(psi, out)
    call("ovl_sign_apply", g.handle, poly._h, defl._h if defl is not None else None, _ptr(out),
         _ptr(psi), nrhs, _spin_dtype(psi), _stream())
    return out


def sign_residual(g: GaugeField, poly: Polynomial, psi, defl: Deflation = None) -> np.ndarray:
    """||S (S psi_r) - psi_r|| / ||psi_r|| per right-hand side for the approximate sign function S
    of sign_apply (the exact one squares to one); FP64 reductions on the device."""
    nrhs = _check_spinor(psi, g.dims)
    r = (ctypes.c_double * nrhs)()
    call("ovl_sign_residual", g.handle, poly._h, defl._h if defl is not None else None,
         _ptr(psi), nrhs, _spin_dtype(psi), r, _stream())
    return np.array(r[:], dtype=np.float64)


def overlap_apply(g: GaugeField, poly: Polynomial, psi, mu: float, defl: Deflation = None,
                  dagger: bool = False, out=None):
    """D[mu] psi (Sec. 2, eq. 1), or D[mu]^+ psi when dagger."""
    nrhs = _check_spinor(psi, g.dims)
    out = _out_like(psi, out)
    call("ovl_overlap_apply", g.handle, poly._h, defl._h if defl is not None else None, float(mu),
         1 if dagger else 0, _ptr(out), _ptr(psi), nrhs, _spin_dtype(psi), _stream())
    return out


def overlap_solve(g: GaugeField, poly: Polynomial, b, mu: float, defl: Deflation = None,
                  g_inner: GaugeField = None, defl_inner: Deflation = None, tol: float = 1e-10,
                  max_iter: int = 10000, out=None):
    """x with D[mu] x = b (FP64): FP64 defect correction around CG on the normal equations, the
    CG in the precision of g_inner (FP32 or BF16 links) when given.  Returns (x, iterations,
    relative residual); raises OvlError (OVL_EDIVERGED) if tol is not reached."""
    if b.dtype != torch.complex128:
        raise TypeError("b must be complex128")
    _check_spinor(b, g.dims)
    x = _out_like(b, out)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0)
    call("ovl_overlap_solve", g.handle, poly._h, defl._h if defl is not None else None, float(mu),
         _ptr(x), _ptr(b), g_inner.handle if g_inner is not None else None,
         defl_inner._h if defl_inner is not None else None, float(tol), int(max_iter),
         ctypes.byref(it), ctypes.byref(res), _stream())
    return x, it.value, res.value


def overlap_solve_gmresr(g: GaugeField, poly: Polynomial, b, mu: float, defl: Deflation = None,
                         g_inner: GaugeField = None, defl_inner: Deflation = None,
                         tol: float = 1e-13, inner_tol: float = 0.1, inner_poly_tol: float = 0.03,
                         relax: bool = True, max_outer: int = 64, max_inner: int = 20000,
                         out=None):
    """x with D[mu] x = b (FP64) by GMRESR around inner CG solves in the precision of g_inner
    with a truncated sign polynomial (ovl_overlap_solve_gmresr).  Returns (x, outer steps, inner
    iterations, relative residual with the full polynomial)."""
    if b.dtype != torch.complex128:
        raise TypeError("b must be complex128")
    _check_spinor(b, g.dims)
    x = _out_like(b, out)
    no, ni = ctypes.c_int(0), ctypes.c_int(0)
    res = ctypes.c_double(0)
    call("ovl_overlap_solve_gmresr", g.handle, poly._h, defl._h if defl is not None else None,
         float(mu), _ptr(x), _ptr(b), g_inner.handle if g_inner is not None else None,
         defl_inner._h if defl_inner is not None else None, float(tol), float(inner_tol),
         float(inner_poly_tol), 1 if relax else 0, int(max_outer), int(max_inner),
         ctypes.byref(no), ctypes.byref(ni), ctypes.byref(res), _stream())
    return x, no.value, ni.value, res.value


def _batch_items(problems, outs=None):
    """ovl_batch_item array for a list of (GaugeField, psi) problems, with their outputs."""
    if not 1 <= len(problems) <= 16:
        raise ValueError("between 1 and 16 problems")
    arr = (_lib.BatchItem * len(problems))()
    res = []
    dt = None
    for i, (g, psi) in enumerate(problems):
        nrhs = _check_spinor(psi, g.dims)
        out = _out_like(psi, None if outs is None else outs[i])
        dt = _spin_dtype(psi)
        arr[i] = _lib.BatchItem(g.handle.value, psi.data_ptr(), out.data_ptr(), nrhs)
        res.append(out)
    return arr, res, dt


def batch_sign_apply(poly: Polynomial, problems, outs=None, tune_cache: str = None):
    """sum_m alpha_m T_m(X_i) psi_i for a list of (GaugeField, psi) problems in one launch per
    K application (Sec. 2, eq. 3 without deflation), in the configuration ``autotune`` measured
    for the same problem set (``tune_cache``: a cache file to read first).  Returns the list of
    outputs."""
    arr, res, dt = _batch_items(problems, outs)
    call("ovl_batch_sign_apply", arr, len(problems), poly._h, dt,
         tune_cache.encode() if tune_cache else None, _stream())
    return res


def defl_project(defl: Deflation, psi) -> torch.Tensor:
    """c[r, i] = phi_i^+ psi_r as complex128 (nrhs, n_ev), FP64 accumulation."""
    nrhs = _check_spinor(psi, defl.dims)
    c = torch.empty((nrhs, defl.n_ev), dtype=torch.complex128, device=psi.device)
    call("ovl_defl_project", defl._h, _ptr(c), _ptr(psi), nrhs, _spin_dtype(psi), _stream())
    return c


def defl_correct(defl: Deflation, psi_inout, c, w):
    """psi_r += sum_i phi_i w_i c[r, i] in place."""
    nrhs = _check_spinor(psi_inout, defl.dims)
    c = c.to(torch.complex128).contiguous()
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    if c.shape != (nrhs, defl.n_ev) or w.shape != (defl.n_ev,):
        raise ValueError("c must be (nrhs, n_ev) and w (n_ev,)")
    call("ovl_defl_correct", defl._h, _ptr(psi_inout), _ptr(c),
         w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nrhs, _spin_dtype(psi_inout),
         _stream())
    return psi_inout


def _g_like(g: GaugeField, psi, out):
    lx, ly, lz, lt = g.dims
    shape = (4, 3, 3, lt, lz, ly, lx)
    if out is None:
        return torch.empty(shape, dtype=psi.dtype, device=psi.device)
    if tuple(out.shape) != shape or out.dtype != psi.dtype:
        raise ValueError("G must be (4, 3, 3, T, Z, Y, X) of the spinor dtype")
    return out


def wilson_link_vjp(g: GaugeField, chi, psi, out=None, accumulate: bool = False):
    """G = dRe<chi, D_W psi>/dRe U + i dRe<chi, D_W psi>/dIm U (single right-hand side)."""
    if _check_spinor(chi, g.dims) != 1 or _check_spinor(psi, g.dims) != 1:
        raise ValueError("single right-hand side expected")
    out = _g_like(g, psi, out)
    call("ovl_wilson_link_vjp", g.handle, _ptr(out), _ptr(chi), _ptr(psi), _spin_dtype(psi),
         1 if accumulate else 0, _stream())
    return out


def sign_force(g: GaugeField, poly: Polynomial, chi, psi, ckpt_stride: int = 0, out=None):
    """G = d Re<chi, p(X) psi> / dU (lmax fixed, no deflation term), checkpointed sweep."""
    if _check_spinor(chi, g.dims) != 1 or _check_spinor(psi, g.dims) != 1:
        raise ValueError("single right-hand side expected")
    out = _g_like(g, psi, out)
    call("ovl_sign_force", g.handle, poly._h, _ptr(out), _ptr(chi), _ptr(psi), int(ckpt_stride),
         _spin_dtype(psi), _stream())
    return out


class SignFunction(torch.autograd.Function):
    """y = p(X) psi with X = gamma5 (D_W[U] - m_W) / lmax, differentiable in U and psi.

    Backward (torch's complex convention, grad = dL/dRe + i dL/dIm): grad_psi = p(X) grad_y
    (p(X) is Hermitian) and grad_U = ovl_sign_force(chi = grad_y, psi).
    """

    @staticmethod
    def forward(ctx, u, psi, poly: Polynomial, store: str = "f64"):
        g = GaugeField(u.detach(), store)
        ctx.save_for_backward(psi)
        ctx.g = g
        ctx.poly = poly
        return sign_apply(g, poly, psi.detach().contiguous())

    @staticmethod
    def backward(ctx, grad_y):
        (psi,) = ctx.saved_tensors
        grad_y = grad_y.contiguous()
        grad_u = grad_psi = None
        if ctx.needs_input_grad[0]:
            grad_u = sign_force(ctx.g, ctx.poly, grad_y, psi.detach().contiguous())
        if ctx.needs_input_grad[1]:
            grad_psi = sign_apply(ctx.g, ctx.poly, grad_y)
        return grad_u, grad_psi, None, None


def autotune(problems, poly: Polynomial = None, cache_path: str = None, outs=None) -> float:
    """Pick the fastest launch configuration of the fused Chebyshev step for a problem set: a list
    of (GaugeField, psi) problems (the batched launch) or one such pair (the single-problem launch
    of every operator).  Returns its microseconds per step; the choice applies to every later
    launch of the same problem set in this process.  The outputs (``outs`` or temporaries) are
    overwritten."""
    if isinstance(problems, tuple) and len(problems) == 2 and isinstance(problems[0], GaugeField):
        problems = [problems]
    arr, _, dt = _batch_items(problems, outs)
    us = ctypes.c_double(0)
    call("ovl_autotune", arr, len(problems), poly._h if poly is not None else None, dt,
         cache_path.encode() if cache_path else None, ctypes.byref(us), _stream())
    return us.value


def batch_launch_config(problems):
    """(sites per workgroup, order, XCD remap, right-hand-side block) an evaluation of this
    problem set (a list of (GaugeField, psi) pairs, or one pair) will use."""
    if isinstance(problems, tuple) and len(problems) == 2 and isinstance(problems[0], GaugeField):
        problems = [problems]
    outs = [torch.empty_like(psi) for _, psi in problems]   # distinct outputs for the checks
    arr, _, dt = _batch_items(problems, outs)
    out = (ctypes.c_int * 4)()
    call("ovl_batch_launch_config", arr, len(problems), dt, out)
    return tuple(out)


def autotune_load(cache_path: str) -> int:
    n = _lib.load().ovl_autotune_load(cache_path.encode())
    if n < 0:
        raise _lib.OvlError("ovl_autotune_load", n, _lib.load().ovl_last_error().decode())
    return n


def launch_config(g: GaugeField, nrhs: int = 1, dtype=None):
    """(sites per workgroup, tile order on, XCD remap on) the library will use."""
    dt = _spin_dtype(torch.empty(0, dtype=dtype or g.spin_dtype))
    out = (ctypes.c_int * 3)()
    call("ovl_launch_config", g.handle, int(nrhs), dt, out)
    return tuple(out)


def graph_enable(on: bool = True):
    """Replay the plain recurrence steps of repeated small sign evaluations from cached HIP
    graphs (on by default; results are bitwise the same either way)."""
    call("ovl_graph_enable", 1 if on else 0)


def timing_enable(on: bool = True):
    call("ovl_timing_enable", 1 if on else 0)


def timing_read(kind: int = 0):
    """(total milliseconds, launches) since the last read of this kind: 0 = the fused Chebyshev
    step kernel (runs of plain recurrence steps), 1 = link-VJP launches of the force."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    call("ovl_timing_read", int(kind), ctypes.byref(ms), ctypes.byref(n))
    return ms.value, n.value


STREAM_READ, STREAM_COPY, STREAM_3TO1 = 0, 1, 2


def stream_probe(kind: int, dst, src, nbytes: int):
    """One plain device-memory stream (bandwidth ceiling): read, copy or three-to-one, on the
    current stream (see ovl_stream_probe)."""
    call("ovl_stream_probe", int(kind), _ptr(dst), _ptr(src), int(nbytes), _stream())


# ------------------------------------------------------------------------------------------------
# stout smearing of the links (Sec. 2: 3 steps of over-improved stout smearing, rho = 0.1,
# eps = -0.25) and its chain rule (the HMC force on the thin links, Sec. 1)
def _check_links64(u, name="U"):
    if not u.is_cuda or u.dim() != 7 or tuple(u.shape[:3]) != (4, 3, 3):
        raise ValueError(f"{name} must be a CUDA tensor of shape (4, 3, 3, T, Z, Y, X)")
    if u.dtype != torch.complex128 or not u.is_contiguous():
        raise ValueError(f"{name} must be contiguous complex128")
    return (int(u.shape[6]), int(u.shape[5]), int(u.shape[4]), int(u.shape[3]))


def stout_smear(u, rho: float = 0.1, eps: float = -0.25, steps: int = 3, out=None):
    """Links after `steps` stout steps with the over-improved staples of weight eps (eps = 1:
    plain stout smearing); FP64 in and out."""
    dims = _check_links64(u)
    out = torch.empty_like(u) if out is None else out
    _check_links64(out, "out")
    call("ovl_stout_smear", _dims_arr(dims), _ptr(out), _ptr(u), float(rho), float(eps),
         int(steps), _stream())
    return out


def stout_backward(u_thin, g_smeared, rho: float = 0.1, eps: float = -0.25, steps: int = 3,
                   out=None):
    """dL/dRe U + i dL/dIm U of the thin links from the same derivative of the smeared links."""
    dims = _check_links64(u_thin, "U_thin")
    if _check_links64(g_smeared, "G_smeared") != dims:
        raise ValueError("G_smeared and U_thin differ in shape")
    out = torch.empty_like(u_thin) if out is None else out
    _check_links64(out, "out")
    call("ovl_stout_backward", _dims_arr(dims), _ptr(out), _ptr(g_smeared), _ptr(u_thin),
         float(rho), float(eps), int(steps), _stream())
    return out


class StoutFunction(torch.autograd.Function):
    """U_smeared = stout(U); backward carries dL/dU_smeared to the thin links (torch's complex
    gradient convention dL/dRe + i dL/dIm).  Composes with SignFunction for the force of
    Re<chi, p(X[stout(U)]) psi> on U."""

    @staticmethod
    def forward(ctx, u, rho: float = 0.1, eps: float = -0.25, steps: int = 3):
        u = u.detach().contiguous()
        ctx.save_for_backward(u)
        ctx.par = (float(rho), float(eps), int(steps))
        return stout_smear(u, *ctx.par)

    @staticmethod
    def backward(ctx, grad):
        (u,) = ctx.saved_tensors
        g = grad.contiguous()
        if g.dtype != torch.complex128:
            g = g.to(torch.complex128)
        return stout_backward(u, g, *ctx.par), None, None, None
