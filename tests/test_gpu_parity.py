"""GPU parity: every C-ABI operator against the FP64 oracle on the same seeded inputs.

Operators of Cundy & Lee, Sec. 2: D_W (eq. 2), K, the deflated Chebyshev sign function (eq. 3),
the overlap operator (eq. 1), deflation projection/correction and the link derivatives.
Tolerances: 1e-12 relative for the FP64 path (the GPU evaluates the polynomial by Clenshaw's
recurrence, the oracle by the forward recurrence, so they agree only up to rounding that grows
with the degree), 1e-6 for the FP32 path.  Mixed-precision results are compared with the oracle
run on the same rounded inputs (link rounding is an input, not kernel error).
"""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import deflation as odefl
from oracle import force as oforce
from oracle import overlap as oov
from oracle import wilson as ow
from tests.conftest import complete_third_row, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LMAX = 6.5


@pytest.fixture(scope="module")
def ovl():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1510_06897_amd as m
    m.load()
    return m


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.complex128).numpy()


def max_rel(a, b):
    """max |a - b| over max |b| (element-wise bound) and the norm ratio."""
    return max(float(np.abs(a - b).max() / np.abs(b).max()), rel_err(a, b))


DIMS_SMALL = [(4, 4, 4, 4), (2, 3, 4, 5), (1, 3, 2, 2), (5, 2, 3, 7)]


@pytest.mark.parametrize("dims", DIMS_SMALL + [(8, 8, 8, 16)])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_wilson_kernel_fp64(ovl, dims, nrhs):
    u = latgen.random_su3_field(dims, 10100, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20100, nrhs=nrhs)
    g = ovl.GaugeField(dev(u), "f64")
    d_psi = dev(psi)
    got_dw = host(ovl.wilson_apply(g, d_psi, m_w=0.0))
    got_dag = host(ovl.wilson_apply(g, d_psi, m_w=1.5, dagger=True))
    got_k = host(ovl.kernel_apply(g, d_psi, m_w=1.5))
    for r in range(nrhs):
        assert max_rel(got_dw[r], ow.dw(u, psi[r])) < 1e-14
        ref_dag = ow.gamma5(ow.dw_minus_mass(u, ow.gamma5(psi[r]), 1.5))
        assert max_rel(got_dag[r], ref_dag) < 1e-14
        assert max_rel(got_k[r], ow.kop(u, psi[r])) < 1e-14


@pytest.mark.parametrize("dims", [(20, 12, 12, 24), (24, 6, 10, 48), (16, 16, 16, 16)])
def test_kernel_large_orders(ovl, dims):
    """Lattices above 64K sites: the t-streaming tile order (Lx x 4 x 4, Lx x 8 x 8) and the
    memory-order fallback when no tile divides the extents, FP64, two right-hand sides."""
    u = latgen.random_su3_field(dims, 10150, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20150, nrhs=2)
    g = ovl.GaugeField(dev(u), "f64")
    got = host(ovl.kernel_apply(g, dev(psi)))
    for r in range(2):
        assert max_rel(got[r], ow.kop(u, psi[r])) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 5, 2, 4), (8, 8, 8, 16)])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_kernel_mixed(ovl, dims, store):
    u = latgen.smeared_field(dims, 10200, steps=1)
    psi = latgen.gaussian_spinor(dims, 20200, nrhs=2)
    u_r = latgen.round_to_f32(u) if store == "f32" else latgen.round_to_bf16(u)
    psi_r = latgen.round_to_f32(psi)
    g = ovl.GaugeField(dev(u), store)
    got = host(ovl.kernel_apply(g, dev(psi, torch.complex64)))
    for r in range(2):
        ref_same = ow.kop(u_r, psi_r[r])
        assert max_rel(got[r], ref_same) < 1e-6                  # kernel arithmetic
        end_to_end = rel_err(got[r], ow.kop(u, psi[r]))
        assert end_to_end < (1e-6 if store == "f32" else 1e-2)   # includes link rounding


@pytest.mark.parametrize("dims,spw", [((20, 12, 12, 24), 128), ((16, 16, 16, 16), 128),
                                      ((15, 8, 8, 72), 64)])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_kernel_pairs(ovl, tmp_path, dims, spw, store):
    """Two x-adjacent sites per lane (selected through a tuning-cache entry): memory order (no
    tile divides 20 x 12 x 12), the tile order (16^4), and the one-site kernel for an odd Lx."""
    prec = {"f32": 1, "bf16": 2}[store]
    cache = tmp_path / "pairs.txt"
    cache.write_text(" ".join(map(str, dims)) + f" {prec} 1 128 1 1 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.random_su3_field(dims, 10160, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20160)
    u_r = latgen.round_to_f32(u) if store == "f32" else latgen.round_to_bf16(u)
    g = ovl.GaugeField(dev(u), store)
    assert ovl.launch_config(g, 1)[0] == spw
    got = host(ovl.kernel_apply(g, dev(psi, torch.complex64)))
    assert max_rel(got, ow.kop(u_r, latgen.round_to_f32(psi))) < 1e-6


def test_kernel_pairs_unaligned_vectors(ovl, tmp_path):
    """Vectors that are not 16-byte aligned fall back to one site per lane, same result."""
    dims = (16, 16, 16, 16)
    cache = tmp_path / "pairs.txt"
    cache.write_text(" ".join(map(str, dims)) + " 1 1 128 1 1 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.random_su3_field(dims, 10161)
    psi = latgen.gaussian_spinor(dims, 20161)
    g = ovl.GaugeField(dev(u), "f32")
    n = psi.size
    buf = torch.zeros(2 * n + 1, dtype=torch.complex64, device="cuda")
    x = buf[1:n + 1].view(psi.shape)
    x.copy_(dev(psi, torch.complex64))
    y = buf[n + 1:].view(psi.shape)
    ovl.kernel_apply(g, x, out=y)
    ref = ow.kop(latgen.round_to_f32(u), latgen.round_to_f32(psi))
    assert max_rel(host(y), ref) < 1e-6
    assert max_rel(host(ovl.kernel_apply(g, x)), ref) < 1e-6


def test_sign_overlap_pairs_deflated(ovl, tmp_path):
    """The final fused step (deflation, norms, overlap combine) in the two-sites-per-lane form,
    both D and D^dagger, against the oracle."""
    dims = (16, 16, 8, 32)
    cache = tmp_path / "pairs.txt"
    cache.write_text(" ".join(map(str, dims)) + " 1 1 128 1 1 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.smeared_field(dims, 10162, steps=1)
    psi = latgen.gaussian_spinor(dims, 20162)
    phi, lam = random_basis(dims, 5, 20163)
    alpha = och.coeffs_sign_interp(21, 0.1)
    g = ovl.GaugeField(dev(u), "f32")
    assert ovl.launch_config(g, 1)[0] == 128
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f32")
    x = dev(psi, torch.complex64)
    s = host(ovl.sign_apply(g, p, x, defl=d))
    assert rel_err(s, och.sign_apply(u, psi, alpha, LMAX, phi, lam)) < 1e-6
    o = host(ovl.overlap_apply(g, p, x, 0.05, defl=d))
    assert rel_err(o, oov.overlap_apply(u, psi, 0.05, alpha, LMAX, phi, lam)) < 1e-6
    od = host(ovl.overlap_apply(g, p, x, 0.05, defl=d, dagger=True))
    assert rel_err(od, oov.overlap_dagger_apply(u, psi, 0.05, alpha, LMAX, phi, lam)) < 1e-6
    assert g.flags() == 0


@pytest.mark.parametrize("dims", [(3, 3, 3, 3), (2, 3, 4, 5), (6, 4, 2, 4)])
@pytest.mark.parametrize("spb", [8, 16])
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_kernel_small_launch_forms(ovl, tmp_path, dims, spb, store):
    """Eight threads per site (forward and backward hops on separate threads, 8 sites per
    workgroup) and four (16 sites), forced through a tuning-cache entry, on volumes that leave a
    ragged last workgroup; two right-hand sides."""
    prec = {"f64": 0, "f32": 1, "bf16": 2}[store]
    cache = tmp_path / "small.txt"
    cache.write_text(" ".join(map(str, dims)) + f" {prec} 2 {spb} 0 1 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.random_su3_field(dims, 10175, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20175, nrhs=2)
    g = ovl.GaugeField(dev(u), store)
    assert ovl.launch_config(g, 2) == (spb, 0, 1)
    if store == "f64":
        got = host(ovl.kernel_apply(g, dev(psi)))
        for r in range(2):
            assert max_rel(got[r], ow.kop(u, psi[r])) < 1e-14
        return
    u_r = latgen.round_to_f32(u) if store == "f32" else latgen.round_to_bf16(u)
    got = host(ovl.kernel_apply(g, dev(psi, torch.complex64)))
    for r in range(2):
        assert max_rel(got[r], ow.kop(u_r, latgen.round_to_f32(psi[r]))) < 1e-6


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_sign_overlap_eight_threads_deflated(ovl, tmp_path, store):
    """Every step of a deflated sign and overlap evaluation with eight threads per site, on a
    volume (225 sites) that leaves a ragged last workgroup."""
    dims = (5, 5, 3, 3)
    prec = {"f64": 0, "f32": 1}[store]
    cache = tmp_path / "small.txt"
    cache.write_text(" ".join(map(str, dims)) + f" {prec} 1 8 0 1 0\n")
    ovl.autotune_load(str(cache))
    u = latgen.smeared_field(dims, 10176, steps=1)
    psi = latgen.gaussian_spinor(dims, 20176)
    phi, lam = random_basis(dims, 4, 20177)
    alpha = och.coeffs_sign_interp(31, 0.1)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    tol = 1e-12 if store == "f64" else 1e-6
    g = ovl.GaugeField(dev(u), store)
    assert ovl.launch_config(g, 1) == (8, 0, 1)
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, store)
    x = dev(psi, cdt)
    s = host(ovl.sign_apply(g, p, x, defl=d))
    assert rel_err(s, och.sign_apply(u, psi, alpha, LMAX, phi, lam)) < tol
    o = host(ovl.overlap_apply(g, p, x, 0.05, defl=d))
    assert rel_err(o, oov.overlap_apply(u, psi, 0.05, alpha, LMAX, phi, lam)) < tol
    od = host(ovl.overlap_apply(g, p, x, 0.05, defl=d, dagger=True))
    assert rel_err(od, oov.overlap_dagger_apply(u, psi, 0.05, alpha, LMAX, phi, lam)) < tol
    assert g.flags() == 0


SLAB_CASES = [((16, 8, 4, 6), 64), ((16, 8, 6, 4), 128), ((24, 16, 2, 4), 192), ((8, 8, 4, 6), 64)]


@pytest.mark.parametrize("dims,spb", SLAB_CASES)
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_kernel_slab(ovl, tmp_path, dims, spb, store):
    """The slab order (whole x lines staged in LDS with the periodic y halo rows), forced through
    a tuning-cache entry, against the oracle; two right-hand sides."""
    prec = {"f64": 0, "f32": 1, "bf16": 2}[store]
    cache = tmp_path / "slab.txt"
    cache.write_text(" ".join(map(str, dims)) + f" {prec} 2 {spb} 2 1 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.random_su3_field(dims, 10170, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20170, nrhs=2)
    g = ovl.GaugeField(dev(u), store)
    assert ovl.launch_config(g, 2) == (spb, 2, 1)
    if store == "f64":
        got = host(ovl.kernel_apply(g, dev(psi)))
        for r in range(2):
            assert max_rel(got[r], ow.kop(u, psi[r])) < 1e-14
        return
    u_r = latgen.round_to_f32(u) if store == "f32" else latgen.round_to_bf16(u)
    got = host(ovl.kernel_apply(g, dev(psi, torch.complex64)))
    for r in range(2):
        assert max_rel(got[r], ow.kop(u_r, latgen.round_to_f32(psi[r]))) < 1e-6


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_sign_overlap_slab_deflated(ovl, tmp_path, store):
    """Every step of a deflated sign and overlap evaluation in the slab order."""
    dims = (16, 8, 6, 6)
    prec = {"f64": 0, "f32": 1}[store]
    cache = tmp_path / "slab.txt"
    cache.write_text(" ".join(map(str, dims)) + f" {prec} 1 128 2 1 0\n")
    ovl.autotune_load(str(cache))
    u = latgen.smeared_field(dims, 10171, steps=1)
    psi = latgen.gaussian_spinor(dims, 20171)
    phi, lam = random_basis(dims, 4, 20172)
    alpha = och.coeffs_sign_interp(31, 0.1)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    tol = 1e-12 if store == "f64" else 1e-6
    g = ovl.GaugeField(dev(u), store)
    assert ovl.launch_config(g, 1) == (128, 2, 1)
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, store)
    x = dev(psi, cdt)
    s = host(ovl.sign_apply(g, p, x, defl=d))
    assert rel_err(s, och.sign_apply(u, psi, alpha, LMAX, phi, lam)) < tol
    o = host(ovl.overlap_apply(g, p, x, 0.05, defl=d, dagger=True))
    assert rel_err(o, oov.overlap_dagger_apply(u, psi, 0.05, alpha, LMAX, phi, lam)) < tol
    assert g.flags() == 0


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_kernel_many_rhs(ovl, store):
    """Nine right-hand sides on 8^3x16 in one launch (four waves per workgroup, one site per
    lane, right-hand side fastest in the workgroup order)."""
    dims = (8, 8, 8, 16)
    u = latgen.random_su3_field(dims, 10180, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20180, nrhs=9)
    u_r = latgen.round_to_f32(u) if store == "f32" else latgen.round_to_bf16(u)
    g = ovl.GaugeField(dev(u), store)
    assert ovl.launch_config(g, 9)[0] == 64
    got = host(ovl.kernel_apply(g, dev(psi, torch.complex64)))
    for r in range(9):
        assert max_rel(got[r], ow.kop(u_r, latgen.round_to_f32(psi[r]))) < 1e-6


def test_sign_overlap_many_rhs_deflated(ovl):
    """Six right-hand sides through a deflated sign and overlap evaluation in one launch per
    step (per-right-hand-side projections, norms and flags)."""
    dims = (8, 8, 8, 24)
    u = latgen.smeared_field(dims, 10181, steps=1)
    psi = latgen.gaussian_spinor(dims, 20181, nrhs=6)
    phi, lam = random_basis(dims, 3, 20182)
    alpha = och.coeffs_sign_interp(21, 0.1)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f32")
    x = dev(psi, torch.complex64)
    s = host(ovl.sign_apply(g, p, x, defl=d))
    o = host(ovl.overlap_apply(g, p, x, 0.01, defl=d))
    for r in range(6):
        assert rel_err(s[r], och.sign_apply(u, psi[r], alpha, LMAX, phi, lam)) < 1e-6
        assert rel_err(o[r], oov.overlap_apply(u, psi[r], 0.01, alpha, LMAX, phi, lam)) < 1e-6
    assert g.flags() == 0


@pytest.mark.parametrize("dims,spb,order,rb", [((16, 8, 8, 8), 64, 0, 2), ((16, 8, 8, 8), 16, 0, 4),
                                               ((16, 16, 16, 16), 64, 1, 4),
                                               ((16, 16, 16, 16), 16, 1, 2)])
@pytest.mark.parametrize("store", ["f64", "f32"])
def test_sign_overlap_rhs_blocks(ovl, tmp_path, dims, spb, order, rb, store):
    """Right-hand-side blocks (one link read per thread for rb right-hand sides), forced through
    a tuning-cache entry: five right-hand sides (a ragged last block), deflated sign and overlap
    evaluations, memory and tile order."""
    prec = {"f64": 0, "f32": 1}[store]
    nrhs = 5
    cache = tmp_path / "rb.txt"
    cache.write_text(f"B {prec} 0 1 {' '.join(map(str, dims))} {nrhs} {spb} {order} 1 {rb} 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.smeared_field(dims, 10183, steps=1)
    psi = latgen.gaussian_spinor(dims, 20183, nrhs=nrhs)
    phi, lam = random_basis(dims, 3, 20184)
    alpha = och.coeffs_sign_interp(11, 0.1)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    tol = 1e-12 if store == "f64" else 1e-6
    g = ovl.GaugeField(dev(u), store)
    x = dev(psi, cdt)
    assert ovl.batch_launch_config((g, x)) == (spb, order, 1, rb)
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, store)
    s = host(ovl.sign_apply(g, p, x, defl=d))
    od = host(ovl.overlap_apply(g, p, x, 0.05, defl=d, dagger=True))
    for r in range(nrhs):
        assert rel_err(s[r], och.sign_apply(u, psi[r], alpha, LMAX, phi, lam)) < tol
        assert rel_err(od[r], oov.overlap_dagger_apply(u, psi[r], 0.05, alpha, LMAX, phi,
                                                       lam)) < tol
    assert g.flags() == 0


@pytest.mark.parametrize("store,cdt,tol", [("f64", torch.complex128, 1e-14),
                                           ("f32", torch.complex64, 1e-6)])
def test_kernel_axpby(ovl, store, cdt, tol):
    """out = c K psi + a src + b w in one launch, also in place over w and over src."""
    dims = (4, 6, 2, 8)
    u = latgen.random_su3_field(dims, 10195)
    psi, src, w = (latgen.gaussian_spinor(dims, 20195 + i, nrhs=2) for i in range(3))
    if store == "f32":
        u, psi, src, w = (latgen.round_to_f32(a) for a in (u, psi, src, w))
    g = ovl.GaugeField(dev(u), store)
    c, a, b = 0.37, -1.25, 0.5
    ref = np.stack([c * ow.kop(u, psi[r]) + a * src[r] + b * w[r] for r in range(2)])
    got = host(ovl.kernel_axpby(g, dev(psi, cdt), c, src=dev(src, cdt), a=a, w=dev(w, cdt), b=b))
    assert max_rel(got, ref) < tol
    wd = dev(w, cdt)
    ovl.kernel_axpby(g, dev(psi, cdt), c, src=dev(src, cdt), a=a, w=wd, b=b, out=wd)
    assert max_rel(host(wd), ref) < tol
    sd = dev(src, cdt)
    ovl.kernel_axpby(g, dev(psi, cdt), c, src=sd, a=a, out=sd)
    ref2 = np.stack([c * ow.kop(u, psi[r]) + a * src[r] for r in range(2)])
    assert max_rel(host(sd), ref2) < tol
    ref3 = np.stack([c * ow.kop(u, psi[r]) for r in range(2)])
    assert max_rel(host(ovl.kernel_axpby(g, dev(psi, cdt), c)), ref3) < tol


def c1_inputs():
    dims = (4, 4, 4, 4)
    u = latgen.random_su3_field(dims, latgen.seed_for("gauge", 1))
    psi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 1))
    from oracle.eigen import low_modes
    lam, _, _ = low_modes(u, 1, LMAX, filter_degree=16)
    eps = abs(lam[0]) / LMAX
    alpha = och.coeffs_sign_interp(64, eps)
    return dims, u, psi, alpha


def test_sign_overlap_c1_fp64(ovl):
    dims, u, psi, alpha = c1_inputs()
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d_psi = dev(psi)
    s = host(ovl.sign_apply(g, p, d_psi))
    ref_s = och.sign_apply(u, psi, alpha, LMAX)
    assert max_rel(s, ref_s) < 1e-12
    for dag in (False, True):
        o = host(ovl.overlap_apply(g, p, d_psi, 0.1, dagger=dag))
        ref = (oov.overlap_dagger_apply if dag else oov.overlap_apply)(u, psi, 0.1, alpha, LMAX)
        assert max_rel(o, ref) < 1e-12
    assert g.flags() == 0


@pytest.mark.parametrize("n_alpha", [2, 3, 4, 5])
def test_sign_low_degrees(ovl, n_alpha):
    """Degree 1..4, including even top index: exercises the folded first Clenshaw steps."""
    dims = (3, 2, 4, 2)
    u = latgen.random_su3_field(dims, 7)
    psi = latgen.gaussian_spinor(dims, 8, nrhs=2)
    alpha = np.random.default_rng(n_alpha).standard_normal(n_alpha) * 0.5
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    s = host(ovl.sign_apply(g, p, dev(psi)))
    for r in range(2):
        assert max_rel(s[r], och.poly_apply(u, psi[r], alpha, LMAX)) < 1e-13


def random_basis(dims, n_ev, seed):
    raw = latgen.gaussian_spinor(dims, seed, nrhs=n_ev)
    phi = odefl.cgs2(raw)
    lam = np.linspace(-0.52, 0.52, n_ev) + 0.003
    return phi, lam


@pytest.fixture(scope="module")
def deflated_8x8x8x16():
    dims = (8, 8, 8, 16)
    u = latgen.smeared_field(dims, latgen.seed_for("gauge", 2))
    psi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 2))
    phi, lam = random_basis(dims, 12, 777)
    alpha = och.coeffs_sign_interp(200, 0.077)
    ref_s = och.sign_apply(u, psi, alpha, LMAX, phi, lam)
    return dims, u, psi, phi, lam, alpha, ref_s


def test_sign_8x8x8x16_deflated_fp64(ovl, deflated_8x8x8x16):
    dims, u, psi, phi, lam, alpha, ref_s = deflated_8x8x8x16
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    d_psi = dev(psi)
    s = host(ovl.sign_apply(g, p, d_psi, defl=d))
    assert max_rel(s, ref_s) < 1e-12
    for mu in (0.01, 0.05):
        o = host(ovl.overlap_apply(g, p, d_psi, mu, defl=d))
        ref = 0.5 * ((1 + mu) * psi + (1 - mu) * ow.gamma5(ref_s))
        assert max_rel(o, ref) < 1e-12
    assert g.flags() == 0


def test_sign_8x8x8x16_deflated_fp32(ovl, deflated_8x8x8x16):
    dims, u, psi, phi, lam, alpha, ref_s = deflated_8x8x8x16
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f32")
    s = host(ovl.sign_apply(g, p, dev(psi, torch.complex64), defl=d))
    err = rel_err(s, ref_s)
    assert err < 1e-6, err
    assert g.flags() == 0


def test_overlap_dagger_deflated_fp64(ovl):
    dims = (4, 4, 2, 4)
    u = latgen.smeared_field(dims, 31)
    psi = latgen.gaussian_spinor(dims, 32)
    phi, lam = random_basis(dims, 5, 33)
    alpha = och.coeffs_sign_interp(41, 0.08)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    o = host(ovl.overlap_apply(g, p, dev(psi), 0.05, defl=d, dagger=True))
    ref = oov.overlap_dagger_apply(u, psi, 0.05, alpha, LMAX, phi, lam)
    assert max_rel(o, ref) < 1e-12


def test_deflation_exact_on_true_eigenvectors(ovl):
    from oracle.eigen import dense_eigs
    dims = (4, 4, 2, 4)
    u = latgen.random_su3_field(dims, 41, noise=0.6)
    lam_all, vec_all = dense_eigs(u)
    lam, phi = lam_all[:6], vec_all[:6]
    alpha = och.coeffs_sign_interp(63, 0.05)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    s = host(ovl.sign_apply(g, p, dev(phi), defl=d))
    for i in range(6):
        assert rel_err(s[i], np.sign(lam[i]) * phi[i]) < 1e-12


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_defl_project_correct(ovl, store):
    dims = (4, 2, 4, 6)
    phi, lam = random_basis(dims, 7, 51)
    psi = latgen.gaussian_spinor(dims, 52, nrhs=3)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    d = ovl.Deflation(dev(phi), lam, store)
    basis = host(d.basis())
    assert rel_err(basis, phi) < 1e-13
    c = host(ovl.defl_project(d, dev(psi, cdt)))
    psi_in = latgen.round_to_f32(psi) if store == "f32" else psi
    phi_in = latgen.round_to_f32(phi) if store == "f32" else phi
    tol = 1e-13 if store == "f64" else 1e-6
    c_ref = np.stack([odefl.project(phi_in, psi_in[r]) for r in range(3)])
    for r in range(3):
        assert max_rel(c[r], c_ref[r]) < tol
    # the correction takes the oracle's projections as its input on both sides
    w = np.linspace(-1.0, 2.0, 7)
    out = dev(psi, cdt)
    ovl.defl_correct(d, out, dev(c_ref), w)
    out = host(out)
    for r in range(3):
        ref = odefl.correct(phi_in, psi_in[r], c_ref[r], w)
        assert max_rel(out[r], ref) < tol


@pytest.mark.parametrize("n_ev,nrhs", [(20, 10), (12, 1), (3, 9), (16, 8)])
def test_defl_project_mfma_tiles(ovl, n_ev, nrhs):
    """FP32 projection on the matrix cores: partial and several MFMA tiles in both the
    eigenvector and the right-hand-side direction, a volume that leaves ragged chunks, FP64
    oracle on the rounded data."""
    dims = (5, 3, 4, 6)
    phi, lam = random_basis(dims, n_ev, 55)
    psi = latgen.gaussian_spinor(dims, 56, nrhs=nrhs)
    d = ovl.Deflation(dev(phi), lam, "f32")
    c = host(ovl.defl_project(d, dev(psi, torch.complex64)))
    phi_r, psi_r = latgen.round_to_f32(phi), latgen.round_to_f32(psi)
    for r in range(nrhs):
        ref = odefl.project(phi_r, psi_r[r])
        assert max_rel(c[r], ref) < 1e-6


def test_overlap_dagger_deflated_fp32(ovl):
    """gamma5 applied to the source inside the FP32 matrix-core projection (the adjoint)."""
    dims = (4, 4, 2, 4)
    u = latgen.smeared_field(dims, 34)
    psi = latgen.gaussian_spinor(dims, 35)
    phi, lam = random_basis(dims, 5, 36)
    alpha = och.coeffs_sign_interp(41, 0.08)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f32")
    o = host(ovl.overlap_apply(g, p, dev(psi, torch.complex64), 0.05, defl=d, dagger=True))
    ref = oov.overlap_dagger_apply(u, psi, 0.05, alpha, LMAX, phi, lam)
    assert rel_err(o, ref) < 1e-6


def test_defl_rank_deficient(ovl):
    dims = (2, 2, 2, 2)
    raw = latgen.gaussian_spinor(dims, 61, nrhs=3)
    raw[2] = 2.0 * raw[0] - raw[1]
    with pytest.raises(ovl.OvlError) as e:
        ovl.Deflation(dev(raw), np.array([0.1, 0.2, 0.3]), "f64")
    assert e.value.status == "OVL_EDEFL"


@pytest.mark.parametrize("kind", ["gaussian", "near_dependent"])
def test_defl_cgs2_raw_vectors(ovl, kind):
    """The device's FP64 classical Gram-Schmidt applied twice, on vectors that are not
    orthonormal, element by element against the oracle's CGS2 of the same raw vectors: Gaussian
    vectors (norms ~ sqrt(12 V), overlaps ~ 1/sqrt(12 V)), and vectors each within a small angle of
    the span of the previous ones, where the projection removal carries the result."""
    dims = (4, 4, 4, 6)
    n_ev = 9
    raw = latgen.gaussian_spinor(dims, 20190, nrhs=n_ev) * 3.0
    if kind == "near_dependent":
        for j in range(1, n_ev):
            raw[j] = raw[j - 1] - 0.5 * raw[j // 2] + 1e-4 * raw[j]
    ref = odefl.cgs2(raw)
    d = ovl.Deflation(dev(raw), np.linspace(-0.4, 0.4, n_ev), "f64")
    got = host(d.basis())
    # conditioning: the near-dependent vectors lose about log10(1e4) digits in both
    tol = 1e-13 if kind == "gaussian" else 1e-9
    for j in range(n_ev):
        assert max_rel(got[j], ref[j]) < tol, j
    gram = got.reshape(n_ev, -1).conj() @ got.reshape(n_ev, -1).T
    assert np.abs(gram - np.eye(n_ev)).max() < 1e-13


def test_link_vjp_fp64(ovl):
    dims = (4, 3, 2, 4)
    u = latgen.random_su3_field(dims, 71)
    chi = latgen.gaussian_spinor(dims, 72)
    psi = latgen.gaussian_spinor(dims, 73)
    g = ovl.GaugeField(dev(u), "f64")
    got = host(ovl.wilson_link_vjp(g, dev(chi), dev(psi)))
    assert max_rel(got, oforce.wilson_link_vjp(chi, psi)) < 1e-14
    acc = ovl.wilson_link_vjp(g, dev(chi), dev(psi))
    ovl.wilson_link_vjp(g, dev(chi), dev(psi), out=acc, accumulate=True)
    assert max_rel(host(acc), 2 * oforce.wilson_link_vjp(chi, psi)) < 1e-14


@pytest.mark.parametrize("dims", [(6, 3, 4, 2), (2, 2, 3, 4), (5, 4, 2, 3), (16, 16, 16, 16)])
def test_link_vjp_fp32(ovl, dims):
    """FP32 link VJP against the oracle on the same FP32-rounded spinors, on extent-2, odd and
    (16^4, 64K sites) t-streaming tile-ordered launches; accumulate adds to the existing G."""
    chi = latgen.round_to_f32(latgen.gaussian_spinor(dims, 74))
    psi = latgen.round_to_f32(latgen.gaussian_spinor(dims, 75))
    g = ovl.GaugeField(dev(latgen.random_su3_field(dims, 76)), "f32")
    got = ovl.wilson_link_vjp(g, dev(chi, torch.complex64), dev(psi, torch.complex64))
    ref = oforce.wilson_link_vjp(chi, psi)
    assert max_rel(host(got), ref) < 1e-6
    ovl.wilson_link_vjp(g, dev(chi, torch.complex64), dev(psi, torch.complex64), out=got,
                        accumulate=True)
    assert max_rel(host(got), 2 * ref) < 1e-6


def test_link_vjp_fp64_tile_order(ovl):
    """FP64 link VJP on a lattice large enough for the tile order (16^3 x 16)."""
    dims = (16, 16, 16, 16)
    chi = latgen.gaussian_spinor(dims, 77)
    psi = latgen.gaussian_spinor(dims, 78)
    g = ovl.GaugeField(dev(latgen.random_su3_field(dims, 79)), "f64")
    got = host(ovl.wilson_link_vjp(g, dev(chi), dev(psi)))
    assert max_rel(got, oforce.wilson_link_vjp(chi, psi)) < 1e-14


@pytest.mark.parametrize("dims", [(6, 4, 2, 4), (3, 4, 4, 2)])
def test_sign_force_fp32_lattices(ovl, dims):
    """Checkpointed FP32 force (segments over two runs of ring slots, FP64 running sum) on even
    and odd extents against the oracle gradient on the same rounded inputs."""
    u = latgen.smeared_field(dims, 87, steps=1)
    chi = latgen.gaussian_spinor(dims, 88)
    psi = latgen.gaussian_spinor(dims, 89)
    alpha = och.coeffs_sign_interp(41, 0.1)
    u32, chi32, psi32 = latgen.round_to_f32(u), latgen.round_to_f32(chi), latgen.round_to_f32(psi)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    got = host(ovl.sign_force(g, p, dev(chi, torch.complex64), dev(psi, torch.complex64),
                              ckpt_stride=5))
    assert rel_err(got, oforce.sign_force(u32, chi32, psi32, alpha, LMAX)) < 1e-6


@pytest.mark.parametrize("aligned", [True, False])
def test_sign_force_fp32_pair_form_twins(ovl, tmp_path, aligned):
    """The FP32 force with its single and twin (two-right-hand-side) steps forced into the
    two-sites-per-lane form, against the oracle on the same rounded inputs; with chi and psi at an
    8-byte offset (not 16-byte aligned) the steps that read them fall back to one site per lane."""
    dims = (8, 4, 4, 6)
    cache = tmp_path / "pairs.txt"
    cache.write_text(f"B 1 0 1 {' '.join(map(str, dims))} 1 128 1 1 1 0\n"
                     f"B 1 0 1 {' '.join(map(str, dims))} 2 128 1 1 1 0\n")
    assert ovl.autotune_load(str(cache)) == 2
    u = latgen.smeared_field(dims, 90, steps=1)
    chi = latgen.gaussian_spinor(dims, 91)
    psi = latgen.gaussian_spinor(dims, 92)
    alpha = och.coeffs_sign_interp(41, 0.1)
    u32, chi32, psi32 = latgen.round_to_f32(u), latgen.round_to_f32(chi), latgen.round_to_f32(psi)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    x = dev(psi, torch.complex64)
    c = dev(chi, torch.complex64)
    assert ovl.batch_launch_config((g, x))[0] == 128
    if not aligned:
        n = psi.size
        buf = torch.zeros(2 * n + 1, dtype=torch.complex64, device="cuda")
        xo = buf[1:n + 1].view(psi.shape)
        co = buf[n + 1:].view(chi.shape)
        xo.copy_(x)
        co.copy_(c)
        x, c = xo, co
    got = host(ovl.sign_force(g, p, c, x, ckpt_stride=5))
    assert rel_err(got, oforce.sign_force(u32, chi32, psi32, alpha, LMAX)) < 1e-6


@pytest.mark.parametrize("stride", [0, 1, 5, 63])
def test_sign_force_fp64(ovl, stride):
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 81, steps=1)
    chi = latgen.gaussian_spinor(dims, 82)
    psi = latgen.gaussian_spinor(dims, 83)
    alpha = och.coeffs_sign_interp(63, 0.07)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    got = host(ovl.sign_force(g, p, dev(chi), dev(psi), ckpt_stride=stride))
    ref = oforce.sign_force(u, chi, psi, alpha, LMAX)
    assert max_rel(got, ref) < 1e-12


def test_sign_force_fp32(ovl):
    """FP32 recurrence vectors, outer products summed in FP64: within the 1e-6 mixed-path
    tolerance against the oracle on the same FP32-rounded inputs and on the exact ones."""
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 84, steps=1)
    chi = latgen.gaussian_spinor(dims, 85)
    psi = latgen.gaussian_spinor(dims, 86)
    alpha = och.coeffs_sign_interp(63, 0.07)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    got = host(ovl.sign_force(g, p, dev(chi, torch.complex64), dev(psi, torch.complex64)))
    same = oforce.sign_force(latgen.round_to_f32(u), latgen.round_to_f32(chi),
                             latgen.round_to_f32(psi), alpha, LMAX)
    assert rel_err(got, same) < 1e-6
    assert rel_err(got, oforce.sign_force(u, chi, psi, alpha, LMAX)) < 1e-6


@pytest.fixture(scope="module")
def force299():
    """The force workload's polynomial (degree 299, eps 0.05) and checkpoint stride
    (ceil(sqrt 299) = 18) on a 4^4 lattice of 3-step stout-smeared links."""
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, latgen.seed_for("gauge", 5, 7))
    chi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 5, 8))
    psi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 5, 9))
    alpha = och.coeffs_sign_interp(300, 0.05)
    assert len(alpha) == 300   # N = 299
    return dims, u, chi, psi, alpha


@pytest.mark.parametrize("stride", [18, 0])
def test_sign_force_degree299_fp64(ovl, force299, stride):
    dims, u, chi, psi, alpha = force299
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    got = host(ovl.sign_force(g, p, dev(chi), dev(psi), ckpt_stride=stride))
    assert max_rel(got, oforce.sign_force(u, chi, psi, alpha, LMAX)) < 1e-12


def test_sign_force_degree299_fp32(ovl, force299):
    """The force workload's FP32 form at its full degree and stride on smeared links: the two
    errors of a mixed result, against the oracle on the same rounded inputs and on the exact
    ones, both within 1e-6."""
    dims, u, chi, psi, alpha = force299
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    got = host(ovl.sign_force(g, p, dev(chi, torch.complex64), dev(psi, torch.complex64),
                              ckpt_stride=18))
    same = oforce.sign_force(latgen.round_to_f32(u), latgen.round_to_f32(chi),
                             latgen.round_to_f32(psi), alpha, LMAX)
    assert rel_err(got, same) < 1e-6
    assert rel_err(got, oforce.sign_force(u, chi, psi, alpha, LMAX)) < 1e-6


def test_autograd_sign_function(ovl):
    dims = (2, 2, 2, 4)
    u = latgen.random_su3_field(dims, 91)
    psi = latgen.gaussian_spinor(dims, 92)
    chi = latgen.gaussian_spinor(dims, 93)
    alpha = och.coeffs_sign_interp(15, 0.1)
    p = ovl.Polynomial(alpha, LMAX)
    du = dev(u).requires_grad_(True)
    dpsi = dev(psi).requires_grad_(True)
    y = ovl.SignFunction.apply(du, dpsi, p, "f64")
    loss = torch.real(torch.vdot(dev(chi).reshape(-1), y.reshape(-1)))
    loss.backward()
    assert max_rel(host(du.grad), oforce.sign_force(u, chi, psi, alpha, LMAX)) < 1e-12
    assert max_rel(host(dpsi.grad), och.poly_apply(u, chi, alpha, LMAX)) < 1e-12


def test_gauge_covariance_gpu(ovl):
    dims = (4, 4, 2, 4)
    u = latgen.random_su3_field(dims, 101, noise=0.6)
    psi = latgen.gaussian_spinor(dims, 102)
    om = latgen.random_gauge_transform(dims, 103)
    alpha = och.coeffs_sign_interp(31, 0.08)
    p = ovl.Polynomial(alpha, LMAX)
    a = host(ovl.sign_apply(ovl.GaugeField(dev(latgen.gauge_transform_links(u, om)), "f64"), p,
                            dev(latgen.gauge_transform_spinor(psi, om))))
    b = latgen.gauge_transform_spinor(host(ovl.sign_apply(ovl.GaugeField(dev(u), "f64"), p,
                                                          dev(psi))), om)
    assert rel_err(a, b) < 1e-13


def test_divergence_flag(ovl):
    dims = (4, 4, 4, 4)
    u = latgen.random_su3_field(dims, 111)
    psi = latgen.gaussian_spinor(dims, 112)
    alpha = och.coeffs_sign_interp(63, 0.1)
    g = ovl.GaugeField(dev(u), "f64")
    ovl.sign_apply(g, ovl.Polynomial(alpha, LMAX), dev(psi))
    assert g.flags() == 0
    ovl.sign_apply(g, ovl.Polynomial(alpha, 3.0), dev(psi))     # lmax below ||K||
    assert g.flags() & 0x2
    assert g.flags() == 0                                         # cleared by the read


def test_alias_rejected(ovl):
    dims = (2, 2, 2, 2)
    g = ovl.GaugeField(dev(latgen.random_su3_field(dims, 1)), "f64")
    x = dev(latgen.gaussian_spinor(dims, 2))
    with pytest.raises(ovl.OvlError) as e:
        ovl.wilson_apply(g, x, out=x)
    assert e.value.status == "OVL_EALIAS"
    with pytest.raises(ovl.OvlError) as e:
        ovl.kernel_apply(g, dev(latgen.gaussian_spinor(dims, 2), torch.complex64))
    assert e.value.status == "OVL_EDTYPE"


def test_repeatable_bitwise(ovl):
    dims = (8, 8, 8, 16)
    u = latgen.random_su3_field(dims, 121)
    psi = dev(latgen.gaussian_spinor(dims, 122), torch.complex64)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(och.coeffs_sign_interp(99, 0.08), LMAX)
    phi, lam = random_basis(dims, 4, 123)
    d = ovl.Deflation(dev(phi), lam, "f32")
    a = ovl.overlap_apply(g, p, psi, 0.05, defl=d)
    b = ovl.overlap_apply(g, p, psi, 0.05, defl=d)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_dw_full_size_24x24x24x48(ovl):
    """The force lattice at full size, in the launch configuration the benchmark times."""
    dims = (24, 24, 24, 48)
    u = latgen.random_su3_field(dims, latgen.seed_for("gauge", 5))
    psi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 5))
    ref = ow.kop(u, psi)
    g64 = ovl.GaugeField(dev(u), "f64")
    assert max_rel(host(ovl.kernel_apply(g64, dev(psi))), ref) < 1e-14
    g32 = ovl.GaugeField(dev(u), "f32")
    got32 = host(ovl.kernel_apply(g32, dev(psi, torch.complex64)))
    assert rel_err(got32, ref) < 1e-6
    # two-row link reads, as the benchmark times them beside the full reads
    g64.reconstruct()
    assert max_rel(host(ovl.kernel_apply(g64, dev(psi))), ref) < 1e-13
    g32.reconstruct()
    got32 = host(ovl.kernel_apply(g32, dev(psi, torch.complex64)))
    assert rel_err(got32, ref) < 1e-6
    gbf = ovl.GaugeField(dev(u), "bf16")
    gbf.reconstruct()
    u_r = complete_third_row(latgen.round_to_bf16(u))
    got = host(ovl.kernel_apply(gbf, dev(psi, torch.complex64)))
    assert max_rel(got, ow.kop(u_r, latgen.round_to_f32(psi))) < 1e-6


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_sign_residual_vs_oracle(ovl, store):
    """||S(S psi) - psi|| / ||psi|| (the sign function squares to one) with deflation, two
    right-hand sides, against the oracle's S applied twice (FP32 on the same rounded inputs)."""
    dims = (4, 4, 2, 6)
    u = latgen.smeared_field(dims, 10180, steps=1)
    psi = latgen.gaussian_spinor(dims, 20180, nrhs=2)
    psi[1] *= 3.0
    phi, lam = random_basis(dims, 3, 20181)
    alpha = och.coeffs_sign_interp(31, 0.1)
    p = ovl.Polynomial(alpha, LMAX)
    if store == "f64":
        u_r, psi_r, phi_r = u, psi, phi
        x = dev(psi)
    else:
        u_r, psi_r, phi_r = (latgen.round_to_f32(a) for a in (u, psi, phi))
        x = dev(psi, torch.complex64)
    g = ovl.GaugeField(dev(u), store)
    d = ovl.Deflation(dev(phi), lam, store)
    got = ovl.sign_residual(g, p, x, defl=d)
    for r in range(2):
        s1 = och.sign_apply(u_r, psi_r[r], alpha, LMAX, phi_r, lam)
        s2 = och.sign_apply(u_r, s1, alpha, LMAX, phi_r, lam)
        ref = np.linalg.norm(s2 - psi_r[r]) / np.linalg.norm(psi_r[r])
        assert 1e-4 < ref < 1.0
        if store == "f64":
            assert abs(got[r] - ref) < 1e-10 * ref
        else:
            assert abs(got[r] - ref) < 1e-5
    zero = torch.zeros_like(x)
    assert np.all(ovl.sign_residual(g, p, zero, defl=d) == 0.0)


def test_ginsparg_wilson_residual_gpu(ovl):
    """At mu = 0, gamma5 D + D gamma5 - 2 D gamma5 D = -1/2 gamma5 (S^2 - 1) for any Hermitian S:
    the Ginsparg-Wilson residual of the device's overlap operator equals half the device's
    sign-function residual (FP64, deflated)."""
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 10182, steps=1)
    psi = latgen.gaussian_spinor(dims, 20182)
    phi, lam = random_basis(dims, 4, 20183)
    alpha = och.coeffs_sign_interp(31, 0.1)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    x = dev(psi)
    g5 = torch.tensor([1.0, 1.0, -1.0, -1.0], dtype=torch.float64, device="cuda").view(4, 1, 1, 1, 1, 1)
    dx = ovl.overlap_apply(g, p, x, 0.0, defl=d)
    dg5x = ovl.overlap_apply(g, p, g5 * x, 0.0, defl=d)
    dg5dx = ovl.overlap_apply(g, p, g5 * dx, 0.0, defl=d)
    gw = g5 * dx + dg5x - 2.0 * dg5dx
    lhs = float(torch.linalg.vector_norm(gw) / torch.linalg.vector_norm(x))
    rs = float(ovl.sign_residual(g, p, x, defl=d)[0])
    assert rs > 1e-4
    assert abs(lhs - 0.5 * rs) < 1e-10 * rs


_R12_FORMS = [((4, 4, 4, 4), 8, 0), ((6, 4, 2, 4), 16, 0), ((8, 8, 4, 6), 64, 1),
              ((8, 8, 4, 6), 128, 1), ((16, 8, 4, 6), 128, 2)]


# two sites per lane (128 sites per workgroup outside the slab order) take FP32 spinors
@pytest.mark.parametrize("store,dims,spb,tiles",
                         [(st, d, sp, ti) for st in ("f64", "f32", "bf16") for d, sp, ti in _R12_FORMS
                          if not (st == "f64" and sp == 128 and ti == 1)])
def test_two_row_links_kernel(ovl, tmp_path, store, dims, spb, tiles):
    """K with links read as two rows (third completed as for SU(3)) in every launch form, against
    the oracle on the links the kernel sees; two right-hand sides."""
    prec = {"f64": 0, "f32": 1, "bf16": 2}[store]
    cache = tmp_path / "r12.txt"
    # the tuning key includes the link read mode: an entry for two-row reads (r12 = 1)
    cache.write_text(f"B {prec} 1 1 {' '.join(map(str, dims))} 2 {spb} {tiles} 1 1 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.random_su3_field(dims, 10185, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20185, nrhs=2)
    g = ovl.GaugeField(dev(u), store)
    dev_max = g.reconstruct()
    assert dev_max < {"f64": 1e-14, "f32": 1e-6, "bf16": 2e-2}[store]
    assert ovl.launch_config(g, 2) == (spb, tiles, 1)
    if store == "f64":
        got = host(ovl.kernel_apply(g, dev(psi)))
        for r in range(2):
            assert max_rel(got[r], ow.kop(u, psi[r])) < 1e-13
        return
    u_r = complete_third_row(latgen.round_to_f32(u) if store == "f32" else latgen.round_to_bf16(u))
    got = host(ovl.kernel_apply(g, dev(psi, torch.complex64)))
    for r in range(2):
        assert max_rel(got[r], ow.kop(u_r, latgen.round_to_f32(psi[r]))) < 1e-6


def test_two_row_links_refused_for_non_su3(ovl):
    """A field that is not SU(3) is refused (status EINVAL, deviation reported) and keeps full
    reads."""
    dims = (4, 4, 2, 4)
    rng = np.random.default_rng(7)
    shape = (4, 3, 3) + tuple(reversed(dims))
    u = (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * 0.5
    psi = latgen.gaussian_spinor(dims, 20186)
    g = ovl.GaugeField(dev(u), "f64")
    with pytest.raises(ovl.OvlError) as e:
        g.reconstruct()
    assert e.value.status == "OVL_EINVAL"
    got = host(ovl.kernel_apply(g, dev(psi)))
    assert max_rel(got, ow.kop(u, psi)) < 1e-14


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_two_row_links_sign_overlap_and_graphs(ovl, store):
    """Deflated sign and overlap with two-row links (replayed from the step graph on repeated
    calls), then back to full reads: each against the oracle on the links it reads."""
    dims = (4, 6, 4, 8)
    u = latgen.smeared_field(dims, 10187, steps=1)
    psi = latgen.gaussian_spinor(dims, 20187)
    phi, lam = random_basis(dims, 3, 20188)
    alpha = och.coeffs_sign_interp(31, 0.1)
    cdt = torch.complex128 if store == "f64" else torch.complex64
    tol = 1e-12 if store == "f64" else 1e-6
    g = ovl.GaugeField(dev(u), store)
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, store)
    x = dev(psi, cdt)
    u_full = u if store == "f64" else latgen.round_to_f32(u)
    u_two = complete_third_row(u_full)
    ref_full = och.sign_apply(u_full, psi, alpha, LMAX, phi, lam)
    ref_two = och.sign_apply(u_two, psi, alpha, LMAX, phi, lam)
    out = torch.empty_like(x)
    for _ in range(3):
        ovl.sign_apply(g, p, x, defl=d, out=out)
    full = host(out)
    assert rel_err(full, ref_full) < tol
    g.reconstruct()
    for _ in range(3):
        ovl.sign_apply(g, p, x, defl=d, out=out)
        assert rel_err(host(out), ref_two) < tol
    o = host(ovl.overlap_apply(g, p, x, 0.05, defl=d))
    assert rel_err(o, oov.overlap_apply(u_two, psi, 0.05, alpha, LMAX, phi, lam)) < tol
    g.reconstruct(False)
    for _ in range(2):
        ovl.sign_apply(g, p, x, defl=d, out=out)
        assert np.array_equal(host(out), full)
    assert g.flags() == 0


def test_two_row_links_batch(ovl):
    """A batch whose items all read two rows equals the one-problem launches bitwise; with one
    item on full reads the whole launch reads full links and equals those launches bitwise."""
    alpha = och.coeffs_sign_interp(15, 0.08)
    p = ovl.Polynomial(alpha, LMAX)
    probs = []
    # volumes whose one-problem launches take the batch's launch form (16 sites per workgroup)
    for i, dims in enumerate([(8, 8, 8, 8), (6, 6, 8, 16), (8, 8, 6, 12)]):
        u = latgen.random_su3_field(dims, 10189 + i)
        psi = latgen.gaussian_spinor(dims, 20189 + i, nrhs=1 + i % 2)
        g = ovl.GaugeField(dev(u), "f32")
        g.reconstruct()
        probs.append((g, dev(psi, torch.complex64)))
    outs = ovl.batch_sign_apply(p, probs)
    for (g, x), o in zip(probs, outs):
        assert torch.equal(ovl.sign_apply(g, p, x), o)
    probs[1][0].reconstruct(False)
    outs = ovl.batch_sign_apply(p, probs)
    for (g, x), o in zip(probs, outs):
        g.reconstruct(False)
        assert torch.equal(ovl.sign_apply(g, p, x), o)


def test_zero_right_hand_sides_rejected(ovl):
    """An empty batch of right-hand sides is an argument error (EINVAL) before any launch, for
    the stencil, the sign function, the residual diagnostic and the batched form."""
    dims = (4, 4, 2, 2)
    g = ovl.GaugeField(dev(latgen.random_su3_field(dims, 1)), "f64")
    p = ovl.Polynomial(och.coeffs_sign_interp(7, 0.1), LMAX)
    empty = torch.zeros((0, 4, 3) + tuple(reversed(dims)), dtype=torch.complex128, device="cuda")
    for call in (lambda: ovl.kernel_apply(g, empty), lambda: ovl.sign_apply(g, p, empty),
                 lambda: ovl.sign_residual(g, p, empty),
                 lambda: ovl.batch_sign_apply(p, [(g, empty)])):
        with pytest.raises(ovl.OvlError) as e:
            call()
        assert e.value.status == "OVL_EINVAL"
    # the handle still works afterwards
    x = dev(latgen.gaussian_spinor(dims, 2))
    assert max_rel(host(ovl.kernel_apply(g, x)), ow.kop(latgen.random_su3_field(dims, 1),
                                                         latgen.gaussian_spinor(dims, 2))) < 1e-14


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_two_row_links_force(ovl, store):
    """The checkpointed force with two-row link reads against the oracle gradient on the links the
    kernels see (ragged segments: degree 63, stride ceil(sqrt 63) = 8)."""
    dims = (4, 4, 4, 4)
    u = latgen.smeared_field(dims, 10195, steps=1)
    chi = latgen.gaussian_spinor(dims, 20195)
    psi = latgen.gaussian_spinor(dims, 20196)
    alpha = och.coeffs_sign_interp(63, 0.07)
    g = ovl.GaugeField(dev(u), store)
    g.reconstruct()
    p = ovl.Polynomial(alpha, LMAX)
    if store == "f64":
        got = host(ovl.sign_force(g, p, dev(chi), dev(psi)))
        assert max_rel(got, oforce.sign_force(u, chi, psi, alpha, LMAX)) < 1e-12
        return
    u_two = complete_third_row(latgen.round_to_f32(u))
    got = host(ovl.sign_force(g, p, dev(chi, torch.complex64), dev(psi, torch.complex64)))
    ref = oforce.sign_force(u_two, latgen.round_to_f32(chi), latgen.round_to_f32(psi), alpha, LMAX)
    assert rel_err(got, ref) < 1e-6


# more than 16 right-hand sides run in groups of four in the workgroup order (the last group
# ragged for 17 and 19); every launch form that takes right-hand-side blocks
_GROUP_FORMS = [(16, 0, 1), (16, 0, 2), (64, 0, 4), (64, 1, 1), (8, 0, 1)]


@pytest.mark.parametrize("nrhs", [17, 19, 24])
@pytest.mark.parametrize("spb,tiles,rb", _GROUP_FORMS)
@pytest.mark.parametrize("store,cdt,tol", [("f64", torch.complex128, 1e-13),
                                           ("f32", torch.complex64, 1e-6)])
def test_kernel_many_rhs_groups(ovl, tmp_path, nrhs, spb, tiles, rb, store, cdt, tol):
    """K on 17 to 24 right-hand sides (workgroups in right-hand-side groups) in a forced launch
    form, every right-hand side against the oracle."""
    dims = (6, 4, 4, 6)
    prec = {"f64": 0, "f32": 1}[store]
    cache = tmp_path / "groups.txt"
    cache.write_text(f"B {prec} 0 1 {' '.join(map(str, dims))} {nrhs} {spb} {tiles} 1 {rb} 0\n")
    assert ovl.autotune_load(str(cache)) == 1
    u = latgen.random_su3_field(dims, 10190, noise=0.5)
    psi = latgen.gaussian_spinor(dims, 20190, nrhs=nrhs)
    g = ovl.GaugeField(dev(u), store)
    assert ovl.batch_launch_config((g, dev(psi, cdt))) == (spb, tiles, 1, rb)
    got = host(ovl.kernel_apply(g, dev(psi, cdt)))
    u_r = u if store == "f64" else latgen.round_to_f32(u)
    for r in range(nrhs):
        psi_r = psi[r] if store == "f64" else latgen.round_to_f32(psi[r])
        assert max_rel(got[r], ow.kop(u_r, psi_r)) < tol, r


@pytest.mark.parametrize("nrhs", [17, 19])
def test_sign_many_rhs_groups_norms(ovl, nrhs):
    """The deflated sign function on 17 and 19 right-hand sides in one call: outputs against the
    oracle and the FP64 norm partials of the final step (indexed by site block and right-hand
    side) consistent with the bound (no flag raised)."""
    dims = (4, 4, 2, 4)
    u = latgen.smeared_field(dims, 10191, steps=1)
    psi = latgen.gaussian_spinor(dims, 20191, nrhs=nrhs)
    phi, lam = random_basis(dims, 3, 20192)
    alpha = och.coeffs_sign_interp(21, 0.1)
    g = ovl.GaugeField(dev(u), "f64")
    p = ovl.Polynomial(alpha, LMAX)
    d = ovl.Deflation(dev(phi), lam, "f64")
    got = host(ovl.sign_apply(g, p, dev(psi), defl=d))
    for r in range(nrhs):
        assert rel_err(got[r], och.sign_apply(u, psi[r], alpha, LMAX, phi, lam)) < 1e-12, r
    assert g.flags() == 0
