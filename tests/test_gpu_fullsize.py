"""Parity at the full sizes of the measured workloads, in the launch configurations the benchmark
times.  The batched workload also runs at its full degree, with the lattices the oracle evaluates
in seconds compared element by element.  Elsewhere the oracle cannot run the benchmark's
Chebyshev degrees at these volumes in a test, so the polynomial degree is lowered: every launch is the same kernel in the same configuration as in the
benchmark (the degree only sets how many steps run), and every output element is compared with
the FP64 oracle on the same rounded inputs."""
import json
import os

import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import deflation as odefl
from oracle import force as oforce
from tests.conftest import complete_third_row, rel_err

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

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


def test_bf16_links_24_modes_16x16x16x32(ovl):
    """16^3x32 stout-smeared links stored in BF16, FP32 spinors, 24 deflated vectors through the
    FP32 matrix-core projection; degree 9 instead of 399."""
    dims = (16, 16, 16, 32)
    u = latgen.smeared_field(dims, latgen.seed_for("gauge", 3))
    psi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 3))
    phi = odefl.cgs2(latgen.gaussian_spinor(dims, 30301, nrhs=24))
    lam = np.linspace(-0.5, 0.5, 24) + 0.004
    lmax = LMAX * (1 + 2.0 ** -6)
    alpha = och.coeffs_sign_interp(9, 0.08)
    g = ovl.GaugeField(dev(u), "bf16")
    p = ovl.Polynomial(alpha, lmax)
    d = ovl.Deflation(dev(phi), lam, "f32")
    got = host(ovl.sign_apply(g, p, dev(psi, torch.complex64), defl=d))
    ref = och.sign_apply(latgen.round_to_bf16(u), latgen.round_to_f32(psi), alpha, lmax,
                         latgen.round_to_f32(phi), lam)
    assert rel_err(got, ref) < 1e-6
    assert g.flags() == 0


def test_batched_mixed_volumes_full_size(ovl):
    """12 point sources on 16^3x32 with 4 x 8^3x16 and 2 x 12^3x24 in one launch per step, FP32;
    degree 3 instead of 299."""
    alpha = och.coeffs_sign_interp(3, 0.05)
    p = ovl.Polynomial(alpha, LMAX)
    shapes = [((16, 16, 16, 32), 12)] + [((8, 8, 8, 16), 1)] * 4 + [((12, 12, 12, 24), 1)] * 2
    fields, probs = [], []
    for i, (dims, nrhs) in enumerate(shapes):
        u = latgen.random_su3_field(dims, latgen.seed_for("gauge", 4, i))
        if nrhs == 12:
            src = np.stack([latgen.point_source(dims, s, c) for s in range(4) for c in range(3)])
        else:
            src = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 4, i), nrhs=1)
        fields.append((u, src))
        probs.append((ovl.GaugeField(dev(u), "f32"), dev(src, torch.complex64)))
    outs = ovl.batch_sign_apply(p, probs)
    for (u, src), out in zip(fields, outs):
        got = host(out)
        u_r, s_r = latgen.round_to_f32(u), latgen.round_to_f32(src)
        for r in range(src.shape[0]):
            assert rel_err(got[r], och.sign_apply(u_r, s_r[r], alpha, LMAX)) < 1e-6


def test_batched_full_degree_sampled(ovl):
    """The batched workload as the benchmark runs it -- stout-smeared fields, two-row link reads,
    the tuned launch configuration, degree 300 (299 K applications) -- with the 8^3x16 and 12^3x24
    outputs (sampled lattices the oracle evaluates in seconds) compared element by element with
    the oracle on the same rounded inputs; the 16^3x32 sources are checked for finiteness and
    against the single-problem launch."""
    alpha = och.coeffs_sign_interp(300, 0.05)
    p = ovl.Polynomial(alpha, LMAX)
    shapes = [((16, 16, 16, 32), 12)] + [((8, 8, 8, 16), 1)] * 4 + [((12, 12, 12, 24), 1)] * 2
    fields, probs = [], []
    for i, (dims, nrhs) in enumerate(shapes):
        u = latgen.smeared_field(dims, latgen.seed_for("gauge", 4, i))
        if nrhs == 12:
            src = np.stack([latgen.point_source(dims, s, c) for s in range(4) for c in range(3)])
        else:
            src = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 4, i), nrhs=1)
        g = ovl.GaugeField(dev(u), "f32")
        g.reconstruct()
        fields.append((u, src))
        probs.append((g, dev(src, torch.complex64)))
    outs = [torch.empty_like(x) for _, x in probs]
    ovl.autotune(probs, p, outs=outs)
    print(f"batch launch configuration {ovl.batch_launch_config(probs)}", flush=True)
    outs = ovl.batch_sign_apply(p, probs, outs)
    for item in (1, 5):
        u, src = fields[item]
        ref = och.poly_apply(complete_third_row(latgen.round_to_f32(u)),
                             latgen.round_to_f32(src[0]), alpha, LMAX)
        assert rel_err(host(outs[item])[0], ref) < 1e-6
    got0 = host(outs[0])
    assert np.isfinite(got0).all()
    single = host(ovl.sign_apply(probs[0][0], p, probs[0][1]))
    assert rel_err(got0, single) < 1e-6
    for g, _ in probs:
        assert g.flags() == 0


def test_force_24x24x24x48(ovl):
    """d Re<chi, p(X) psi>/dU on 24^3x48 in FP32 with the checkpointed reverse recurrence
    (stride ceil(sqrt 5) = 3: two segments, a partial one); degree 5 instead of 299."""
    dims = (24, 24, 24, 48)
    u = latgen.random_su3_field(dims, latgen.seed_for("gauge", 5))
    psi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 5))
    chi = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 5, 1))
    alpha = och.coeffs_sign_interp(5, 0.05)
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, LMAX)
    got = host(ovl.sign_force(g, p, dev(chi, torch.complex64), dev(psi, torch.complex64)))
    ref = oforce.sign_force(latgen.round_to_f32(u), latgen.round_to_f32(chi),
                            latgen.round_to_f32(psi), alpha, LMAX)
    assert rel_err(got, ref) < 1e-6


def test_force_24x24x24x48_full_degree_directional(ovl):
    """The force workload as the benchmark runs it -- 24^3x48 stout-smeared links, FP32, degree 299,
    checkpoint stride 18 -- projected on seeded Gaussian directions Y: Re sum tr(G^+ Y) against
    the oracle's forward-mode derivative along Y (tests/golden/force_directional_24x24x24x48.json,
    written by make_force_directional.py from oracle/ only), on the same FP32-rounded inputs and
    on the exact ones."""
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "force_directional_24x24x24x48.json")))
    dims = tuple(ref["dims"])
    u = latgen.smeared_field(dims, ref["seeds"]["gauge"])
    psi = latgen.gaussian_spinor(dims, ref["seeds"]["psi"])
    chi = latgen.gaussian_spinor(dims, ref["seeds"]["chi"])
    alpha = och.coeffs_sign_interp(ref["degree"], ref["eps"])
    g = ovl.GaugeField(dev(u), "f32")
    p = ovl.Polynomial(alpha, ref["lmax"])
    G = host(ovl.sign_force(g, p, dev(chi, torch.complex64), dev(psi, torch.complex64),
                            ckpt_stride=18))
    for k, seed in enumerate(ref["direction_seeds"]):
        rng = np.random.Generator(np.random.PCG64(seed))
        y = rng.standard_normal(G.shape) + 1j * rng.standard_normal(G.shape)
        dl = float(np.real(np.vdot(G, y)))
        same, exact = ref["values"]["f32_rounded"][k], ref["values"]["exact"][k]
        print(f"direction {seed}: device {dl:.9e}, oracle (rounded inputs) {same:.9e}, "
              f"(exact inputs) {exact:.9e}", flush=True)
        assert abs(dl - same) < 1e-6 * abs(same)
        assert abs(dl - exact) < 1e-6 * abs(exact)
