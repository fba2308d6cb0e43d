#!/usr/bin/env python3
"""Benchmark of the overlap-operator hot path on one MI355X.

Headline workload (one "step"): the Chebyshev sign function of Cundy & Lee, Sec. 2, eq. 3,
sign(K) psi ~ sum_m alpha_m T_m(K/lmax) psi with K = gamma5 (D_W - m_W), m_W = 1.5, of degree 300
(N = 299 fused stencil + Clenshaw kernels, eps = 0.05), applied to a batch of lattice problems in
one kernel launch per K application: 12 spin-colour point sources on a 16^3x32 lattice plus
4 x 8^3x16 and 2 x 12^3x24 lattices with one Gaussian source each, every lattice with its own
synthetic near-unit SU(3) field smeared by 3 plain stout steps (rho = 0.1).  FP32 storage and
arithmetic, two-row link reads (the third row of each SU(3) link completed in registers), the
launch configuration chosen by the library's autotuner for this problem set.  `value` is
right-hand-side sign(K) psi applications per second.  Beside it: the same batch with full link
reads, in the default configuration, unbatched, and in plain FP64; the BF16-link 16^3x32 form with
24 deflated modes; the FP32 force on 24^3x48 smeared links; the deflated overlap operator on
8^3x16; K and sign(K) psi at 24^3x48; device-memory stream ceilings; the FP64 oracle's errors on
every form and its time on the host cores.

Prints ONE JSON line.  `python bench.py --gpus N --steps K --warmup W`.
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sign(K)psi applies/s + D_W HBM GB/s, mixed/batched vs FP64 plain at stated rel err"
HBM_PEAK_GBPS = 8000.0
LMAX = 6.5
LMAX_BF16 = LMAX * (1 + 2.0 ** -6)   # BF16 links are not unitary: margin on ||K||
# batched workload (lattice, right-hand sides); item 0 carries the 12 point sources
BATCH_SHAPES = [((16, 16, 16, 32), 12)] + [((8, 8, 8, 16), 1)] * 4 + [((12, 12, 12, 24), 1)] * 2
BATCH_DEGREE, BATCH_EPS = 300, 0.05
BF16_DIMS, BF16_DEGREE, BF16_NEV = (16, 16, 16, 32), 400, 24
FORCE_DIMS, FORCE_DEGREE, FORCE_EPS, FORCE_STRIDE = (24, 24, 24, 48), 300, 0.05, 18
OVL_DIMS, OVL_DEGREE, OVL_NEV, MUS = (8, 8, 8, 16), 200, 12, (0.01, 0.05)
# algorithmic bytes per site: each link, input and output read or written once
BYTES_LINK = {"f64": 576, "f32": 288, "bf16": 144}          # 4 x 3 x 3 complex
BYTES_LINK_R12 = {"f64": 384, "f32": 192, "bf16": 96}       # two rows read
BYTES_SPIN = {"f64": 192, "f32": 96, "bf16": 96}            # 12 complex (BF16: FP32 spinors)
STEP_STREAMS = 3.5   # Clenshaw step: b_{k+1}, b_{k+2}, b_k, and psi on odd k only
GOLDEN_FORCE = os.path.join(ROOT, "tests", "golden", "force_directional_24x24x24x48.json")


def step_bytes(store, r12=False):
    return (BYTES_LINK_R12 if r12 else BYTES_LINK)[store] + STEP_STREAMS * BYTES_SPIN[store]


def dw_bytes(store, r12=False):
    return (BYTES_LINK_R12 if r12 else BYTES_LINK)[store] + 2 * BYTES_SPIN[store]


def counter_traffic(tag, cfg=None):
    """HBM-side bytes per launch from the committed counter summary profiles/<tag>_counters.md
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy of known size), or None when the
    kernel sources changed after the counters were taken.  With cfg (a launch configuration), the
    summary's figure for that configuration, or None when it holds none."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{tag}_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    key = "traffic_bytes_per_launch" if cfg is None else \
        "traffic_bytes_per_launch[" + ",".join(str(int(c)) for c in cfg) + "]"
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in (key, "sources_sha256"):
            k, v = line.split(":", 1)
            fields["traffic_bytes_per_launch" if k == key else k] = v.strip()
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1510_06897_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    if fields.get("sources_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the FP64 oracle leg (CPU baseline and errors vs the oracle)")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the BF16/24-mode, force, overlap, 24^3x48 and "
                         "stream measurements")
    ap.add_argument("--config", default=None,
                    help="with --profile batch or bf16: run in this launch configuration "
                         "(spb,order,remap,rb) instead of the autotuned one")
    ap.add_argument("--profile", choices=["batch", "bf16", "force", "stout", "overlap", "dw", "dw2", "proj",
                                          "copy"],
                    help="run one part only, for rocprofv3: batch = the timed batched loop of the "
                         "headline (--steps batches), bf16 = the BF16 24-mode loop, force = the "
                         "FP32 force at 24^3x48, overlap = the FP32 overlap loop, dw = K at 24^3x48 "
                         "in FP64/FP32/BF16 (dw2: two-row link reads), proj = the FP32 "
                         "matrix-core projection at 16^3x32 with 24 vectors, copy = two plain "
                         "256 MiB device copies (scale of the byte counters)")
    return ap.parse_args()


def gpu_ms(torch, fn, reps, warmup=1):
    """Average milliseconds of fn() on the current stream (HIP events)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ------------------------------------------------------------------------------------------------
# inputs (host, seeded)
_FIELDS = {}


def batch_inputs(latgen):
    """[(dims, links, sources)] of the batched workload (cached)."""
    if "batch" not in _FIELDS:
        out = []
        for i, (dims, nrhs) in enumerate(BATCH_SHAPES):
            u = latgen.smeared_field(dims, latgen.seed_for("gauge", 4, i))
            if nrhs == 12:
                src = np.stack([latgen.point_source(dims, s, c) for s in range(4) for c in range(3)])
            else:
                src = latgen.gaussian_spinor(dims, latgen.seed_for("spinor", 4, i), nrhs=1)
            out.append((dims, u, src))
        _FIELDS["batch"] = out
    return _FIELDS["batch"]


def force_inputs(latgen):
    """Links, psi, chi of the force workload: the seeds of the stored oracle derivatives."""
    if "force" not in _FIELDS:
        u = latgen.smeared_field(FORCE_DIMS, latgen.seed_for("gauge", 5))
        psi = latgen.gaussian_spinor(FORCE_DIMS, latgen.seed_for("spinor", 5))
        chi = latgen.gaussian_spinor(FORCE_DIMS, latgen.seed_for("spinor", 5, 1))
        _FIELDS["force"] = (u, psi, chi)
    return _FIELDS["force"]


# ------------------------------------------------------------------------------------------------
# headline: the batched sign function
def batch_handles(ovl, torch, dev, latgen, store, two_row):
    probs = []
    cdt = torch.complex128 if store == "f64" else torch.complex64
    for dims, u, src in batch_inputs(latgen):
        g = ovl.GaugeField(torch.from_numpy(u).to(dev), store)
        if two_row:
            g.reconstruct()
        probs.append((g, torch.from_numpy(src).to(dev).to(cdt)))
    return probs


def batch_bytes_per_step(store, two_row):
    link = (BYTES_LINK_R12 if two_row else BYTES_LINK)[store]
    total = 0.0
    for dims, nrhs in BATCH_SHAPES:
        v = int(np.prod(dims))
        total += v * (link + nrhs * STEP_STREAMS * BYTES_SPIN[store])
    return total


def kernel_name(cfg, store, two_row, table=True):
    spb, order, remap, rb = cfg
    c, se, le = {"f64": ("double", "double2", "double2"), "f32": ("float", "float2", "float2"),
                 "bf16": ("float", "float2", "bf16c")}[store]
    if order == 2:
        return f"step_slab_kernel<{c},{se},{le},NW={spb // 64},TABLE={int(table)},R12={int(two_row)}>"
    if spb == 128:
        return f"step2_kernel<{le},64,TABLE={int(table)},R12={int(two_row)}>"
    nq = 8 if spb == 8 else 4
    return (f"step_kernel<{c},{se},{le},SPB={spb},TABLE={int(table)},NQ={nq},"
            f"R12={int(two_row)},RB={rb}>")


def measure_batch(ovl, torch, dev, latgen, steps, warmup, profile=False, force_cfg=None):
    t0 = time.time()
    alpha = ovl.cheb_sign_coeffs(BATCH_DEGREE, BATCH_EPS)
    p32 = ovl.Polynomial(alpha, LMAX)
    probs = batch_handles(ovl, torch, dev, latgen, "f32", two_row=True)
    outs = [torch.empty_like(x) for _, x in probs]
    n_rhs = sum(nrhs for _, nrhs in BATCH_SHAPES)
    log(f"batch inputs {time.time() - t0:.1f} s")
    res = {}
    if not profile:
        cfg_default = ovl.batch_launch_config(probs)
        ms_default = gpu_ms(torch, lambda: ovl.batch_sign_apply(p32, probs, outs), 3)
        res["default_config"] = {"config": list(cfg_default), "ms_per_batch": round(ms_default, 3)}
    if profile and force_cfg:
        # a profiled run in a given configuration (counters per configuration)
        cache = os.path.join(tempfile.gettempdir(), f"ovl_batch_cfg_{os.getpid()}.txt")
        items = " ".join(f"{d[0]} {d[1]} {d[2]} {d[3]} {n}" for d, n in BATCH_SHAPES)
        with open(cache, "w") as f:
            f.write(f"B 1 1 {len(BATCH_SHAPES)} {items} {' '.join(map(str, force_cfg))} 0\n")
        ovl.autotune_load(cache)
        os.remove(cache)
        us_tune = float("nan")
    else:
        us_tune = ovl.autotune(probs, p32, outs=outs)
    cfg = ovl.batch_launch_config(probs)
    log(f"batch autotuned {cfg} ({us_tune:.1f} us per step in the tuner)")
    # the timed loop: warm-up, then exactly `steps` batches, with the library's event pair around
    # the consecutive plain steps of every evaluation (the dominant kernel's average duration)
    for _ in range(warmup):
        ovl.batch_sign_apply(p32, probs, outs)
    torch.cuda.synchronize()
    ovl.timing_read(0)
    ovl.timing_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ovl.batch_sign_apply(p32, probs, outs)
    e1.record()
    torch.cuda.synchronize()
    ovl.timing_enable(False)
    k_ms, k_n = ovl.timing_read(0)
    ms = e0.elapsed_time(e1) / steps
    log(f"batch FP32 two-row: {ms:.3f} ms/batch, step kernel {1e3 * k_ms / k_n:.2f} us")
    if profile:
        return None
    for g, _ in probs:
        assert g.flags() == 0
    res.update({"config": list(cfg), "ms_per_batch": ms, "kernel_ms": k_ms, "kernel_launches": k_n,
                "tuner_us_per_step": round(us_tune, 2), "n_rhs": n_rhs})
    res["speedup_tuned_vs_default"] = round(res["default_config"]["ms_per_batch"] / ms, 3)
    del probs
    # full link reads (tuned for that form), unbatched FP32 and plain FP64
    probs_f = batch_handles(ovl, torch, dev, latgen, "f32", two_row=False)
    ovl.autotune(probs_f, p32, outs=outs)
    ms_full = gpu_ms(torch, lambda: ovl.batch_sign_apply(p32, probs_f, outs), 5)
    res["full_link_reads"] = {"config": list(ovl.batch_launch_config(probs_f)),
                              "ms_per_batch": round(ms_full, 3),
                              "rhs_applies_per_s": round(n_rhs * 1e3 / ms_full, 2)}
    ms_u = gpu_ms(torch, lambda: [ovl.sign_apply(g, p32, x, out=o)
                                  for (g, x), o in zip(probs_f, outs)], 3)
    del probs_f
    probs64 = batch_handles(ovl, torch, dev, latgen, "f64", two_row=False)
    outs64 = [torch.empty_like(x) for _, x in probs64]
    ms_64 = gpu_ms(torch, lambda: [ovl.sign_apply(g, p32, x, out=o)
                                   for (g, x), o in zip(probs64, outs64)], 2)
    del probs64, outs64
    res["unbatched_f32_ms"] = round(ms_u, 3)
    res["plain_f64_ms"] = round(ms_64, 3)
    res["speedup_vs_unbatched_f32"] = round(ms_u / ms, 3)
    res["speedup_vs_plain_f64"] = round(ms_64 / ms, 3)
    log(f"batch: full reads {ms_full:.2f} ms, unbatched {ms_u:.2f} ms, plain FP64 {ms_64:.2f} ms")
    return res


# ------------------------------------------------------------------------------------------------
def measure_bf16(ovl, torch, dev, latgen, low_modes, reps, profile=False, force_cfg=None):
    """BF16 links, FP32 spinors/accumulation, FP64 reductions, degree 400 (N = 399), 24 deflated
    modes found on the device, FP32 matrix-core projection."""
    t0 = time.time()
    u = latgen.smeared_field(BF16_DIMS, latgen.seed_for("gauge", 3))
    psi = latgen.gaussian_spinor(BF16_DIMS, latgen.seed_for("spinor", 3))
    du = torch.from_numpy(u).to(dev)
    g64 = ovl.GaugeField(du, "f64")
    gbf = ovl.GaugeField(du, "bf16")
    # a 128-vector block holds the 48-mode doubler cluster around the 24th eigenvalue whole
    t1 = time.time()
    lam, phi, res_e, eps = low_modes(g64, BF16_NEV, LMAX, block=128, cut=1.0)
    t_eig = time.time() - t1
    alpha = ovl.cheb_sign_coeffs(BF16_DEGREE, eps)
    pbf = ovl.Polynomial(alpha, LMAX_BF16)
    dbf = ovl.Deflation(phi, lam, "f32")
    x32 = torch.from_numpy(psi).to(dev).to(torch.complex64)
    y32 = torch.empty_like(x32)
    log(f"BF16/24-mode set-up {time.time() - t0:.1f} s (eigen-solve {t_eig:.1f} s, residual {res_e.max():.1e})")
    if profile:
        if force_cfg:
            # a profiled run in a given configuration (counters per configuration)
            cache = os.path.join(tempfile.gettempdir(), f"ovl_bf16_cfg_{os.getpid()}.txt")
            with open(cache, "w") as f:
                f.write(f"B 2 0 1 {' '.join(map(str, BF16_DIMS))} 1 {' '.join(map(str, force_cfg))} 0\n")
            ovl.autotune_load(cache)
            os.remove(cache)
        else:
            ovl.autotune((gbf, x32), pbf, outs=[y32])
        log(f"bf16 configuration {ovl.batch_launch_config((gbf, x32))}")
        for _ in range(reps):
            ovl.sign_apply(gbf, pbf, x32, defl=dbf, out=y32)
        torch.cuda.synchronize()
        return None
    cfg_default = ovl.batch_launch_config((gbf, x32))
    ovl.autotune((gbf, x32), pbf, outs=[y32])
    cfg = ovl.batch_launch_config((gbf, x32))
    ovl.sign_apply(gbf, pbf, x32, defl=dbf, out=y32)
    torch.cuda.synchronize()
    ovl.timing_read(0)
    ovl.timing_enable(True)
    ms_bf = gpu_ms(torch, lambda: ovl.sign_apply(gbf, pbf, x32, defl=dbf, out=y32), reps, warmup=0)
    ovl.timing_enable(False)
    k_ms, k_n = ovl.timing_read(0)
    d64 = ovl.Deflation(phi, lam, "f64")
    p64 = ovl.Polynomial(alpha, LMAX_BF16)
    x64 = torch.from_numpy(psi).to(dev)
    y64 = torch.empty_like(x64)
    ms_64 = gpu_ms(torch, lambda: ovl.sign_apply(g64, p64, x64, defl=d64, out=y64), 3)
    gbf.reconstruct()
    ms_r12 = gpu_ms(torch, lambda: ovl.sign_apply(gbf, pbf, x32, defl=dbf, out=y32), reps)
    ms_proj = gpu_ms(torch, lambda: ovl.defl_project(dbf, x32), 20)
    assert gbf.flags() == 0
    vol = int(np.prod(BF16_DIMS))
    proj_flops = 8.0 * BF16_NEV * 12 * vol    # complex multiply-add = 8 real flops
    out = {"ms_per_apply": ms_bf, "kernel_ms": k_ms, "kernel_launches": k_n,
           "config": list(cfg), "default_config": list(cfg_default),
           "plain_f64_ms_per_apply": round(ms_64, 3),
           "speedup_vs_plain_f64": round(ms_64 / ms_bf, 3),
           "two_row_links_ms_per_apply": round(ms_r12, 3),
           "eps": round(float(eps), 5), "lmax": LMAX_BF16, "degree": len(alpha) - 1,
           "eigen_solve_s": round(t_eig, 1), "eigen_residual_max": float(res_e.max()),
           "projection_us": round(ms_proj * 1e3, 2),
           "projection_mfma_TFLOPs": round(proj_flops / (ms_proj * 1e-3) / 1e12, 3),
           "projection_frac_of_fp32_matrix_peak": round(proj_flops / (ms_proj * 1e-3) / 157.3e12, 5),
           "projection_GBps": round(BF16_NEV * 12 * vol * 8 / (ms_proj * 1e-3) / 1e9, 1)}
    log(f"BF16 24 modes: {ms_bf:.2f} ms/apply (two-row {ms_r12:.2f}), FP64 {ms_64:.2f} ms")
    _FIELDS["bf16"] = (u, psi, float(eps))
    return out


# ------------------------------------------------------------------------------------------------
def measure_force(ovl, torch, dev, latgen, reps, profile=False):
    t0 = time.time()
    u, psi, chi = force_inputs(latgen)
    g32 = ovl.GaugeField(torch.from_numpy(u).to(dev), "f32")
    pf = ovl.Polynomial(ovl.cheb_sign_coeffs(FORCE_DEGREE, FORCE_EPS), LMAX)
    G = torch.empty((4, 3, 3) + tuple(psi.shape[-4:]), dtype=torch.complex64, device=dev)
    x32 = torch.from_numpy(psi).to(dev).to(torch.complex64)
    c32 = torch.from_numpy(chi).to(dev).to(torch.complex64)
    log(f"force inputs {time.time() - t0:.1f} s")
    # the stencil steps of the force are single-problem launches on this lattice: tune them
    ovl.autotune((g32, x32), pf, outs=[torch.empty_like(x32)])
    step_cfg = ovl.batch_launch_config((g32, x32))
    # the twin steps (checkpoint recomputation beside the reverse sweep) launch as a
    # two-right-hand-side problem on the same lattice
    x2 = x32.reshape((1,) + tuple(x32.shape[-6:])).expand((2,) + tuple(x32.shape[-6:])).contiguous()
    twin_cfg = ovl.batch_launch_config((g32, x2))
    del x2
    if profile:
        for _ in range(reps):
            ovl.sign_force(g32, pf, c32, x32, ckpt_stride=FORCE_STRIDE, out=G)
        torch.cuda.synchronize()
        return None
    ovl.sign_force(g32, pf, c32, x32, ckpt_stride=FORCE_STRIDE, out=G)
    torch.cuda.synchronize()
    ovl.timing_read(1)
    ovl.timing_enable(True)
    ms_f = gpu_ms(torch, lambda: ovl.sign_force(g32, pf, c32, x32, ckpt_stride=FORCE_STRIDE, out=G),
                  reps, warmup=0)
    ovl.timing_enable(False)
    v_ms, v_n = ovl.timing_read(1)
    # one segment: every t_m regenerated into HBM once (N vectors) instead of sqrt(N) checkpoints
    ms_all = gpu_ms(torch, lambda: ovl.sign_force(g32, pf, c32, x32, ckpt_stride=FORCE_DEGREE,
                                                  out=G), 1)
    g32.reconstruct()
    ms_r12 = gpu_ms(torch, lambda: ovl.sign_force(g32, pf, c32, x32, ckpt_stride=FORCE_STRIDE,
                                                  out=G), reps)
    # the HMC chain on thin links (Sec. 1; Sec. 2: 3 steps of over-improved stout smearing,
    # rho 0.1, eps -0.25): smear on the device, force on the smeared links, chain rule back
    u_thin = torch.from_numpy(latgen.random_su3_field(FORCE_DIMS, latgen.seed_for("gauge", 5))).to(dev)
    us = torch.empty_like(u_thin)
    ms_smear = gpu_ms(torch, lambda: ovl.stout_smear(u_thin, 0.1, -0.25, 3, out=us), 2)
    g_s = ovl.GaugeField(us, "f32")
    ms_fs = gpu_ms(torch, lambda: ovl.sign_force(g_s, pf, c32, x32, ckpt_stride=FORCE_STRIDE, out=G), 1)
    g64 = G.to(torch.complex128)
    gt = torch.empty_like(u_thin)
    ms_back = gpu_ms(torch, lambda: ovl.stout_backward(u_thin, g64, 0.1, -0.25, 3, out=gt), 2)
    assert torch.isfinite(torch.view_as_real(gt)).all()
    del u_thin, us, g_s, g64, gt
    chain = {"stout_smear_3_steps_ms": round(ms_smear, 2), "force_on_smeared_links_ms": round(ms_fs, 2),
             "stout_chain_rule_3_steps_ms": round(ms_back, 2),
             "thin_link_force_ms": round(ms_smear + ms_fs + ms_back, 2),
             "smearing": "over-improved stout, rho 0.1, eps -0.25, 3 steps (FP64 on the device)"}
    log(f"force chain on thin links: smear {ms_smear:.1f} ms, force {ms_fs:.1f} ms, chain rule "
        f"{ms_back:.1f} ms")
    # bytes of the link-VJP launches: every pair reads a and t once (FP32 spinors), the FP64
    # running sum of G is written by the first segment, read and written by the middle ones and
    # read by the last, which writes G in FP32
    vol = int(np.prod(FORCE_DIMS))
    n = FORCE_DEGREE - 1
    nseg = (n + FORCE_STRIDE - 1) // FORCE_STRIDE
    vjp_bytes = vol * (n * 2 * BYTES_SPIN["f32"] + (nseg - 1) * 2 * 36 * 16 + 36 * 8)
    out = {"ms_per_force": ms_f, "forces_per_s": round(1e3 / ms_f, 3),
           "stencil_step_config": list(step_cfg), "twin_step_config": list(twin_cfg),
           "ms_per_force_stride_299": round(ms_all, 2),
           "ms_per_force_two_row_links": round(ms_r12, 2),
           "vjp_ms": v_ms, "vjp_launches": v_n, "vjp_launches_per_force": v_n // reps,
           "vjp_bytes_per_force": vjp_bytes, "hmc_chain_thin_links": chain}
    log(f"force 24^3x48: {ms_f:.1f} ms (link VJP {v_ms / reps:.1f} ms of it; "
        f"two-row {ms_r12:.1f}, stride 299 {ms_all:.1f})")
    return out


# ------------------------------------------------------------------------------------------------
def measure_overlap(ovl, torch, dev, latgen, low_modes, reps, profile=False):
    t0 = time.time()
    u = latgen.smeared_field(OVL_DIMS, latgen.seed_for("gauge", 2))
    psi = latgen.gaussian_spinor(OVL_DIMS, latgen.seed_for("spinor", 2))
    d_u = torch.from_numpy(u).to(dev)
    g64 = ovl.GaugeField(d_u, "f64")
    g32 = ovl.GaugeField(d_u, "f32")
    # the smooth synthetic fields keep K close to its free spectrum: 48 near-degenerate doubler
    # modes at |lambda| ~ 0.5, so the filtered block (64) must hold that whole cluster
    lam, phi, res_e, eps = low_modes(g64, OVL_NEV, LMAX, block=64, cut=1.0)
    alpha = ovl.cheb_sign_coeffs(OVL_DEGREE, eps)
    poly = ovl.Polynomial(alpha, LMAX)
    defl64 = ovl.Deflation(phi, lam, "f64")
    defl32 = ovl.Deflation(phi, lam, "f32")
    psi64 = torch.from_numpy(psi).to(dev)
    psi32 = psi64.to(torch.complex64)
    out64 = torch.empty_like(psi64)
    out32 = torch.empty_like(psi32)
    log(f"overlap 8^3x16 set-up {time.time() - t0:.1f} s (eps {eps:.4f})")

    def step(form, i):
        mu = MUS[i % 2]
        if form == "f32":
            ovl.overlap_apply(g32, poly, psi32, mu, defl=defl32, out=out32)
        else:
            ovl.overlap_apply(g64, poly, psi64, mu, defl=defl64, out=out64)

    for i in range(3):
        step("f32", i)
        step("f64", i)
    torch.cuda.synchronize()
    if profile:
        for i in range(reps):
            step("f32", i)
        torch.cuda.synchronize()
        return None
    ms32 = gpu_ms(torch, lambda: [step("f32", i) for i in range(reps)], 1, warmup=0) / reps
    ms64 = gpu_ms(torch, lambda: [step("f64", i) for i in range(reps)], 1, warmup=0) / reps
    psi12 = torch.from_numpy(latgen.gaussian_spinor(OVL_DIMS, latgen.seed_for("spinor", 2, 1),
                                                    nrhs=12)).to(dev).to(torch.complex64)
    out12 = torch.empty_like(psi12)
    ms12 = gpu_ms(torch, lambda: ovl.overlap_apply(g32, poly, psi12, MUS[0], defl=defl32,
                                                   out=out12), 5)
    solves = {}
    for label, gi, di in (("cg_f64", None, None), ("cg_f32_inner", g32, defl32)):
        torch.cuda.synchronize()
        t0s = time.perf_counter()
        _, its, sres = ovl.overlap_solve(g64, poly, psi64, MUS[1], defl=defl64, g_inner=gi,
                                         defl_inner=di, tol=1e-13)
        torch.cuda.synchronize()
        solves[label] = {"s": round(time.perf_counter() - t0s, 4), "cg_iterations": its,
                         "rel_residual": sres}
    # the paper's solver form: GMRESR around FP32 inner CG on a truncated polynomial, relaxed
    # FP64 outer products (Sec. 2), to the paper's overlap accuracy 1e-13 (Sec. 3)
    for label, relax in (("gmresr_f32_inner_relaxed", True), ("gmresr_f32_inner", False)):
        torch.cuda.synchronize()
        t0s = time.perf_counter()
        _, n_out, n_in, sres = ovl.overlap_solve_gmresr(g64, poly, psi64, MUS[1], defl=defl64,
                                                        g_inner=g32, defl_inner=defl32, tol=1e-13,
                                                        relax=relax)
        torch.cuda.synchronize()
        solves[label] = {"s": round(time.perf_counter() - t0s, 4), "outer_steps": n_out,
                         "inner_cg_iterations": n_in, "rel_residual": sres}
    assert g32.flags() == 0 and g64.flags() == 0
    log(f"overlap 8^3x16: FP32 {ms32:.3f} ms, FP64 {ms64:.3f} ms, 12 sources {ms12:.3f} ms")
    _FIELDS["overlap"] = (u, psi, float(eps))
    return {"ms_per_apply_f32": round(ms32, 4), "ms_per_apply_f64": round(ms64, 4),
            "applies_per_s_f32": round(1e3 / ms32, 1), "applies_per_s_f64": round(1e3 / ms64, 1),
            "speedup_f32_over_f64": round(ms64 / ms32, 3),
            "twelve_sources_ms_per_call": round(ms12, 4),
            "twelve_sources_rhs_applies_per_s": round(12e3 / ms12, 1),
            "eps": round(float(eps), 5), "degree": len(alpha) - 1,
            "eigen_residual_max": float(res_e.max()),
            "solve_mu0.05_to_1e-13": solves}


# ------------------------------------------------------------------------------------------------
def measure_big(ovl, torch, dev, latgen, profile=None, reps=50):
    """K and sign(K) psi at 24^3x48 (the force lattice; working set above the 256 MB Infinity
    Cache) in FP64, FP32 and BF16-link storage, full and two-row link reads."""
    u, psi, _ = force_inputs(latgen)
    d_u = torch.from_numpy(u).to(dev)
    d_p = torch.from_numpy(psi).to(dev)
    vol = int(np.prod(FORCE_DIMS))
    dw, sign_big = {}, {}
    p_big = ovl.Polynomial(ovl.cheb_sign_coeffs(OVL_DEGREE, 0.05), LMAX_BF16)
    for store in ("f64", "f32", "bf16"):
        gb = ovl.GaugeField(d_u, store)
        x = d_p if store == "f64" else d_p.to(torch.complex64)
        y = torch.empty_like(x)
        if profile in ("dw", "dw2"):
            if profile == "dw2":
                gb.reconstruct()
            for _ in range(reps):
                ovl.kernel_apply(gb, x, out=y)
            torch.cuda.synchronize()
            gb.close()
            continue
        row = {}
        for r12 in (False, True):
            if r12:
                gb.reconstruct()
            us = 1e3 * gpu_ms(torch, lambda: ovl.kernel_apply(gb, x, out=y), reps, warmup=3)
            gbps = dw_bytes(store, r12) * vol / (us * 1e-6) / 1e9
            ovl.sign_apply(gb, p_big, x, out=y)
            torch.cuda.synchronize()
            ovl.timing_read(0)
            ovl.timing_enable(True)
            ms = gpu_ms(torch, lambda: ovl.sign_apply(gb, p_big, x, out=y), 3, warmup=0)
            ovl.timing_enable(False)
            k_ms, k_n = ovl.timing_read(0)
            kus = 1e3 * k_ms / k_n
            sgbps = step_bytes(store, r12) * vol / (kus * 1e-6) / 1e9
            key = "two_row_links" if r12 else "full_links"
            row[key] = {"K_us_per_apply": round(us, 2), "K_GBps": round(gbps, 1),
                        "K_frac_of_8TBps": round(gbps / HBM_PEAK_GBPS, 4),
                        "K_bytes_per_site": dw_bytes(store, r12),
                        "sign_ms_per_apply": round(ms, 3), "step_kernel_us": round(kus, 2),
                        "step_GBps": round(sgbps, 1),
                        "step_frac_of_8TBps": round(sgbps / HBM_PEAK_GBPS, 4),
                        "step_bytes_per_site": step_bytes(store, r12)}
        dw[store] = row
        log(f"24^3x48 {store}: K {row['full_links']['K_us_per_apply']} us "
            f"(two-row {row['two_row_links']['K_us_per_apply']}), step "
            f"{row['full_links']['step_kernel_us']} us")
        gb.close()
    return dw


def measure_streams(ovl, torch, dev):
    """Plain device-memory streams of 4 GiB (read, copy, three-to-one) and torch's copy."""
    nb = 4 << 30
    src = torch.empty(3 * nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    sink = torch.empty(8 << 20, dtype=torch.uint8, device=dev)
    out = {}
    for kind, name, moved in ((0, "read", 1), (1, "copy", 2), (2, "three_to_one", 4)):
        d = sink if kind == 0 else dst
        ms = gpu_ms(torch, lambda: ovl.stream_probe(kind, d, src, nb), 5, warmup=2)
        out[name] = {"GBps": round(moved * nb / (ms * 1e-3) / 1e9, 1),
                     "frac_of_8TBps": round(moved * nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    a = src[: nb // 4]
    ms = gpu_ms(torch, lambda: dst.copy_(a), 5, warmup=2)
    out["torch_copy"] = {"GBps": round(2 * nb / (ms * 1e-3) / 1e9, 1)}
    log(f"streams 4 GiB: {out}")
    return out


# ------------------------------------------------------------------------------------------------
# FP64 oracle leg: errors of every form against the oracle (on the exact FP64 inputs and on the
# same rounded inputs) and the oracle's time on the host.  The oracle never receives anything the
# GPU computed: its inputs come from latgen and its own coefficient rule and Gram-Schmidt.
def _oracle_job(job):
    """One oracle evaluation in a worker process (single-threaded NumPy)."""
    from threadpoolctl import threadpool_limits
    from oracle import chebyshev as och
    from oracle import overlap as oov
    name, kind, args = job
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        if kind == "poly":
            u, psi, alpha, lmax = args
            y = och.poly_apply(u, psi, alpha, lmax)
        elif kind == "sign":
            u, psi, alpha, lmax, phi, lam = args
            y = och.sign_apply(u, psi, alpha, lmax, phi, lam)
        else:
            u, psi, mu, alpha, lmax, phi, lam = args
            y = oov.overlap_apply(u, psi, mu, alpha, lmax, phi, lam)
    return name, y, time.perf_counter() - t0


def oracle_leg(ovl, torch, dev, latgen, results, workers=8):
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import chebyshev as och
    from oracle import deflation as odefl
    r32, rbf = latgen.round_to_f32, latgen.round_to_bf16
    jobs, gpu = [], {}
    # the batched headline form (FP32, two-row links, tuned batch launch) with the oracle's
    # coefficients; sampled right-hand sides: point source 5 of the 16^3x32 lattice, the first
    # 8^3x16 and the first 12^3x24 lattice
    bat = batch_inputs(latgen)
    alpha4 = och.coeffs_sign_interp(BATCH_DEGREE, BATCH_EPS)
    p4 = ovl.Polynomial(alpha4, LMAX)
    probs = batch_handles(ovl, torch, dev, latgen, "f32", two_row=True)
    outs = ovl.batch_sign_apply(p4, probs)
    torch.cuda.synchronize()
    for item, r in ((0, 5), (1, 0), (5, 0)):
        dims, u, src = bat[item]
        name = f"batch_{'x'.join(map(str, dims))}_rhs{r}"
        gpu[name] = outs[item][r].cpu().to(torch.complex128).numpy()
        jobs.append((name + "|exact", "poly", (u, src[r], alpha4, LMAX)))
        jobs.append((name + "|same", "poly", (r32(u), r32(src[r]), alpha4, LMAX)))
    del probs, outs
    # BF16 links; a Gaussian basis orthonormalised by the oracle stands in for the low modes
    # (same cost), with fixed eigenvalues
    if "bf16" in _FIELDS:
        u, psi, eps = _FIELDS["bf16"]
        phi_o = odefl.cgs2(latgen.gaussian_spinor(BF16_DIMS, 30301, nrhs=BF16_NEV))
        lam_o = np.linspace(-0.5, 0.5, BF16_NEV) + 0.004
        alpha3 = och.coeffs_sign_interp(BF16_DEGREE, eps)
        gbf = ovl.GaugeField(torch.from_numpy(u).to(dev), "bf16")
        d3 = ovl.Deflation(torch.from_numpy(phi_o).to(dev), lam_o, "f32")
        p3 = ovl.Polynomial(alpha3, LMAX_BF16)
        gpu["bf16"] = ovl.sign_apply(gbf, p3, torch.from_numpy(psi).to(dev).to(torch.complex64),
                                   defl=d3).cpu().to(torch.complex128).numpy()
        jobs.append(("bf16|exact", "sign", (u, psi, alpha3, LMAX_BF16, phi_o, lam_o)))
        jobs.append(("bf16|same", "sign", (rbf(u), r32(psi), alpha3, LMAX_BF16, r32(phi_o), lam_o)))
        del gbf, d3
    # the deflated overlap operator on 8^3x16, FP32 and FP64
    if "overlap" in _FIELDS:
        u, psi, eps = _FIELDS["overlap"]
        phi_o = odefl.cgs2(latgen.gaussian_spinor(OVL_DIMS, 777, nrhs=OVL_NEV))
        lam_o = np.linspace(-0.52, 0.52, OVL_NEV) + 0.003
        alpha2 = och.coeffs_sign_interp(OVL_DEGREE, eps)
        p2 = ovl.Polynomial(alpha2, LMAX)
        du = torch.from_numpy(u).to(dev)
        dphi = torch.from_numpy(phi_o).to(dev)
        x = torch.from_numpy(psi).to(dev)
        for store in ("f32", "f64"):
            g = ovl.GaugeField(du, store)
            d = ovl.Deflation(dphi, lam_o, store)
            xs = x if store == "f64" else x.to(torch.complex64)
            gpu[f"overlap_{store}"] = ovl.overlap_apply(g, p2, xs, MUS[1], defl=d).cpu().to(
                torch.complex128).numpy()
        jobs.append(("overlap|exact", "overlap", (u, psi, MUS[1], alpha2, LMAX, phi_o, lam_o)))
        jobs.append(("overlap|same", "overlap", (r32(u), r32(psi), MUS[1], alpha2, LMAX, r32(phi_o),
                                            lam_o)))
    torch.cuda.synchronize()
    # CPU baseline: the oracle on a bounded sample of the headline batch, one thread, in this
    # process: full-degree applies on one 8^3x16 and one 12^3x24 source, and 60 of the 299
    # K applications on one 16^3x32 source (scaled linearly to 299)
    base = {}
    with threadpool_limits(limits=1):
        for item, nk in ((1, BATCH_DEGREE - 1), (5, BATCH_DEGREE - 1), (0, 60)):
            dims, u, src = bat[item]
            a = alpha4[: nk + 1]
            t0 = time.perf_counter()
            och.poly_apply(u, src[0], a, LMAX)
            base[item] = (time.perf_counter() - t0) * (BATCH_DEGREE - 1) / nk
    n_rhs = sum(nrhs for _, nrhs in BATCH_SHAPES)
    t_batch = 12 * base[0] + 4 * base[1] + 2 * base[5]
    sampled = sum(base[i] * (60 if i == 0 else BATCH_DEGREE - 1) / (BATCH_DEGREE - 1) for i in base)
    cpu = {"value": round(n_rhs / t_batch, 5), "unit": "sign(K)psi right-hand-side applies/s",
           "cores": 1, "kind": "oracle",
           "sample": f"FP64 NumPy oracle (forward Chebyshev recurrence), one thread: degree 299 on "
                     f"one 8^3x16 source ({base[1]:.1f} s) and one 12^3x24 source "
                     f"({base[5]:.1f} s), 60 of 299 steps on one 16^3x32 source (scaled: "
                     f"{base[0]:.1f} s); {sampled:.1f} s of CPU work; the batch of 18 sources "
                     f"extrapolated to {t_batch:.0f} s ({len(os.sched_getaffinity(0))} cores "
                     f"visible)"}
    log(f"oracle baseline: {cpu['sample']}")
    # the oracle evaluations for the errors, in parallel worker processes (spawned: they never
    # touch the GPU)
    t0 = time.time()
    with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
        done = pool.map(_oracle_job, jobs, chunksize=1)
    log(f"oracle leg: {len(jobs)} evaluations in {time.time() - t0:.0f} s")
    refs = {name: (y, sec) for name, y, sec in done}
    errs = {}
    for key in gpu:
        base_name = key if not key.startswith("overlap_") else "overlap"
        ex, same = refs[base_name + "|exact"][0], refs[base_name + "|same"][0]
        if key.endswith("_f64"):
            same = ex   # FP64 storage: the device sees the exact inputs
        errs[key] = {"vs_oracle_exact_inputs": rel(gpu[key], ex),
                     "vs_oracle_same_rounded_inputs": rel(gpu[key], same),
                     "oracle_s": round(refs[base_name + "|exact"][1], 1)}
    # the force: the stored oracle derivatives along seeded directions (tests/golden)
    if os.path.exists(GOLDEN_FORCE) and "force" in _FIELDS:
        ref = json.load(open(GOLDEN_FORCE))
        u, psi, chi = force_inputs(latgen)
        g32 = ovl.GaugeField(torch.from_numpy(u).to(dev), "f32")
        pf = ovl.Polynomial(och.coeffs_sign_interp(ref["degree"], ref["eps"]), ref["lmax"])
        G = ovl.sign_force(g32, pf, torch.from_numpy(chi).to(dev).to(torch.complex64),
                           torch.from_numpy(psi).to(dev).to(torch.complex64),
                           ckpt_stride=FORCE_STRIDE).cpu().to(torch.complex128).numpy()
        del g32
        e_ex, e_same = [], []
        for k, seed in enumerate(ref["direction_seeds"]):
            rng = np.random.Generator(np.random.PCG64(seed))
            y = rng.standard_normal(G.shape) + 1j * rng.standard_normal(G.shape)
            dl = float(np.real(np.vdot(G, y)))
            e_ex.append(abs(dl - ref["values"]["exact"][k]) / abs(ref["values"]["exact"][k]))
            e_same.append(abs(dl - ref["values"]["f32_rounded"][k])
                          / abs(ref["values"]["f32_rounded"][k]))
        errs["force"] = {"vs_oracle_exact_inputs": max(e_ex),
                            "vs_oracle_same_rounded_inputs": max(e_same),
                            "measure": "relative error of Re sum tr(G^+ Y) against the oracle's "
                                       "forward-mode derivative along seeded Gaussian directions "
                                       "Y (tests/golden/force_directional_24x24x24x48.json), "
                                       "max over directions"}
    for k, v in errs.items():
        log(f"error vs oracle {k}: exact inputs {v['vs_oracle_exact_inputs']:.2e}, same rounded "
            f"inputs {v['vs_oracle_same_rounded_inputs']:.2e}")
    return cpu, errs


# ------------------------------------------------------------------------------------------------
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import latgen
    import paper_1510_06897_amd as ovl
    from paper_1510_06897_amd.eigsolve import low_modes

    ovl.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile == "copy":
        # a plain device copy of known size: 256 MiB read + 256 MiB written per copy
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(2):
            ovl.stream_probe(1, b, a, 256 << 20)
        torch.cuda.synchronize()
        log("copied 256 MiB twice")
        return
    if args.profile == "batch":
        force_cfg = tuple(int(c) for c in args.config.split(",")) if args.config else None
        measure_batch(ovl, torch, dev, latgen, args.steps, args.warmup, profile=True,
                      force_cfg=force_cfg)
        return
    if args.profile == "bf16":
        force_cfg = tuple(int(c) for c in args.config.split(",")) if args.config else None
        measure_bf16(ovl, torch, dev, latgen, low_modes, args.steps, profile=True,
                     force_cfg=force_cfg)
        return
    if args.profile == "force":
        measure_force(ovl, torch, dev, latgen, args.steps, profile=True)
        return
    if args.profile == "stout":
        # the smearing and chain-rule kernels of the HMC chain on 24^3x48 thin links
        u_thin = torch.from_numpy(latgen.random_su3_field(FORCE_DIMS, latgen.seed_for("gauge", 5))).to(dev)
        us = torch.empty_like(u_thin)
        g_s = torch.from_numpy(latgen.gaussian_spinor(FORCE_DIMS, latgen.seed_for("spinor", 5), nrhs=3)
                               ).to(dev).reshape(u_thin.shape)
        gt = torch.empty_like(u_thin)
        for _ in range(args.steps):
            ovl.stout_smear(u_thin, 0.1, -0.25, 3, out=us)
            ovl.stout_backward(u_thin, g_s, 0.1, -0.25, 3, out=gt)
        torch.cuda.synchronize()
        log(f"stout smear + chain rule x {args.steps}")
        return
    if args.profile == "overlap":
        measure_overlap(ovl, torch, dev, latgen, low_modes, args.steps, profile=True)
        return
    if args.profile in ("dw", "dw2"):
        measure_big(ovl, torch, dev, latgen, profile=args.profile, reps=args.steps)
        return
    if args.profile == "proj":
        gen = torch.Generator(device=dev).manual_seed(7)
        shape = (BF16_NEV, 4, 3) + tuple(reversed(BF16_DIMS))
        phi = torch.randn(shape, dtype=torch.complex128, device=dev, generator=gen)
        psi = torch.randn(shape[1:], dtype=torch.complex64, device=dev, generator=gen)
        d = ovl.Deflation(phi, np.linspace(-0.5, 0.5, BF16_NEV), "f32")
        for _ in range(args.steps):
            ovl.defl_project(d, psi)
        torch.cuda.synchronize()
        return

    t_start = time.time()
    bt = measure_batch(ovl, torch, dev, latgen, args.steps, args.warmup)
    extra = {}
    if not args.no_extra:
        extra["bf16_24modes_16x16x16x32"] = measure_bf16(ovl, torch, dev, latgen, low_modes, 5)
        extra["force_24x24x24x48"] = measure_force(ovl, torch, dev, latgen, 2)
        extra["overlap_8x8x8x16"] = measure_overlap(ovl, torch, dev, latgen, low_modes, 20)
        extra["k_and_sign_24x24x24x48"] = measure_big(ovl, torch, dev, latgen)
        extra["streams_4GiB"] = measure_streams(ovl, torch, dev)
    cpu, errs = (None, {})
    if not args.no_cpu:
        cpu, errs = oracle_leg(ovl, torch, dev, latgen, extra)

    # ---- roofline of each form's dominant kernel (algorithmic bytes / average launch) ----
    def roofline(kernel, bytes_per_launch, k_ms, k_n, tag=None, cfg=None):
        avg_us = 1e3 * k_ms / k_n
        ach = bytes_per_launch / (avg_us * 1e-6) / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                "traffic": counter_traffic(tag, cfg) if tag else None,
                "avg_launch_us": round(avg_us, 3), "launches": k_n,
                "bytes_per_launch": int(bytes_per_launch)}

    batch_bytes = batch_bytes_per_step("f32", True)
    # the counters of the configuration this run's tuner chose (the summary holds the forms the
    # tuner picks between)
    rl = roofline(kernel_name(bt["config"], "f32", True), batch_bytes, bt["kernel_ms"],
                  bt["kernel_launches"], tag="step2_kernel_sign_batch", cfg=bt["config"])
    rl["bytes_model"] = ("per step: every lattice's links once (two rows, 192 B/site) + "
                         "3.5 FP32 spinor streams (96 B each) per site and right-hand side")
    if "bf16_24modes_16x16x16x32" in extra:
        bf = extra["bf16_24modes_16x16x16x32"]
        bf["roofline"] = roofline(kernel_name(bf["config"], "bf16", False, False),
                                  step_bytes("bf16") * int(np.prod(BF16_DIMS)), bf.pop("kernel_ms"),
                                  bf.pop("kernel_launches"), tag="step_kernel_sign_bf16_16x16x16x32",
                                  cfg=bf["config"])
        bf["roofline"]["note"] = "62.9 MB per launch: the working set stays in the 256 MB Infinity Cache"
        bf["applies_per_s"] = round(1e3 / bf["ms_per_apply"], 2)
        bf["ms_per_apply"] = round(bf["ms_per_apply"], 3)
        bf["errors"] = errs.get("bf16")
    if "force_24x24x24x48" in extra:
        f = extra["force_24x24x24x48"]
        nv = f.pop("vjp_launches")
        f["roofline"] = roofline("link_vjp_kernel<float,float2,float2>",
                                 f["vjp_bytes_per_force"] / f["vjp_launches_per_force"],
                                 f.pop("vjp_ms"), nv, tag="link_vjp_kernel_24x24x24x48")
        f["roofline"]["bytes_model"] = ("per force: every (b_{m+1}, t_m) pair's two FP32 spinors "
                                        "once, the FP64 running sum of G between segments, G once")
        f["ms_per_force"] = round(f["ms_per_force"], 2)
        f["errors"] = errs.get("force")
    if "overlap_8x8x8x16" in extra:
        extra["overlap_8x8x8x16"]["errors"] = {k: errs.get(f"overlap_{k}") for k in ("f32", "f64")}

    # the same figures against the measured device-memory stream ceilings (a plain 4 GiB read,
    # copy and three-reads-one-write stream; the stencil reads several streams and writes one)
    st = extra.get("streams_4GiB")
    if st:
        ceil = {k: st[k]["GBps"] for k in ("read", "copy", "three_to_one")}
        rl["measured_ceilings_GBps"] = ceil
        rl["frac_of_three_to_one_stream"] = round(rl["achieved"] / ceil["three_to_one"], 4)
        for store, row in extra.get("k_and_sign_24x24x24x48", {}).items():
            for form in row.values():
                form["K_frac_of_three_to_one_stream"] = round(form["K_GBps"] / ceil["three_to_one"], 4)
                form["step_frac_of_three_to_one_stream"] = round(form["step_GBps"] / ceil["three_to_one"], 4)
        if "force_24x24x24x48" in extra:
            f = extra["force_24x24x24x48"]["roofline"]
            f["frac_of_three_to_one_stream"] = round(f["achieved"] / ceil["three_to_one"], 4)
    n_rhs = bt["n_rhs"]
    ms = bt["ms_per_batch"]
    line = {
        "metric": METRIC,
        "value": round(n_rhs * 1e3 / ms, 2),
        "unit": "sign(K)psi right-hand-side applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched sign(K) psi, Chebyshev degree 300 (299 K applications, eps 0.05, "
                        "no deflation): 12 spin-colour point sources on 16^3x32 + 4 x 8^3x16 + "
                        "2 x 12^3x24 (one Gaussian source each), every lattice its own 3-step "
                        "stout-smeared (rho 0.1) synthetic SU(3) field; FP32 storage and "
                        "arithmetic, two-row link reads, one launch per K application for the "
                        "whole batch, autotuned launch configuration",
            "lattices": ["16x16x16x32 x12 rhs", "8x8x8x16 x4", "12x12x12x24 x2"],
            "degree": BATCH_DEGREE - 1, "lmax": LMAX, "launch_config": bt["config"],
        },
        "roofline": rl,
        "cpu_baseline": cpu,
        "rel_err": {k: v for k, v in errs.items() if k.startswith("batch_")} or None,
        "batch": {k: v for k, v in bt.items() if k not in ("kernel_ms", "kernel_launches")},
        **extra,
        "wall_s": round(time.time() - t_start, 1),
    }
    line["batch"]["ms_per_batch"] = round(ms, 4)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
