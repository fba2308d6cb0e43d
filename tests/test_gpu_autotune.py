"""Launch-configuration autotuner of the fused Chebyshev step: the chosen configuration is used by
later calls (single problems and batches), persists through the cache file, and every
configuration gives the oracle's answer."""
import numpy as np
import pytest

import latgen
from oracle import chebyshev as och
from oracle import wilson as ow
from tests.conftest import rel_err

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


def last_entry(path):
    """(spb, order, remap, rb) of the last line an autotune call appended."""
    f = open(path).read().split("\n")
    toks = [t for t in f if t.strip()][-1].split()
    assert toks[0] == "B"
    return tuple(int(v) for v in toks[-5:-1])


def test_autotune_single_and_results(ovl, tmp_path):
    dims = (16, 16, 16, 16)
    u = latgen.random_su3_field(dims, 3)
    psi = latgen.gaussian_spinor(dims, 4, nrhs=2)
    ref = [ow.kop(u, psi[r]) for r in range(2)]
    for store, cdt, tol in (("f64", torch.complex128, 1e-14), ("f32", torch.complex64, 1e-6)):
        g = ovl.GaugeField(dev(u), store)
        x = dev(psi, cdt)
        cache = str(tmp_path / f"tune_{store}.txt")
        us = ovl.autotune((g, x), cache_path=cache)
        assert us > 0
        spb, order, remap, rb = last_entry(cache)
        assert ovl.batch_launch_config((g, x)) == (spb, order, remap, rb)
        cfg = ovl.launch_config(g, nrhs=2)
        assert cfg == (spb, order, remap)
        # any candidate may win: one site per lane (8, 16, 64 sites per workgroup, with 1, 2 or 4
        # right-hand sides per thread at 16 and 64), two sites per lane (128, FP32 only) or an
        # LDS slab (order 2, 64 to 256 sites)
        if order == 2:
            assert spb in (64, 128, 192, 256) and rb == 1
        else:
            assert spb in ((8, 16, 64) if store == "f64" else (8, 16, 64, 128))
            assert rb in ((1, 2) if spb in (16, 64) else (1,))
        assert ovl.autotune_load(cache) == 1
        got = ovl.kernel_apply(g, x).cpu().numpy()
        for r in range(2):
            assert rel_err(got[r], ref[r]) < tol


def batch_problems(ovl, store):
    shapes = [((8, 8, 8, 8), 4), ((4, 4, 4, 8), 1), ((6, 4, 4, 4), 3)]
    cdt = torch.complex128 if store == "f64" else torch.complex64
    probs, refs_in = [], []
    for i, (dims, nrhs) in enumerate(shapes):
        u = latgen.smeared_field(dims, 10450 + i, steps=1)
        psi = latgen.gaussian_spinor(dims, 20450 + i, nrhs=nrhs)
        u_in = u if store == "f64" else latgen.round_to_f32(u)
        psi_in = psi if store == "f64" else latgen.round_to_f32(psi)
        probs.append((ovl.GaugeField(dev(u), store), dev(psi, cdt)))
        refs_in.append((u_in, psi_in))
    return probs, refs_in


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_batch_autotune_used_by_the_batch(ovl, tmp_path, store):
    """ovl_autotune on a mixed-volume batch: the batch then runs in the configuration it chose
    (and in a forced right-hand-side-block configuration read from a cache file), with the
    oracle's result either way."""
    probs, refs_in = batch_problems(ovl, store)
    alpha = och.coeffs_sign_interp(21, 0.08)
    p = ovl.Polynomial(alpha, LMAX)
    tol = 1e-12 if store == "f64" else 1e-6
    cache = str(tmp_path / "batch.txt")
    us = ovl.autotune(probs, p, cache_path=cache)
    assert us > 0
    tuned = last_entry(cache)
    assert ovl.batch_launch_config(probs) == tuned

    def check():
        outs = ovl.batch_sign_apply(p, probs)
        torch.cuda.synchronize()
        for (g, _), out, (u_in, psi_in) in zip(probs, outs, refs_in):
            got = out.cpu().to(torch.complex128).numpy()
            for r in range(psi_in.shape[0]):
                assert rel_err(got[r], och.poly_apply(u_in, psi_in[r], alpha, LMAX)) < tol
            assert g.flags() == 0

    check()
    # right-hand-side blocks of 4 and 2 (ragged last blocks: 4 -> 4, 1 -> 1, 3 -> 3 and 2 + 1)
    prec = 0 if store == "f64" else 1
    items = " ".join(f"{g.dims[0]} {g.dims[1]} {g.dims[2]} {g.dims[3]} {x.shape[0]}"
                     for g, x in probs)
    for rb, spb in ((4, 64), (2, 16)):
        forced = tmp_path / f"rb{rb}.txt"
        forced.write_text(f"B {prec} 0 {len(probs)} {items} {spb} 0 1 {rb} 0\n")
        ovl.batch_sign_apply(p, probs, tune_cache=str(forced))   # reads the file once
        assert ovl.batch_launch_config(probs) == (spb, 0, 1, rb)
        check()
