"""Launch-configuration autotuner of the fused stencil: the chosen configuration is used by later
calls, persists through the cache file, and every configuration gives the oracle's answer."""
import numpy as np
import pytest

import latgen
from oracle import wilson as ow
from tests.conftest import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_and_results(tmp_path):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1510_06897_amd as ovl
    dims = (16, 16, 16, 16)
    u = latgen.random_su3_field(dims, 3)
    psi = latgen.gaussian_spinor(dims, 4, nrhs=2)
    ref = [ow.kop(u, psi[r]) for r in range(2)]
    for store, cdt, tol in (("f64", torch.complex128, 1e-14), ("f32", torch.complex64, 1e-6)):
        g = ovl.GaugeField(torch.from_numpy(u).cuda(), store)
        cache = str(tmp_path / f"tune_{store}.txt")
        us = ovl.autotune(g, nrhs=2, cache_path=cache)
        assert us > 0
        cfg = ovl.launch_config(g, nrhs=2)
        # any candidate may win: one site per lane (8, 16, 64 sites per workgroup), two sites per
        # lane (128, FP32 only) or an LDS slab (order 2, 64 to 256 sites)
        if cfg[1] == 2:
            assert cfg[0] in (64, 128, 192, 256)
        else:
            assert cfg[0] in ((8, 16, 64) if store == "f64" else (8, 16, 64, 128))
        assert ovl.autotune_load(cache) == 1
        got = ovl.kernel_apply(g, torch.from_numpy(psi).cuda().to(cdt)).cpu().numpy()
        for r in range(2):
            assert rel_err(got[r], ref[r]) < tol
