"""MI355X-native overlap-operator library (Cundy & Lee, "Overlap fermions on GPUs", arXiv:1510.06897).

The compute path is libovl.so (hand-written HIP kernels for gfx950 behind a C ABI, include/ovl.h);
this package is its PyTorch binding.  Importing the operators loads the library and raises if it
has not been built (``python -m paper_1510_06897_amd.build``).
"""
from ._lib import OvlError, load  # noqa: F401
from .api import (  # noqa: F401
    M_W, Deflation, GaugeField, Polynomial, SignFunction, autotune, autotune_load,
    batch_launch_config, batch_sign_apply, cheb_sign_coeffs, defl_correct, defl_project, graph_enable, kernel_apply,
    kernel_axpby,
    launch_config, overlap_apply, overlap_solve, overlap_solve_gmresr, sign_apply, sign_force, sign_residual, stout_backward, stout_smear, StoutFunction, stream_probe, timing_enable,
    timing_read, wilson_apply, wilson_link_vjp,
)
