"""MI355X-native hot path of finite-temperature PEPS-VMC (arXiv 2409.05285).

The computation lives in libpeps.so (HIP for gfx950, C ABI in
include/peps.h); this package only marshals arguments.  Importing it fails
if the library has not been built (python paper_2409_05285_amd/build.py).
"""
from .api import (Desc, PepsLogAmp, Trace, check, new_status, peps_eval_batch, peps_grad_batch,  # noqa: F401
                  peps_orow_count, peps_param_count, peps_sample_stats,
                  peps_sample_sweep, peps_slot_count, peps_vjp_batch, peps_workspace_bytes, sr_cg_solve,
                  sr_cg_solve_noalloc, peps_direct_workspace_bytes, peps_direct_sample, peps_importance_weights,
                  workspace_bytes, peps_observables_batch, thermal_observables, OBS_NAMES,
                  nnn_spin_correlation, specific_heat, peps_simple_update, peps_su_absorb, su_bond_count)
from .api import peps_autotune_compression  # noqa: F401
from .autotune import tune as tune_compression  # noqa: F401
from .cooling import cool  # noqa: F401
from ._lib import (LIB_PATH, MODEL_HEISENBERG, MODEL_HUBBARD, PREC_FP64, PREC_MIXED, PepsError,  # noqa: F401
                   COMPRESS_AUTO, COMPRESS_REGISTER, COMPRESS_LDS, COMPRESS_WORKSPACE)
