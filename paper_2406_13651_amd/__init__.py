"""MI355X-native CLAMP forward-model agent (HIP kernels for gfx950 behind a C ABI).

Import raises when libclamp.so is missing: there is no CPU fallback.
"""

from . import _clamp  # noqa: F401
from ._clamp import (  # noqa: F401
    ClampError, Plan, Scene, clamp_aperture_op, clamp_fwd_agent, clamp_fwd_init, clamp_mace_step,
    clamp_plan_create, clamp_plan_pupil_index, clamp_plan_pupil_info, clamp_plan_workspace_size,
    clamp_prior_gauss, clamp_fwd_refresh, make_params, CLAMP_FWD, CLAMP_ADJ, CLAMP_NORMAL,
    DG_GAMMA, DG_DD, DG_AD, DG_H0, DG_H1, DG_MURES, DG_WD, DG_R2,
)
from .clamp import ClampBatchGPU, ClampGPU, agent_weights, beta_schedule  # noqa: F401
