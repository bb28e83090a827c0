"""CPU float64 oracle of CLAMP's forward-model agent, prior and consensus step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
GPU library never calls it and shares no code with it.

Each function is a plain, slow transcription of the passage it cites in
"CLAMP: Majorized Plug-and-Play for Coherent 3D Lidar Imaging" (Allen, Rabb,
Buzzard, Bouman).  numpy's FFT serves as the DFT primitive; everything else is
written out in the paper's order and notation.

Pinned against closed forms, brute force and invariants (tests/test_oracle_*):
operator (brute-force 2D and 3D DFT, Parseval, adjoint, projector, the 3D
form with a full range box against the per-slice form), gradient (finite
differences), step size (numerical line search, exact decrement), aperture
ablation (one-step closed form), r-update (exact-prox cubic, sigma^2 -> inf
limit, monotone on downward moves), exact surrogate prox (global minimum on a
dense grid, stationarity, sigma^2 limits), Mann iteration (quadratic-agent consensus
optimum), Gaussian prior (dense circular convolution), U-Net prior (brute-force
pooling and transposed convolution, adjoint and linearity identities, batch
normalisation closed forms and finite differences, folded against unfolded
evaluation, whole-network loss gradient by finite differences).  The full trajectory of
Algorithm 2 on a synthetic scene has no printed value in the paper: parity
unpinned beyond those invariants and the vanishing consensus error.
"""

from .operator import (  # noqa: F401
    pupil_mask, aperture_fraction, dft2, idft2, apply_A, apply_AH, apply_AHA,
    range_box, cylinder_mask, dft3, idft3,
)
from .agent import (  # noqa: F401
    noise_floor_weight, h_objective, neg_grad_h, exact_step, cov_diag,
    qs_prox, forward_agent, beta_schedule, exact_prox, surrogate_prox_objective,
)
from .prior import gaussian_taps, gaussian_smooth  # noqa: F401
from .mace import (  # noqa: F401
    agent_weights, weighted_average, mann_step, convergence_error, mu_residual,
)
from .clamp import ClampState, clamp_init, clamp_iteration, clamp_run  # noqa: F401
from .metrics import scale_fit, nrmse, psnr, point_cloud, point_cloud_metrics  # noqa: F401
from .regularizers import (  # noqa: F401
    l21_prox, l21_norm, grad3, div3, tv_norm, tv_prox, tv_dual_gap, speckle_average,
)
