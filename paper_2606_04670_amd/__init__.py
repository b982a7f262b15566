"""MI355X (gfx950) implementation of the all-pairs Lipschitz bound evaluation
of optimal Lipschitz interpolation with monotonicity constraints: the
envelopes H_up / H_lo (Eq. 2), the interpolant g (Eq. 3) with directional
distances on monotone coordinates (Eq. 4), the data-side consistency check
and Lipschitz-constant estimates, subgradients, batched fits and a
BF16-MFMA l2 variant, the step-function local constants M_k(t) of
Sec. 4.3 and the penalty objective of the smoothing problem (Sec. 4.4).  The work runs in hand-written HIP kernels behind the
C ABI of include/lipfit.h; this package only binds it.
"""
from ._lib import LipError, load  # noqa: F401
from .api import (LipFitFn, Metric, Plan, StepModel, autotune, backward, bounds,  # noqa: F401
                  consistency, estimate_M, fit_eval, fit_eval_k, fit_eval_steps, lipfit, local_knots,
                  local_steps, smooth_lipschitz, smooth_objective, tune_clear, tune_get,
                  tune_load, tune_save, tune_set)
