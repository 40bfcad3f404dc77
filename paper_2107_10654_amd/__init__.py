"""MI355X (gfx950) library for the ridge-leverage-score-sampled Tucker core update.

Fahrbach, Ghadiri, Fu, "Fast Low-Rank Tensor Decomposition by Ridge Leverage
Score Sampling" (arXiv 2107.10654): Alg. 3 (FastCoreTensorUpdate) with Alg. 1
(ApproximateRidgeRegression) inside Alg. 2 (ALS), as hand-written HIP kernels
behind the C ABI of ``include/tucker.h``.  The Python functions here only
marshal arguments; see ``tucker.py``.
"""
from .tucker import (  # noqa: F401
    BatchedSketchedUpdate, TuckerError, PRECISIONS, als, core_update_exact, core_update_sketched,
    core_update_sketched_adjoint, core_update_sketched_batched, core_update_sketched_noalloc,
    factor_update, leverage_scores,
    loss, make_problem, masked_sample_bound, release_workspace, ridge_tables, sample, sample_augmented, sample_count,
    sample_count_augmented, sample_ridge, sketched_system, tune_batched,
)
from .autograd import SketchedCoreUpdate, sketched_core_update  # noqa: F401
