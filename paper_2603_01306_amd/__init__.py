"""MI355X-native certified lower bounds for k-sparse GLM branch-and-bound nodes.

The solver (FISTA with duality-gap restarts on the perspective relaxation,
arXiv 2603.01306) lives in the HIP library libpr.so behind the C ABI of
include/pr.h; this package is its Python binding.
"""
from ._binding import (Context, Node, prox, prox_noalloc, regularizer, gemm, default_opts, load, PrError,  # noqa: F401
                       mlp_forward, mlp_grad, mlp_adam, mlp_workspace, MLP_NFEAT, MLP_NPARAM, time_prox, time_read,
                       CONVERGED, MAXITER, INFEASIBLE, CUTOFF_PRUNE, CUTOFF_BRANCH,
                       FREE, ZERO, ONE, LSQ, LOGISTIC, FISTA_GAP, FISTA, FISTA_FV, PGD, ACFGM_GAP, ACFGM, FISTA_BT_GAP, FISTA_BT, L1_REG, L1_BALL, BNB_OPTIMAL, BNB_NODE_LIMIT, BNB_TIME_LIMIT, F64, F32, BF16, EXPORTS, LIB_PATH, PROX_NOALLOC_MAX_P, DEBUG_GRAM_RECHECK, DEBUG_FORCE_BATCH)
