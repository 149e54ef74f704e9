"""Randomized SVD, interpolative (ID) and CUR decompositions on AMD MI355X.

Python binding of librsvd.so (include/rsvd.h): argument marshalling only.
Every step of the computation runs in the library's HIP kernels; PyTorch is
used for device memory and streams.  Names follow the C entry points:

    svd(A, k, p, q, seed)        -> U, S, V, info      (Alg. 5, s = 1)
    svd_noalloc(A, k, p, q, seed) -> the same without a workspace (static scratch)
    id(A, k, p, q, seed)         -> J, T, info         (ID from B = Q^T A)
    id_left(A, k, p, q, seed)    -> J, T, info         (ID from Y = Omega~ A, Alg. 6)
    qb(A, b, M, q, tol, seed)    -> Q, B, resid, R, info (blocked adaptive QB, Alg. 7)
    cur(A, k, p, q, seed)        -> Jc, Jr, U, info    (CUR from the two-sided ID)
    svd_grad(A, k, p, q, seed, dU, dS, dV, dres) -> dA (adjoint, sketch fixed)
    svd_diff(A, k, p, q, seed)   -> U, S, V, resid2    (torch.autograd.Function)
    BatchPlan(ms, ns, ks, p, q)  -> batched RSVD of FP32 matrices in one persistent launch
    decompose(A, k, p, q, seed)  -> dict with all three from one range finder

    svd_ex(A, k, p, q, seed, scales, want_Q) -> U, S, V, info, Q (also FP8 A with column scales)
    quantize(A, BF16 | F8E4M3)   -> BF16 A, or (E4M3 codes, column scales), from FP64

and the single steps sketch, philox, pass_, pass_f8, orth, small_svd, cpqr.
"""

from .api import (  # noqa: F401
    RsvdError, handle, svd, svd_noalloc, id, id_left, qb, cur, svd_grad, svd_diff, BatchPlan, decompose,
    workspace_bytes, sketch, philox, pass_, orth, small_svd, cpqr, INFO_ORTH_FALLBACK,
    INFO_JACOBI_CAP, INFO_RANK, INFO_NONFINITE, INFO_BARRIER, F64, F32, BF16, F8E4M3, set_option,
    quantize, svd_ex, pass_f8,
    OPT_JACOBI_MAX_SWEEPS, OPT_TEST_WAIT_GIVEUP,
)
