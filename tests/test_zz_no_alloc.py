"""The allocation-free randomized SVD (rsvd_svd_noalloc, static device
scratch) against the workspace entry point rsvd_svd (needs a GPU).

Two calls in a row on the same device, the second smaller than the first, so
the second runs on scratch that holds the first call's leftovers.  Both
entry points run the same kernels on the same inputs: sigma within 1e-12
relative and U, V within 1e-10 (the FP64 parity bar of the path is 1e-10).
"""

import numpy as np
import pytest
import torch

from paper_1502_05366_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_workspace_call(R, dtype):
    cases = [(3000, 1700, 40, 10, 1, 0x5EED0003, 2), (900, 700, 12, 8, 2, 0x5EED0004, 3)]
    for m, n, k, p, q, seed, kind in cases:
        print("noalloc vs rsvd_svd:", m, n, k, p, q, dtype, flush=True)
        A, _ = W.logspace_type(m, n, kind, seed=m)
        Ad = torch.as_tensor(A, dtype=dtype, device="cuda")
        U0, S0, V0, i0 = R.svd(Ad, k, p, q, seed)
        U1, S1, V1, i1 = R.svd_noalloc(Ad, k, p, q, seed)
        torch.cuda.synchronize()
        assert int(i1.cpu()[0]) == int(i0.cpu()[0]) == 0
        S0, S1 = S0.cpu().numpy(), S1.cpu().numpy()
        assert np.abs(S1 - S0).max() <= 1e-12 * S0[0]
        tol = 1e-10 if dtype == torch.float64 else 1e-5
        assert (U1 - U0).abs().max().item() <= tol
        assert (V1 - V0).abs().max().item() <= tol


def test_noalloc_rejects_oversized(R):
    import ctypes
    from paper_1502_05366_amd import _lib
    lib = _lib.load()
    m, n, k = 20000, 10000, 200
    need = lib.rsvd_svd_noalloc_bytes(R.F64, m, n, k, 20, 2)
    assert need > (64 << 20)
    A = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    p = ctypes.c_void_p(A.data_ptr())
    rc = lib.rsvd_svd_noalloc(R.handle(), R.F64, m, n, k, 20, 2, 1, p, n, p, k, p, p, k,
                              ctypes.c_void_p(info.data_ptr()), None)
    assert rc == 5   # RSVD_ERR_SCRATCH: rejected before any launch
