"""Failure handling of the GPU path (needs a GPU): non-finite input, the
Jacobi sweep cap, and the bounded cross-workgroup waits giving up.

Every condition is forced from the host, so every kernel still runs to its
end: NaN entries in the input; a sweep cap of 1 on a factor that needs more
sweeps; and the handle's test mode in which every cross-workgroup wait of the
pivoted QR and of the block Jacobi waits for a value no workgroup posts,
with a small spin cap.  The status bits are those of the rank / failure
reporting of Sec. 2.6 (frank) extended with the library's own conditions.
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


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def info_word(info):
    return int(info.cpu()[0])


@pytest.mark.parametrize("nan_cols", [[3], [0, 5, 17, 40], "all"])
def test_cpqr_nonfinite_columns(R, nan_cols):
    # B (r x c) by columns; NaN columns are still chosen (after every finite
    # column), so J stays a permutation and the call reports NONFINITE
    r, c, k = 24, 300, 20
    g = np.random.default_rng(11)
    Bc = g.standard_normal((c, r))
    cols = list(range(c)) if nan_cols == "all" else nan_cols
    Bc[cols, 2] = np.nan
    print("cpqr NaN columns", nan_cols, flush=True)
    J, T, pv, info = R.cpqr(dev(Bc), r, k)
    J = J.cpu().numpy()
    assert np.array_equal(np.sort(J), np.arange(c))
    assert info_word(info) & R.INFO_NONFINITE
    if nan_cols != "all" and len(cols) < c - k:
        # the finite columns come first, in the oracle's order of norms
        assert not np.any(np.isin(J[:k], cols))


def test_decompose_nonfinite_input(R):
    A, _ = W.logspace_type(400, 300, 2, seed=3)
    A[17, 33] = np.nan
    print("decompose with a NaN entry", flush=True)
    out = R.decompose(dev(A), 12, 8, 1, 0x5EED0000)
    torch.cuda.synchronize()
    info = info_word(out["info"])
    assert info & R.INFO_NONFINITE
    J = out["J"].cpu().numpy()
    assert np.array_equal(np.sort(J), np.arange(300))
    Jr = out["Jr"].cpu().numpy()
    assert np.all((Jr >= 0) & (Jr < 400))


def test_jacobi_sweep_cap(R):
    g = np.random.default_rng(4)
    l = 100
    Rh = np.triu(g.standard_normal((l, l))) + 3 * np.eye(l)
    try:
        R.set_option(R.OPT_JACOBI_MAX_SWEEPS, 1)
        print("small_svd with a sweep cap of 1", flush=True)
        S, Uh, Vh, info = R.small_svd(dev(Rh), 10)
        assert info_word(info) & R.INFO_JACOBI_CAP
    finally:
        R.set_option(R.OPT_JACOBI_MAX_SWEEPS, 40)
    S, Uh, Vh, info = R.small_svd(dev(Rh), 10)
    assert info_word(info) == 0
    ref = np.linalg.svd(Rh, compute_uv=False)[:10]
    assert np.abs(S.cpu().numpy() - ref).max() <= 1e-12 * ref[0]


def test_option_arguments(R):
    with pytest.raises(R.RsvdError):
        R.set_option(R.OPT_JACOBI_MAX_SWEEPS, 0)
    with pytest.raises(R.RsvdError):
        R.set_option(99, 1)


@pytest.mark.parametrize("what", ["cpqr", "small_svd", "decompose"])
def test_wait_giveup_reports_barrier(R, what):
    g = np.random.default_rng(6)
    try:
        R.set_option(R.OPT_TEST_WAIT_GIVEUP, 1)
        print("forced wait give-up:", what, flush=True)
        if what == "cpqr":
            r, c, k = 40, 5000, 30
            J, T, pv, info = R.cpqr(dev(g.standard_normal((c, r))), r, k)
            J = J.cpu().numpy()
            assert np.all((J >= 0) & (J < c))
        elif what == "small_svd":
            l = 120                               # above 64: the block iteration
            Rh = np.triu(g.standard_normal((l, l))) + 2 * np.eye(l)
            S, Uh, Vh, info = R.small_svd(dev(Rh), 20)
        else:
            A, _ = W.logspace_type(2000, 1500, 2, seed=8)
            out = R.decompose(dev(A), 100, 20, 1, 0x5EED0000)
            info = out["info"]
        torch.cuda.synchronize()
        assert info_word(info) & R.INFO_BARRIER
    finally:
        R.set_option(R.OPT_TEST_WAIT_GIVEUP, 0)
    # the handle works normally again
    r, c, k = 40, 5000, 30
    Bc = g.standard_normal((c, r))
    J, T, pv, info = R.cpqr(dev(Bc), r, k)
    assert info_word(info) == 0
    assert np.array_equal(np.sort(J.cpu().numpy()), np.arange(c))
