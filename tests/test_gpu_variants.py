"""Parity of the paper's variants with the FP64 oracle on the same A and seed
(needs a GPU): the left-sketch randomized ID (Alg. 6 with the power scheme of
eq. (Ypower)) and the blocked adaptive QB (Alg. 7).

Bar, as for the ID from B: skeleton indices identical up to the first near-tie
of the oracle's pivot norms (margin 1e-8), T within a rounding-level
tolerance where all k pivots agree, J a permutation, exact results where the
mathematics fixes them (exact rank, separated skeleton).  Blocked QB: the same
number of blocks as the oracle, Q and B equal to the oracle's to 1e-9 (both
orthonormalize with the positive-diagonal QR, so each Q_i is unique), the
residual norm to 1e-9 relative, and the deflation identities.
"""

import numpy as np
import pytest
import torch

from oracle import rsvd as O
from paper_1502_05366_amd import workloads as W
from tests.helpers import pivot_prefix

pytestmark = pytest.mark.gpu
SEED = 0x5EED0000


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def id_error(A, J, T):
    V = O.interp_matrix(J, T, A.shape[1])
    return np.linalg.norm(A - A[:, J[:T.shape[0]]] @ V.T, 2)


def check_against_oracle(J, T, d, k, ttol):
    n = len(J)
    assert np.array_equal(np.sort(J), np.arange(n))
    npre = pivot_prefix(d["pivot_norms"], d["second_norms"], 1e-8)
    assert npre >= 1
    assert np.array_equal(J[:npre], d["J"][:npre])
    if npre == k and n > k:
        assert np.array_equal(J, d["J"])
        assert np.abs(T - d["T"]).max() <= ttol * max(1.0, np.abs(d["T"]).max())
    return npre


@pytest.mark.parametrize("m,n,k,p,q", [(2000, 1000, 20, 10, 1), (333, 517, 17, 5, 0),
                                       (1000, 300, 30, 10, 2), (300, 1000, 25, 7, 1),
                                       (64, 48, 48, 0, 1)])
def test_id_left_vs_oracle(R, m, n, k, p, q):
    if (m, n) == (2000, 1000):
        A, _ = W.c1_matrix()
    else:
        A, _ = W.logspace_type(m, n, 2, seed=m + 7 * n)
    J, T, info = R.id_left(dev(A), k, p, q, SEED)
    J, T = J.cpu().numpy(), T.cpu().numpy()
    assert int(info.cpu()[0]) & ~R.INFO_RANK == 0
    d = O.id_left(A, k, p, q, SEED)
    check_against_oracle(J, T, d, k, 1e-8)


@pytest.mark.parametrize("q", [0, 2])
def test_id_left_exact_rank(R, q):
    A, s, _, _ = W.exact_rank_matrix(1500, 900, 11, seed=3)
    J, T, info = R.id_left(dev(A), 15, 5, q, SEED)
    J, T = J.cpu().numpy(), T.cpu().numpy()
    assert id_error(A, J, T) <= 1e-11 * s[0]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_id_left_separated_skeleton(R, dtype):
    A, pi, _ = W.separated_skeleton_matrix(3000, 5000, 60, seed=17)
    k, p, q = 40, 20, 1
    J, T, info = R.id_left(dev(A, dtype), k, p, q, SEED)
    assert list(J.cpu().numpy()[:k]) == list(pi[:k])


def test_id_left_deterministic(R):
    A, _ = W.logspace_type(1200, 800, 2, seed=5)
    Ad = dev(A)
    a = R.id_left(Ad, 30, 10, 1, SEED)
    b = R.id_left(Ad, 30, 10, 1, SEED)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_id_left_args(R):
    lib = R.api._lib.load()
    assert lib.rsvd_id_left_workspace_bytes(0, 100, 50, 60, 5, 1) == 0     # k > min(m, n)
    assert lib.rsvd_id_left_workspace_bytes(7, 100, 50, 10, 5, 1) == 0     # bad dtype
    A = dev(np.zeros((100, 50)))
    with pytest.raises(R.RsvdError):
        R.id_left(A, 10, 5, -1, SEED)


# ---------------------------------------------------------- blocked QB ----

@pytest.mark.parametrize("m,n,b,M,q,tolf", [(600, 400, 16, 6, 1, 0.0), (2000, 1000, 10, 5, 1, 0.0),
                                            (333, 517, 7, 9, 0, 0.02), (512, 512, 32, 8, 2, 0.01)])
def test_qb_vs_oracle(R, m, n, b, M, q, tolf):
    if (m, n) == (2000, 1000):
        A, _ = W.c1_matrix()
    else:
        A, _ = W.logspace_type(m, n, 2, seed=m + n)
    tol = tolf * np.linalg.norm(A)
    Q, B, res, Rd, info = R.qb(dev(A), b, M, q, tol, SEED)
    Q, B, Rd = Q.cpu().numpy(), B.cpu().numpy(), Rd.cpu().numpy()
    d = O.qb_blocked(A, b, M, tol, q, SEED)
    assert Q.shape[1] == d["Q"].shape[1], (Q.shape, d["nblocks"])
    nA = np.linalg.norm(A)
    assert np.abs(Q - d["Q"]).max() <= 1e-9
    assert np.abs(B - d["B"]).max() <= 1e-9 * nA
    assert abs(res - d["norms"][-1]) <= 1e-9 * nA
    assert np.abs(Rd - (A - Q @ B)).max() <= 1e-11 * nA
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-12


def test_qb_exact_rank(R):
    A, s, _, _ = W.exact_rank_matrix(1200, 700, 20, seed=9)
    nA = np.linalg.norm(A)
    Q, B, res, Rd, info = R.qb(dev(A), 8, 10, 1, 1e-10 * nA, SEED)
    assert Q.shape[1] == 24
    assert res < 1e-12 * nA
    Q = Q.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(24)).max() < 1e-12


def test_qb_args(R):
    lib = R.api._lib.load()
    assert lib.rsvd_qb_workspace_bytes(0, 100, 50, 16, 4, 1) == 0      # b*M > min(m, n)
    assert lib.rsvd_qb_workspace_bytes(1, 100, 50, 8, 4, 1) == 0       # FP32 not built
    with pytest.raises(R.RsvdError):
        R.qb(dev(np.zeros((100, 50)), torch.float32), 8, 4, 1, 0.0, SEED)
