"""The randomized SVD at the sample size of the mixed-precision workload,
l = k + p = 576 (needs a GPU): the block orthonormalization (column blocks of
at most 256, each projected twice against the columns before it), the block
Jacobi SVD of the 576 x 576 factor, and the passes with more than one column
tile, against the FP64 oracle at sizes it finishes in seconds.

Bars: orth as for l <= 256 (Q orthonormal to 1e-12, R equal to the oracle's
unique positive-diagonal R); small SVD as for l <= 256; FP64 RSVD sigma
within 1e-10 relative (the FP64 target); BF16 RSVD sigma within 1e-3 relative
of the oracle run on the same BF16 values of A (the BF16 target).
"""

import numpy as np
import pytest
import torch

from oracle import rsvd as O, dense as OD, quant as QZ
from paper_1502_05366_amd import workloads as W
from tests.helpers import align_signs, orth_err

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("rows,l,decay", [(5000, 576, 3), (3000, 300, 2), (2000, 513, 4)])
def test_orth_blocks_vs_oracle(R, rows, l, decay):
    g = np.random.default_rng(rows + l)
    Y = g.standard_normal((rows, l)) @ np.diag(np.logspace(0, -decay, l)) @ \
        np.linalg.qr(g.standard_normal((l, l)))[0]
    print("orth l=%d rows=%d" % (l, rows), flush=True)
    Q, Rm, info = R.orth(dev(Y))
    Q, Rm = Q.cpu().numpy(), Rm.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    assert orth_err(Q) < 1e-12
    kappa = 10.0 ** decay
    assert np.abs(Q @ Rm - Y).max() < 1e-13 * np.abs(Y).max() * max(1.0, kappa / 10)
    assert np.all(np.diag(Rm) > 0) and np.array_equal(np.triu(Rm), Rm)
    Qo, Ro = OD.householder_qr(Y)
    assert np.abs(Rm - Ro).max() <= 1e-13 * kappa * np.abs(Ro).max()
    assert np.abs(Q - Qo).max() <= 1e-12 * kappa


def test_orth_blocks_fp32(R):
    g = np.random.default_rng(12)
    Y = g.standard_normal((6000, 576)).astype(np.float32)
    Q, Rm, info = R.orth(dev(Y, torch.float32))
    Q = Q.cpu().numpy().astype(np.float64)
    assert orth_err(Q) < 1e-5
    assert np.abs(Q @ Rm.cpu().numpy() - Y).max() < 1e-5 * np.abs(Y).max()


def test_orth_blocks_rank_deficient(R):
    # a dependent column in the second block is replaced, and the replacement is
    # orthogonal to the first block too
    g = np.random.default_rng(13)
    rows, l = 4000, 400
    Y = g.standard_normal((rows, l))
    Y[:, 300] = Y[:, 10] - 2.0 * Y[:, 250]
    Q, Rm, info = R.orth(dev(Y), seed=3)
    Q = Q.cpu().numpy()
    assert int(info.cpu()[0]) & R.INFO_ORTH_FALLBACK
    assert orth_err(Q) < 1e-12
    assert np.abs(Q @ (Q.T @ Y) - Y).max() < 1e-12 * np.abs(Y).max()


def test_small_svd_l576(R):
    l, k = 576, 512
    g = np.random.default_rng(576)
    U0 = np.linalg.qr(g.standard_normal((l, l)))[0]
    V0 = np.linalg.qr(g.standard_normal((l, l)))[0]
    s0 = np.arange(1, l + 1, dtype=np.float64) ** -1.5
    Rh = np.triu((U0 * s0) @ V0.T)
    print("small SVD l=576", flush=True)
    S, Uh, Vh, info = R.small_svd(dev(Rh), k)
    S, Uh, Vh = S.cpu().numpy(), Uh.cpu().numpy(), Vh.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    Uo, so, Vo, _, _ = OD.jacobi_svd(Rh)
    assert np.all(np.abs(S - so[:k]) <= np.maximum(1e-12 * so[:k], 50 * l * EPS * so[0]))
    # the iteration stops when every column pair is orthogonal to l eps relative
    # to the column norms, so U is orthonormal to a small multiple of l eps; V
    # collects the rotations of every sweep (26 here): measured against the
    # oracle's own V
    assert orth_err(Uh) < 2 * l * EPS
    assert orth_err(Vh) < max(2 * l * EPS, 3 * orth_err(Vo[:, :k]))
    assert np.abs(Rh @ Vh - Uh * S[None, :]).max() < 50 * l * EPS * so[0]
    gaps = np.minimum(np.r_[np.inf, so[:-1] - so[1:]][:k], np.r_[so[:-1] - so[1:], np.inf][:k])
    ok = gaps > 1e-6 * so[0]
    assert np.abs(align_signs(Vh, Vo[:, :k]) - Vo[:, :k])[:, ok].max(initial=0) < 1e-8


@pytest.fixture(scope="module")
def graded():
    """4096 x 2048 with sigma_j = j^(-1.5) (the spectrum of the mixed-precision
    workload), Haar factors."""
    m, n = 4096, 2048
    s = np.arange(1, n + 1, dtype=np.float64) ** -1.5
    A, _, _ = W.spectrum_matrix(m, n, s, seed=0xC0FFEE12)
    return A


K, P, Q, SEED = 512, 64, 2, 0x5EED0012


def test_rsvd_l576_fp64_vs_oracle(R, graded):
    A = graded
    print("FP64 RSVD l=576 on the GPU", flush=True)
    U, S, V, info = R.svd(dev(A), K, P, Q, SEED)
    S = S.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    print("oracle", flush=True)
    Uo, So, Vo = O.rsvd(A, K, P, Q, SEED)
    assert np.max(np.abs(S - So) / So) <= 1e-10
    U, V = U.cpu().numpy(), V.cpu().numpy()
    assert orth_err(U) < 1e-12 and orth_err(V) < 1e-12
    # U^T A V = diag(S), a property of the method at any size
    assert np.abs(U.T @ A @ V - np.diag(S)).max() <= 1e-12


def test_rsvd_l576_bf16_vs_oracle(R, graded):
    A = graded
    Ab = QZ.bf16_round(A)
    Ad = torch.as_tensor(Ab, device="cuda").to(torch.bfloat16)   # exact: Ab is BF16
    print("BF16 RSVD l=576 on the GPU", flush=True)
    U, S, V, info = R.svd(Ad, K, P, Q, SEED)
    S = S.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    print("oracle on the BF16 values", flush=True)
    _, So, _ = O.rsvd(Ab, K, P, Q, SEED)
    assert np.max(np.abs(S - So) / So) <= 1e-3
    U = U.cpu().numpy().astype(np.float64)
    assert orth_err(U) < 1e-5
