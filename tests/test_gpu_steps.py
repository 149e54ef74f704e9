"""Parity of each step of the GPU path with the FP64 oracle (needs a GPU).

Steps: Philox words (bit-exact), Gaussian sketch, passes over A (exact on
integer data, bounded rounding otherwise), orth (CholeskyQR2), the Jacobi
SVD of the small factor, and the k-step column-pivoted QR with T.
"""

import numpy as np
import pytest
import torch

from oracle import philox as OP, dense as OD
from paper_1502_05366_amd import workloads as W
from tests.helpers import align_signs, orth_err, pivot_prefix

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


# ------------------------------------------------------------- sketch -----

@pytest.mark.parametrize("seed,sid,batch,first,count", [
    (0x5EED0000, 0, 0, 0, 4096),
    (0x123456789ABCDEF0, 7, 3, 0xFFFFFF00, 1000),     # crosses 2^32
    (1, 0, 0, (1 << 64) - 16, 16),
])
def test_philox_words_bit_exact(R, seed, sid, batch, first, count):
    got = R.philox(seed, sid, batch, first, count).cpu().numpy().view(np.uint32)
    ref = OP.raw_words(seed, sid, first, count, batch)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,l,ldo", [(1000, 30, 30), (10000, 220, 224), (77, 13, 16), (1, 1, 1)])
def test_sketch_matches_oracle(R, n, l, ldo):
    seed = 0x5EED0001
    om = R.sketch(n, l, seed, torch.float64, ldo=ldo).cpu().numpy()
    ref = OP.sketch(seed, n, l)
    # the same Philox words and Box-Muller formula on both sides; only the
    # device and host libm log / sqrt / sin / cos differ, each by at most an
    # ulp or two: per entry within 4 ulps of the oracle's value (measured: at
    # most 3, with 96% of the entries bit-identical)
    ulps = np.abs(om[:, :l] - ref) / np.spacing(np.abs(ref))
    assert ulps.max() <= 4.0
    assert np.mean(om[:, :l] == ref) >= 0.9
    assert np.all(om[:, l:] == 0.0)
    om32 = R.sketch(n, l, seed, torch.float32).cpu().numpy()
    # FP32 sketch = FP64 normals rounded to FP32 (a 1-ulp flip where the two
    # FP64 values straddle a rounding boundary)
    assert np.abs(om32 - ref.astype(np.float32)).max() <= np.spacing(np.float32(6.0))


# -------------------------------------------------------------- passes ----

@pytest.mark.parametrize("m,n,l", [(333, 517, 30), (1000, 2000, 220), (130, 70, 1), (16, 16, 16),
                                   (2047, 129, 257 - 1), (2048, 1024, 64), (1001, 3000, 33),
                                   (5000, 200, 48), (300, 20000, 17), (20000, 400, 30)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pass_exact_on_integers(R, m, n, l, dtype):
    A = W.integer_matrix(m, n, seed=m + n)
    Xn = W.integer_matrix(n, l, seed=l + 1)
    Xm = W.integer_matrix(m, l, seed=l + 2)
    Y = R.pass_(dev(A, dtype), dev(Xn, dtype), trans=False).cpu().numpy()
    Z = R.pass_(dev(A, dtype), dev(Xm, dtype), trans=True).cpu().numpy()
    # every partial sum is an integer below 2^24: exact in FP32 and FP64
    assert np.array_equal(Y.astype(np.float64), A @ Xn)
    assert np.array_equal(Z.astype(np.float64), A.T @ Xm)


@pytest.mark.parametrize("m,n,l", [(2000, 1000, 30), (3001, 1777, 220), (4000, 3000, 64),
                                   (3001, 1776, 40)])
def test_pass_random_vs_oracle(R, m, n, l):
    g = np.random.default_rng(1)
    A = g.standard_normal((m, n))
    X = g.standard_normal((n, l))
    Xm = g.standard_normal((m, l))
    Y = R.pass_(dev(A), dev(X)).cpu().numpy()
    Z = R.pass_(dev(A), dev(Xm), trans=True).cpu().numpy()
    bound_y = 2 * n * EPS * (np.abs(A) @ np.abs(X))
    bound_z = 2 * m * EPS * (np.abs(A.T) @ np.abs(Xm))
    assert np.all(np.abs(Y - A @ X) <= bound_y)
    assert np.all(np.abs(Z - A.T @ Xm) <= bound_z)
    # FP32 pass: within FP32 rounding of the same product
    A32, X32 = A.astype(np.float32), X.astype(np.float32)
    Y32 = R.pass_(dev(A32, torch.float32), dev(X32, torch.float32)).cpu().numpy()
    ref = A32.astype(np.float64) @ X32.astype(np.float64)
    b32 = 2 * n * np.finfo(np.float32).eps * (np.abs(A32) @ np.abs(X32))
    assert np.all(np.abs(Y32 - ref) <= b32)


# ---------------------------------------------------------------- orth ----

@pytest.mark.parametrize("rows,l,decay", [(1000, 30, 3), (20000, 220, 2), (50, 50, 1), (333, 17, 0),
                                          (2000, 64, 5), (3000, 100, 6)])
def test_orth_cholqr2(R, rows, l, decay):
    g = np.random.default_rng(rows + l)
    Y = g.standard_normal((rows, l)) @ np.diag(np.logspace(0, -decay, l)) @ \
        np.linalg.qr(g.standard_normal((l, l)))[0]
    Q, Rm, info = R.orth(dev(Y))
    Q, Rm = Q.cpu().numpy(), Rm.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    assert orth_err(Q) < 1e-12
    assert np.abs(Q @ Rm - Y).max() < 1e-13 * np.abs(Y).max() * max(1.0, 10.0 ** decay / 10)
    assert np.all(np.diag(Rm) > 0) and np.array_equal(np.triu(Rm), Rm)
    # the positive-diagonal QR of a full-rank Y is unique: the oracle's R
    Qo, Ro = OD.householder_qr(Y)
    kappa = 10.0 ** decay
    assert np.abs(Rm - Ro).max() <= 1e-13 * kappa * np.abs(Ro).max()
    assert np.abs(Q - Qo).max() <= 1e-12 * kappa


def test_orth_rank_deficient_fallback(R):
    g = np.random.default_rng(5)
    r, l, rows = 12, 30, 4000
    Y = g.standard_normal((rows, r)) @ g.standard_normal((r, l))
    Q, Rm, info = R.orth(dev(Y), seed=9)
    Q = Q.cpu().numpy()
    assert int(info.cpu()[0]) & R.INFO_ORTH_FALLBACK
    assert orth_err(Q) < 1e-12
    # range(Y) is inside range(Q)
    P = Q @ (Q.T @ Y)
    assert np.abs(P - Y).max() < 1e-12 * np.abs(Y).max()


def test_orth_fp32(R):
    g = np.random.default_rng(8)
    Y = g.standard_normal((5000, 40)).astype(np.float32)
    Q, Rm, info = R.orth(dev(Y, torch.float32))
    Q = Q.cpu().numpy().astype(np.float64)
    assert orth_err(Q) < 1e-5
    assert np.abs(Q @ Rm.cpu().numpy() - Y).max() < 1e-5 * np.abs(Y).max()


# ---------------------------------------------------------- small SVD ----

@pytest.mark.parametrize("l,k,decay", [(30, 20, 3), (64, 64, 6), (220, 200, 2.5), (1, 1, 0),
                                       (131, 7, 1), (80, 64, 4), (96, 96, 5), (65, 30, 3),
                                       (97, 50, 3), (17, 5, 2)])
def test_small_svd_vs_oracle(R, l, k, decay):
    g = np.random.default_rng(l)
    U0 = np.linalg.qr(g.standard_normal((l, l)))[0]
    V0 = np.linalg.qr(g.standard_normal((l, l)))[0]
    Rh = np.triu((U0 * np.logspace(0, -decay, l)) @ V0.T)
    S, Uh, Vh, info = R.small_svd(dev(Rh), k)
    S, Uh, Vh = S.cpu().numpy(), Uh.cpu().numpy(), Vh.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    Uo, so, Vo, _, _ = OD.jacobi_svd(Rh)
    # both Jacobi iterations are accurate to a few ulps relative where sigma is
    # not tiny, and to a multiple of eps * sigma_1 everywhere
    assert np.all(np.abs(S - so[:k]) <= np.maximum(1e-12 * so[:k], 50 * l * EPS * so[0]))
    assert np.abs(np.linalg.svd(Rh, compute_uv=False)[:k] - S).max() < 50 * l * EPS * so[0]
    assert orth_err(Uh) < 1e-13 and orth_err(Vh) < 1e-13
    # Rh Vh = Uh diag(S)
    assert np.abs(Rh @ Vh - Uh * S[None, :]).max() < 50 * l * EPS * so[0]
    # vectors agree with the oracle's up to sign where sigma is well separated
    gaps = np.minimum(np.r_[np.inf, so[:-1] - so[1:]][:k], np.r_[so[:-1] - so[1:], np.inf][:k])
    ok = gaps > 1e-6 * so[0]
    assert np.abs(align_signs(Vh, Vo[:, :k]) - Vo[:, :k])[:, ok].max(initial=0) < 1e-8
    assert np.abs(align_signs(Uh, Uo[:, :k]) - Uo[:, :k])[:, ok].max(initial=0) < 1e-8


# ---------------------------------------------------------------- CPQR ----

@pytest.mark.parametrize("r,c,k", [(30, 1000, 20), (220, 10000, 200), (12, 12, 12), (40, 333, 1),
                                   (64, 5000, 64)])
def test_cpqr_vs_oracle(R, r, c, k):
    g = np.random.default_rng(r * 7 + c)
    B = g.standard_normal((r, c)) * g.uniform(0.05, 10.0, c)[None, :]
    J, T, pv, info = R.cpqr(dev(B.T.copy()), r, k)
    J, T, pv = J.cpu().numpy(), T.cpu().numpy(), pv.cpu().numpy()
    f = OD.cpqr(B, k)
    npre = pivot_prefix(f['pivot_norms'], f['second_norms'], 1e-8)
    assert npre >= min(k, 1)
    assert np.array_equal(J[:npre], f['J'][:npre])
    if npre == k:
        assert np.array_equal(J, f['J'])
        To = OD.solve_upper(f['S11'], f['S12'])
        assert np.abs(T - To).max(initial=0) <= 1e-9 * max(1.0, np.abs(To).max(initial=0))
        assert np.allclose(pv, f['pivot_norms'], rtol=1e-12)
    # J is a permutation; the residual columns ascend
    assert np.array_equal(np.sort(J), np.arange(c))
    assert np.all(np.diff(J[k:]) > 0)
    assert int(info.cpu()[0]) & R.INFO_BARRIER == 0


def test_cpqr_rank_deficient_reports_rank(R):
    g = np.random.default_rng(3)
    B = g.standard_normal((20, 5)) @ g.standard_normal((5, 300))
    J, T, pv, info = R.cpqr(dev(B.T.copy()), 20, 10)
    info = info.cpu().numpy()
    assert info[0] & R.INFO_RANK
    assert info[1] == 5
    f = OD.cpqr(B, 10)
    assert f['frank'] == 5


@pytest.mark.parametrize("decay", [0.0, 3.0, 5.0])
def test_orth_fp32_conditioning(R, decay):
    """FP32 bases across conditioning: well-conditioned Y takes the rounding
    copy after the first pass, ill-conditioned Y (kappa ~1e5) the full second
    pass; both give an FP32-orthonormal Q spanning range(Y)."""
    g = np.random.default_rng(31 + int(decay))
    rows, l = 6000, 48
    Y = (g.standard_normal((rows, l)) @ np.diag(np.logspace(0, -decay, l))
         @ np.linalg.qr(g.standard_normal((l, l)))[0]).astype(np.float32)
    Q, Rm, info = R.orth(dev(Y, torch.float32))
    Q = Q.cpu().numpy().astype(np.float64)
    assert int(info.cpu()[0]) == 0
    assert orth_err(Q) < 1e-5
    Y64 = Y.astype(np.float64)
    # range(Y) inside range(Q), relative to the size of Y
    assert np.linalg.norm(Y64 - Q @ (Q.T @ Y64)) <= 1e-5 * np.linalg.norm(Y64)
