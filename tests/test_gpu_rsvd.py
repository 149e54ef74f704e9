"""End-to-end parity of rsvd_svd / rsvd_id / rsvd_cur / rsvd_decompose with
the FP64 oracle on the same A and seed (needs a GPU).

Bar: sigma relative error <= 1e-10 (FP64), singular vectors equal up to sign
where the spectrum is separated, ID skeleton indices identical up to the first
near-tie of the pivot norms (margin 1e-8), T and the CUR factor within a
rounding-level tolerance, and exact results where the paper fixes them
(exact rank, separated skeleton).
"""

import numpy as np
import pytest
import torch

from oracle import rsvd as O
from paper_1502_05366_amd import workloads as W
from tests.helpers import align_signs, orth_err, pivot_prefix, subspace_gap

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
SEED = 0x5EED0000


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def check_svd(A, U, S, V, Uo, So, Vo, rtol=1e-10):
    k = len(So)
    assert np.max(np.abs(S - So) / So) <= rtol
    assert orth_err(U) < 1e-12 and orth_err(V) < 1e-12
    gap = np.minimum(np.r_[np.inf, So[:-1] - So[1:]], np.r_[So[:-1] - So[1:], np.inf])
    ok = gap > 1e-3 * So
    Ua, Va = align_signs(U, Uo), align_signs(V, Vo)
    assert np.abs(Ua - Uo)[:, ok].max(initial=0) < 1e-7
    assert np.abs(Va - Vo)[:, ok].max(initial=0) < 1e-7


@pytest.fixture(scope="module")
def c1():
    A, s = W.c1_matrix()
    return A, s


def test_c1_svd(R, c1):
    A, s = c1
    k, p, q = 20, 10, 1
    U, S, V, info = R.svd(dev(A), k, p, q, SEED)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    Uo, So, Vo = O.rsvd(A, k, p, q, SEED)
    check_svd(A, U, S, V, Uo, So, Vo)
    # and the approximation is as good as the oracle's
    e = np.linalg.norm(A - (U * S) @ V.T, 2)
    eo = np.linalg.norm(A - (Uo * So) @ Vo.T, 2)
    assert abs(e - eo) <= 1e-9 * s[0]


def test_c1_id_and_cur(R, c1):
    A, s = c1
    k, p, q = 20, 10, 1
    J, T, info = R.id(dev(A), k, p, q, SEED)
    J, T = J.cpu().numpy(), T.cpu().numpy()
    d = O.qb_id(A, k, p, q, SEED)
    npre = pivot_prefix(d['pivot_norms'], d['second_norms'], 1e-8)
    assert npre == k
    assert np.array_equal(J, d['J'])
    assert np.abs(T - d['T']).max() <= 1e-8 * max(1.0, np.abs(d['T']).max())
    Jc, Jr, Uc, info = R.cur(dev(A), k, p, q, SEED)
    Jc, Jr, Uc = Jc.cpu().numpy(), Jr.cpu().numpy(), Uc.cpu().numpy()
    c = O.cur(A, k, p, q, SEED)
    assert np.array_equal(Jc, c['Jc'])
    nr = pivot_prefix(c['row_pivot_norms'], c['row_second_norms'], 1e-8)
    assert nr == k
    assert np.array_equal(Jr, c['Jr'])
    assert np.abs(Uc - c['U']).max() <= 1e-7 * np.abs(c['U']).max()
    err = np.linalg.norm(A - A[:, Jc] @ Uc @ A[Jr, :], 2)
    erro = np.linalg.norm(A - A[:, c['Jc']] @ c['U'] @ A[c['Jr'], :], 2)
    assert abs(err - erro) <= 1e-8 * s[0]


@pytest.mark.parametrize("m,n,k,p,q", [
    (517, 333, 13, 7, 2),      # ragged tiles everywhere
    (300, 900, 25, 5, 0),      # m < n, no power step
    (64, 48, 40, 30, 1),       # k + p > min(m, n): l clamps to n
    (1000, 1000, 1, 0, 1),     # k = 1, p = 0
    (4000, 250, 200, 20, 2),   # the C2 sample size on a small matrix
])
def test_shapes_svd_id(R, m, n, k, p, q):
    A, s = W.logspace_type(m, n, 3, seed=m * 3 + n)
    out = R.decompose(dev(A), k, p, q, SEED, svd=True, id=True, cur=False)
    U, S, V = (out[x].cpu().numpy() for x in ("U", "S", "V"))
    Uo, So, Vo, det = O.rsvd(A, k, p, q, SEED, return_details=True)
    check_svd(A, U, S, V, Uo, So, Vo)
    d = O.qb_id(A, k, p, q, SEED)
    npre = pivot_prefix(d['pivot_norms'], d['second_norms'], 1e-8)
    J = out["J"].cpu().numpy()
    assert np.array_equal(J[:npre], d['J'][:npre])
    if npre == k:
        T = out["T"].cpu().numpy()
        assert np.abs(T - d['T']).max() <= 1e-7 * max(1.0, np.abs(d['T']).max())


def test_exact_rank_recovery(R):
    A, s, _, _ = W.exact_rank_matrix(700, 400, 9, seed=4)
    k, p, q = 12, 8, 1                     # rank 9 < l = 20: orth meets dependent columns
    U, S, V, info = R.svd(dev(A), k, p, q, SEED)
    U, S, V, info = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info.cpu().numpy()
    assert info[0] & R.INFO_ORTH_FALLBACK
    assert np.max(np.abs(S[:9] - s) / s) < 1e-12
    assert np.all(S[9:] < 1e-13 * s[0])
    assert np.linalg.norm(A - (U * S) @ V.T, 2) < 1e-13 * s[0]
    assert orth_err(U[:, :9]) < 1e-12 and orth_err(V[:, :9]) < 1e-12


def test_separated_skeleton(R):
    m, n, r = 3000, 5000, 60
    A, pi, d = W.separated_skeleton_matrix(m, n, r, seed=17)
    k, p, q = 40, 20, 1                    # l = r: Q Q^T A = A
    J, T, info = R.id(dev(A), k, p, q, SEED)
    assert list(J.cpu().numpy()[:k]) == list(pi[:k])


def test_fp32_path(R, c1):
    A, s = c1
    A32 = A.astype(np.float32)
    k, p, q = 20, 10, 1
    U, S, V, info = R.svd(dev(A32, torch.float32), k, p, q, SEED)
    S = S.cpu().numpy()
    U, V = U.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
    Uo, So, Vo = O.rsvd(A32.astype(np.float64), k, p, q, SEED)
    # FP32 storage and passes: sigma to ~1e-5 relative of sigma_1
    assert np.abs(S - So).max() < 1e-5 * So[0]
    assert orth_err(U) < 1e-5 and orth_err(V) < 1e-5
    assert subspace_gap(U[:, :10], Uo[:, :10]) < 1e-3


def test_deterministic(R, c1):
    A, _ = c1
    Ad = dev(A)
    a = R.decompose(Ad, 20, 10, 1, SEED)
    b = R.decompose(Ad, 20, 10, 1, SEED)
    for key in ("U", "S", "V", "J", "T", "Jr", "Ucur"):
        assert torch.equal(a[key], b[key]), key


def test_decompose_matches_single_calls(R, c1):
    A, _ = c1
    Ad = dev(A)
    out = R.decompose(Ad, 20, 10, 1, SEED)
    U, S, V, _ = R.svd(Ad, 20, 10, 1, SEED)
    J, T, _ = R.id(Ad, 20, 10, 1, SEED)
    Jc, Jr, Uc, _ = R.cur(Ad, 20, 10, 1, SEED)
    assert torch.equal(out["S"], S) and torch.equal(out["U"], U)
    assert torch.equal(out["J"], J) and torch.equal(out["T"], T)
    assert torch.equal(out["Jr"], Jr) and torch.equal(out["Ucur"], Uc)


def test_zero_matrix(R):
    # every sample column is dependent: orth replaces them all, sigma = 0,
    # the pivoted QR reports numerical rank 0 and picks the lowest indices
    A = np.zeros((300, 200))
    out = R.decompose(dev(A), 5, 5, 1, SEED)
    info = out["info"].cpu().numpy()
    assert np.all(out["S"].cpu().numpy() == 0.0)
    assert info[0] & R.INFO_ORTH_FALLBACK
    assert info[0] & R.INFO_RANK and info[1] == 0
    assert orth_err(out["U"].cpu().numpy()) < 1e-12
    J = out["J"].cpu().numpy()
    assert np.array_equal(np.sort(J), np.arange(200))
    assert np.all(np.isfinite(out["T"].cpu().numpy()))


def test_rank_one(R):
    g = np.random.default_rng(11)
    u, v = g.standard_normal(400), g.standard_normal(250)
    A = np.outer(u, v)
    U, S, V, info = R.svd(dev(A), 3, 4, 1, SEED)
    S = S.cpu().numpy()
    s1 = np.linalg.norm(u) * np.linalg.norm(v)
    assert abs(S[0] - s1) <= 1e-13 * s1
    assert np.all(S[1:] <= 1e-13 * s1)


@pytest.mark.parametrize("m,n,k,p,q", [(150, 900, 12, 6, 1), (900, 150, 12, 6, 2), (96, 96, 96, 0, 0),
                                       (1, 40, 1, 3, 1), (40, 1, 1, 0, 0)])
def test_shapes_id_cur(R, m, n, k, p, q):
    A, s = W.logspace_type(m, n, 2, seed=m + 7 * n)
    out = R.decompose(dev(A), k, p, q, SEED)
    c = O.cur(A, k, p, q, SEED)
    J, Jr = out["J"].cpu().numpy(), out["Jr"].cpu().numpy()
    npre = pivot_prefix(c["pivot_norms"], c["second_norms"], 1e-8)
    assert np.array_equal(J[:npre], c["J"][:npre])
    assert np.array_equal(np.sort(J), np.arange(n))
    if npre == k:
        nr = pivot_prefix(c["row_pivot_norms"], c["row_second_norms"], 1e-8)
        assert np.array_equal(Jr[:nr], c["Jr"][:nr])
        if nr == k:
            Uc = out["Ucur"].cpu().numpy()
            assert np.abs(Uc - c["U"]).max() <= 1e-6 * max(1.0, np.abs(c["U"]).max())
