"""Parity at full size: the 20000 x 10000 FP64 matrix with sigma_j = 1/j plus
N(0, (1e-6)^2) noise, k = 200, p = 20, q = 2, in the launch configuration the
benchmark times (one rsvd_decompose call with every output), against the FP64
oracle on the same A and seed (needs a GPU; the oracle takes ~40 s).

Bar: sigma relative error <= 1e-10; U, V orthonormal and U^T A V = diag(S)
(a property of the method at any size: U^T A V = Vh^T B Qh Uh = diag(S));
skeleton and CUR row indices identical to the oracle's up to the first
near-tie of the pivot norms (margin 1e-8); T and the CUR factor within a
rounding-level tolerance where the indices agree.

The same step with A stored in BF16, against the oracle run on the BF16
values of A: sigma within 1e-3 relative, the range-finder residual
||A - Q Q^T A||_F within 1% of the oracle's, and the skeleton identical up to
the first pivot margin below 1e-2.
"""

import numpy as np
import pytest
import torch

from oracle import rsvd as O
from paper_1502_05366_amd import workloads as W
from tests.helpers import orth_err, pivot_prefix

pytestmark = pytest.mark.gpu
K, P, Q, SEED = 200, 20, 2, 0x5EED0001


@pytest.fixture(scope="module")
def c2():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print("C2: generating A", flush=True)
    A, _ = W.c2_matrix()
    Ad = torch.from_numpy(A).cuda()
    print("C2: rsvd_decompose on the GPU", flush=True)
    out = R.decompose(Ad, K, P, Q, SEED)
    torch.cuda.synchronize()
    print("C2: oracle", flush=True)
    Uo, So, Vo, det = O.rsvd(A, K, P, Q, SEED, return_details=True)
    c = O.cur(A, K, P, Q, SEED, Q=det["Q"])
    return dict(A=A, Ad=Ad, out=out, So=So, c=c)


def test_c2_sigma_and_info(c2):
    S = c2["out"]["S"].cpu().numpy()
    So = c2["So"]
    assert np.max(np.abs(S - So) / So) <= 1e-10
    assert int(c2["out"]["info"].cpu()[0]) == 0


def test_c2_singular_vectors(c2):
    U, S, V = (c2["out"][x] for x in ("U", "S", "V"))
    assert orth_err(U.cpu().numpy()) < 1e-12 and orth_err(V.cpu().numpy()) < 1e-12
    # U^T A V = diag(S): each entry is a sum of m n terms, rounding ~ n eps ||A||
    M = (U.T @ (c2["Ad"] @ V)).cpu().numpy()
    D = np.diag(S.cpu().numpy())
    assert np.abs(M - D).max() <= 1e-11


def test_c2_id(c2):
    J = c2["out"]["J"].cpu().numpy()
    T = c2["out"]["T"].cpu().numpy()
    c = c2["c"]
    npre = pivot_prefix(c["pivot_norms"], c["second_norms"], 1e-8)
    assert npre >= 1
    assert np.array_equal(J[:npre], c["J"][:npre])
    assert np.array_equal(np.sort(J), np.arange(len(J)))
    if npre == K:
        assert np.array_equal(J, c["J"])
        assert np.abs(T - c["T"]).max() <= 1e-8 * max(1.0, np.abs(c["T"]).max())


def test_c2_cur(c2):
    c = c2["c"]
    Jr = c2["out"]["Jr"].cpu().numpy()
    Uc = c2["out"]["Ucur"].cpu().numpy()
    npre = pivot_prefix(c["pivot_norms"], c["second_norms"], 1e-8)
    nr = pivot_prefix(c["row_pivot_norms"], c["row_second_norms"], 1e-8)
    if npre < K:
        pytest.skip("column pivots not unique at this seed (near-tie at step %d)" % npre)
    assert np.array_equal(Jr[:nr], c["Jr"][:nr])
    if nr == K:
        assert np.abs(Uc - c["U"]).max() <= 1e-7 * np.abs(c["U"]).max()


def test_c2_fp32(c2):
    """The same matrix stored in FP32 (passes on the FP32 matrix cores, FP64
    after them), against the FP64 oracle on the FP64 matrix. Rounding A to
    FP32 moves each sigma by at most ||A - fl32(A)||_2 <= 2^-24 ||A||_F
    (~8e-8 here); the passes add O(sqrt(n) 2^-24 sigma_1). Bar 1e-5 sigma_1,
    as for the small FP32 case."""
    import paper_1502_05366_amd as R
    A32 = c2["Ad"].float()
    out = R.decompose(A32, K, P, Q, SEED)
    torch.cuda.synchronize()
    So = c2["So"]
    S = out["S"].cpu().numpy()
    assert int(out["info"].cpu()[0]) == 0
    assert np.abs(S - So).max() <= 1e-5 * So[0]
    U = out["U"].double()
    V = out["V"].double()
    assert orth_err(U.cpu().numpy()) < 1e-5 and orth_err(V.cpu().numpy()) < 1e-5
    M = (U.T @ (A32.double() @ V)).cpu().numpy()
    assert np.abs(M - np.diag(S)).max() <= 1e-5 * So[0]
    c = c2["c"]
    J = out["J"].cpu().numpy()
    npre = pivot_prefix(c["pivot_norms"], c["second_norms"], 1e-4)
    assert np.array_equal(J[:npre], c["J"][:npre])
    assert np.array_equal(np.sort(J), np.arange(len(J)))


def test_c2_id_left(c2):
    """The left-sketch ID (Alg. 6, eq. (Ypower)) at full size against the
    oracle's: skeleton up to the first near-tie of the pivot norms, T where
    all pivots agree."""
    import paper_1502_05366_amd as R
    J, T, info = R.id_left(c2["Ad"], K, P, Q, SEED)
    torch.cuda.synchronize()
    J, T = J.cpu().numpy(), T.cpu().numpy()
    d = O.id_left(c2["A"], K, P, Q, SEED)
    assert np.array_equal(np.sort(J), np.arange(len(J)))
    npre = pivot_prefix(d["pivot_norms"], d["second_norms"], 1e-8)
    assert npre >= 1
    assert np.array_equal(J[:npre], d["J"][:npre])
    if npre == K:
        assert np.array_equal(J, d["J"])
        assert np.abs(T - d["T"]).max() <= 1e-8 * max(1.0, np.abs(d["T"]).max())


def test_c2_qb(c2):
    """Blocked adaptive QB (Alg. 7) at full size, b = 32, q = 1, tol = 0.07, at
    most 10 blocks (on sigma_j = 1/j the residual crosses tol with the 8th):
    the same blocks, Q, B and residual as the oracle's."""
    import paper_1502_05366_amd as R
    A = c2["A"]
    Q, B, res, Rd, info = R.qb(c2["Ad"], 32, 10, 1, 0.07, SEED)
    Q, B = Q.cpu().numpy(), B.cpu().numpy()
    del Rd
    d = O.qb_blocked(A, 32, 10, 0.07, 1, SEED)
    assert d["nblocks"] < 10 and d["norms"][-1] < 0.07
    assert Q.shape[1] == d["Q"].shape[1]
    assert np.abs(Q - d["Q"]).max() <= 1e-9
    assert np.abs(B - d["B"]).max() <= 1e-9
    assert abs(res - d["norms"][-1]) <= 1e-9


@pytest.fixture(scope="module")
def c2_bf16(c2):
    """The same workload with A stored in BF16 (rounded to nearest even from
    FP64), against the oracle run on those BF16 values."""
    import paper_1502_05366_amd as R
    from oracle import quant as QZ
    Ab = QZ.bf16_round(c2["A"])
    Ad = torch.as_tensor(Ab, device="cuda").to(torch.bfloat16)     # exact
    print("C2 BF16: rsvd_decompose and rsvd_svd_ex on the GPU", flush=True)
    out = R.decompose(Ad, K, P, Q, SEED)
    _, Sx, _, info, Qb = R.svd_ex(Ad, K, P, Q, SEED, want_Q=True)
    torch.cuda.synchronize()
    print("C2 BF16: oracle", flush=True)
    Uo, So, Vo, det = O.rsvd(Ab, K, P, Q, SEED, return_details=True)
    c = O.cur(Ab, K, P, Q, SEED, Q=det["Q"])
    return dict(Ab=Ab, out=out, Sx=Sx.cpu().numpy(), Qb=Qb.cpu().numpy().astype(np.float64),
                So=So, Qo=det["Q"], c=c)


def test_c2_bf16_sigma(c2_bf16):
    d = c2_bf16
    S = d["out"]["S"].cpu().numpy()
    assert np.max(np.abs(S - d["So"]) / d["So"]) <= 1e-3
    assert np.max(np.abs(d["Sx"] - d["So"]) / d["So"]) <= 1e-3
    assert int(d["out"]["info"].cpu()[0]) == 0


def test_c2_bf16_range_residual(c2_bf16):
    # ||A - Q Q^T A||_F with the GPU's basis against the oracle's (same BF16 A)
    d = c2_bf16
    Ab, Qg, Qo = d["Ab"], d["Qb"], d["Qo"]
    rg = np.linalg.norm(Ab - Qg @ (Qg.T @ Ab))
    ro = np.linalg.norm(Ab - Qo @ (Qo.T @ Ab))
    print("C2 BF16 ||A - QQ^T A||_F: GPU %.6e oracle %.6e" % (rg, ro), flush=True)
    assert abs(rg / ro - 1.0) <= 1e-2


def test_c2_bf16_skeleton_prefix(c2_bf16):
    # identical skeleton up to the first pivot whose margin is below 1e-2 (the
    # BF16 passes perturb B by ~1e-3 relative, so closer pivots may swap)
    d = c2_bf16
    J = d["out"]["J"].cpu().numpy()
    c = d["c"]
    npre = pivot_prefix(c["pivot_norms"], c["second_norms"], 1e-2)
    print("C2 BF16 skeleton prefix with margin >= 1e-2: %d" % npre, flush=True)
    assert np.array_equal(J[:npre], c["J"][:npre])
    assert np.array_equal(np.sort(J), np.arange(len(J)))
