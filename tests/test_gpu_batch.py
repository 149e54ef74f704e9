"""Parity of the batched randomized SVD (one persistent launch over many
uneven FP32 matrices) with the FP64 oracle (needs a GPU), through the C-ABI
entry points rsvd_batch_*.

The oracle is oracle.rsvd.batch_rsvd: matrix i of the batch with the sketch
of Philox batch index i, on the FP32 values of A_i taken exactly in FP64.
The GPU path runs the products on the FP32 matrix cores (FP32 accumulation),
so its perturbation of B is of the order of the FP32 rounding of the passes,
~ sqrt(n) eps_32 sigma_1 ~ 2e-6 sigma_1.  Hence, per singular value, sigma_i
within 1e-5 sigma_i + 32 eps_32 sigma_1 of the oracle's (relative where
sigma_i is large, the FP32 floor in the tail); the singular vectors, once
their signs are aligned, within 64 eps_32 sigma_1 / gap_i + 1e-5 element by
element (gap_i the distance of sigma_i to its neighbours) wherever that
bound is below 0.05; ||U S V^T - U_o S_o V_o^T||_F within 2e-5 sigma_1.
Also: U and V orthonormal to 1e-5, exact recovery at exact rank <= k, edge
shapes (l = min(m, n), l = 80, tiny m or n, k = 1), q = 0, 1, 2, replays of
a captured graph equal to the eager call bit for bit, determinism, and the
4096-matrix workload (sampled matrices against the oracle, properties on
all of them).
"""

import numpy as np
import pytest
import torch

from oracle import rsvd as O
from paper_1502_05366_amd import workloads as W
from tests.helpers import align_signs

pytestmark = pytest.mark.gpu
SEED = 0x5EED0004


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def spectrum_batch(ms, ns, seed):
    return [W.spectrum_matrix(int(m), int(n), W.c4_spectrum(int(m), int(n)), seed + i)[0]
            .astype(np.float32) for i, (m, n) in enumerate(zip(ms, ns))]


def run_batch(R, As, ms, ns, ks, p, q, seed=SEED, variants=None):
    plan = R.BatchPlan(ms, ns, ks, p, q, variants=variants)
    buf = plan.pack([torch.from_numpy(A) for A in As])
    U, S, V, info = plan.run(buf, seed)
    torch.cuda.synchronize()
    res = [(u.cpu().numpy().astype(np.float64), s.cpu().numpy(), v.cpu().numpy().astype(np.float64))
           for u, s, v in plan.unpack(U, S, V)]
    return res, info.cpu().numpy(), plan


def check_against_oracle(As, ks, res, p, q, seed=SEED, idx=None):
    """As, ks, res indexed by the matrices' batch indices (lists or dicts)."""
    idx = range(len(As)) if idx is None else idx
    for i in idx:
        A = As[i].astype(np.float64)
        Uo, So, Vo = O.rsvd(A, int(ks[i]), p, q, seed, batch=i)
        U, S, V = res[i]
        s1 = So[0]
        eps32 = float(np.finfo(np.float32).eps)
        assert np.all(np.isfinite(S)) and np.all(np.diff(S) <= 0), i
        assert np.all(np.abs(S - So) <= 1e-5 * So + 32 * eps32 * s1), \
            (i, (np.abs(S - So) / So).max())
        # sign-aligned singular vectors where sigma_i is separated
        gaps = np.minimum(np.r_[np.inf, So[:-1] - So[1:]], np.r_[So[:-1] - So[1:], So[-1]])
        tol = 64 * eps32 * s1 / np.maximum(gaps, 1e-300) + 1e-5
        ok = tol < 0.05
        Ua, Va = align_signs(U, Uo), align_signs(V, Vo)
        if np.any(ok):
            assert np.all(np.abs(Ua - Uo).max(axis=0)[ok] <= tol[ok]), i
            assert np.all(np.abs(Va - Vo).max(axis=0)[ok] <= tol[ok]), i
        d = np.linalg.norm((U * S) @ V.T - (Uo * So) @ Vo.T)
        assert d <= 2e-5 * s1, (i, d / s1)
        k = U.shape[1]
        assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5, i
        assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-5, i


@pytest.mark.parametrize("q", [1, 0, 2])
def test_batch_parity_uneven(R, q):
    g = np.random.default_rng(40 + q)
    count = 24 if q == 1 else 10
    ms = g.integers(16, 601, count)
    ns = g.integers(16, 401, count)
    ks = np.minimum(g.integers(1, 65, count), np.minimum(ms, ns))
    print("batch parity q=%d count=%d" % (q, count), flush=True)
    As = spectrum_batch(ms, ns, 100 * q)
    res, info, _ = run_batch(R, As, ms, ns, ks, 8, q)
    assert info[0] == 0, info
    check_against_oracle(As, ks, res, 8, q)


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_batch_pass_shapes(R, shape):
    """Every pass shape of the autotuner's menu gives the oracle's result (the
    shapes change only the order of the FP32 sums): sizes across one and
    several row and column tiles of each shape (128 and 256), ragged."""
    g = np.random.default_rng(60 + shape)
    ms = np.r_[g.integers(16, 900, 9), 255, 257, 513]
    ns = np.r_[g.integers(16, 700, 9), 300, 129, 64]
    ks = np.minimum(np.r_[g.integers(1, 73, 9), 60, 8, 40], np.minimum(ms, ns))
    print("batch pass shape %d" % shape, flush=True)
    As = spectrum_batch(ms, ns, 300 + shape)
    res, info, plan = run_batch(R, As, ms, ns, ks, 8, 1, variants=shape)
    assert np.all(plan.variants == shape)
    assert info[0] == 0, info
    check_against_oracle(As, ks, res, 8, 1)


def test_batch_plan_uses_tuned_table(R):
    from paper_1502_05366_amd import batch_tune
    ms, ns, ks = np.array([100, 600, 1500, 2000]), np.array([90, 1500, 300, 2000]), \
        np.array([5, 40, 60, 20])
    plan = R.BatchPlan(ms, ns, ks, 8, 1)
    ls = np.minimum(ks + 8, np.minimum(ms, ns))
    assert np.array_equal(plan.variants, batch_tune.choose(ms, ns, ls))


def test_batch_edge_shapes(R):
    # l = min(m, n); l = 80 exactly; tiny m / n; k = 1; k = min(m, n); 1 x 1
    shapes = [(16, 16, 16), (40, 24, 20), (500, 300, 72), (3, 5, 1), (1, 1, 1), (7, 200, 7),
              (300, 9, 2), (129, 130, 64), (2048, 64, 60), (64, 1024, 33)]
    ms = np.array([s[0] for s in shapes])
    ns = np.array([s[1] for s in shapes])
    ks = np.array([s[2] for s in shapes])
    print("batch edge shapes", flush=True)
    As = spectrum_batch(ms, ns, 7)
    res, info, plan = run_batch(R, As, ms, ns, ks, 8, 1)
    assert info[0] == 0, info
    check_against_oracle(As, ks, res, 8, 1)
    assert np.all(plan.lda % 4 == 0) and np.all(plan.lda >= plan.ns)
    assert np.all(plan.a_off % 4 == 0)


def test_batch_exact_rank(R):
    ms, ns, ks = np.array([300, 120, 77]), np.array([200, 260, 77]), np.array([12, 9, 20])
    As = []
    for i, (m, n, k) in enumerate(zip(ms, ns, ks)):
        A, _, _, _ = W.exact_rank_matrix(int(m), int(n), int(k) - 2, seed=30 + i)
        As.append(A.astype(np.float32))
    print("batch exact rank", flush=True)
    res, info, _ = run_batch(R, As, ms, ns, ks, 6, 1)
    # the samples of rank k - 2 < l have dependent columns: they are replaced
    # by fresh Gaussian columns (info bit 1), so the bases stay orthonormal
    assert info[0] & R.INFO_ORTH_FALLBACK
    assert not info[0] & (R.INFO_NONFINITE | R.INFO_JACOBI_CAP)
    for A, (U, S, V) in zip(As, res):
        A = A.astype(np.float64)
        assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-5 * np.linalg.norm(A)
        k = U.shape[1]
        assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-5
        assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-5


def test_batch_nonfinite_reported(R):
    ms, ns, ks = np.array([200, 150]), np.array([120, 90]), np.array([10, 8])
    As = spectrum_batch(ms, ns, 17)
    As[1][5, 7] = np.nan
    print("batch with a NaN entry", flush=True)
    res, info, _ = run_batch(R, As, ms, ns, ks, 6, 1)
    assert info[0] & R.INFO_NONFINITE
    # the finite matrix is unaffected
    Uo, So, Vo = O.rsvd(As[0].astype(np.float64), 10, 6, 1, SEED, batch=0)
    assert np.abs(res[0][1] - So).max() <= 1e-5 * So[0]


def test_batch_graph_replay_and_determinism(R):
    g = np.random.default_rng(9)
    count = 40
    ms = g.integers(16, 700, count)
    ns = g.integers(16, 500, count)
    ks = np.minimum(g.integers(1, 65, count), np.minimum(ms, ns))
    As = spectrum_batch(ms, ns, 55)
    plan = R.BatchPlan(ms, ns, ks, 8, 1)
    buf = plan.pack([torch.from_numpy(A) for A in As])
    print("batch graph replay", flush=True)
    out = plan.outputs()
    plan.run(buf, SEED, out)
    torch.cuda.synchronize()
    ref = [t.clone() for t in out[:3]]
    plan.run(buf, SEED, out)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(out[:3], ref))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(buf, SEED, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(buf, SEED, out)
    for rep in range(3):
        for t in out[:3]:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(out[:3], ref)), rep
        assert int(out[3][0].item()) == 0


def test_batch_unsupported(R):
    with pytest.raises(R.RsvdError):
        R.BatchPlan([200], [100], [80], 8, 1)          # l = 88 > 80
    with pytest.raises(R.RsvdError):
        R.BatchPlan([20], [10], [11], 8, 1)            # k > min(m, n)


def test_batch_c4_full(R):
    """The 4096-matrix workload: m ~ U{64..2048}, n ~ U{64..1024},
    k ~ U{4..64}, p = 8, q = 1, sigma_j = exp(-j/8).  Eight sampled matrices
    (the largest, the smallest, six others) against the oracle; on all:
    sigma_1 within the interlacing bound, and on every 97th matrix S finite
    and descending, U and V orthonormal."""
    ms, ns, ks = W.c4_dims()
    print("batch C4 generate", flush=True)
    As = W.c4_batch_torch(ms, ns, 0xC0FFEE04, "cuda")
    plan = R.BatchPlan(ms, ns, ks, 8, 1)
    buf = plan.pack(As)
    print("batch C4 run", flush=True)
    U, S, V, info = plan.run(buf, SEED)
    torch.cuda.synchronize()
    assert int(info[0].item()) == 0
    views = plan.unpack(U, S, V)
    s1 = torch.stack([s[0] for _, s, _ in views]).cpu().numpy()
    # interlacing: the singular values of Q^T A never exceed those of A (up
    # to the FP32 rounding of A and of the passes, the 1e-5 sigma_1 of the
    # parity bar); with l as small as 12 on this slowly decaying spectrum the
    # randomized sigma_1 lies up to ~1e-3 below the exact value
    assert np.all(s1 <= np.exp(-1 / 8) * (1 + 1e-5))
    assert np.all(s1 >= np.exp(-1 / 8) * (1 - 5e-3))
    for u, s, v in views[::97]:
        sn = s.cpu().numpy()
        assert np.all(np.isfinite(sn)) and np.all(np.diff(sn) <= 0)
        un, vn = u.double().cpu().numpy(), v.double().cpu().numpy()
        k = un.shape[1]
        assert np.abs(un.T @ un - np.eye(k)).max() <= 1e-5
        assert np.abs(vn.T @ vn - np.eye(k)).max() <= 1e-5
    work = ms * ns
    others = np.random.default_rng(3).choice(len(ms), 6, replace=False)
    pick = [int(np.argmax(work)), int(np.argmin(work))] + [int(i) for i in others]
    print("batch C4 oracle on %s" % pick, flush=True)
    res = {i: (views[i][0].double().cpu().numpy(), views[i][1].cpu().numpy(),
               views[i][2].double().cpu().numpy()) for i in pick}
    Anp = {i: As[i].cpu().numpy() for i in pick}
    check_against_oracle(Anp, ks, res, 8, 1, idx=pick)


def test_batch_single_matrix_max_l(R):
    """A batch of one (a grid of one workgroup) at l = 80, q = 2."""
    ms, ns, ks = np.array([700]), np.array([450]), np.array([72])
    print("batch single matrix", flush=True)
    As = spectrum_batch(ms, ns, 77)
    res, info, _ = run_batch(R, As, ms, ns, ks, 8, 2)
    assert info[0] == 0, info
    check_against_oracle(As, ks, res, 8, 2)


def test_batch_rejects_unprepared_workspace(R):
    """A workspace that did not receive the descriptors is refused before
    any launch."""
    import ctypes
    from paper_1502_05366_amd import _lib
    plan = R.BatchPlan([100, 80], [60, 90], [5, 6], 8, 1)
    buf = plan.pack([torch.zeros(100, 60), torch.zeros(80, 90)])
    U, S, V, info = plan.outputs()
    other = torch.empty_like(plan.work)
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _lib.load().rsvd_batch_svd(plan._plan, 1, P(buf), P(U), P(S), P(V), P(other),
                                    other.numel(), P(info), stream)
    assert rc == -7
    plan.run(buf, 1)                                      # the prepared one works
    torch.cuda.synchronize()
