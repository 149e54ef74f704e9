"""Throughput of the randomized SVD + ID + CUR path on one MI355X.

One step = one rsvd_decompose call on the 20000 x 10000 FP64 matrix with
sigma_j = 1/j plus N(0, (1e-6)^2) noise, k = 200, p = 20, q = 2: the Gaussian
sketch, 6 passes over A with CholeskyQR2 between them, the Jacobi SVD of the
small factor with U, V, the k-step pivoted QR of B with T, and the CUR
post-processing.  A is resident in HBM before timing starts.

GFLOP/s counts the algorithmic work of the RSVD only:
  F = 2(2q+2) m n l + (q+1)(2 m l^2 - 2/3 l^3) + (q+1)(2 n l^2 - 2/3 l^3)
      + 2 (m + n) l k
(passes, Householder-count orthonormalization, U and V); the ID and CUR work
is timed but not credited.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
                       [--grad-only] [--batch-only]
"""

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RSVD GFLOP/s + % HBM roofline; BF16 vs FP64 speedup at stated σ error"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0


# HBM bytes of one pass over A (Y = A X and Z = A^T X averaged), from the
# FETCH_SIZE and WRITE_SIZE counters of two rocprofv3 --pmc runs of this
# script, each scaled by counter/bytes of the plain 1 GiB copy kernel timed
# below; valid only while the pass kernel's sources hash to "sources".
PASS_TRAFFIC = {"sources": "fc2a4138c2a8871c57e6d256b627da01351229dcf28ef61f39e02b7dbe4b90c7",
                "bytes": 4589000000}
PASS_SOURCES = ("paper_1502_05366_amd/csrc/gemm.hip",)


def pass_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pass_traffic():
    if PASS_TRAFFIC is None or PASS_TRAFFIC["sources"] != pass_sources_hash():
        return None
    return PASS_TRAFFIC["bytes"]


def alg_flops(m, n, k, p, q):
    l = min(k + p, m, n)
    return (2 * (2 * q + 2) * m * n * l + (q + 1) * (2 * m * l * l - 2 * l ** 3 / 3)
            + (q + 1) * (2 * n * l * l - 2 * l ** 3 / 3) + 2 * (m + n) * l * k)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, k, p, q, seed, single_run_s=20.0):
    """The FP64 oracle (RSVD + ID + CUR) on the same 20000 x 10000 A and seed
    as the GPU step, on all host threads: median of 3 runs, or one run when a
    run takes longer than single_run_s.  Plus the oracle's RSVD on the
    2000 x 1000 plain-RSVD workload on one thread (median of 3)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import rsvd as O
    from paper_1502_05366_amd import workloads as W

    m, n = A.shape
    times = []
    while True:
        t0 = time.perf_counter()
        O.rsvd(A, k, p, q, seed)
        O.cur(A, k, p, q, seed)
        times.append(time.perf_counter() - t0)
        if len(times) == 3 or times[0] > single_run_s:
            break
    t = float(np.median(times))
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    f = alg_flops(m, n, k, p, q)
    A1, _ = W.c1_matrix()
    t1 = []
    with threadpool_limits(1):
        for _ in range(3):
            t0 = time.perf_counter()
            O.rsvd(A1, 20, 10, 1, 0x5EED0000)
            t1.append(time.perf_counter() - t0)
    t1m = float(np.median(t1))
    return {"value": round(f / t / 1e9, 3), "unit": "GFLOP/s", "cores": int(threads),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "oracle RSVD+ID+CUR on the full %d x %d matrix of the GPU step (same A and "
                      "seed), k=%d p=%d q=%d; median of %d run(s): %s s; GFLOP/s with the same "
                      "RSVD flop count" % (m, n, k, p, q, len(times),
                                           ", ".join("%.1f" % x for x in times)),
            "c1_one_thread": {"ms": round(1e3 * t1m, 1),
                              "value_gflops": round(alg_flops(2000, 1000, 20, 10, 1) / t1m / 1e9,
                                                    3),
                              "runs_ms": [round(1e3 * x, 1) for x in t1],
                              "sample": "oracle RSVD on the 2000 x 1000 plain-RSVD matrix "
                                        "(sigma_j = 10^(-j/10)), k=20 p=10 q=1, one thread, "
                                        "median of 3"}}


def c1_graph_step(lib, h, args, stream, sp, P, e0, e1):
    """The plain-RSVD workload (2000 x 1000 FP64, sigma_j = 10^(-j/10), k = 20,
    p = 10, q = 1): one rsvd_svd call captured into a graph and replayed; the
    per-call wall time of the replays and the sigma error against the oracle."""
    import numpy as np
    import torch
    from oracle import rsvd as O
    from paper_1502_05366_amd import api, workloads as W

    dev = torch.device("cuda:0")
    A_np, _ = W.c1_matrix()
    A = torch.from_numpy(A_np).to(dev)
    m, n = A.shape
    k, p, q, seed = 20, 10, 1, 0x5EED0000
    wb = lib.rsvd_workspace_bytes(api.OP_SVD, api.F64, m, n, k, p, q)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    U = torch.empty((m, k), dtype=torch.float64, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=torch.float64, device=dev)

    def call(st):
        rc = lib.rsvd_svd(h, api.F64, m, n, k, p, q, seed, P(A), n, P(U), k, P(S), P(V), k,
                          P(work), wb, P(info), ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError("rsvd_svd returned %d" % rc)

    call(stream)
    torch.cuda.synchronize()
    S_eager = S.cpu().numpy().copy()
    # eager timing
    e0.record(stream)
    for _ in range(50):
        call(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / 50
    # capture on a side stream, replay on it
    gs = torch.cuda.Stream(device=dev)
    gs.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(g, stream=gs):
            call(gs)
    torch.cuda.synchronize()
    ok = True
    for _ in range(3):
        S.zero_()
        g.replay()
        torch.cuda.synchronize()
        ok = ok and np.array_equal(S.cpu().numpy(), S_eager)
    reps = 200
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) / reps * 1e3
    _, So, _ = O.rsvd(A_np, k, p, q, seed)
    rel = float(np.max(np.abs(S_eager - So) / So))
    return {"workload": "plain RSVD, FP64 A 2000x1000, sigma_j=10^(-j/10), k=20 p=10 q=1",
            "graph_replay_wall_ms": round(wall_ms, 4), "eager_event_ms": round(eager_ms, 4),
            "value_gflops": round(alg_flops(m, n, k, p, q) / (wall_ms * 1e-3) / 1e9, 1),
            "replays_match_eager": bool(ok), "sigma_rel_err_vs_oracle": rel,
            "info": [int(x) for x in info.cpu().numpy()]}


def id_left_flops(m, n, k, p, q):
    """Algorithmic flops of the left-sketch ID (Alg. 6 with eq. (Ypower)):
    2q+1 passes over A and 2q orthonormalizations at the Householder count
    (the pivoted QR of the l x n sample and T are not credited)."""
    l = min(k + p, m, n)
    return (2 * (2 * q + 1) * m * n * l + q * (2 * m * l * l - 2 * l ** 3 / 3)
            + q * (2 * n * l * l - 2 * l ** 3 / 3))


def id_left_step(lib, h, A, m, n, k, p, q, seed, args, stream, sp, P, e0, e1):
    """Time rsvd_id_left (FP64 A resident in HBM) at the benchmark's shape."""
    import torch
    from paper_1502_05366_amd import api

    dev = A.device
    wb = lib.rsvd_id_left_workspace_bytes(api.F64, m, n, k, p, q)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    J = torch.empty(n, dtype=torch.int64, device=dev)
    T = torch.empty((k, n - k), dtype=torch.float64, device=dev)

    def step():
        rc = lib.rsvd_id_left(h, api.F64, m, n, k, p, q, seed, P(A), n, P(J), P(T), n - k,
                              P(work), wb, P(info), sp)
        if rc != 0:
            raise RuntimeError("rsvd_id_left returned %d" % rc)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log("id_left: %.3f ms/call" % ms)
    st = info.cpu().numpy()
    return {"ms_per_call": round(ms, 4),
            "value_gflops": round(id_left_flops(m, n, k, p, q) / (ms * 1e-3) / 1e9, 2),
            "passes": 2 * q + 1,
            "info": [int(st[0]), int(st[1])],
            "note": "rsvd_id_left, FP64 A, same k, p, q and seed; GFLOP/s = 2(2q+1)mnl + "
                    "q(2ml^2 - 2l^3/3) + q(2nl^2 - 2l^3/3) per call"}


QB_B, QB_M, QB_Q, QB_TOL = 32, 10, 1, 0.07


def qb_step(lib, h, A, m, n, seed, args, stream, sp, P, e0, e1):
    """Time rsvd_qb (blocked adaptive QB, FP64) on a fresh copy of A per call
    (the call deflates its A in place; the copy is outside the timed region).
    b = 32, at most 10 blocks, q = 1, tol = 0.07: on sigma_j = 1/j the residual
    is 0.0704 after 7 blocks and drops below tol with the 8th."""
    import ctypes
    import torch
    from paper_1502_05366_amd import api

    dev = A.device
    b, M, q, tol = QB_B, QB_M, QB_Q, QB_TOL
    wb = lib.rsvd_qb_workspace_bytes(api.F64, m, n, b, M, q)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    Q = torch.empty((m, b * M), dtype=torch.float64, device=dev)
    B = torch.empty((b * M, n), dtype=torch.float64, device=dev)
    Aw = torch.empty_like(A)
    nb = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)

    def call():
        rc = lib.rsvd_qb(h, api.F64, m, n, b, M, q, tol, seed, P(Aw), n, P(Q), b * M, P(B), n,
                         ctypes.byref(nb), ctypes.byref(res), P(work), wb, P(info), sp)
        if rc != 0:
            raise RuntimeError("rsvd_qb returned %d" % rc)

    tot = 0.0
    reps = max(1, min(args.steps, 5))
    for it in range(args.warmup + reps):
        Aw.copy_(A)
        torch.cuda.synchronize()
        e0.record(stream)
        call()
        e1.record(stream)
        torch.cuda.synchronize()
        if it >= args.warmup:
            tot += e0.elapsed_time(e1)
    ms = tot / reps
    k = nb.value
    # per block: 2q+2 passes over A (2mnb flops each), the deflation (2mnb),
    # and the projection on the earlier blocks (4 m (ib) b)
    flops = sum((2 * q + 3) * 2.0 * m * n * b + 4.0 * m * (i * b) * b for i in range(k))
    abytes = k * ((2 * q + 2) * 8.0 * m * n + 16.0 * m * n)
    log("qb: %.3f ms/call, %d blocks, resid %.4g" % (ms, k, res.value))
    st = info.cpu().numpy()
    return {"ms_per_call": round(ms, 4), "blocks": k, "block_size": b, "q": q, "tol": tol,
            "resid_fro": res.value,
            "value_gflops": round(flops / (ms * 1e-3) / 1e9, 2),
            "a_traffic_GBs": round(abytes / (ms * 1e-3) / 1e9, 1),
            "info": [int(st[0]), int(st[1])],
            "note": "rsvd_qb on a fresh FP64 copy of A; flops = sum over blocks of "
                    "(2q+3) 2mnb + 4m(ib)b; a_traffic = (2q+2) reads of A + one read and "
                    "write per block, per second"}


GRAD_K, GRAD_P, GRAD_Q, GRAD_SEED = 64, 16, 2, 0x5EED0005


def grad_step(lib, h, args, stream, sp, P, e0, e1):
    """Time rsvd_svd_grad on the 8192 x 4096 sigma_j = 1/j Kronecker-Haar A
    (k = 64, p = 16, q = 2) in FP64: the recomputed forward alone (U, S, V and
    ||A - Q Q^T A||_F^2), and forward + adjoint for the two losses sum sigma_i
    and ||A - Q Q^T A||_F^2 (cotangents dS = 1, dres = 1)."""
    import torch
    from paper_1502_05366_amd import api, workloads as W

    dev = torch.device("cuda:0")
    k, p, q, seed = GRAD_K, GRAD_P, GRAD_Q, GRAD_SEED
    A_np, _ = W.c5_matrix()
    m, n = A_np.shape
    l = min(k + p, m, n)
    A = torch.from_numpy(A_np).to(dev)
    del A_np
    wb = lib.rsvd_svd_grad_workspace_bytes(api.F64, m, n, k, p, q)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    U = torch.empty((m, k), dtype=torch.float64, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=torch.float64, device=dev)
    r2 = torch.empty(1, dtype=torch.float64, device=dev)
    dS = torch.ones(k, dtype=torch.float64, device=dev)
    dres = torch.ones(1, dtype=torch.float64, device=dev)
    dA = torch.empty((m, n), dtype=torch.float64, device=dev)

    def call(backward):
        rc = lib.rsvd_svd_grad(h, api.F64, m, n, k, p, q, seed, P(A), n, None, k, P(dS), None, k,
                               P(dres), P(dA) if backward else None, n, P(U), k, P(S), P(V), k,
                               P(r2), P(work), wb, P(info), sp)
        if rc != 0:
            raise RuntimeError("rsvd_svd_grad returned %d" % rc)

    res = {}
    reps = max(1, min(args.steps, 10))
    for key, bwd in (("forward", False), ("forward_backward", True)):
        for _ in range(max(1, args.warmup)):
            call(bwd)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            call(bwd)
        e1.record(stream)
        torch.cuda.synchronize()
        res[key] = e0.elapsed_time(e1) / reps
    ms_f, ms_fb = res["forward"], res["forward_backward"]
    # reads of A: forward 2q+2 passes + the residual; adjoint 2q+1 passes +
    # the 2 dres A term; one write of dA
    a_bytes = 8.0 * m * n
    fb_bytes = a_bytes * ((2 * q + 3) + (2 * q + 2) + 1)
    fb_flops = 2.0 * m * n * l * ((2 * q + 3) + (2 * q + 1) + (2 * q + 2))
    st = info.cpu().numpy()
    log("grad: forward %.3f ms, forward+adjoint %.3f ms" % (ms_f, ms_fb))
    out = {"ms_forward": round(ms_f, 4), "ms_forward_backward": round(ms_fb, 4),
           "ms_adjoint": round(ms_fb - ms_f, 4),
           "value_gflops": round(fb_flops / (ms_fb * 1e-3) / 1e9, 2),
           "a_traffic_GBs": round(fb_bytes / (ms_fb * 1e-3) / 1e9, 1),
           "sigma_1": float(S[0].item()), "resid2": float(r2.item()),
           "info": [int(st[0]), int(st[1])],
           "workload": "FP64 A %dx%d, sigma_j=1/j, Kronecker-Haar factors, k=%d p=%d q=%d; "
                       "losses sum sigma_i and ||A - QQ^T A||_F^2 (dS = 1, dres = 1)"
                       % (m, n, k, p, q),
           "note": "one rsvd_svd_grad call per step (recomputed forward, then the adjoint); "
                   "flops = 2mnl ((2q+3) forward + (2q+1) adjoint passes + (2q+2) rank-l "
                   "terms of dA); a_traffic = (4q+6) reads of A + one write of dA, per "
                   "second"}
    del A, dA, work
    torch.cuda.empty_cache()
    return out


BATCH_P, BATCH_Q, BATCH_SEED = 8, 1, 0x5EED0004


def batch_step(lib, args, stream, e0, e1):
    """Time the batched randomized SVD of the 4096 uneven FP32 matrices
    (m ~ U{64..2048}, n ~ U{64..1024}, k ~ U{4..64}, p = 8, q = 1,
    sigma_j = exp(-j/8)): one rsvd_batch_svd call (queue reset + one
    persistent kernel) per step, eagerly and as replays of a captured graph."""
    import numpy as np
    import torch
    import paper_1502_05366_amd as R
    from paper_1502_05366_amd import workloads as W

    ms, ns, ks = W.c4_dims()
    p, q = BATCH_P, BATCH_Q
    As = W.c4_batch_torch(ms, ns, 0xC0FFEE04, "cuda")
    plan = R.BatchPlan(ms, ns, ks, p, q)
    buf = plan.pack(As)
    del As
    torch.cuda.empty_cache()
    out = plan.outputs()
    reps = max(1, min(args.steps, 5))
    for _ in range(max(1, args.warmup)):
        plan.run(buf, BATCH_SEED, out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        plan.run(buf, BATCH_SEED, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / reps
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(buf, BATCH_SEED, out)
    graph.replay()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / reps
    ls = np.minimum(ks + p, np.minimum(ms, ns)).astype(np.float64)
    mf, nf, kf = ms.astype(np.float64), ns.astype(np.float64), ks.astype(np.float64)
    flops = float(np.sum(2 * (2 * q + 2) * mf * nf * ls
                         + (q + 1) * (2 * mf * ls ** 2 - 2.0 / 3 * ls ** 3)
                         + (q + 1) * (2 * nf * ls ** 2 - 2.0 / 3 * ls ** 3)
                         + 2 * (mf + nf) * ls * kf))
    abytes = float(np.sum(4.0 * mf * nf)) * (2 * q + 2)
    st = out[3].cpu().numpy()
    log("batch: %.3f ms per batch (graph replay %.3f ms)" % (ms_eager, ms_graph))
    return {"ms_per_batch": round(ms_eager, 4), "ms_per_batch_graph": round(ms_graph, 4),
            "matrices": int(len(ms)), "matrices_per_s": round(len(ms) / (ms_graph * 1e-3), 1),
            "value_gflops": round(flops / (ms_graph * 1e-3) / 1e9, 2),
            "a_traffic_GBs": round(abytes / (ms_graph * 1e-3) / 1e9, 1),
            "a_bytes_per_batch": abytes, "info": [int(st[0]), int(st[1])],
            "workload": "4096 FP32 matrices, m~U{64..2048}, n~U{64..1024}, k~U{4..64}, "
                        "p=8, q=1, sigma_j=exp(-j/8); one persistent launch per batch",
            "note": "GFLOP/s = sum over matrices of 2(2q+2)mnl + (q+1)(2ml^2-2l^3/3) + "
                    "(q+1)(2nl^2-2l^3/3) + 2(m+n)lk per graph replay; a_traffic = (2q+2) "
                    "reads of every A_i per replay"}


def lowp_step(lib, h, A, m, n, k, p, q, seed, l, args, stream, sp, P, e0, e1, bf16):
    """Time rsvd_decompose with A stored in BF16 (bf16=True) or FP32, and one
    pass over A of that storage type."""
    import torch
    from paper_1502_05366_amd import api

    dev = A.device
    dt = api.BF16 if bf16 else api.F32
    name = "BF16" if bf16 else "FP32"
    Ab = A.to(torch.bfloat16 if bf16 else torch.float32)   # round to nearest even
    ops = api.OP_SVD | api.OP_ID | api.OP_CUR
    wb = lib.rsvd_workspace_bytes(ops, dt, m, n, k, p, q)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    U = torch.empty((m, k), dtype=torch.float32, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=torch.float32, device=dev)
    J = torch.empty(n, dtype=torch.int64, device=dev)
    T = torch.empty((k, n - k), dtype=torch.float64, device=dev)
    Jr = torch.empty(k, dtype=torch.int64, device=dev)
    Uc = torch.empty((k, k), dtype=torch.float64, device=dev)

    def step():
        rc = lib.rsvd_decompose(h, dt, m, n, k, p, q, seed, P(Ab), n, P(U), k, P(S), P(V),
                                k, P(J), P(T), n - k, P(Jr), P(Uc), k, P(work), wb, P(info), sp)
        if rc != 0:
            raise RuntimeError("rsvd_decompose (%s) returned %d" % (name, rc))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log("%s: %.3f ms/step" % (name, ms))
    # one pass in each direction (X in FP32; with BF16 A it is rounded inside)
    X = torch.randn((n, l), dtype=torch.float32, device=dev)
    Xm = torch.randn((m, l), dtype=torch.float32, device=dev)
    Y = torch.empty((m, l), dtype=torch.float32, device=dev)
    Z = torch.empty((n, l), dtype=torch.float32, device=dev)
    pw = max(lib.rsvd_pass_workspace_bytes(dt, 0, m, n, l),
             lib.rsvd_pass_workspace_bytes(dt, 1, m, n, l))
    pwork = torch.empty(pw, dtype=torch.uint8, device=dev)
    pass_ms = {}
    for trans, Xt, Yt, name in ((0, X, Y, "A_X"), (1, Xm, Z, "At_X")):
        for _ in range(3):
            lib.rsvd_pass(h, dt, trans, m, n, l, P(Ab), n, P(Xt), l, P(Yt), l, P(pwork), pw, sp)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.pass_reps):
            lib.rsvd_pass(h, dt, trans, m, n, l, P(Ab), n, P(Xt), l, P(Yt), l, P(pwork), pw, sp)
        e1.record(stream)
        torch.cuda.synchronize()
        pass_ms[name] = e0.elapsed_time(e1) / args.pass_reps
    t_pass = 0.5 * (pass_ms["A_X"] + pass_ms["At_X"])
    st = info.cpu().numpy()
    out = {"ms_per_step": round(ms, 4),
           "value_gflops": round(alg_flops(m, n, k, p, q) / (ms * 1e-3) / 1e9, 2),
           "pass_ms": {kk: round(v, 4) for kk, v in pass_ms.items()},
           "info": [int(st[0]), int(st[1])],
           "S": S.cpu().numpy()}
    if bf16:
        a_gbs = 2.0 * m * n / (t_pass * 1e-3) / 1e9
        out["dtype"] = "bf16 passes (FP32 accumulation), f64 orth / Jacobi / pivoted QR"
        out["pass_roofline"] = {"bound": "hbm", "achieved": round(a_gbs, 1), "peak": PEAK_HBM_GBS,
                                "unit": "GB/s", "frac": round(a_gbs / PEAK_HBM_GBS, 4),
                                "traffic": None,
                                "note": "achieved = 2mn bytes of A per pass / mean pass time"}
    else:
        tf = 2.0 * m * n * l / (t_pass * 1e-3) / 1e12
        out["dtype"] = "f32 passes (FP32 MFMA), f64 orth / Jacobi / pivoted QR"
        out["pass_roofline"] = {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP32_TFLOPS,
                                "unit": "TFLOP/s", "frac": round(tf / PEAK_FP32_TFLOPS, 4),
                                "traffic": None}
    return out


def mhbm_step(lib, h, A, args, stream, sp, P, e0, e1):
    """The HBM-bound supplement: the 20000 x 10000 matrix with k = 20, p = 10,
    q = 1 (l = 30, 7.5 flop per byte of FP64 A: below the ridge points), A in
    FP64 and in FP32.  One rsvd_svd call per step, and one pass over A in each
    direction; the pass rate is the bytes of A per pass over the pass time."""
    import torch
    from paper_1502_05366_amd import api

    dev = A.device
    m, n = A.shape
    k, p, q, seed = 20, 10, 1, 0x5EED0001
    l = min(k + p, m, n)
    out = {"workload": "C2's A (20000x10000, sigma_j=1/j + noise) with k=20 p=10 q=1 (l=30)",
           "k": k, "p": p, "q": q, "l": l}
    for name, dt, tt in (("fp64", api.F64, torch.float64), ("fp32", api.F32, torch.float32)):
        Ax = A if tt == torch.float64 else A.to(tt)
        wb = lib.rsvd_workspace_bytes(api.OP_SVD, dt, m, n, k, p, q)
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
        info = torch.zeros(2, dtype=torch.int32, device=dev)
        U = torch.empty((m, k), dtype=tt, device=dev)
        S = torch.empty(k, dtype=torch.float64, device=dev)
        V = torch.empty((n, k), dtype=tt, device=dev)

        def step():
            rc = lib.rsvd_svd(h, dt, m, n, k, p, q, seed, P(Ax), n, P(U), k, P(S), P(V), k,
                              P(work), wb, P(info), sp)
            if rc != 0:
                raise RuntimeError("rsvd_svd returned %d" % rc)

        for _ in range(2):
            step()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        X = torch.randn((n, l), dtype=tt, device=dev)
        Xm = torch.randn((m, l), dtype=tt, device=dev)
        Y = torch.empty((m, l), dtype=tt, device=dev)
        Z = torch.empty((n, l), dtype=tt, device=dev)
        pw = max(lib.rsvd_pass_workspace_bytes(dt, 0, m, n, l),
                 lib.rsvd_pass_workspace_bytes(dt, 1, m, n, l))
        pwork = torch.empty(max(pw, 1), dtype=torch.uint8, device=dev)
        pass_ms = {}
        for trans, Xt, Yt, key in ((0, X, Y, "A_X"), (1, Xm, Z, "At_X")):
            for _ in range(3):
                lib.rsvd_pass(h, dt, trans, m, n, l, P(Ax), n, P(Xt), l, P(Yt), l, P(pwork), pw,
                              sp)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.pass_reps):
                lib.rsvd_pass(h, dt, trans, m, n, l, P(Ax), n, P(Xt), l, P(Yt), l, P(pwork), pw,
                              sp)
            e1.record(stream)
            torch.cuda.synchronize()
            pass_ms[key] = e0.elapsed_time(e1) / args.pass_reps
        esz = 8 if tt == torch.float64 else 4
        gbs = {kk: esz * m * n / (v * 1e-3) / 1e9 for kk, v in pass_ms.items()}
        t_pass = 0.5 * (pass_ms["A_X"] + pass_ms["At_X"])
        a = esz * m * n / (t_pass * 1e-3) / 1e9
        st = info.cpu().numpy()
        out[name] = {"ms_per_step": round(ms, 4),
                     "value_gflops": round(alg_flops(m, n, k, p, q) / (ms * 1e-3) / 1e9, 1),
                     "info": [int(st[0]), int(st[1])],
                     "pass_ms": {kk: round(v, 4) for kk, v in pass_ms.items()},
                     "pass_roofline": {"bound": "hbm", "achieved": round(a, 1),
                                       "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                       "frac": round(a / PEAK_HBM_GBS, 4),
                                       "per_direction_GBs": {kk: round(v, 1)
                                                             for kk, v in gbs.items()}}}
        log("mhbm %s: %.3f ms/step, passes %s" % (name, ms, out[name]["pass_ms"]))
        del work, U, V, X, Xm, Y, Z, pwork
    return out


def c3_step(lib, h, args, stream, sp, P, e0, e1):
    """The mixed-precision workload: A 65536 x 32768, sigma_j = j^-1.5
    (Kronecker-Haar factors), k = 512, p = 64, q = 2, one rsvd_svd_ex call
    per step with A stored in BF16, in FP8 E4M3 with FP32 column scales, and
    in FP64 (the reference for the speedups).  Errors against the FP64 oracle
    on the same A (tests/golden/c3_oracle.json, written by the committed
    script beside it): sigma relative errors and the range-finder residual
    ||A - Q Q^T A||_F (Q the returned basis, the product formed in FP64)."""
    import numpy as np
    import torch
    from paper_1502_05366_amd import api, workloads as W

    dev = torch.device("cuda:0")
    m, n = W.C3_SHAPE
    k, p, q, seed = 512, 64, 2, 0x5EED0002
    l = min(k + p, m, n)
    gpath = os.path.join(ROOT, "tests", "golden", "c3_oracle.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    log("c3: generating A %dx%d (FP64, on the device)" % (m, n))
    A = W.c3_matrix_torch(dev)
    Ab = api.quantize(A, api.BF16)
    A8, sc = api.quantize(A, api.F8E4M3)
    torch.cuda.synchronize()
    res = {"workload": "A 65536x32768 = (U1[:, :128] kron U2) diag(j^-1.5) (V1 kron V2)^T, "
                       "k=512 p=64 q=2; one rsvd_svd_ex call per step; A resident in HBM in the "
                       "storage format",
           "m": m, "n": n, "k": k, "p": p, "q": q, "l": l}
    sig_o = np.array(golden["fp64"]["sigma"]) if golden else None
    A_fro = float(torch.linalg.vector_norm(A).item())

    def resid_fro(Qb):
        Q64 = Qb.to(torch.float64)
        B = Q64.T @ A
        s2 = 0.0
        for i in range(0, m, 8192):
            D = A[i:i + 8192] - Q64[i:i + 8192] @ B
            s2 += float((D * D).sum().item())
        return s2 ** 0.5

    specs = (("bf16", api.BF16, Ab, None, torch.float32, args.c3_steps),
             ("fp8", api.F8E4M3, A8, sc, torch.float32, args.c3_steps),
             ("fp64", api.F64, A, None, torch.float64, max(2, args.c3_steps // 3)))
    for name, dt, Ax, scales, ot, steps in specs:
        wb = lib.rsvd_workspace_bytes(api.OP_SVD, dt, m, n, k, p, q)
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
        info = torch.zeros(2, dtype=torch.int32, device=dev)
        U = torch.empty((m, k), dtype=ot, device=dev)
        S = torch.empty(k, dtype=torch.float64, device=dev)
        V = torch.empty((n, k), dtype=ot, device=dev)
        Qb = torch.empty((m, l), dtype=ot, device=dev)
        sptr = P(scales) if scales is not None else None

        def step():
            rc = lib.rsvd_svd_ex(h, dt, m, n, k, p, q, seed, P(Ax), Ax.stride(0), sptr, P(U), k,
                                 P(S), P(V), k, P(Qb), l, P(work), wb, P(info), sp)
            if rc != 0:
                raise RuntimeError("rsvd_svd_ex (%s) returned %d" % (name, rc))

        step()
        torch.cuda.synchronize()
        log("c3 %s: warmup done" % name)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        log("c3 %s: %.3f ms/step" % (name, ms))
        S_np = S.cpu().numpy()
        st = info.cpu().numpy()
        r = {"ms_per_step": round(ms, 3), "steps": steps,
             "value_gflops": round(alg_flops(m, n, k, p, q) / (ms * 1e-3) / 1e9, 1),
             "info": [int(st[0]), int(st[1])],
             "qb_resid_fro": resid_fro(Qb)}
        if golden:
            rel = np.abs(S_np - sig_o) / sig_o
            r["sigma_rel_err_vs_fp64_oracle"] = {"max": float(rel.max()),
                                                 "max_first_64": float(rel[:64].max()),
                                                 "max_first_256": float(rel[:256].max()),
                                                 "median": float(np.median(rel))}
            r["qb_resid_rel_diff_vs_fp64_oracle"] = (r["qb_resid_fro"] / golden["fp64"]["qb_resid_fro"]
                                                    - 1.0)
            same = golden[name]["sigma"]
            r["sigma_rel_err_vs_oracle_same_storage"] = float(np.max(np.abs(S_np - same) /
                                                                     np.array(same)))
        # one pass over A in each direction in this storage (X FP32 or FP64)
        xt = torch.float64 if dt == api.F64 else torch.float32
        X = torch.randn((n, l), dtype=xt, device=dev)
        Xm = torch.randn((m, l), dtype=xt, device=dev)
        Y = torch.empty((m, l), dtype=xt, device=dev)
        Z = torch.empty((n, l), dtype=xt, device=dev)
        if dt == api.F8E4M3:
            pw = max(lib.rsvd_pass_f8_workspace_bytes(0, m, n, l),
                     lib.rsvd_pass_f8_workspace_bytes(1, m, n, l))
        else:
            pw = max(lib.rsvd_pass_workspace_bytes(dt, 0, m, n, l),
                     lib.rsvd_pass_workspace_bytes(dt, 1, m, n, l))
        pwork = torch.empty(max(pw, 1), dtype=torch.uint8, device=dev)

        def one_pass(trans, Xt, Yt):
            if dt == api.F8E4M3:
                rc = lib.rsvd_pass_f8(h, trans, m, n, l, P(Ax), Ax.stride(0), sptr, P(Xt), l,
                                      P(Yt), l, 0, P(pwork), pw, sp)
            else:
                rc = lib.rsvd_pass(h, dt, trans, m, n, l, P(Ax), Ax.stride(0), P(Xt), l, P(Yt), l,
                                   P(pwork), pw, sp)
            if rc != 0:
                raise RuntimeError("pass (%s) returned %d" % (name, rc))

        reps = 3 if dt == api.F64 else 10
        pass_ms = {}
        for trans, Xt, Yt, key in ((0, X, Y, "A_X"), (1, Xm, Z, "At_X")):
            one_pass(trans, Xt, Yt)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                one_pass(trans, Xt, Yt)
            e1.record(stream)
            torch.cuda.synchronize()
            pass_ms[key] = e0.elapsed_time(e1) / reps
        t_pass = 0.5 * (pass_ms["A_X"] + pass_ms["At_X"])
        tf = 2.0 * m * n * l / (t_pass * 1e-3) / 1e12
        peak = {"bf16": PEAK_BF16_TFLOPS, "fp8": PEAK_FP8_TFLOPS, "fp64": PEAK_FP64_TFLOPS}[name]
        ebytes = {"bf16": 2, "fp8": 1, "fp64": 8}[name]
        r["pass_ms"] = {kk: round(v, 4) for kk, v in pass_ms.items()}
        r["pass_roofline"] = {"bound": "mfma", "achieved": round(tf, 2), "peak": peak,
                              "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                              "a_hbm_GBs": round(ebytes * m * n / (t_pass * 1e-3) / 1e9, 1)}
        res[name] = r
        del work, U, V, Qb, X, Xm, Y, Z, pwork
    res["speedup_bf16_vs_fp64"] = round(res["fp64"]["ms_per_step"] / res["bf16"]["ms_per_step"], 3)
    res["speedup_fp8_vs_fp64"] = round(res["fp64"]["ms_per_step"] / res["fp8"]["ms_per_step"], 3)
    res["a_fro"] = A_fro
    if golden:
        res["oracle_qb_resid_fro"] = golden["fp64"]["qb_resid_fro"]
    del A, Ab, A8, sc
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pass-reps", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32, BF16, left-sketch ID, blocked QB, gradient and batch "
                         "sections "
                         "(for counter runs of the FP64 step and pass)")
    ap.add_argument("--grad-only", action="store_true",
                    help="run only the gradient section and print its JSON object "
                         "(for kernel traces of rsvd_svd_grad)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched section and print its JSON object")
    ap.add_argument("--mhbm-only", action="store_true",
                    help="run only the HBM-bound supplement (l = 30 on the 20000 x 10000 matrix) "
                         "and print its JSON object")
    ap.add_argument("--c3-only", action="store_true",
                    help="run only the mixed-precision section (65536 x 32768, l = 576) and "
                         "print its JSON object")
    ap.add_argument("--c3-steps", type=int, default=6,
                    help="timed steps of the BF16 and FP8 runs of the mixed-precision section "
                         "(the FP64 run takes a third of them, at least 2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1502_05366_amd import _lib, api, workloads as W

    lib = _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.batch_only:
        stream = torch.cuda.current_stream(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        print(json.dumps({"batch": batch_step(lib, args, stream, e0, e1)}), flush=True)
        return
    if args.c3_only:
        stream = torch.cuda.current_stream(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        r = c3_step(lib, api.handle(dev), args, stream, ctypes.c_void_p(stream.cuda_stream), P,
                    e0, e1)
        print(json.dumps({"c3": r}), flush=True)
        return
    if args.grad_only:
        stream = torch.cuda.current_stream(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        r = grad_step(lib, api.handle(dev), args, stream, ctypes.c_void_p(stream.cuda_stream), P,
                      e0, e1)
        print(json.dumps({"grad": r}), flush=True)
        return
    m, n = W.C2_SHAPE
    k, p, q, seed = 200, 20, 2, 0x5EED0001
    l = min(k + p, m, n)
    log("generating A %dx%d" % (m, n))
    t0 = time.perf_counter()
    A_np, _ = W.c2_matrix()
    A = torch.from_numpy(A_np).to(dev)
    torch.cuda.synchronize()
    log("generated in %.1f s" % (time.perf_counter() - t0))

    h = api.handle(dev)
    if args.mhbm_only:
        stream = torch.cuda.current_stream(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        r = mhbm_step(lib, h, A, args, stream, ctypes.c_void_p(stream.cuda_stream), P, e0, e1)
        print(json.dumps({"mhbm": r}), flush=True)
        return
    ops = api.OP_SVD | api.OP_ID | api.OP_CUR
    wb = lib.rsvd_workspace_bytes(ops, api.F64, m, n, k, p, q)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    U = torch.empty((m, k), dtype=torch.float64, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty((n, k), dtype=torch.float64, device=dev)
    J = torch.empty(n, dtype=torch.int64, device=dev)
    T = torch.empty((k, n - k), dtype=torch.float64, device=dev)
    Jr = torch.empty(k, dtype=torch.int64, device=dev)
    Uc = torch.empty((k, k), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731

    def step():
        rc = lib.rsvd_decompose(h, api.F64, m, n, k, p, q, seed, P(A), n, P(U), k, P(S), P(V), k,
                                P(J), P(T), n - k, P(Jr), P(Uc), k, P(work), wb, P(info), sp)
        if rc != 0:
            raise RuntimeError("rsvd_decompose returned %d" % rc)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    log("timed %d steps: %.3f ms/step (wall %.3f s)" % (args.steps, ms, wall))
    flops = alg_flops(m, n, k, p, q)
    gflops = flops / (ms * 1e-3) / 1e9
    st = info.cpu().numpy()

    # dominant kernel: one pass over A (Y = A X and Z = A^T X on the matrix
    # cores), timed with events on the stream it runs on
    X = torch.randn((n, l), dtype=torch.float64, device=dev)
    Xm = torch.randn((m, l), dtype=torch.float64, device=dev)
    Y = torch.empty((m, l), dtype=torch.float64, device=dev)
    Z = torch.empty((n, l), dtype=torch.float64, device=dev)
    pw = max(lib.rsvd_pass_workspace_bytes(api.F64, 0, m, n, l),
             lib.rsvd_pass_workspace_bytes(api.F64, 1, m, n, l))
    pwork = torch.empty(pw, dtype=torch.uint8, device=dev)
    pass_ms = {}
    for trans, Xt, Yt, name in ((0, X, Y, "A_X"), (1, Xm, Z, "At_X")):
        for _ in range(3):
            lib.rsvd_pass(h, api.F64, trans, m, n, l, P(A), n, P(Xt), l, P(Yt), l, P(pwork), pw, sp)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.pass_reps):
            lib.rsvd_pass(h, api.F64, trans, m, n, l, P(A), n, P(Xt), l, P(Yt), l, P(pwork), pw, sp)
        e1.record(stream)
        torch.cuda.synchronize()
        pass_ms[name] = e0.elapsed_time(e1) / args.pass_reps
    # a plain device copy of known size: the HBM rate a streaming kernel
    # reaches on this part, and the calibration kernel of the HBM byte counters
    cn = (1 << 30) // 8
    src = torch.ones(cn, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        torch.neg(src, out=dst)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * cn * 8 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    del src, dst

    pass_flops = 2.0 * m * n * l
    t_pass = 0.5 * (pass_ms["A_X"] + pass_ms["At_X"])
    achieved = pass_flops / (t_pass * 1e-3) / 1e12
    a_bytes = 8.0 * m * n
    log("pass A X %.3f ms, A^T X %.3f ms" % (pass_ms["A_X"], pass_ms["At_X"]))

    # the same step with A stored in BF16 (passes on the BF16 matrix cores,
    # FP32 accumulation, FP64 after the passes); A is converted once, untimed
    S64 = S.cpu().numpy()
    lowp = {}
    for key, is_bf16 in (() if args.no_extras else (("fp32", False), ("bf16", True))):
        r = lowp_step(lib, h, A, m, n, k, p, q, seed, l, args, stream, sp, P, e0, e1, is_bf16)
        Sl = r.pop("S")
        r["sigma_rel_err_vs_fp64"] = float(np.max(np.abs(Sl - S64) / S64))
        r["speedup_vs_fp64"] = round(ms / r["ms_per_step"], 3)
        lowp[key] = r

    idl = qbr = grd = bat = c3r = mh = c1g = None
    if not args.no_extras:
        idl = id_left_step(lib, h, A, m, n, k, p, q, seed, args, stream, sp, P, e0, e1)
        qbr = qb_step(lib, h, A, m, n, seed, args, stream, sp, P, e0, e1)
        grd = grad_step(lib, h, args, stream, sp, P, e0, e1)
        bat = batch_step(lib, args, stream, e0, e1)
        mh = mhbm_step(lib, h, A, args, stream, sp, P, e0, e1)
        c1g = c1_graph_step(lib, h, args, stream, sp, P, e0, e1)
        c3r = c3_step(lib, h, args, stream, sp, P, e0, e1)

    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "RSVD+ID+CUR, FP64 A 20000x10000, sigma_j=1/j + N(0,1e-12) noise, "
                               "k=200 p=20 q=2, one rsvd_decompose call per step",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "l": l},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": pass_traffic(),
                     "traffic_unit": "bytes per pass",
                     "kernel": "pass over A (gemm_sk_kernel + fix-up), FP64 MFMA 16x16x4",
                     "pass_ms": {kk: round(v, 4) for kk, v in pass_ms.items()},
                     "pass_hbm_GBs": round(a_bytes / (t_pass * 1e-3) / 1e9, 1),
                     "copy_kernel_GBs": round(copy_gbs, 1)},
        "end_to_end_frac_of_fp64_peak": round(gflops / 1e3 / PEAK_FP64_TFLOPS, 4),
        "info": [int(st[0]), int(st[1])],
    }
    if not args.no_extras:
        out["fp32"] = lowp["fp32"]
        out["bf16"] = lowp["bf16"]
        out["id_left"] = idl
        out["qb"] = qbr
        out["grad"] = grd
        out["batch"] = bat
        out["mhbm"] = mh
        out["c1_graph"] = c1g
        out["c3"] = c3r
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(A_np, k, p, q, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
