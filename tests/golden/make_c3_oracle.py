"""Writes tests/golden/c3_oracle.json: the FP64 oracle's results on the
mixed-precision workload, which is too large to recompute in a test.

Workload: A = (U1[:, :128] kron U2) diag(sigma) (V1 kron V2)^T, 65536 x 32768,
sigma_j = j^(-1.5) (seed 0xC0FFEE02), rank k = 512, oversampling p = 64,
q = 2 power steps, sketch seed 0x5EED0002 (Alg. 5 with re-orthonormalization
after every product, Sec. 3.2).  Three oracle runs, each on the matrix the
GPU path factorizes in that storage format:

* fp64: A itself;
* bf16: A rounded to BF16 (to nearest even, from FP64);
* fp8:  A quantized to FP8 E4M3 with per-column FP32 scales, dequantized.

Each run stores sigma_1..k, the range-finder residual ||A_v - Q Q^T A_v||_F
(A_v the run's matrix) and ||A - Q Q^T A||_F against the FP64 A, and the
rank-k residual ||A - U_k diag(sigma) V_k^T||_F against the FP64 A.

Calls only oracle/ and the seeded generator.  Needs about 40 GB of memory and
half an hour on 8 cores.  Usage: python tests/golden/make_c3_oracle.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rsvd as O, quant as QZ          # noqa: E402
from paper_1502_05366_amd import workloads as W    # noqa: E402

K, P, QP, SEED = 512, 64, 2, 0x5EED0002
CHUNK = 4096


def log(msg):
    print("[%7.1f s] %s" % (time.perf_counter() - T0, msg), flush=True)


def resid_fro(A, Q, Bt):
    """||A - Q Bt^T||_F by row blocks."""
    s = 0.0
    for i in range(0, A.shape[0], CHUNK):
        D = A[i:i + CHUNK] - Q[i:i + CHUNK] @ Bt.T
        s += float(np.einsum('ij,ij->', D, D))
    return float(np.sqrt(s))


def rankk_fro(A, U, S, V):
    s = 0.0
    VS = V * S[None, :]
    for i in range(0, A.shape[0], CHUNK):
        D = A[i:i + CHUNK] - U[i:i + CHUNK] @ VS.T
        s += float(np.einsum('ij,ij->', D, D))
    return float(np.sqrt(s))


def run(name, Av, A):
    log("%s: oracle RSVD" % name)
    U, S, V, det = O.rsvd(Av, K, P, QP, SEED, return_details=True)
    Q, Bt = det["Q"], det["Bt"]
    log("%s: residuals" % name)
    out = dict(sigma=[float(x) for x in S],
               qb_resid_fro=resid_fro(Av, Q, Bt),
               rankk_resid_fro=rankk_fro(A, U, S, V),
               jacobi_sweeps=int(det["sweeps"]))
    if Av is not A:
        out["qb_resid_fro_vs_fp64_A"] = resid_fro(A, Q, A.T @ Q)
    else:
        out["qb_resid_fro_vs_fp64_A"] = out["qb_resid_fro"]
    log("%s: sigma_1 %.6e sigma_k %.6e qb %.6e" % (name, S[0], S[-1], out["qb_resid_fro"]))
    return out


def main():
    log("generating A (65536 x 32768, FP64)")
    A, sig = W.c3_matrix()
    m, n = A.shape
    res = dict(workload="C3: A 65536x32768 = (U1[:, :128] kron U2) diag(j^-1.5) (V1 kron V2)^T, "
                        "matrix seed 0xC0FFEE02", m=m, n=n, k=K, p=P, q=QP, seed=SEED,
               a_fro=float(np.sqrt(np.sum(sig ** 2))), sigma_exact_k=[float(x) for x in sig[:K]])
    res["fp64"] = run("fp64", A, A)
    # FP8 E4M3 with per-column scales (scales from the whole column)
    mx = np.zeros(n)
    for i in range(0, m, CHUNK):
        mx = np.maximum(mx, np.abs(A[i:i + CHUNK]).max(axis=0))
    scales = np.where(mx == 0.0, 1.0, (mx / QZ.E4M3_MAX).astype(np.float32)).astype(np.float32)
    Av = np.empty_like(A)
    for i in range(0, m, CHUNK):
        codes = QZ.e4m3_encode(A[i:i + CHUNK] / scales.astype(np.float64)[None, :])
        Av[i:i + CHUNK] = QZ.e4m3_dequantize_columns(codes, scales)
    res["fp8"] = run("fp8", Av, A)
    for i in range(0, m, CHUNK):
        Av[i:i + CHUNK] = QZ.bf16_round(A[i:i + CHUNK])
    res["bf16"] = run("bf16", Av, A)
    with open(os.path.join(HERE, "c3_oracle.json"), "w") as f:
        json.dump(res, f, indent=1)
    log("wrote c3_oracle.json")


if __name__ == "__main__":
    T0 = time.perf_counter()
    main()
