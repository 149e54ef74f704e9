"""The FP8 half of the mixed-precision path (needs a GPU): A stored as FP8
E4M3 codes with FP32 column scales, passes on the FP8 matrix cores with FP32
accumulation, everything after the passes in FP64 (the re-orthonormalization
of Sec. 3.2 between the narrow passes).

* The storage formats (rsvd_quantize) equal the oracle's quantizers bit for
  bit: BF16 patterns, E4M3 codes and column scales.
* The FP8 pass is exact on inputs whose every rounding is exact: small
  integer codes with unit scales, and skinny columns whose largest entry is
  7, so that X / t = 64 X are E4M3 values and t = 1/64 (FP32 sums of integers
  below 2^24).
* On random data the pass stays within the quantization of the skinny
  operand (half a step of a 3-bit significand, 2^-4 relative; 2^-8 with the
  two-term split) plus FP32 accumulation, against the exact product with the
  dequantized A.
* The FP8 randomized SVD (l = 576) against the FP64 oracle run on the
  dequantized A: its singular values within the error that the FP8 passes
  leave (bounds stated in the test).
"""

import numpy as np
import pytest
import torch

from oracle import rsvd as O, quant as QZ
from paper_1502_05366_amd import workloads as W
from tests.helpers import orth_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def codes_dev(codes):
    """uint8 codes on the GPU with rows padded to 16 bytes."""
    m, n = codes.shape
    P = torch.zeros((m, (n + 15) // 16 * 16), dtype=torch.uint8, device="cuda")
    P[:, :n] = torch.from_numpy(np.ascontiguousarray(codes))
    return P[:, :n]


def test_quantize_bit_exact(R):
    g = np.random.default_rng(21)
    m, n = 1000, 333
    A = g.standard_normal((m, n)) * np.logspace(-6, 3, n)[None, :]
    A[:, 5] = 0.0
    A[7, 9] = 1e-300            # below both formats' subnormals in its column
    A[::97, 11] *= 1e6          # one column with a few large entries
    Ad = dev(A)
    Bq = R.quantize(Ad, R.BF16)
    bits = Bq.contiguous().view(torch.int16).cpu().numpy().astype(np.uint16)
    assert np.array_equal(bits, QZ.bf16_bits(A))
    codes, sc = R.quantize(Ad, R.F8E4M3)
    oc, osc = QZ.e4m3_quantize_columns(A)
    assert np.array_equal(sc.cpu().numpy(), osc)
    assert np.array_equal(codes.cpu().numpy(), oc)


@pytest.mark.parametrize("m,n,l", [(300, 520, 30), (1000, 2000, 220), (130, 72, 1),
                                   (2047, 136, 256), (700, 900, 576), (257, 1003, 17),
                                   # n a multiple of 128: A X on the direct-to-LDS kernel
                                   (1000, 1024, 220), (300, 2048, 576), (129, 128, 17),
                                   (4100, 256, 300)])
def test_f8_pass_exact_on_integers(R, m, n, l):
    g = np.random.default_rng(m + n + l)
    A = g.integers(-8, 9, size=(m, n)).astype(np.float64)
    codes = QZ.e4m3_encode(A)
    ones = torch.ones(n, dtype=torch.float32, device="cuda")

    def skinny(rows):
        X = g.integers(-7, 8, size=(rows, l)).astype(np.float64)
        X[g.integers(0, rows, size=l), np.arange(l)] = 7.0      # column max exactly 7
        return X

    Xn, Xm = skinny(n), skinny(m)
    A8 = codes_dev(codes)
    Y = R.pass_f8(A8, ones, dev(Xn, torch.float32)).cpu().numpy().astype(np.float64)
    Z = R.pass_f8(A8, ones, dev(Xm, torch.float32), trans=True).cpu().numpy().astype(np.float64)
    assert np.array_equal(Y, A @ Xn)
    assert np.array_equal(Z, A.T @ Xm)


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("split", [False, True])
def test_f8_pass_random_bound(R, trans, split):
    g = np.random.default_rng(31 + trans + 2 * split)
    m, n, l = 3001, 1777, 200
    A = g.standard_normal((m, n)) * np.logspace(-2, 1, n)[None, :]
    codes, sc = QZ.e4m3_quantize_columns(A)
    A8 = QZ.e4m3_decode(codes)
    s64 = sc.astype(np.float64)
    X = g.standard_normal((m if trans else n, l)).astype(np.float32)
    X64 = X.astype(np.float64)
    Y = R.pass_f8(codes_dev(codes), dev(sc, torch.float32), dev(X, torch.float32), trans=trans,
                  split=split).cpu().numpy().astype(np.float64)
    # Y = A8 X' with X' = diag(s) X (scales folded into the skinny operand), or
    # Z = diag(s) A8^T X; the reference is the exact product with dequantized A
    if trans:
        Op, Xp, outs = A8.T, X64, s64[:, None]
    else:
        Op, Xp, outs = A8, s64[:, None] * X64, 1.0
    ref = outs * (Op @ Xp)
    t = np.abs(Xp).max(axis=0) / 448.0
    # an E4M3 code is within 2^-4 relative of its value (normal range) or 2^-10
    # t absolute (subnormal); the split leaves 2^-8 relative and 2^-12 t
    rel, sub = (2.0 ** -8, 2.0 ** -12) if split else (2.0 ** -4, 2.0 ** -10)
    absop = np.abs(Op)
    K = Op.shape[1]
    bound = outs * (rel * (absop @ np.abs(Xp)) + sub * (absop @ np.ones((K, 1))) * t[None, :]
                    + (K + 8) * 2.0 ** -24 * 1.07 * (absop @ np.abs(Xp)))
    assert np.all(np.abs(Y - ref) <= bound)


@pytest.fixture(scope="module")
def graded():
    m, n = 4096, 2048
    s = np.arange(1, n + 1, dtype=np.float64) ** -1.5
    A, _, _ = W.spectrum_matrix(m, n, s, seed=0xC0FFEE12)
    return A


K, P, Q, SEED = 512, 64, 2, 0x5EED0012


def test_rsvd_f8_l576_vs_oracle(R, graded):
    A = graded
    codes, sc = R.quantize(dev(A), R.F8E4M3)
    oc, osc = QZ.e4m3_quantize_columns(A)
    assert np.array_equal(codes.cpu().numpy(), oc)
    Adq = QZ.e4m3_dequantize_columns(oc, osc)
    print("FP8 RSVD l=576 on the GPU", flush=True)
    U, S, V, info, Qb = R.svd_ex(codes, K, P, Q, SEED, scales=sc, want_Q=True)
    S = S.cpu().numpy()
    assert int(info.cpu()[0]) == 0
    print("oracle on the dequantized A", flush=True)
    _, So, _, det = O.rsvd(Adq, K, P, Q, SEED, return_details=True)
    rel = np.abs(S - So) / So
    print("FP8 sigma rel err: max %.3e, first 64 %.3e, first 256 %.3e"
          % (rel.max(), rel[:64].max(), rel[:256].max()), flush=True)
    # the basis is orthonormal to FP32 precision
    Qn = Qb.cpu().numpy().astype(np.float64)
    assert orth_err(Qn) < 1e-5
    # range-finder residual within 5% of the oracle's on the same matrix
    res_gpu = np.linalg.norm(Adq - Qn @ (Qn.T @ Adq))
    res_orc = np.linalg.norm(Adq - det["Q"] @ (det["Q"].T @ Adq))
    print("||A - QQ^T A||_F: GPU %.6e oracle %.6e" % (res_gpu, res_orc), flush=True)
    assert res_gpu <= 1.05 * res_orc
    # sigma: the last projection carries ~8 significand bits of Q, the earlier
    # passes ~4 bits of their operands, so sigma is accurate to about 2^-8
    # relative where the basis has converged (the leading values) and to the
    # range finder's own accuracy in the tail
    assert rel[:64].max() <= 2.0 ** -7
    assert rel.max() <= 0.1
