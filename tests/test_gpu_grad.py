"""Parity of the library's reverse-mode derivative of the randomized SVD with
the FP64 oracle (needs a GPU), through the C-ABI entry rsvd_svd_grad.

* dA element by element against oracle.grad.rsvd_grad on the same A, seed
  and cotangents, for q = 0, 1, 2, tall, wide, ragged and l = min(m, n)
  shapes, each cotangent alone and all at once.  The singular pairs of the
  two sides may differ by a joint sign per column: the cotangents on U and V
  are given the GPU's signs before the oracle is called.
* Properties of the GPU result alone: central differences of the GPU forward,
  and d(sum sigma)/dA = U_k V_k^T on A of exact rank <= l.
* The recomputed forward equals rsvd_svd bit for bit.
* The differentiable wrapper (torch.autograd.Function) returns the entry
  point's dA.
* The 8192 x 4096, sigma_j = 1/j, k = 64, p = 16, q = 2 workload in FP64:
  dA of the two losses sum sigma_i and ||A - Q Q^T A||_F^2 against the
  oracle element by element.

Tolerance: |dA - dA_oracle| <= TOL * max|dA_oracle|.  The two forwards agree
to ~1e-13 (both form the positive-diagonal QR; rounding differs), and the
adjoint multiplies such differences by at most ||R^{-1}|| ||R|| of the bases
and by 1 / min relative gap of the singular values, each below 1e3 on these
inputs: TOL = 1e-8 leaves a wide margin above the ~1e-12 observed.
"""

import numpy as np
import pytest
import torch

from oracle import grad as G
from oracle import rsvd as O
from paper_1502_05366_amd import workloads as W

pytestmark = pytest.mark.gpu
SEED = 0x5EED0000
TOL = 1e-8


@pytest.fixture(scope="module")
def R():
    import paper_1502_05366_amd as R
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return R


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def pair_signs(U_gpu, U_or):
    sg = np.sign(np.sum(U_gpu * U_or, axis=0))
    sg[sg == 0] = 1.0
    return sg


def gpu_grad(R, A, k, p, q, seed, dU=None, dS=None, dV=None, dres=None):
    dA, U, S, V, r2 = R.svd_grad(dev(A), k, p, q, seed,
                                 dU=None if dU is None else dev(dU),
                                 dS=None if dS is None else dev(dS),
                                 dV=None if dV is None else dev(dV),
                                 dres=None if dres is None else dev(np.array([dres])),
                                 outputs=True)
    torch.cuda.synchronize()
    return (host(dA) if dA is not None else None), host(U), host(S), host(V), float(r2.item())


def check_parity(R, A, k, p, q, seed, which, rng):
    m, n = A.shape
    dU = rng.standard_normal((m, k)) if "U" in which else None
    dS = rng.standard_normal(k) if "S" in which else None
    dV = rng.standard_normal((n, k)) if "V" in which else None
    dres = 0.37 if "r" in which else None
    print("grad parity m=%d n=%d k=%d p=%d q=%d cot=%s" % (m, n, k, p, q, which), flush=True)
    dA, U, S, V, r2 = gpu_grad(R, A, k, p, q, seed, dU, dS, dV, dres)
    f = G.rsvd_forward_tape(A, k, p, q, seed)
    sg = pair_signs(U, f["U"])
    dAo, _ = G.rsvd_grad(A, k, p, q, seed,
                         dU=None if dU is None else dU * sg, dS=dS,
                         dV=None if dV is None else dV * sg, dres=dres)
    assert np.all(np.isfinite(dA))
    err = np.abs(dA - dAo).max()
    scale = np.abs(dAo).max()
    print("  max |dA - dA_oracle| / max |dA_oracle| = %.2e" % (err / scale), flush=True)
    assert err <= TOL * scale, "max err %.3e scale %.3e" % (err, scale)
    assert np.abs(S - f["S"]).max() <= 1e-10 * f["S"][0]
    assert abs(r2 - f["resid2"]) <= 1e-10 * max(np.sum(A * A), 1.0)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_grad_parity_all_cotangents(R, q):
    A, _ = W.logspace_type(300, 200, 1, seed=3)
    check_parity(R, A, 10, 6, q, SEED + q, "USVr", np.random.default_rng(q))


@pytest.mark.parametrize("which", ["U", "S", "V", "r"])
def test_grad_parity_single_cotangent(R, which):
    A, _ = W.logspace_type(260, 190, 1, seed=4)
    check_parity(R, A, 9, 7, 1, SEED + 7, which, np.random.default_rng(11))


@pytest.mark.parametrize("shape", [(333, 177, 7, 5, 1), (150, 260, 9, 7, 1), (40, 24, 20, 10, 1),
                                   (210, 130, 12, 0, 2), (1000, 70, 16, 9, 3)])
def test_grad_parity_shapes(R, shape):
    m, n, k, p, q = shape
    A, _ = W.logspace_type(m, n, 1, seed=m + n)
    check_parity(R, A, k, p, q, SEED + m, "USVr", np.random.default_rng(m))


def test_grad_forward_equals_svd(R):
    A, _ = W.logspace_type(300, 200, 1, seed=3)
    k, p, q = 10, 6, 2
    print("grad forward vs svd", flush=True)
    _, U, S, V, _ = R.svd_grad(dev(A), k, p, q, SEED, outputs=True)
    U2, S2, V2, _ = R.svd(dev(A), k, p, q, SEED)
    torch.cuda.synchronize()
    assert torch.equal(U, U2) and torch.equal(S, S2) and torch.equal(V, V2)


def test_grad_central_difference(R):
    """Directional derivative of the GPU forward against <dA, E>."""
    m, n, k, p, q = 220, 150, 8, 6, 1
    A, _ = W.logspace_type(m, n, 1, seed=9)
    g = np.random.default_rng(5)
    dU, dS, dV = g.standard_normal((m, k)), g.standard_normal(k), g.standard_normal((n, k))
    dres = 0.5
    E = g.standard_normal((m, n))
    print("grad central difference", flush=True)
    dA, U0, _, _, _ = gpu_grad(R, A, k, p, q, SEED, dU, dS, dV, dres)
    h = 1e-6

    def L(M):
        _, U, S, V, r2 = gpu_grad(R, M, k, p, q, SEED)
        sg = pair_signs(U, U0)           # follow the unperturbed branch
        return np.sum(dU * U * sg) + np.sum(dS * S) + np.sum(dV * V * sg) + dres * r2
    # fourth-order central difference: the singular values of the small factor
    # lie close together on this slowly decaying spectrum (gaps ~1e-3), so
    # the second-order formula's truncation error at h = 1e-6 is ~2e-6
    # relative, while this one's is ~1e-10
    fd = (8 * (L(A + h * E) - L(A - h * E)) - (L(A + 2 * h * E) - L(A - 2 * h * E))) / (12 * h)
    assert abs(fd - np.sum(dA * E)) <= 1e-7 * max(1.0, abs(fd))


def test_grad_exact_rank_sum_sigma(R):
    """rank(A) <= l: Q Q^T A = A to first order, so d(sum sigma)/dA = U_k V_k^T."""
    A, _, _, _ = W.exact_rank_matrix(300, 200, 8, seed=4)
    k, p, q = 8, 4, 1
    print("grad exact rank", flush=True)
    dA, U, _, V, _ = gpu_grad(R, A, k, p, q, SEED, dS=np.ones(k))
    assert np.abs(dA - U @ V.T).max() <= 1e-10


def test_grad_autograd_function(R):
    A, _ = W.logspace_type(180, 120, 1, seed=2)
    k, p, q = 6, 4, 1
    g = np.random.default_rng(3)
    cU = dev(g.standard_normal((180, k)))
    print("grad autograd function", flush=True)
    Ad = dev(A).requires_grad_(True)
    U, S, V, r2 = R.svd_diff(Ad, k, p, q, SEED)
    loss = S.sum() + 0.25 * r2 + (U * cU).sum()
    loss.backward()
    dA = R.svd_grad(dev(A), k, p, q, SEED, dU=cU, dS=torch.ones(k, dtype=torch.float64,
                                                                 device="cuda"),
                    dres=torch.tensor(0.25, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(Ad.grad, dA)
    # an unused output contributes nothing
    Ad.grad = None
    U, S, V, r2 = R.svd_diff(Ad, k, p, q, SEED)
    S.sum().backward()
    dS_only = R.svd_grad(dev(A), k, p, q, SEED, dS=torch.ones(k, dtype=torch.float64,
                                                                device="cuda"))
    assert torch.equal(Ad.grad, dS_only)


def test_grad_unsupported(R):
    A = torch.zeros((64, 48), dtype=torch.float32, device="cuda")
    with pytest.raises(R.RsvdError):
        R.svd_grad(A, 4, 2, 1, SEED, dS=torch.ones(4, device="cuda"))
    with pytest.raises(R.RsvdError):
        R.svd_grad(A.double(), 4, 2, 9, SEED, dS=torch.ones(4, device="cuda"))


def test_grad_c5_full_size(R):
    """8192 x 4096, sigma_j = 1/j, k = 64, p = 16, q = 2 in FP64: dA of
    sum sigma_i + ||A - Q Q^T A||_F^2 against the oracle element by element."""
    A, _ = W.c5_matrix()
    k, p, q = 64, 16, 2
    print("grad C5 full size", flush=True)
    dA, U, S, V, r2 = gpu_grad(R, A, k, p, q, SEED, dS=np.ones(k), dres=1.0)
    dAo, f = G.rsvd_grad(A, k, p, q, SEED, dS=np.ones(k), dres=1.0)
    err = np.abs(dA - dAo).max()
    scale = np.abs(dAo).max()
    print("  max |dA - dA_oracle| / max |dA_oracle| = %.2e" % (err / scale), flush=True)
    assert err <= TOL * scale, "max err %.3e scale %.3e" % (err, scale)
    assert np.abs(S - f["S"]).max() <= 1e-10 * f["S"][0]
    assert abs(r2 - f["resid2"]) <= 1e-10 * f["resid2"]
    # sigma_i of the randomized SVD are those of A to the accuracy the
    # spectrum allows: the leading ones to 1e-6 (gap-independent check that
    # the forward is the right workload)
    Uo, So, Vo = O.rsvd(A, k, p, q, SEED)
    assert np.abs(So - S).max() <= 1e-10
    assert np.abs(S[:8] - 1.0 / np.arange(1, 9)).max() <= 1e-6
