"""Seeded synthetic test matrices shaped like the paper's workloads.

This module holds input generators only; it contains none of the
factorization arithmetic.  The paper's experiments (Sec. 5) use
A = U D V^* with U, V random matrices with orthonormal columns and a
prescribed diagonal D (log-spaced spectra, "types I, II, III"); every
generator below follows that recipe with an exactly known spectrum.

Randomness comes from numpy's PCG64 generator seeded by the caller.  Haar
(uniformly distributed) orthonormal factors come from the QR factorization of
a Gaussian matrix with the column signs fixed by sign(diag(R)) (Mezzadri,
"How to generate random matrices from the classical compact groups", 2007).
"""

import numpy as np

C1_SHAPE = (2000, 1000)
C2_SHAPE = (20000, 10000)


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def haar(g, m, r):
    """m x r matrix with orthonormal columns, Haar distributed."""
    G = g.standard_normal((m, r))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def from_factors(U, s, V):
    """U diag(s) V^T."""
    return (U * s[None, :]) @ V.T


def spectrum_matrix(m, n, s, seed):
    """A = U diag(s) V^T with Haar U (m x r), V (n x r), r = len(s)."""
    g = rng(seed)
    r = len(s)
    U = haar(g, m, r)
    V = haar(g, n, r)
    return from_factors(U, np.asarray(s, dtype=np.float64), V), U, V


def logspace_type(m, n, kind, seed):
    """Sec. 5 test matrices: sigma = logspace(0, -e, min(m,n)) with
    e = 0.5 (type I), 2 (type II), 3.5 (type III)."""
    e = {1: 0.5, 2: 2.0, 3: 3.5}[kind]
    r = min(m, n)
    s = np.logspace(0.0, -e, r)
    A, U, V = spectrum_matrix(m, n, s, seed)
    return A, s


def c1_matrix(seed=0xC0FFEE00):
    """2000 x 1000, sigma_j = 10^(-j/10) (j = 1..1000), Haar U and V."""
    m, n = C1_SHAPE
    s = 10.0 ** (-np.arange(1, n + 1) / 10.0)
    A, _, _ = spectrum_matrix(m, n, s, seed)
    return A, s


def kron_haar_factors(m1, r1, m2, n1, n2, seed):
    """The Haar factors of kron_haar_matrix: U1[:, :r1] (U1 m1 x m1), U2
    (m2 x m2), V1 (n1 x n1), V2 (n2 x n2), drawn in that order."""
    g = rng(seed)
    U1 = haar(g, m1, m1)[:, :r1]
    U2 = haar(g, m2, m2)
    V1 = haar(g, n1, n1)
    V2 = haar(g, n2, n2)
    return U1, U2, V1, V2


def kron_haar_matrix(m1, r1, m2, n1, n2, s, seed):
    """A = (U1[:, :r1] kron U2) diag(s) (V1 kron V2)^T.

    U1 is m1 x m1 Haar, U2 is m2 x m2 Haar, V1 n1 x n1 Haar, V2 n2 x n2 Haar;
    r1 * m2 = n1 * n2 = len(s).  Singular vector j of A is column j of each
    Kronecker factor, so the spectrum is exactly s while A is dense and its
    singular vectors are delocalized.  Assembled without forming the
    Kronecker factors: rows (a, b) of W = diag(s) V^T are mapped by
    U1[:, :r1] on a and by U2 on b.
    """
    U1, U2, V1, V2 = kron_haar_factors(m1, r1, m2, n1, n2, seed)
    r = r1 * m2
    n = n1 * n2
    assert r == len(s) and r == n
    W = np.kron(V1.T, V2.T)                      # (V1 kron V2)^T, n x n
    W *= np.asarray(s, dtype=np.float64)[:, None]
    W = W.reshape(r1, m2, n)
    T1 = np.matmul(U2[None, :, :], W)            # (r1, m2, n): U2 on index b
    del W
    A = np.tensordot(U1, T1, axes=([1], [0]))    # (m1, m2, n): U1 on index a
    return A.reshape(m1 * m2, n)


def kron_haar_matrix_torch(m1, r1, m2, n1, n2, s, seed, device):
    """kron_haar_matrix assembled on a device with torch (FP64), from the same
    factors; it differs from the host assembly only by the order of the
    rounding of the sums (a few units of FP64 rounding per entry)."""
    import torch
    U1, U2, V1, V2 = (torch.as_tensor(x, device=device)
                      for x in kron_haar_factors(m1, r1, m2, n1, n2, seed))
    n = n1 * n2
    W = torch.kron(V1.T.contiguous(), V2.T.contiguous())
    W *= torch.as_tensor(np.asarray(s, dtype=np.float64), device=device)[:, None]
    T1 = torch.matmul(U2, W.view(r1, m2, n))     # (r1, m2, n)
    del W
    A = torch.tensordot(U1, T1, dims=([1], [0]))  # (m1, m2, n)
    return A.reshape(m1 * m2, n)


def c2_matrix(seed=0xC0FFEE01, noise_std=1e-6):
    """20000 x 10000, sigma_j = 1/j (j = 1..10000) plus i.i.d. N(0, noise_std^2).

    Kronecker-Haar factors U = U1[:, :80] kron U2 (U1 160^2, U2 125^2) and
    V = V1 kron V2 (100^2 each).  The noise E has ||E||_2 ~ noise_std *
    (sqrt(m) + sqrt(n)) ~ 2.4e-4, so sigma_j(A) = 1/j +- 2.5e-4 (Weyl)."""
    m, n = C2_SHAPE
    s = 1.0 / np.arange(1, n + 1)
    A = kron_haar_matrix(160, 80, 125, 100, 100, s, seed)
    if noise_std:
        g = rng(seed ^ 0x5A5A5A5A)
        A += noise_std * g.standard_normal(A.shape)
    return A, s


C3_SHAPE = (65536, 32768)
C3_KRON = (256, 128, 256, 128, 256)       # m1, r1, m2, n1, n2


def c3_spectrum():
    """sigma_j = j^(-1.5), j = 1..32768."""
    return np.arange(1, C3_SHAPE[1] + 1, dtype=np.float64) ** -1.5


def c3_matrix(seed=0xC0FFEE02):
    """65536 x 32768, sigma_j = j^(-1.5), Kronecker-Haar factors
    U = U1[:, :128] kron U2 (U1, U2 256^2) and V = V1 kron V2 (128^2, 256^2):
    the mixed-precision workload (stored BF16 or FP8 E4M3 with per-column
    scales).  17.2 GB in FP64."""
    return kron_haar_matrix(*C3_KRON, c3_spectrum(), seed), c3_spectrum()


def c3_matrix_torch(device, seed=0xC0FFEE02):
    """c3_matrix assembled on the device (FP64)."""
    return kron_haar_matrix_torch(*C3_KRON, c3_spectrum(), seed, device)


C5_SHAPE = (8192, 4096)


def c5_matrix(seed=0xC0FFEE05):
    """8192 x 4096, sigma_j = 1/j (j = 1..4096), Kronecker-Haar factors
    U = U1[:, :64] kron U2 (U1 128^2, U2 64^2) and V = V1 kron V2 (64^2 each):
    the workload of the differentiated randomized SVD."""
    m, n = C5_SHAPE
    s = 1.0 / np.arange(1, n + 1)
    return kron_haar_matrix(128, 64, 64, 64, 64, s, seed), s


C4_COUNT = 4096


def c4_dims(count=C4_COUNT, seed=0xC0FFEE04, mmax=2048, nmax=1024, kmax=64):
    """Sizes of a batch of uneven problems: m ~ U{64..mmax}, n ~ U{64..nmax},
    k ~ U{4..kmax} (clamped to min(m, n))."""
    g = rng(seed)
    m = g.integers(min(64, mmax), mmax + 1, size=count).astype(np.int64)
    n = g.integers(min(64, nmax), nmax + 1, size=count).astype(np.int64)
    k = g.integers(min(4, kmax), kmax + 1, size=count)
    k = np.minimum(k, np.minimum(m, n)).astype(np.int32)
    return m, n, k


def c4_spectrum(m, n, rmax=320):
    """sigma_j = exp(-j/8), j = 1 .. min(m, n, rmax)."""
    r = min(m, n, rmax)
    return np.exp(-np.arange(1, r + 1) / 8.0)


def c4_batch_torch(ms, ns, seed, device, rmax=320):
    """The batch's FP32 matrices A_i = U_i diag(sigma) V_i^T generated on a
    device with torch: U_i, V_i are the first r columns of a product of two
    Householder reflectors with Gaussian vectors (orthonormal; a Gaussian
    sketch is rotation-invariant, so the error law of the method depends only
    on sigma), formed in FP64 and rounded to FP32 once."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)

    def factor(rows, r):
        E = torch.eye(rows, r, dtype=torch.float64, device=device)
        for _ in range(2):
            w = torch.randn(rows, 1, dtype=torch.float64, device=device, generator=gen)
            w = w / torch.linalg.vector_norm(w)
            E = E - 2.0 * w @ (w.T @ E)
        return E

    out = []
    for m, n in zip(ms, ns):
        m, n = int(m), int(n)
        s = torch.as_tensor(c4_spectrum(m, n, rmax), device=device)
        r = s.numel()
        U, V = factor(m, r), factor(n, r)
        out.append(((U * s) @ V.T).to(torch.float32))
    return out


def exact_rank_matrix(m, n, r, seed, decay=0.5):
    """Rank-r A = U diag(s) V^T with s_j = decay^j (j = 0..r-1)."""
    s = decay ** np.arange(r)
    A, U, V = spectrum_matrix(m, n, s, seed)
    return A, s, U, V


def separated_skeleton_matrix(m, n, r, seed):
    """A = U_r diag(d) E_pi^T with d_j = 2^(-j/4) (j = 0..r-1).

    U_r is m x r Haar, pi an injective map of 0..r-1 into 0..n-1, and every
    other column of A is zero.  A has rank r and orthogonal nonzero columns
    of norms d_j, so any B with the same row space relation (B = Q^T A with
    Q Q^T A = A) has orthogonal columns of the same norms: k steps of the
    column-pivoted QR must return pi(0), .., pi(k-1) in that order, with a
    16% norm margin between consecutive pivots.  Returns (A, pi, d)."""
    g = rng(seed)
    U = haar(g, m, r)
    pi = g.permutation(n)[:r]
    d = 2.0 ** (-np.arange(r) / 4.0)
    A = np.zeros((m, n))
    A[:, pi] = U * d[None, :]
    return A, pi, d


def integer_matrix(m, n, seed, lo=-8, hi=8):
    """Small-integer entries: every product and sum of a GEMM is exact in
    FP64 (and in FP32 for short enough reductions)."""
    g = rng(seed)
    return g.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
