"""Randomized range finder, RSVD, ID and CUR in FP64 (the oracle).

Test infrastructure (see the package header): only tests, smoke() and the
bench's cpu_baseline leg may use it.

``range_finder``  Alg. 5 (RSVD Version II) lines 1-10 with re-orthonormalization
                  after every product (s = 1, the second scheme of Sec. 3.2):
                  Y = A Omega; q times { Q = orth(Y); Z = A^T Q; Z = orth(Z);
                  Y = A Z }; Q = orth(Y).
``rsvd``          Alg. 5 lines 11-15: B^T = A^T Q, [Qh, Rh] = qr(B^T, 0),
                  [Uh, S, Vh] = svd(Rh), U_k = Q Vh(:, 1:k), V_k = Qh Uh(:, 1:k).
``batch_rsvd``    ``rsvd`` of every matrix of a batch, matrix i with the sketch of
                  batch index i (the matrices are independent, as the blocks
                  of Alg. 8 are).
``rsvd_fig1``     Fig. 1: SVD of B = Q^T A directly (cross-check).
``rsvd_alg4``     Alg. 4 (Version I): eigen-decomposition of B B^T (cross-check).
``qb_id``         ID from B = Q^T A (Sec. 3.5, last part): k-step CPQR of B gives
                  J and T = S11^{-1} S12; V = P [I_k; T^T] (Sec. 2.4).
``two_sided_id``  Sec. 2.5 / Alg. 2: row ID of C = A(:, J(1:k)).
``cur``           Sec. 2.5 / Alg. 3 and Sec. 3.6: C = A(:, Jc), R = A(Jr, :),
                  U = V^T R^dagger with R^dagger from the QR of R^T.
``id_left``       Sec. 3.5 / Alg. 6: ID from the left sample Y = Omega~ A with
                  the power scheme of eq. (Ypower) orthonormalized between
                  products; k steps of column-pivoted QR of Y, T = S11^{-1} S12.
``qb_blocked``    Sec. 3.3 / Alg. 7: blocked adaptive QB with deflation of A
                  and a tolerance on the residual.
"""

import numpy as np

from . import philox
from .dense import householder_qr, jacobi_svd, cpqr, solve_upper


def orth(Y):
    """orth(Y) of Sec. 2.1: the Q of the thin Householder QR."""
    return householder_qr(Y)[0]


def sample_size(m, n, k, p):
    """l = k + p, clamped to min(m, n) (a sketch wider than A adds nothing)."""
    return min(k + p, m, n)


def range_finder(A, k, p, q, seed, batch=0):
    """Q (m x l) with orthonormal columns such that Q Q^T A ~ A.

    Alg. 5 lines 1-10 with s = 1: orthonormalize before every product with
    A or A^T (the second scheme of Sec. 3.2), then a final Q = orth(Y).
    Omega comes from Philox stream 0 with batch index ``batch``.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = sample_size(m, n, k, p)
    Omega = philox.sketch(seed, n, l, batch=batch)
    Y = A @ Omega
    for _ in range(q):
        Qy = orth(Y)
        Z = A.T @ Qy
        Qz = orth(Z)
        Y = A @ Qz
    return orth(Y)


def rsvd(A, k, p, q, seed, return_details=False, batch=0):
    """Rank-k randomized SVD, Alg. 5 (QR of B^T, SVD of the l x l R_hat).

    Returns U_k (m x k), sigma (k,), V_k (n x k) with A ~ U_k diag(sigma) V_k^T.
    """
    A = np.asarray(A, dtype=np.float64)
    Q = range_finder(A, k, p, q, seed, batch=batch)
    Bt = A.T @ Q                              # n x l, = B^T
    Qh, Rh = householder_qr(Bt)               # B^T = Qh Rh
    Uh, s, Vh, sweeps, conv = jacobi_svd(Rh)  # Rh = Uh diag(s) Vh^T
    U = Q @ Vh[:, :k]                         # A ~ (Q Vh) S (Qh Uh)^T
    V = Qh @ Uh[:, :k]
    if return_details:
        return U, s[:k], V, dict(Q=Q, Bt=Bt, Qh=Qh, Rh=Rh, s_all=s,
                                 sweeps=sweeps, converged=conv)
    return U, s[:k], V


def batch_rsvd(As, ks, p, q, seed):
    """The randomized SVD of each matrix of a batch on its own: matrix i uses
    the sketch of Philox stream 0 with batch index i.  Returns a list of
    (U_k, sigma, V_k)."""
    return [rsvd(A, k, p, q, seed, batch=i) for i, (A, k) in enumerate(zip(As, ks))]


def rsvd_fig1(A, k, p, q, seed):
    """Fig. 1 steps 4-7: SVD of B = Q^T A itself (via Jacobi on B^T)."""
    A = np.asarray(A, dtype=np.float64)
    Q = range_finder(A, k, p, q, seed)
    Bt = A.T @ Q
    W, s, Ub, _, _ = jacobi_svd(Bt)           # B^T = W diag(s) Ub^T
    return Q @ Ub[:, :k], s[:k], W[:, :k]     # B = Ub S W^T


def rsvd_alg4(A, k, p, q, seed):
    """Alg. 4: eigen-decomposition of T = B B^T (squares the condition)."""
    A = np.asarray(A, dtype=np.float64)
    Q = range_finder(A, k, p, q, seed)
    B = Q.T @ A
    T = B @ B.T
    # T is symmetric positive semi-definite: its SVD is its eigen-decomposition
    Ut, d, _, _, _ = jacobi_svd(T)
    s = np.sqrt(d[:k])
    U = Q @ Ut[:, :k]
    V = (B.T @ Ut[:, :k]) / s[None, :]
    return U, s, V


def qb_id(A, k, p, q, seed, Q=None):
    """Column ID from B = Q^T A (Sec. 3.5, last part; Alg. 1 applied to B).

    Returns dict(J, T, frank, B, pivot_norms, second_norms, S22norm_F) where
    J[:k] is the skeleton (pivot order), J[k:] the remaining columns in
    ascending order, and T = S11^{-1} S12 is k x (n-k) with its columns in the
    order of J[k:].  V = P [I_k; T^T]: V[J[i], :] = e_i for i < k and
    V[J[k+j], :] = T[:, j].
    """
    A = np.asarray(A, dtype=np.float64)
    if Q is None:
        Q = range_finder(A, k, p, q, seed)
    B = Q.T @ A
    f = cpqr(B, k)
    T = solve_upper(f['S11'], f['S12'])
    return dict(J=f['J'], T=T, frank=f['frank'], B=B, Q=Q,
                pivot_norms=f['pivot_norms'], second_norms=f['second_norms'],
                S22norm_F=f['S22norm_F'], S11=f['S11'], S12=f['S12'])


def interp_matrix(J, T, n):
    """V = P [I_k; T^T], the column interpolation matrix of Sec. 2.4 (n x k)."""
    k = T.shape[0]
    V = np.zeros((n, k))
    V[J[:k], np.arange(k)] = 1.0
    V[J[k:], :] = T.T
    return V


def two_sided_id(A, J, k):
    """Row ID of C = A(:, J(1:k)) (Sec. 2.5, the factorization of C): C = W C(Jr(1:k), :).

    k steps of CPQR on C^T pick Jr; W = C C(Jr, :)^{-1} (the row ID of a rank-k
    C is exact).  Returns (Jr, W)."""
    A = np.asarray(A, dtype=np.float64)
    C = A[:, J[:k]]
    f = cpqr(C.T, k)
    Jr = f['J'][:k]
    M = C[Jr, :]                               # k x k
    Qm, Rm = householder_qr(M.T)               # M^T = Qm Rm, so M^{-1} = Qm Rm^{-T}
    Rinv = solve_upper(Rm, np.eye(k))
    W = (C @ Qm) @ Rinv.T                      # W = C M^{-1}
    return Jr, W, f['frank']


def cur(A, k, p, q, seed, Q=None):
    """Randomized CUR (Sec. 3.6 and Alg. 3): A ~ C U R.

    Column ID from B = Q^T A gives Jc and V; k steps of CPQR on C^T give Jr;
    R = A(Jr, :); with R^T = Qt Rt (thin Householder QR),
    U = V^T R^dagger = (V^T Qt) Rt^{-T}, i.e. the least-squares solution of
    U R = V^T (Sec. 2.5).  Q, when given, is the range finder's basis (saves
    recomputing it).  Returns dict(Jc (k,), Jr (k,), U (k x k), ID fields)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    d = qb_id(A, k, p, q, seed, Q=Q)
    J, T = d['J'], d['T']
    Jc = J[:k]
    C = A[:, Jc]
    fr = cpqr(C.T, k)
    Jr = fr['J'][:k]
    R = A[Jr, :]
    Qt, Rt = householder_qr(R.T)              # R^T = Qt Rt  (n x k, k x k)
    M = Qt[Jc, :] + T @ Qt[J[k:], :]          # V^T Qt
    # U Rt^T = M  <=>  Rt U^T = M^T
    U = solve_upper(Rt, M.T).T
    out = dict(d)
    out.update(Jc=Jc, Jr=Jr, U=U, frank_rows=fr['frank'],
               row_pivot_norms=fr['pivot_norms'],
               row_second_norms=fr['second_norms'])
    return out


def id_left(A, k, p, q, seed):
    """Randomized column ID with the Gaussian sketch on the left (Alg. 6).

    Omega~ is (k+p) x m; its transpose is drawn like the range finder's
    sketch but from stream philox.STREAM_LEFT (Omega~^T[i, j] = normal
    number j*m + i).  The sample is eq. (Ypower), Y = Omega~ A (A^T A)^q,
    with the columns orthonormalized before every product (the listing
    after eq. (Ypower)):
        Y^T = A^T Omega~^T;  q times { Y^T = A orth(Y^T);  Y^T = A^T orth(Y^T) }.
    Then k steps of the column-pivoted QR of Y (l x n) give J and
    T = S11^{-1} S12 as in qb_id (Alg. 6 keeps the first k of the l pivots,
    which are those of k greedy steps).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = sample_size(m, n, k, p)
    Ot = philox.sketch(seed, m, l, sid=philox.STREAM_LEFT)
    Yt = A.T @ Ot
    for _ in range(q):
        Yt = A @ orth(Yt)
        Yt = A.T @ orth(Yt)
    Y = Yt.T.copy()
    f = cpqr(Y, k)
    T = solve_upper(f['S11'], f['S12'])
    return dict(J=f['J'], T=T, frank=f['frank'], Y=Y,
                pivot_norms=f['pivot_norms'], second_norms=f['second_norms'],
                S22norm_F=f['S22norm_F'], S11=f['S11'], S12=f['S12'])


def qb_blocked(A, b, M, tol, q, seed):
    """Blocked adaptive QB decomposition (Alg. 7, scheme QB_2 of Sec. 3.3).

    For i = 1..M: Omega_i (n x b) is the sketch of philox.STREAM_QB with
    batch index i - 1; Q_i = orth(A Omega_i); q times { Q_i = orth(A^T Q_i);
    Q_i = orth(A Q_i) }; Q_i = orth(Q_i - sum_{j<i} Q_j Q_j^T Q_i);
    B_i = Q_i^T A; A = A - Q_i B_i; stop when ||A||_F < tol.  A here is a
    copy that the loop deflates, so the products of block i see
    (I - Qbar Qbar^T) A.  Returns dict(Q (m x bi), B (bi x n), nblocks = i,
    norms (||A||_F after each block), R = the deflated A).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    Qs, Bs, norms = [], [], []
    for i in range(M):
        Om = philox.sketch(seed, n, b, sid=philox.STREAM_QB, batch=i)
        Qi = orth(A @ Om)
        for _ in range(q):
            Qi = orth(A.T @ Qi)
            Qi = orth(A @ Qi)
        if Qs:
            Qbar = np.hstack(Qs)
            Qi = Qi - Qbar @ (Qbar.T @ Qi)
        Qi = orth(Qi)
        Bi = Qi.T @ A
        A = A - Qi @ Bi
        Qs.append(Qi)
        Bs.append(Bi)
        norms.append(np.linalg.norm(A))
        if norms[-1] < tol:
            break
    return dict(Q=np.hstack(Qs), B=np.vstack(Bs), nblocks=len(Qs), norms=np.array(norms), R=A)
