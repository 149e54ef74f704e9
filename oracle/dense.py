"""Dense FP64 factorizations used by the oracle, written out step by step.

Test infrastructure (see the package header): only tests, smoke() and the
bench's cpu_baseline leg may use it.

* ``householder_qr``  -- ``orth`` / ``qr(Y, 0)`` of Sec. 2.1 (notation), done
  with Householder reflections (Golub & Van Loan, Sec. 5.2, the paper's
  reference for QR in Sec. 2.3), thin Q formed explicitly, column signs fixed
  so that diag(R) >= 0 (then the factorization of a full-rank matrix is
  unique).
* ``jacobi_svd``      -- the small SVD ``svd(R_hat)`` of Alg. 5, by one-sided
  (Hestenes) Jacobi rotations in a round-robin pair ordering.
* ``cpqr``            -- k steps of the column-pivoted QR of Sec. 2.3
  (A P = Q S and its truncation after k steps), with exact residual column norms
  recomputed at each step and ties broken by the lowest column index.
* ``solve_upper``     -- back substitution, for T = S11^{-1} S12 (Sec. 2.4)
  and the CUR factor U (Sec. 2.5, Alg. 3).
"""

import numpy as np

EPS = np.finfo(np.float64).eps


def _sign(x):
    """sign with sign(0) = +1."""
    return 1.0 if x >= 0.0 else -1.0


def householder_qr(Y):
    """Thin QR of an m x c matrix (m >= c) by Householder reflections.

    Step j reflects x = R[j:, j] onto -sign(x_0)||x|| e_1 with
    H = I - beta v v^T, v = x + sign(x_0)||x|| e_1, beta = 2 / v^T v, and
    applies H to the trailing columns.  Q is then accumulated backwards from
    the first c columns of the identity.  Finally D = sign(diag(R)) gives
    Q <- Q D, R <- D R so that diag(R) >= 0.  A zero column leaves H = I.
    Returns (Q, R): Q m x c with orthonormal columns, R c x c upper triangular.
    """
    R = np.array(Y, dtype=np.float64, copy=True)
    m, c = R.shape
    if m < c:
        raise ValueError("householder_qr needs m >= c")
    vs, betas = [], []
    for j in range(c):
        x = R[j:, j].copy()
        normx = np.sqrt(np.dot(x, x))
        v = x
        if normx == 0.0:
            beta = 0.0
        else:
            v[0] += _sign(x[0]) * normx
            beta = 2.0 / np.dot(v, v)
        if beta != 0.0:
            w = v @ R[j:, j:]
            R[j:, j:] -= np.outer(beta * v, w)
        vs.append(v)
        betas.append(beta)
    Rout = np.triu(R[:c, :c])
    Q = np.zeros((m, c))
    Q[np.arange(c), np.arange(c)] = 1.0
    for j in range(c - 1, -1, -1):
        v, beta = vs[j], betas[j]
        if beta != 0.0:
            w = v @ Q[j:, j:]
            Q[j:, j:] -= np.outer(beta * v, w)
    d = np.array([_sign(Rout[i, i]) for i in range(c)])
    return Q * d[None, :], Rout * d[:, None]


def round_robin_pairs(c):
    """Round-robin (circle method) schedule of all column pairs of c columns.

    With N = c rounded up to even, position 0 is fixed and positions 1..N-1
    rotate by one each round; round r pairs position i with position N-1-i.
    Pairs that involve the padding column (index c when c is odd) are dropped.
    Each of the N-1 rounds is a list of disjoint pairs (a, b) with a < b, and
    every pair of columns appears in exactly one round.
    """
    N = c + (c % 2)
    rounds = []
    for r in range(N - 1):
        def player(pos):
            return 0 if pos == 0 else ((pos - 1 + r) % (N - 1)) + 1
        pairs = []
        for i in range(N // 2):
            a, b = player(i), player(N - 1 - i)
            if a < c and b < c:
                pairs.append((min(a, b), max(a, b)))
        rounds.append(pairs)
    return rounds


def jacobi_svd(Rm, max_sweeps=60, tol=None):
    """One-sided (Hestenes) Jacobi SVD of a square or tall matrix, FP64.

    Columns a_p, a_q are rotated so that they become orthogonal: with
    alpha = a_p.a_p, beta = a_q.a_q, gamma = a_p.a_q,
    zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| + sqrt(1+zeta^2))
    (sign(0) = +1), c = 1/sqrt(1+t^2), s = c t:
        a_p <- c a_p - s a_q,   a_q <- s a_p + c a_q,
    and the same rotation is accumulated into V (started at I).  A pair is
    skipped when |gamma| <= tol * sqrt(alpha beta); a sweep with no rotation
    ends the iteration.  Rotations of one round act on disjoint pairs, so
    applying them together is the same as applying them one after another.
    On exit A V = W has orthogonal columns; sigma_j = ||w_j||, u_j = w_j/sigma_j
    (u_j = 0 when sigma_j = 0).  Singular values are sorted descending with a
    stable sort.  Returns (U, s, V, sweeps, converged) with A = U diag(s) V^T.
    """
    W = np.array(Rm, dtype=np.float64, copy=True)
    m, c = W.shape
    if tol is None:
        tol = max(m, c) * EPS
    V = np.eye(c)
    rounds = [np.array(r, dtype=np.int64).reshape(-1, 2)
              for r in round_robin_pairs(c)]
    converged = c < 2
    sweeps = 0
    while not converged and sweeps < max_sweeps:
        sweeps += 1
        rotated = False
        for pr in rounds:
            if len(pr) == 0:
                continue
            P, Qi = pr[:, 0], pr[:, 1]
            ap, aq = W[:, P], W[:, Qi]
            alpha = np.einsum('ij,ij->j', ap, ap)
            beta = np.einsum('ij,ij->j', aq, aq)
            gamma = np.einsum('ij,ij->j', ap, aq)
            act = np.abs(gamma) > tol * np.sqrt(alpha * beta)
            if not np.any(act):
                continue
            rotated = True
            P, Qi = P[act], Qi[act]
            alpha, beta, gamma = alpha[act], beta[act], gamma[act]
            zeta = (beta - alpha) / (2.0 * gamma)
            sg = np.where(zeta >= 0.0, 1.0, -1.0)
            t = sg / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta))
            cs = 1.0 / np.sqrt(1.0 + t * t)
            sn = cs * t
            ap, aq = W[:, P], W[:, Qi]
            W[:, P] = cs * ap - sn * aq
            W[:, Qi] = sn * ap + cs * aq
            vp, vq = V[:, P], V[:, Qi]
            V[:, P] = cs * vp - sn * vq
            V[:, Qi] = sn * vp + cs * vq
        if not rotated:
            converged = True
    s = np.sqrt(np.einsum('ij,ij->j', W, W))
    order = np.argsort(-s, kind='stable')
    s = s[order]
    W = W[:, order]
    V = V[:, order]
    U = np.zeros_like(W)
    nz = s > 0.0
    U[:, nz] = W[:, nz] / s[nz]
    return U, s, V, sweeps, converged


def solve_upper(S, B):
    """Solve S X = B for upper-triangular S (c x c), B c x r, by back
    substitution: x_i = (b_i - sum_{j>i} S_ij x_j) / S_ii for i = c-1 .. 0."""
    S = np.asarray(S, dtype=np.float64)
    X = np.array(B, dtype=np.float64, copy=True)
    c = S.shape[0]
    for i in range(c - 1, -1, -1):
        if i + 1 < c:
            X[i] -= S[i, i + 1:] @ X[i + 1:]
        X[i] /= S[i, i]
    return X


def cpqr(B, k, rank_tol=None):
    """k steps of the column-pivoted Householder QR of an r x c matrix B.

    Step s (0-based) computes the squared norms of the residual columns
    B[s:, j] over the columns not yet chosen, picks the largest (lowest
    column index among exact ties), builds the reflector of that column on
    rows s.., and applies it to rows s.. of every column not yet chosen.
    Chosen columns keep their position; the order of the remaining columns is
    ascending column index.  After k steps the factor is
        S11 = W[:k, J_skel] (k x k, upper triangular in pivot order),
        S12 = W[:k, J_res]  (k x (c-k)),
    and ||S22|| is the norm of the remaining residual block (the truncation and the
    identity ||A - A_approx|| = ||S22|| of Sec. 2.3).

    ``frank`` is the first step whose largest residual norm is <= rank_tol
    (default max(r, c) * eps * ||B||_F), or k when there is none.

    Returns dict(J=skeleton+residual indices (c,), S11, S12, S22norm_F,
    frank, pivot_norms (k,), second_norms (k,)) where second_norms[s] is the
    runner-up residual norm at step s (the pivot margin).
    """
    W = np.array(B, dtype=np.float64, copy=True)
    r, c = W.shape
    if not 1 <= k <= min(r, c):
        raise ValueError("cpqr needs 1 <= k <= min(rows, cols)")
    if rank_tol is None:
        rank_tol = max(r, c) * EPS * np.sqrt(np.sum(W * W))
    chosen = np.zeros(c, dtype=bool)
    J_skel = []
    pivot_norms, second_norms = [], []
    frank = k
    for s in range(k):
        free = np.nonzero(~chosen)[0]
        nrm2 = np.einsum('ij,ij->j', W[s:, free], W[s:, free])
        best = int(np.argmax(nrm2))        # first maximum = lowest index
        p = int(free[best])
        pivot_norms.append(np.sqrt(nrm2[best]))
        rest = np.delete(nrm2, best)
        second_norms.append(np.sqrt(rest.max()) if rest.size else 0.0)
        if frank == k and pivot_norms[-1] <= rank_tol:
            frank = s
        x = W[s:, p].copy()
        normx = np.sqrt(np.dot(x, x))
        if normx > 0.0:
            v = x
            v[0] += _sign(x[0]) * normx
            beta = 2.0 / np.dot(v, v)
            cols = free
            w = v @ W[s:, cols]
            W[s:, cols] -= np.outer(beta * v, w)
            W[s + 1:, p] = 0.0
        chosen[p] = True
        J_skel.append(p)
    J_res = np.nonzero(~chosen)[0]
    J = np.concatenate([np.array(J_skel, dtype=np.int64), J_res.astype(np.int64)])
    S11 = np.triu(W[:k, J_skel])
    S12 = W[:k, J_res]
    S22 = W[k:, J_res]
    return dict(J=J, S11=S11, S12=S12, S22norm_F=float(np.sqrt(np.sum(S22 * S22))),
                frank=frank, pivot_norms=np.array(pivot_norms),
                second_norms=np.array(second_norms))
