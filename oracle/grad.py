"""Reverse-mode derivative of the randomized SVD (FP64), with the Gaussian
sketch held fixed.

Test infrastructure, like the rest of this package: only tests, smoke() and
the benchmark's cpu_baseline leg may use it.

The forward map is the one of ``rsvd.rsvd`` (Alg. 5 with re-orthonormalization
after every product, Sec. 3.2):

    Y_0 = A Omega;  for j < q: Q_j, R_j = qr(Y_j); Z_j = A^T Q_j;
                               P_j, S_j = qr(Z_j); Y_{j+1} = A P_j
    Q, R_q = qr(Y_q);  B^T = A^T Q;  Qh, Rh = qr(B^T);  Rh = Uh diag(s) Vh^T
    U_k = Q Vh[:, :k],  V_k = Qh Uh[:, :k],  sigma = s[:k]

Every qr is the thin QR with a positive diagonal (unique for full rank), so
the map is differentiable wherever the Y's and Z's have full rank and the
singular values of Rh are distinct.  The adjoint walks these steps backwards
with the two rules below; a product C = A X contributes dA += dC X^T and
dX = A^T dC.
"""

import numpy as np

from . import philox
from .dense import householder_qr, jacobi_svd
from .rsvd import sample_size


def copyltu(M):
    """The symmetric matrix with the lower triangle of M (diagonal included)."""
    L = np.tril(M)
    return L + np.tril(M, -1).T


def qr_adjoint(Q, R, dQ, dR=None):
    """dY for Y = Q R (thin QR, Q^T Q = I, R upper triangular with positive
    diagonal): dY = (dQ + Q copyltu(M)) R^{-T} with M = R dR^T - dQ^T Q.

    Derivation: from dY = dQ R + Q dR, Q^T dQ is skew and dR R^{-1} upper
    triangular; projecting the first-order identities onto the skew and the
    triangular parts and pairing with the cotangents gives the formula.
    """
    M = -(dQ.T @ Q)
    if dR is not None:
        M = M + R @ dR.T
    C = dQ + Q @ copyltu(M)
    # C R^{-T}: solve R X^T = C^T
    return np.linalg.solve(R, C.T).T


def svd_adjoint(U, s, V, dU, ds, dV):
    """dA for the full SVD A = U diag(s) V^T of a square matrix with distinct
    singular values:
        dA = U [ (F o (U^T dU - dU^T U)) S + diag(ds) + S (F o (V^T dV - dV^T V)) ] V^T,
    F_ij = 1 / (s_j^2 - s_i^2) (i != j), F_ii = 0, S = diag(s)."""
    l = len(s)
    s2 = s * s
    D = s2[None, :] - s2[:, None]
    F = np.zeros((l, l))
    off = ~np.eye(l, dtype=bool)
    F[off] = 1.0 / D[off]
    Ju = F * (U.T @ dU - dU.T @ U)
    Jv = F * (V.T @ dV - dV.T @ V)
    inner = Ju * s[None, :] + np.diag(ds) + s[:, None] * Jv
    return U @ inner @ V.T


def rsvd_forward_tape(A, k, p, q, seed):
    """The forward map above with every intermediate kept."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = sample_size(m, n, k, p)
    Om = philox.sketch(seed, n, l)
    tape = []
    Y = A @ Om
    for _ in range(q):
        Qy, Ry = householder_qr(Y)
        Z = A.T @ Qy
        Qz, Rz = householder_qr(Z)
        tape.append((Qy, Ry, Qz, Rz))
        Y = A @ Qz
    Q, Rq = householder_qr(Y)
    Bt = A.T @ Q
    Qh, Rh = householder_qr(Bt)
    Uh, s, Vh, _, _ = jacobi_svd(Rh)
    return dict(A=A, Om=Om, tape=tape, Q=Q, Rq=Rq, Qh=Qh, Rh=Rh, Uh=Uh, s=s, Vh=Vh, k=k,
                U=Q @ Vh[:, :k], S=s[:k].copy(), V=Qh @ Uh[:, :k],
                resid2=float(np.sum((A - Q @ Bt.T) ** 2)))


def rsvd_grad(A, k, p, q, seed, dU=None, dS=None, dV=None, dres=None):
    """dA = the gradient of <dU, U_k> + <dS, sigma> + <dV, V_k>
    + dres ||A - Q Q^T A||_F^2 with respect to A (cotangents left out count as
    zero).  Returns (dA, forward dict).

    The residual term uses ||A - Q Q^T A||_F^2 = ||A||_F^2 - ||Q^T A||_F^2
    (Q^T Q = I) and ||Q^T A||_F = ||B^T||_F = ||Rh||_F, whose square is the sum
    of all l squared singular values of Rh: its cotangent is 2 dres A directly
    plus ds_i = -2 dres s_i through the chain."""
    f = rsvd_forward_tape(A, k, p, q, seed)
    A = f["A"]
    m, n = A.shape
    Q, Qh, Uh, Vh, s = f["Q"], f["Qh"], f["Uh"], f["Vh"], f["s"]
    l = len(s)
    dQ = np.zeros((m, l))
    dQh = np.zeros((n, l))
    dUh = np.zeros((l, l))
    dVh = np.zeros((l, l))
    ds = np.zeros(l)
    if dU is not None:                 # U_k = Q Vh_k
        dQ += dU @ Vh[:, :k].T
        dVh[:, :k] = Q.T @ dU
    if dV is not None:                 # V_k = Qh Uh_k
        dQh += dV @ Uh[:, :k].T
        dUh[:, :k] = Qh.T @ dV
    if dS is not None:
        ds[:k] = dS
    if dres is not None:
        ds -= 2.0 * dres * s
    dRh = svd_adjoint(Uh, s, Vh, dUh, ds, dVh)
    dBt = qr_adjoint(Qh, f["Rh"], dQh, dRh)
    dA = Q @ dBt.T                     # B^T = A^T Q
    dQ = dQ + A @ dBt
    dY = qr_adjoint(Q, f["Rq"], dQ)
    for Qy, Ry, Qz, Rz in reversed(f["tape"]):
        dA += dY @ Qz.T                # Y = A Qz
        dZ = qr_adjoint(Qz, Rz, A.T @ dY)
        dA += Qy @ dZ.T                # Z = A^T Qy
        dY = qr_adjoint(Qy, Ry, A @ dZ)
    dA += dY @ f["Om"].T               # Y_0 = A Omega
    if dres is not None:
        dA += 2.0 * dres * A
    return dA, f
