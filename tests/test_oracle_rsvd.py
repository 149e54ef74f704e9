"""Pins of the oracle's range finder, RSVD, ID and CUR against what the paper
and the mathematics fix.

* Lemma of Sec. 3 (range(A) in range(Q) iff A = Q Q^T A): exact recovery for
  A of exact rank <= k.
* Eckart-Young (Sec. 2.2): no rank-k result beats sigma_{k+1}.
* The deterministic error bound quoted in Sec. 3 (with the square on the
  left-hand side, as in the cited survey).
* The approximate RSVD bounds of Sec. 3.4.
* Sec. 3.4: Alg. 4, Alg. 5 and Fig. 1 give the same factors.
* Sec. 3.2: the power scheme samples range((A A^T)^q A Omega), with or without
  re-orthonormalization.
* Sec. 2.3-2.5: ID error = ||S22||, the two-sided ID has the same
  approximant, CUR solves U R = V^T in the least-squares sense, and a
  matrix with separated orthogonal columns has a known skeleton.
* Sec. 3.5: the ID-from-B bound.
* Sec. 5: the qualitative claims about q on slow and fast decay.
"""

import numpy as np
import pytest

from oracle import philox, rsvd as O
from oracle.dense import householder_qr
from paper_1502_05366_amd import workloads as W

EPS = np.finfo(np.float64).eps


def spec2(M):
    return np.linalg.norm(M, 2)


@pytest.mark.parametrize("m,n,r,k,p,q", [(80, 60, 5, 5, 5, 0), (60, 90, 7, 10, 4, 1),
                                         (120, 40, 12, 12, 8, 2)])
def test_exact_recovery(m, n, r, k, p, q):
    A, s, _, _ = W.exact_rank_matrix(m, n, r, seed=m + n)
    U, sh, V = O.rsvd(A, k, p, q, seed=7)
    assert np.max(np.abs(sh[:r] - s) / s) < 1e-12
    assert np.all(np.abs(sh[r:]) < 1e-13 * s[0])
    assert spec2(A - (U * sh) @ V.T) < 1e-13 * s[0]
    Q = O.range_finder(A, k, p, q, seed=7)
    assert spec2(A - Q @ (Q.T @ A)) < 1e-13 * s[0]
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13


@pytest.mark.parametrize("kind,k,q", [(1, 10, 0), (2, 15, 1), (3, 20, 2)])
def test_eckart_young_and_interlacing(kind, k, q):
    A, s = W.logspace_type(150, 100, kind, seed=kind)
    U, sh, V = O.rsvd(A, k, 5, q, seed=11)
    E = A - (U * sh) @ V.T
    assert spec2(E) >= s[k] * (1 - 1e-10)
    assert np.linalg.norm(E) >= np.sqrt(np.sum(s[k:] ** 2)) * (1 - 1e-10)
    # Ritz values from a subspace never exceed the true singular values
    assert np.all(sh <= s[:k] * (1 + 1e-12))
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-13


def test_deterministic_bound():
    """||(I - P_Y) A||^2 <= ||Sigma2||^2 + ||Sigma2 Omega2 Omega1^+||^2 (q = 0)."""
    m, n, k, p = 90, 70, 8, 4
    s = 0.7 ** np.arange(n)
    A, U, V = W.spectrum_matrix(m, n, s, seed=3)
    l = k + p
    Om = philox.sketch(21, n, l)
    Q = O.range_finder(A, k, p, 0, seed=21)
    lhs = spec2(A - Q @ (Q.T @ A)) ** 2
    Om1, Om2 = V[:, :k].T @ Om, V[:, k:].T @ Om
    S2 = np.diag(s[k:])
    rhs = spec2(S2) ** 2 + spec2(S2 @ Om2 @ np.linalg.pinv(Om1)) ** 2
    assert lhs <= rhs * (1 + 1e-10)
    # the Frobenius form holds too
    lhsF = np.linalg.norm(A - Q @ (Q.T @ A)) ** 2
    rhsF = np.linalg.norm(S2) ** 2 + np.linalg.norm(S2 @ Om2 @ np.linalg.pinv(Om1)) ** 2
    assert lhsF <= rhsF * (1 + 1e-10)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_paper_bound_sec34(q):
    """||A - U_k S_k V_k^T||_2 <= (k n)^(1/(2(2q+1))) sigma_{k+1} (approximate)."""
    m, n, k = 200, 120, 10
    A, s = W.logspace_type(m, n, 2, seed=5)
    U, sh, V = O.rsvd(A, k, 10, q, seed=13)
    err = spec2(A - (U * sh) @ V.T)
    assert err <= (k * n) ** (1.0 / (2 * (2 * q + 1))) * s[k]


def test_alg4_alg5_fig1_agree():
    A, s = W.logspace_type(120, 90, 3, seed=8)
    k, p, q = 12, 6, 1
    U5, s5, V5 = O.rsvd(A, k, p, q, seed=2)
    U1, s1, V1 = O.rsvd_fig1(A, k, p, q, seed=2)
    U4, s4, V4 = O.rsvd_alg4(A, k, p, q, seed=2)
    assert np.max(np.abs(s5 - s1) / s5) < 1e-12
    assert np.max(np.abs(s5 - s4) / s5) < 1e-10
    for Ua, Ub in ((U5, U1), (U5, U4), (V5, V1), (V5, V4)):
        # singular vectors agree up to sign (the spectrum is simple)
        d = np.abs(np.sum(Ua * Ub, axis=0))
        assert np.max(np.abs(d - 1)) < 1e-8


def test_full_rank_sample_is_exact_svd():
    A, s = W.logspace_type(40, 30, 2, seed=1)
    U, sh, V = O.rsvd(A, 30, 5, 0, seed=1)      # l clamps to min(m, n)
    assert np.max(np.abs(sh - s) / s) < 1e-12
    assert spec2(A - (U * sh) @ V.T) < 1e-13


def test_power_scheme_span():
    """Sec. 3.2: Y = (A A^T)^q A Omega (no re-orthonormalization) spans the
    same space as the re-orthonormalized scheme; its singular values follow
    sigma^(2q+1)."""
    A, s = W.logspace_type(70, 50, 1, seed=4)
    k, p, q = 6, 4, 2
    l = k + p
    Om = philox.sketch(99, 50, l)
    Y = A @ Om
    for _ in range(q):
        Y = A @ (A.T @ Y)
    Qa = householder_qr(Y)[0]
    Qb = O.range_finder(A, k, p, q, seed=99)
    assert spec2(Qa @ Qa.T - Qb @ Qb.T) < 1e-9
    sv = np.linalg.svd(A @ (A.T @ A) @ (A.T @ A), compute_uv=False)
    assert np.allclose(sv, s ** 5, rtol=1e-10, atol=1e-14)


def test_fig3_qualitative_power_helps_slow_decay():
    A, s = W.logspace_type(300, 200, 1, seed=12)   # type I: slow decay
    k = 20
    errs = []
    for q in (0, 1, 2):
        U, sh, V = O.rsvd(A, k, 5, q, seed=3)
        errs.append(spec2(A - (U * sh) @ V.T))
    assert errs[0] > errs[1] > errs[2] >= s[k] * (1 - 1e-10)
    # type III (fast decay): q = 1 is already close to optimal
    A3, s3 = W.logspace_type(300, 200, 3, seed=12)
    U, sh, V = O.rsvd(A3, k, 5, 1, seed=3)
    assert spec2(A3 - (U * sh) @ V.T) < 1.5 * s3[k]


# ------------------------------------------------------------ ID / CUR ----

def test_separated_skeleton_is_recovered():
    m, n, r = 120, 300, 24
    A, pi, d = W.separated_skeleton_matrix(m, n, r, seed=17)
    k, p = 16, 8                                   # l = r: Q Q^T A = A
    res = O.qb_id(A, k, p, 1, seed=5)
    assert list(res['J'][:k]) == list(pi[:k])
    assert np.allclose(res['pivot_norms'], d[:k], rtol=1e-12)


def test_id_error_identity_and_bound():
    A, s = W.logspace_type(150, 120, 3, seed=6)
    k, p, q = 10, 6, 1
    res = O.qb_id(A, k, p, q, seed=8)
    J, T, B, Q = res['J'], res['T'], res['B'], res['Q']
    V = O.interp_matrix(J, T, A.shape[1])
    # exact identity on B (Sec. 2.3/2.4): ||B - B(:, J) V^T|| = ||S22||
    eB = np.linalg.norm(B - B[:, J[:k]] @ V.T)
    assert abs(eB - res['S22norm_F']) < 1e-12 * np.linalg.norm(B)
    # Sec. 3.5 bound with eps = ||A - Q B||
    eps = spec2(A - Q @ B)
    eA = spec2(A - A[:, J[:k]] @ V.T)
    n = A.shape[1]
    assert eA <= (1 + np.sqrt(1 + 4 * k * (n - k))) * eps
    # the ID is never better than the best rank-k approximation
    assert eA >= s[k] * (1 - 1e-10)
    # V has the identity on the skeleton
    assert np.array_equal(V[J[:k]], np.eye(k))


def test_two_sided_id_same_approximant():
    A, s = W.logspace_type(90, 70, 3, seed=9)
    k = 8
    res = O.qb_id(A, k, 6, 1, seed=1)
    J, T = res['J'], res['T']
    V = O.interp_matrix(J, T, A.shape[1])
    Jr, Wm, frank = O.two_sided_id(A, J, k)
    C = A[:, J[:k]]
    assert frank == k
    # C = W C(Jr, :) exactly (rank C = k) and W A(Jr, Jc) V^T = C V^T
    assert np.abs(Wm @ C[Jr, :] - C).max() < 1e-10 * np.abs(C).max()
    assert np.abs(Wm @ A[np.ix_(Jr, J[:k])] @ V.T - C @ V.T).max() < 1e-10
    assert np.array_equal(Wm[Jr], np.eye(k)) or np.abs(Wm[Jr] - np.eye(k)).max() < 1e-12


def test_cur_least_squares_and_exact_rank():
    A, s = W.logspace_type(100, 80, 3, seed=10)
    k = 9
    res = O.cur(A, k, 6, 1, seed=4)
    Jc, Jr, U = res['Jc'], res['Jr'], res['U']
    R = A[Jr, :]
    V = O.interp_matrix(res['J'], res['T'], A.shape[1])
    # normal equations of min ||U R - V^T||_F: (U R - V^T) R^T = 0
    G = (U @ R - V.T) @ R.T
    assert np.abs(G).max() < 1e-12 * max(1.0, np.abs(R).max()) ** 2
    # CUR error is bounded below by sigma_{k+1}
    C = A[:, Jc]
    assert spec2(A - C @ U @ R) >= s[k] * (1 - 1e-10)
    # exact rank k: CUR reproduces A
    Ae, se, _, _ = W.exact_rank_matrix(60, 50, 6, seed=2)
    r2 = O.cur(Ae, 6, 4, 1, seed=3)
    Ce, Re = Ae[:, r2['Jc']], Ae[r2['Jr'], :]
    assert spec2(Ae - Ce @ r2['U'] @ Re) < 1e-11 * se[0]


def test_rank_deficient_id_reports_frank():
    Ae, _, _, _ = W.exact_rank_matrix(50, 40, 4, seed=5)
    res = O.qb_id(Ae, 8, 4, 1, seed=1)
    assert res['frank'] == 4
