"""Pins of the oracle's dense factorizations (Householder QR, one-sided
Jacobi SVD, k-step CPQR, back substitution).

Each is pinned to something other than itself: LAPACK through numpy/scipy
(a different algorithm for QR / SVD / pivoted QR), closed forms, brute force
on tiny inputs, and the exact identities the paper states for CPQR
(Sec. 2.3: ||A - A_approx|| = ||S22||).
"""

import itertools

import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.interpolative as sli

from oracle import dense

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------- QR -------

@pytest.mark.parametrize("m,c", [(7, 1), (20, 20), (50, 12), (300, 31)])
def test_householder_qr_matches_lapack(m, c):
    g = np.random.default_rng(m * 100 + c)
    Y = g.standard_normal((m, c)) * np.logspace(0, -4, c)[None, :]
    Q, R = dense.householder_qr(Y)
    assert np.allclose(np.triu(R), R, atol=0)
    assert np.all(np.diag(R) > 0)
    assert np.abs(Q.T @ Q - np.eye(c)).max() < 20 * c * EPS
    assert np.abs(Q @ R - Y).max() < 20 * c * EPS * np.abs(Y).max()
    # positive-diagonal thin QR of a full-rank matrix is unique: LAPACK's
    # factors, sign-fixed, must agree
    Ql, Rl = np.linalg.qr(Y)
    d = np.sign(np.diag(Rl))
    assert np.abs(Ql * d - Q).max() < 1e-12
    assert np.abs((Rl * d[:, None]) - R).max() < 1e-12 * np.abs(R).max()


def test_householder_qr_zero_and_dependent_columns():
    g = np.random.default_rng(3)
    Y = g.standard_normal((30, 6))
    Y[:, 2] = 0.0
    Y[:, 4] = Y[:, 0] - 2 * Y[:, 1]
    Q, R = dense.householder_qr(Y)
    # Q stays orthonormal; Y is reproduced; the range of Y is inside range(Q)
    assert np.abs(Q.T @ Q - np.eye(6)).max() < 1e-13
    assert np.abs(Q @ R - Y).max() < 1e-13
    assert abs(R[2, 2]) < 1e-14 and abs(R[4, 4]) < 1e-13


def test_householder_qr_closed_form_2x2():
    Y = np.array([[3.0, 1.0], [4.0, 2.0]])
    Q, R = dense.householder_qr(Y)
    # R11 = ||y1|| = 5, R12 = q1.y2 = (3 + 8)/5, R22 = |det| / 5 = 2/5
    assert np.allclose(R, [[5.0, 11.0 / 5.0], [0.0, 2.0 / 5.0]], atol=1e-15)


# ------------------------------------------------------------ Jacobi -------

def test_round_robin_covers_every_pair_once():
    for c in range(1, 12):
        rounds = dense.round_robin_pairs(c)
        seen = []
        for r in rounds:
            cols = [x for pr in r for x in pr]
            assert len(cols) == len(set(cols))           # disjoint
            seen.extend(r)
        assert sorted(seen) == list(itertools.combinations(range(c), 2))


@pytest.mark.parametrize("c,decay", [(2, 0), (9, 2), (30, 3), (64, 6)])
def test_jacobi_matches_lapack_svd(c, decay):
    g = np.random.default_rng(c)
    Ua = np.linalg.qr(g.standard_normal((c, c)))[0]
    Va = np.linalg.qr(g.standard_normal((c, c)))[0]
    s_true = np.logspace(0, -decay, c)
    M = (Ua * s_true) @ Va.T
    U, s, V, sweeps, conv = dense.jacobi_svd(M)
    assert conv and sweeps < 30
    s_lapack = np.linalg.svd(M, compute_uv=False)
    # both are accurate to a small multiple of eps * sigma_1 (the matrix
    # itself carries rounding errors of that size from its construction)
    assert np.max(np.abs(s - s_lapack)) < 20 * c * EPS * s[0]
    assert np.max(np.abs(s - s_true)) < 20 * c * EPS * s[0]
    assert np.abs(U.T @ U - np.eye(c)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(c)).max() < 1e-13
    assert np.abs((U * s) @ V.T - M).max() < 50 * c * EPS


def test_jacobi_closed_form_2x2():
    # sigma of [[a, b], [0, d]]: sigma1 sigma2 = |a d|,
    # sigma1^2 + sigma2^2 = a^2 + b^2 + d^2
    a, b, d = 3.0, -4.0, 0.5
    _, s, _, _, _ = dense.jacobi_svd(np.array([[a, b], [0.0, d]]))
    tr, det = a * a + b * b + d * d, abs(a * d)
    s1 = np.sqrt((tr + np.sqrt(tr * tr - 4 * det * det)) / 2)
    assert abs(s[0] - s1) < 4 * EPS * s1
    assert abs(s[1] - det / s1) < 4 * EPS * s[1]


def test_jacobi_tall_upper_triangular_and_zero():
    g = np.random.default_rng(11)
    R = np.triu(g.standard_normal((20, 20)))
    R[:, 7] = 0.0
    U, s, V, _, conv = dense.jacobi_svd(R)
    assert conv
    assert s[-1] == 0.0 and np.all(U[:, -1] == 0.0)
    assert np.allclose(s, np.linalg.svd(R, compute_uv=False), rtol=1e-12, atol=1e-15)
    assert np.abs((U * s) @ V.T - R).max() < 1e-13


# ------------------------------------------------------ solve_upper -------

def test_solve_upper_matches_lapack_and_exact_integers():
    g = np.random.default_rng(5)
    S = np.triu(g.standard_normal((25, 25))) + 5 * np.eye(25)
    B = g.standard_normal((25, 7))
    X = dense.solve_upper(S, B)
    Xl = scipy.linalg.solve_triangular(S, B, lower=False)
    assert np.abs(X - Xl).max() < 1e-13
    # unit upper triangular integer matrix: back substitution is exact
    Si = np.triu(g.integers(-3, 4, (10, 10)).astype(float), 1) + np.eye(10)
    Xi = g.integers(-5, 6, (10, 3)).astype(float)
    assert np.array_equal(dense.solve_upper(Si, Si @ Xi), Xi)


# -------------------------------------------------------------- CPQR ------

@pytest.mark.parametrize("r,c,k,seed", [(10, 40, 6, 1), (30, 200, 25, 2), (8, 8, 8, 3)])
def test_cpqr_matches_lapack_pivoting(r, c, k, seed):
    g = np.random.default_rng(seed)
    B = g.standard_normal((r, c)) * g.uniform(0.1, 10.0, c)[None, :]
    f = dense.cpqr(B, k)
    _, Rl, Pl = scipy.linalg.qr(B, pivoting=True)
    # LAPACK dgeqp3 picks the same pivots when they are not near-tied
    margin = (f['pivot_norms'] - f['second_norms']) / f['pivot_norms']
    ok = np.cumprod(margin > 1e-6).astype(bool)
    npiv = int(ok.sum())
    assert npiv >= min(3, k)
    assert np.array_equal(f['J'][:npiv], Pl[:npiv])
    # |S11| equals |R| of LAPACK on those steps (rows may differ by sign)
    assert np.allclose(np.abs(f['S11'][:npiv, :npiv]), np.abs(Rl[:npiv, :npiv]),
                       rtol=1e-11, atol=1e-12 * np.abs(Rl[0, 0]))


def test_cpqr_error_identity():
    """||B - B(:, J_skel) V^T||_F = ||S22||_F with V = P [I; T^T] (Sec. 2.3/2.4)."""
    g = np.random.default_rng(9)
    B = g.standard_normal((15, 60)) @ np.diag(np.logspace(0, -3, 60))
    k = 7
    f = dense.cpqr(B, k)
    T = dense.solve_upper(f['S11'], f['S12'])
    V = np.zeros((60, k))
    V[f['J'][:k], np.arange(k)] = 1.0
    V[f['J'][k:], :] = T.T
    err = np.linalg.norm(B - B[:, f['J'][:k]] @ V.T)
    assert abs(err - f['S22norm_F']) < 1e-12 * np.linalg.norm(B)


def test_cpqr_brute_force_greedy():
    """Each pivot maximizes the distance of a column to the span of the
    columns chosen before it (the definition of greedy column pivoting)."""
    g = np.random.default_rng(21)
    B = g.standard_normal((6, 9)) * g.uniform(0.2, 3.0, 9)[None, :]
    k = 5
    f = dense.cpqr(B, k)
    chosen = []
    for s in range(k):
        best, bestd = None, -1.0
        for j in range(9):
            if j in chosen:
                continue
            if chosen:
                Cs = B[:, chosen]
                x = np.linalg.lstsq(Cs, B[:, j], rcond=None)[0]
                dist = np.linalg.norm(B[:, j] - Cs @ x)
            else:
                dist = np.linalg.norm(B[:, j])
            if dist > bestd + 1e-12:
                best, bestd = j, dist
        chosen.append(best)
        assert abs(f['pivot_norms'][s] - bestd) < 1e-12
    assert list(f['J'][:k]) == chosen


def test_cpqr_matches_scipy_interpolative():
    g = np.random.default_rng(4)
    B = g.standard_normal((12, 50)) * g.uniform(0.1, 5.0, 50)[None, :]
    k = 9
    f = dense.cpqr(B, k)
    T = dense.solve_upper(f['S11'], f['S12'])
    idx, proj = sli.interp_decomp(B.copy(order='F'), k, rand=False)
    assert np.array_equal(np.asarray(idx[:k]), f['J'][:k])
    # scipy orders the residual columns as idx[k:]; ours ascend
    order = np.argsort(idx[k:])
    assert np.abs(proj[:, order] - T).max() < 1e-10


def test_cpqr_ties_and_rank():
    # identical columns tie exactly: the lowest index wins
    B = np.zeros((4, 6))
    B[:, 1] = B[:, 4] = [1.0, 2.0, 0.0, 0.0]
    B[:, 3] = [0.0, 0.0, 1.0, 0.0]
    f = dense.cpqr(B, 3)
    assert f['J'][0] == 1
    assert f['J'][1] == 3
    # after two steps nothing is left: numerical rank is 2
    assert f['frank'] == 2
