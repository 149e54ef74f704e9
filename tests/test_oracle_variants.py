"""Pins of the oracle's variants of Sec. 3.3 and 3.5 against what the paper and
the mathematics fix.

Left-sketch ID (Alg. 6, eq. (Ypower)):
* exact rank: the row space of Y is that of A, so the ID reproduces A;
* the orthonormalized power scheme samples the row space of
  Omega~ A (A^T A)^q, the un-orthonormalized form of eq. (Ypower);
* with q >= 1 and orthogonal skeleton columns the pivots are known;
* Eckart-Young from below and the deterministic pivoted-QR ID from above
  (the text of Sec. 3.5: the error stays close to that of the truncated
  pivoted QR when q >= 1).
"""

import numpy as np
import pytest

from oracle import philox, rsvd as O
from oracle.dense import cpqr, solve_upper
from paper_1502_05366_amd import workloads as W


def id_error(A, J, T):
    """||A - A(:, J[:k]) V^T||_2 with V = P [I_k; T^T]."""
    V = O.interp_matrix(J, T, A.shape[1])
    return np.linalg.norm(A - A[:, J[:T.shape[0]]] @ V.T, 2)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_id_left_exact_rank(q):
    A, s, _, _ = W.exact_rank_matrix(150, 90, 9, seed=31)
    d = O.id_left(A, 12, 5, q, seed=3)
    assert id_error(A, d["J"], d["T"]) <= 1e-11 * s[0]


@pytest.mark.parametrize("q", [1, 2])
def test_id_left_power_row_space(q):
    # sigma in [1e-1, 1]: the plain powers lose nothing at these sizes
    m, n, k, p = 120, 80, 10, 6
    A, _ = W.logspace_type(m, n, 1, seed=17)
    d = O.id_left(A, k, p, q, seed=5)
    Ot = philox.sketch(5, m, k + p, sid=philox.STREAM_LEFT)
    Yplain = Ot.T @ A @ np.linalg.matrix_power(A.T @ A, q)
    Q1 = np.linalg.qr(d["Y"].T)[0]
    # sine of the largest principal angle, ||(I - Q2 Q2^T) Q1||_2 (accurate
    # to rounding, unlike sqrt(1 - cos^2))
    def gap(Qa, Qb):
        return np.linalg.norm(Qa - Qb @ (Qb.T @ Qa), 2)
    assert gap(Q1, np.linalg.qr(Yplain.T)[0]) < 1e-10
    # one product too many samples a different space
    Ywrong = Ot.T @ A @ np.linalg.matrix_power(A.T @ A, q + 1)
    assert gap(Q1, np.linalg.qr(Ywrong.T)[0]) > 1e-6


@pytest.mark.parametrize("q", [1, 2])
def test_id_left_separated_skeleton(q):
    A, pi, dd = W.separated_skeleton_matrix(300, 500, 20, seed=23)
    d = O.id_left(A, 12, 8, q, seed=9)
    assert list(d["J"][:12]) == list(pi[:12])


def test_id_left_error_between_bounds():
    m, n, k, p = 300, 200, 15, 10
    A, s = W.logspace_type(m, n, 2, seed=41)
    d = O.id_left(A, k, p, 2, seed=11)
    err = id_error(A, d["J"], d["T"])
    f = cpqr(A, k)
    err_det = id_error(A, f["J"], solve_upper(f["S11"], f["S12"]))
    assert err >= s[k] * (1.0 - 1e-12)
    assert err <= 10.0 * err_det


def test_id_left_sketch_stream():
    # Omega~^T is stream 6 of the generator, not the range finder's stream 0
    a = philox.sketch(1, 40, 6, sid=philox.STREAM_LEFT)
    b = philox.sketch(1, 40, 6)
    assert a.shape == (40, 6) and not np.allclose(a, b)
    assert np.array_equal(a, philox.sketch(1, 40, 6, sid=6))
