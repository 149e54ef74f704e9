"""Pins of the oracle's reverse-mode derivative of the randomized SVD.

* Each adjoint rule against central differences of the map it inverts (thin
  QR with positive diagonal; full SVD of a square matrix).
* The whole adjoint against central differences of the forward map, for
  q = 0, 1, 2 and cotangents on U, sigma and V at once.
* A of exact rank <= l: the range Q Q^T A = A does not move to first order
  in the singular values, so d(sum sigma)/dA = U_k V_k^T exactly.
"""

import numpy as np
import pytest

from oracle import grad as G
from oracle.dense import householder_qr, jacobi_svd
from paper_1502_05366_amd import workloads as W


def fixed_sign(U, V):
    """Flip singular pairs so that the largest entry of each u_i is positive
    (the convention is applied after every evaluation of a finite
    difference, so that the compared vectors follow one continuous branch)."""
    idx = np.argmax(np.abs(U), axis=0)
    sg = np.sign(U[idx, np.arange(U.shape[1])])
    sg[sg == 0] = 1.0
    return U * sg, V * sg, sg


def test_qr_adjoint_central_difference():
    g = np.random.default_rng(1)
    Y = g.standard_normal((30, 8))
    dQ, dR = g.standard_normal((30, 8)), np.triu(g.standard_normal((8, 8)))
    E = g.standard_normal((30, 8))
    Q, R = householder_qr(Y)
    dY = G.qr_adjoint(Q, R, dQ, dR)
    h = 1e-6
    Qp, Rp = householder_qr(Y + h * E)
    Qm, Rm = householder_qr(Y - h * E)
    fd = (np.sum(dQ * (Qp - Qm)) + np.sum(dR * (Rp - Rm))) / (2 * h)
    assert abs(fd - np.sum(dY * E)) < 1e-7 * max(1.0, abs(fd))


def test_svd_adjoint_central_difference():
    g = np.random.default_rng(2)
    l = 7
    A = g.standard_normal((l, l))
    dU, dV, ds = g.standard_normal((l, l)), g.standard_normal((l, l)), g.standard_normal(l)
    E = g.standard_normal((l, l))
    U, s, V, _, _ = jacobi_svd(A)
    U, V, _ = fixed_sign(U, V)
    dA = G.svd_adjoint(U, s, V, dU, ds, dV)
    h = 1e-6

    def L(M):
        u, ss, v, _, _ = jacobi_svd(M)
        u, v, _ = fixed_sign(u, v)
        return np.sum(dU * u) + np.sum(ds * ss) + np.sum(dV * v)
    fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
    assert abs(fd - np.sum(dA * E)) < 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rsvd_grad_central_difference(q):
    m, n, k, p, seed = 60, 45, 6, 4, 11
    A, _ = W.logspace_type(m, n, 1, seed=5)
    g = np.random.default_rng(q)
    dU, dS, dV = g.standard_normal((m, k)), g.standard_normal(k), g.standard_normal((n, k))
    dA, f = G.rsvd_grad(A, k, p, q, seed, dU, dS, dV)
    _, _, sg = fixed_sign(f["U"], f["V"])
    E = g.standard_normal((m, n))
    h = 1e-6

    def L(M):
        r = G.rsvd_forward_tape(M, k, p, q, seed)
        u, v = r["U"] * sg, r["V"] * sg      # the signs of the unperturbed pairs
        return np.sum(dU * u) + np.sum(dS * r["S"]) + np.sum(dV * v)
    # the unperturbed pairs carry their own signs: fold them into the cotangents
    dA_s, _ = G.rsvd_grad(A, k, p, q, seed, dU * sg, dS, dV * sg)
    fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
    assert abs(fd - np.sum(dA_s * E)) < 1e-6 * max(1.0, abs(fd))


def test_rsvd_grad_exact_rank_sum_sigma():
    A, s, _, _ = W.exact_rank_matrix(80, 50, 8, seed=4)
    k, p, q = 8, 4, 1
    dA, f = G.rsvd_grad(A, k, p, q, 3, dS=np.ones(k))
    assert np.abs(dA - f["U"] @ f["V"].T).max() < 1e-10


def test_copyltu():
    M = np.arange(9.0).reshape(3, 3)
    C = G.copyltu(M)
    assert np.array_equal(C, C.T) and np.array_equal(np.tril(C), np.tril(M))


@pytest.mark.parametrize("q", [0, 1])
def test_rsvd_grad_residual_central_difference(q):
    """The residual term: ||A - Q Q^T A||_F^2 is formed directly from Q and A
    in the forward, while its gradient goes through the singular values and
    2 A; central differences of the direct sum check the two agree."""
    m, n, k, p, seed = 50, 40, 5, 3, 21
    A, _ = W.logspace_type(m, n, 1, seed=6)
    g = np.random.default_rng(10 + q)
    dres = 0.7
    dA, f = G.rsvd_grad(A, k, p, q, seed, dres=dres)
    E = g.standard_normal((m, n))
    h = 1e-6
    fp = G.rsvd_forward_tape(A + h * E, k, p, q, seed)["resid2"]
    fm = G.rsvd_forward_tape(A - h * E, k, p, q, seed)["resid2"]
    fd = dres * (fp - fm) / (2 * h)
    assert abs(fd - np.sum(dA * E)) < 1e-6 * max(1.0, abs(fd))
    # the identity behind it: resid2 = ||A||^2 - sum of all l squared values
    assert abs(f["resid2"] - (np.sum(A * A) - np.sum(f["s"] ** 2))) < 1e-12 * np.sum(A * A)
