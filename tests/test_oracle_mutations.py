"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one line of an oracle function (a dropped term, a wrong
sign, a swapped operand, a wrong constant), installs the mutated function for
the duration of the test, and runs a pin that must then fail.  This runs on
the CPU only and touches nothing but the oracle.
"""

import inspect
import textwrap

import numpy as np
import pytest

from oracle import dense, grad as G, philox, rsvd as O
from paper_1502_05366_amd import workloads as W


def _mutated(func, old, new):
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) == 1, (func.__name__, old)
    src = src.replace(old, new)
    ns = dict(func.__globals__)
    exec(compile(src, f"<mutant of {func.__name__}>", "exec"), ns)
    return ns[func.__name__]


def _install(monkeypatch, func, old, new):
    mut = _mutated(func, old, new)
    for mod in (dense, philox, O, G):
        if getattr(mod, func.__name__, None) is func:
            monkeypatch.setattr(mod, func.__name__, mut)
    return mut


# ---- pins reused as checks ----------------------------------------------

def pin_qr():
    g = np.random.default_rng(1)
    Y = g.standard_normal((40, 9))
    Q, R = dense.householder_qr(Y)
    assert np.abs(Q.T @ Q - np.eye(9)).max() < 1e-12
    assert np.abs(Q @ R - Y).max() < 1e-12


def pin_jacobi():
    g = np.random.default_rng(2)
    M = g.standard_normal((12, 12))
    U, s, V, _, conv = dense.jacobi_svd(M, max_sweeps=40)
    assert conv
    assert np.allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-12)
    assert np.abs((U * s) @ V.T - M).max() < 1e-12


def pin_cpqr():
    g = np.random.default_rng(3)
    B = g.standard_normal((6, 9)) * g.uniform(0.2, 3.0, 9)[None, :]
    f = dense.cpqr(B, 4)
    chosen = []
    for s in range(4):
        best, bestd = None, -1.0
        for j in range(9):
            if j in chosen:
                continue
            Cs = B[:, chosen]
            dist = np.linalg.norm(B[:, j] - Cs @ np.linalg.lstsq(Cs, B[:, j], rcond=None)[0]) \
                if chosen else np.linalg.norm(B[:, j])
            if dist > bestd:
                best, bestd = j, dist
        chosen.append(best)
    assert list(f['J'][:4]) == chosen
    T = dense.solve_upper(f['S11'], f['S12'])
    V = O.interp_matrix(f['J'], T, 9)
    assert abs(np.linalg.norm(B - B[:, f['J'][:4]] @ V.T) - f['S22norm_F']) < 1e-12


def pin_solve():
    g = np.random.default_rng(4)
    S = np.triu(g.standard_normal((8, 8))) + 3 * np.eye(8)
    X = g.standard_normal((8, 2))
    assert np.abs(dense.solve_upper(S, S @ X) - X).max() < 1e-12


def pin_exact_recovery():
    A, s, _, _ = W.exact_rank_matrix(60, 45, 5, seed=3)
    U, sh, V = O.rsvd(A, 6, 4, 1, seed=9)
    assert np.abs(A - (U * sh) @ V.T).max() < 1e-12


def pin_power_span():
    A, s = W.logspace_type(50, 40, 1, seed=4)
    Om = philox.sketch(5, 40, 8)
    Y = A @ (A.T @ (A @ Om))
    Qa = dense.householder_qr(Y)[0]
    Qb = O.range_finder(A, 5, 3, 1, seed=5)
    assert np.linalg.norm(Qa @ Qa.T - Qb @ Qb.T, 2) < 1e-9


def pin_kat():
    out = philox.philox4x32_10(0, 0, 0, 0, 0, 0)
    assert [int(x) for x in out] == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]


def pin_box_muller():
    u1, u2 = philox.uniforms(philox.raw_words(3, 0, 0, 2))
    r = np.sqrt(-2.0 * np.log(u1))
    z = philox.normals(3, 0, 0, 4)
    assert np.array_equal(z[0::2], r * np.cos(philox.TWO_PI * u2))
    assert np.array_equal(z[1::2], r * np.sin(philox.TWO_PI * u2))


def pin_cur_normal_equations():
    A, s = W.logspace_type(60, 50, 3, seed=10)
    res = O.cur(A, 6, 4, 1, seed=4)
    R = A[res['Jr'], :]
    V = O.interp_matrix(res['J'], res['T'], 50)
    assert np.abs((res['U'] @ R - V.T) @ R.T).max() < 1e-12


def pin_grad():
    # central difference of the whole randomized SVD, q = 1, cotangents on
    # U, sigma and V (the signs of the unperturbed singular pairs are kept
    # for the perturbed ones)
    m, n, k, p = 40, 30, 5, 3
    A, _ = W.logspace_type(m, n, 1, seed=5)
    g = np.random.default_rng(7)
    dU, dS, dV = g.standard_normal((m, k)), g.standard_normal(k), g.standard_normal((n, k))
    f0 = G.rsvd_forward_tape(A, k, p, 1, 11)

    def align(U, V):
        d = np.sign(np.sum(U * f0["U"], axis=0))
        return U * d, V * d
    dA, _ = G.rsvd_grad(A, k, p, 1, 11, dU, dS, dV)
    E = g.standard_normal((m, n))
    h = 1e-6

    def L(M):
        r = G.rsvd_forward_tape(M, k, p, 1, 11)
        u, v = align(r["U"], r["V"])
        return np.sum(dU * u) + np.sum(dS * r["S"]) + np.sum(dV * v)
    fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
    assert abs(fd - np.sum(dA * E)) < 1e-6 * max(1.0, abs(fd))


def pin_grad_residual():
    # central difference of ||A - Q Q^T A||_F^2 formed directly from Q and A
    m, n, k, p = 40, 30, 5, 3
    A, _ = W.logspace_type(m, n, 1, seed=6)
    g = np.random.default_rng(8)
    dA, _ = G.rsvd_grad(A, k, p, 1, 11, dres=1.0)
    E = g.standard_normal((m, n))
    h = 1e-6
    fp = G.rsvd_forward_tape(A + h * E, k, p, 1, 11)["resid2"]
    fm = G.rsvd_forward_tape(A - h * E, k, p, 1, 11)["resid2"]
    fd = (fp - fm) / (2 * h)
    assert abs(fd - np.sum(dA * E)) < 1e-6 * max(1.0, abs(fd))


MUTANTS = [
    (G.rsvd_grad, "ds -= 2.0 * dres * s", "ds += 2.0 * dres * s", pin_grad_residual),
    (G.rsvd_grad, "dA += 2.0 * dres * A", "pass", pin_grad_residual),
    (G.qr_adjoint, "C = dQ + Q @ copyltu(M)", "C = dQ + Q @ np.tril(M)", pin_grad),
    (G.qr_adjoint, "M = -(dQ.T @ Q)", "M = dQ.T @ Q", pin_grad),
    (G.svd_adjoint, "F[off] = 1.0 / D[off]", "F[off] = -1.0 / D[off]", pin_grad),
    (G.rsvd_grad, "dA += Qy @ dZ.T", "pass", pin_grad),
    (dense.householder_qr, "beta = 2.0 / np.dot(v, v)", "beta = 1.0 / np.dot(v, v)", pin_qr),
    (dense.householder_qr, "Q[j:, j:] -= np.outer(beta * v, w)", "Q[j:, j:] += np.outer(beta * v, w)", pin_qr),
    (dense.jacobi_svd, "sn = cs * t", "sn = -cs * t", pin_jacobi),
    (dense.jacobi_svd, "order = np.argsort(-s, kind='stable')", "order = np.argsort(s, kind='stable')", pin_jacobi),
    (dense.jacobi_svd, "V[:, Qi] = sn * vp + cs * vq", "V[:, Qi] = sn * vq + cs * vp", pin_jacobi),
    (dense.cpqr, "best = int(np.argmax(nrm2))", "best = int(np.argmin(nrm2))", pin_cpqr),
    (dense.cpqr, "W[s:, cols] -= np.outer(beta * v, w)", "pass", pin_cpqr),
    (dense.solve_upper, "X[i] /= S[i, i]", "X[i] /= S[i, i] ** 2", pin_solve),
    (dense.solve_upper, "X[i] -= S[i, i + 1:] @ X[i + 1:]", "X[i] -= S[i + 1:, i] @ X[i + 1:]", pin_solve),
    (O.rsvd, "U = Q @ Vh[:, :k]", "U = Q @ Uh[:, :k]", pin_exact_recovery),
    (O.rsvd, "V = Qh @ Uh[:, :k]", "V = Qh @ Vh[:, :k]", pin_exact_recovery),
    (O.range_finder, "Z = A.T @ Qy", "Z = Omega", pin_power_span),
    (O.range_finder, "for _ in range(q):", "for _ in range(q - 1):", pin_power_span),
    (philox.philox4x32_10, "k1 = (k1 + PHILOX_W1) & MASK32", "k1 = (k1 + PHILOX_W0) & MASK32", pin_kat),
    (philox.philox4x32_10, "hi0 ^ c3 ^ np.uint64(k1)", "hi0 ^ c3 ^ np.uint64(k0)", pin_kat),
    (philox.normals, "pair[0::2] = r * np.cos(theta)", "pair[0::2] = r * np.sin(theta)", pin_box_muller),
    (O.cur, "M = Qt[Jc, :] + T @ Qt[J[k:], :]", "M = Qt[Jc, :]", pin_cur_normal_equations),
]


@pytest.mark.parametrize("func,old,new,pin", MUTANTS,
                         ids=[f"{m[0].__name__}:{i}" for i, m in enumerate(MUTANTS)])
def test_mutant_is_caught(monkeypatch, func, old, new, pin):
    pin()                                   # the pin holds for the real oracle
    _install(monkeypatch, func, old, new)
    with pytest.raises(Exception):
        pin()
