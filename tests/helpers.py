"""Shared helpers for the tests (no GPU needed to import)."""

import numpy as np


def align_signs(X, Xref):
    """Flip the columns of X so that each has a non-negative inner product
    with the same column of Xref (singular vectors are unique up to sign)."""
    d = np.sum(X * Xref, axis=0)
    s = np.where(d < 0, -1.0, 1.0)
    return X * s[None, :]


def orth_err(Q):
    return np.abs(Q.T @ Q - np.eye(Q.shape[1])).max()


def subspace_gap(U1, U2):
    """Largest sine of the principal angles between range(U1) and range(U2)
    (both with orthonormal columns)."""
    s = np.linalg.svd(U1.T @ U2, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def pivot_prefix(pivot_norms, second_norms, delta):
    """Length of the prefix of CPQR steps whose pivot margin
    (best - second) / best is at least delta (steps after the first
    near-tie may legitimately differ between two correct implementations)."""
    n = 0
    for b, s in zip(pivot_norms, second_norms):
        if b <= 0 or (b - s) / b < delta:
            break
        n += 1
    return n
