"""Column interpolative decomposition by column-pivoted Householder QR.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.1: a column ID writes A ~= A(:, J) X, where J holds r skeleton
columns and X (r x c) has bounded entries, with the rank chosen so that the
Frobenius residual is at most eps times the Frobenius norm of A.  The paper
computes it by rank-revealing QR; this is the textbook column-pivoted
Householder QR (Businger-Golub) written out step by step:

  A P = Q [R11 R12; 0 R22],   J = first r pivots,   X(:, J) = I,
  X(:, rest) = R11^{-1} R12,  and  ||A - A(:, J) X||_F = ||R22||_F exactly.

Rules fixed here (the paper does not state them):
  * pivot: at step k take, among the remaining columns whose residual norm is
    at least (1 - 1e-10) times the largest one, the column with the lowest
    original index (ties are exact for unit-modulus kernels);
  * trailing residual norms are recomputed at every step (no downdating);
  * rank: r = min{k >= 1 : ||R[k:, k:]||_F <= eps ||A||_F}, never above
    min(m, c); a zero matrix gets rank 1 (first column, X = e_1^T).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TIE_REL = 1e-10


@dataclass
class ColumnID:
    rank: int
    skel: np.ndarray     # (r,) original column indices, in pivot order
    X: np.ndarray        # (r, c) interpolation matrix, X[:, skel] = I
    tail: float          # ||A - A(:, skel) X||_F as given by ||R22||_F
    normA: float


def householder_cpqr(A: np.ndarray, eps: float):
    """Column-pivoted Householder QR stopped at the Frobenius-tail rank.

    Returns (rank, perm, R) where A[:, perm] = Q R on the first ``rank``
    columns' worth of reflections (R is the partially reduced matrix).
    """
    A = np.array(A, dtype=np.complex128)
    m, c = A.shape
    R = A.copy()
    perm = np.arange(c)
    normA = float(np.linalg.norm(A))
    kmax = min(m, c)
    rank = kmax
    for k in range(kmax):
        trailing = np.linalg.norm(R[k:, k:], axis=0)
        tail = float(np.sqrt(np.sum(trailing ** 2)))
        if k >= 1 and tail <= eps * normA:
            rank = k
            break
        # pivot rule: lowest original index among the near-maximal norms
        big = trailing >= (1.0 - TIE_REL) * trailing.max()
        cand = np.nonzero(big)[0]
        j = k + cand[np.argmin(perm[k + cand])]
        if j != k:
            R[:, [k, j]] = R[:, [j, k]]
            perm[[k, j]] = perm[[j, k]]
        # Householder reflector zeroing R[k+1:, k]
        x = R[k:, k]
        xnorm = np.linalg.norm(x)
        if xnorm == 0.0:
            continue
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        alpha = -phase * xnorm
        v = x.copy()
        v[0] -= alpha
        v /= np.linalg.norm(v)
        R[k:, k:] -= 2.0 * np.outer(v, np.conj(v) @ R[k:, k:])
        R[k + 1:, k] = 0.0
    return rank, perm, R, normA


def column_id(A: np.ndarray, eps: float) -> ColumnID:
    """Column ID A ~= A[:, skel] @ X at relative Frobenius tolerance eps."""
    A = np.asarray(A, dtype=np.complex128)
    m, c = A.shape
    rank, perm, R, normA = householder_cpqr(A, eps)
    if normA == 0.0:
        X = np.zeros((1, c), dtype=np.complex128)
        X[0, 0] = 1.0
        return ColumnID(1, np.array([0]), X, 0.0, 0.0)
    r = rank
    R11 = R[:r, :r]
    R12 = R[:r, r:]
    T = np.linalg.solve(R11, R12) if r < c else np.zeros((r, 0), np.complex128)
    X = np.zeros((r, c), dtype=np.complex128)
    X[:, perm[:r]] = np.eye(r)
    X[:, perm[r:]] = T
    tail = float(np.linalg.norm(R[r:, r:])) if r < min(m, c) else 0.0
    return ColumnID(r, perm[:r].copy(), X, tail, normA)
