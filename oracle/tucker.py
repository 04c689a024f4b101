"""Tucker-type interpolative decomposition of a small, fully formed tensor.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 3.1: every one of the 2d modes of K(tau, nu) is compressed by a
column ID of the unfolding along that mode, with the mode's indices as
columns; the core is the subtensor of K at the skeleton indices of all modes
and each mode is expanded back by its interpolation matrix.  With the row-form
ID used here (unfolding ~= unfolding(:, J) X, X of size r x n_q), every
mode-q fibre satisfies k ~= X^T k[J], so

    K ~= K(J_1, ..., J_2d) x_1 X_1^T x_2 ... x_2d X_2d^T.

Section 3.1 states a Frobenius bound of eps sqrt(2d) ||K||_F for the result;
the tests check it with slack, since ID projectors are oblique.
"""
from __future__ import annotations

import numpy as np

from .idqr import column_id


def unfolding(T: np.ndarray, q: int) -> np.ndarray:
    """Mode-q unfolding: rows range over the other modes, columns over q."""
    return np.moveaxis(T, q, -1).reshape(-1, T.shape[q])


def mode_product(T: np.ndarray, M: np.ndarray, q: int) -> np.ndarray:
    """T x_q M: every mode-q fibre t of T is replaced by M t."""
    return np.moveaxis(np.tensordot(M, T, axes=(1, q)), 0, q)


def tucker_id(K: np.ndarray, eps: float):
    """Return (skeletons, interpolation matrices, core) of the Tucker-ID."""
    skels, mats = [], []
    for q in range(K.ndim):
        cid = column_id(unfolding(K, q), eps)
        skels.append(cid.skel)
        mats.append(cid.X)
    core = K[np.ix_(*skels)]
    return skels, mats, core


def tucker_reconstruct(core: np.ndarray, mats) -> np.ndarray:
    out = core
    for q, X in enumerate(mats):
        out = mode_product(out, X.T, q)
    return out
