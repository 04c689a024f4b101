"""Pins of the oracle's column ID (section 2.1, rank-revealing QR)."""
import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.interpolative as sli

from oracle.idqr import column_id, householder_cpqr


def _rand(m, c, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, c)) + 1j * rng.standard_normal((m, c))


def _lowrank(m, c, k, seed, decay=None):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))
    C = rng.standard_normal((k, c)) + 1j * rng.standard_normal((k, c))
    if decay is not None:
        B = B * decay[None, :]
    return B @ C


@pytest.mark.parametrize("eps", [1e-2, 1e-6, 1e-10])
def test_residual_identity_and_identity_block(eps):
    s = np.logspace(0, -12, 20)
    A = _lowrank(300, 20, 20, 0, decay=s)
    cid = column_id(A, eps)
    resid = np.linalg.norm(A - A[:, cid.skel] @ cid.X)
    # the residual of the ID is exactly ||R22||_F, which is at most eps ||A||
    assert resid == pytest.approx(cid.tail, rel=1e-6, abs=1e-13 * cid.normA)
    assert resid <= eps * np.linalg.norm(A) * (1 + 1e-8)
    np.testing.assert_allclose(cid.X[:, cid.skel], np.eye(cid.rank), atol=1e-13)
    # the rank is the smallest that meets the tolerance
    if cid.rank > 1:
        _, perm, R, normA = householder_cpqr(A, 0.0)
        tail_prev = np.linalg.norm(R[cid.rank - 1:, cid.rank - 1:])
        assert tail_prev > eps * normA


@pytest.mark.parametrize("k", [1, 4, 7, 12])
def test_exact_recovery_of_low_rank(k):
    A = _lowrank(200, 16, k, k)
    cid = column_id(A, 1e-12)
    assert cid.rank == k
    assert np.linalg.norm(A - A[:, cid.skel] @ cid.X) <= 1e-12 * np.linalg.norm(A)


def test_pivots_match_lapack_geqp3():
    # Away from ties the greedy pivot sequence of column-pivoted QR is unique;
    # LAPACK (norm downdating) and this oracle (recomputed norms) agree.
    for seed in range(5):
        A = _lowrank(120, 14, 14, 10 + seed, decay=np.logspace(0, -8, 14))
        _, perm_l = scipy.linalg.qr(A, mode="r", pivoting=True)
        rank, perm, R, _ = householder_cpqr(A, 0.0)
        assert list(perm[:10]) == list(perm_l[:10])
        Rl = scipy.linalg.qr(A[:, perm_l], mode="r")[0]
        np.testing.assert_allclose(np.abs(np.diag(R))[:10],
                                   np.abs(np.diag(Rl))[:10], rtol=1e-8)


def test_rank_comparable_to_scipy_interpolative():
    A = _lowrank(400, 24, 24, 3, decay=np.logspace(0, -10, 24))
    for eps in (1e-3, 1e-6, 1e-9):
        cid = column_id(A, eps)
        k, idx, proj = sli.interp_decomp(A, eps, rand=False)
        err_s = np.linalg.norm(A - sli.reconstruct_matrix_from_id(A[:, idx[:k]], idx, proj))
        err_o = np.linalg.norm(A - A[:, cid.skel] @ cid.X)
        assert abs(cid.rank - k) <= 2
        assert err_o <= eps * np.linalg.norm(A) * (1 + 1e-8)
        assert err_s < 10 * eps * np.linalg.norm(A)


def test_tie_rule_lowest_original_index():
    # unit-modulus columns all have the same norm: the first pivot is column 0
    n = 16
    x = np.arange(n)[:, None]
    k = np.arange(5, 13)[None, :]
    A = np.exp(-2j * np.pi * x * k / n)
    cid = column_id(A, 1e-12)
    assert cid.skel[0] == 0
    # exactly orthogonal equal-norm columns: every step is a tie
    assert list(cid.skel) == list(range(8))


def test_zero_matrix_and_shapes():
    cid = column_id(np.zeros((5, 3)), 1e-6)
    assert cid.rank == 1 and cid.X.shape == (1, 3)
    # wide matrix: rank never exceeds the number of rows
    A = _rand(3, 7, 1)
    cid = column_id(A, 1e-14)
    assert cid.rank == 3
    assert np.linalg.norm(A - A[:, cid.skel] @ cid.X) < 1e-12 * np.linalg.norm(A)


def test_interpolation_entries_bounded_for_strong_rrqr_like_inputs():
    # Section 2.1 asks for bounded interpolation entries; greedy pivoting keeps
    # them modest on well-behaved kernels (checked, not guaranteed).
    n = 64
    x = (np.arange(n) + 0.5)[:, None] / n
    y = 3.0 + np.arange(12)[None, :] / 12
    A = 1.0 / np.abs(x - y)
    cid = column_id(A, 1e-10)
    assert np.abs(cid.X).max() < 10.0
