"""The plain definition u = K f and its adjoint v = K^H g (reference results).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The operator maps an input tensor F in C^{n x ... x n x n_v} to
G = K x_{d+1..2d} F, which is the matrix product G = K F of the
matricizations (section 3.2).  Layout used throughout: arrays of shape
(n_v, n, ..., n), row-major, mode d fastest; multi-index i flattens to
sum_k i_k n^(d-1-k).

Routes (all FP64):
  brute force   u_i = sum_j K(x_i, y_j) f_j, chunked over targets; any kernel.
  Fourier       exp(-2 pi i (i.k)/n) depends on k mod n only, so u is the
                FFT of the input re-indexed by k mod n (exact for any f).
  Helmholtz     x_i - y_j = (i - j)/n - (2,0,0) depends on i - j only
                (translational invariance, section 3.3), so u is a linear
                convolution, computed by a zero-padded FFT on a (2n)^d grid.
"""
from __future__ import annotations

import numpy as np

from .kernels import DFT, FOURIER, HELMHOLTZ, Operator, bit_reverse


def grid_indices(n: int, d: int) -> np.ndarray:
    """All multi-indices of [0, n)^d in row-major order, shape (n^d, d)."""
    axes = np.meshgrid(*([np.arange(n)] * d), indexing="ij")
    return np.stack([a.reshape(-1) for a in axes], axis=-1).astype(np.int64)


def _as_batch(f: np.ndarray, n: int, d: int) -> np.ndarray:
    f = np.asarray(f, dtype=np.complex128)
    if f.shape == (n,) * d:
        f = f[None]
    if f.shape[1:] != (n,) * d:
        raise ValueError(f"expected (nv,{n}^{d}) input, got {f.shape}")
    return f


def apply_brute(op: Operator, f: np.ndarray, rows: np.ndarray | None = None,
                chunk: int = 256) -> np.ndarray:
    """u_i = sum_j K(x_i, y_j) f_j by direct summation.

    ``rows`` (flat target indices) restricts the output to those targets; the
    result then has shape (nv, len(rows)).  Otherwise (nv, n, ..., n).
    """
    n, d = op.n, op.d
    f = _as_batch(f, n, d)
    nv = f.shape[0]
    src = grid_indices(n, d)
    fmat = f.reshape(nv, -1).T                      # (n^d, nv)
    tgt_all = grid_indices(n, d)
    sel = np.arange(n ** d) if rows is None else np.asarray(rows, np.int64)
    out = np.empty((len(sel), nv), dtype=np.complex128)
    for c0 in range(0, len(sel), chunk):
        ti = tgt_all[sel[c0:c0 + chunk]]
        kblk = op.entries(ti[:, None, :], src[None, :, :])
        out[c0:c0 + chunk] = kblk @ fmat
    if rows is None:
        return out.T.reshape((nv,) + (n,) * d)
    return out.T


def adjoint_brute(op: Operator, g: np.ndarray, cols: np.ndarray | None = None,
                  chunk: int = 256) -> np.ndarray:
    """v_j = sum_i conj(K(x_i, y_j)) g_i by direct summation."""
    n, d = op.n, op.d
    g = _as_batch(g, n, d)
    nv = g.shape[0]
    tgt = grid_indices(n, d)
    gmat = g.reshape(nv, -1).T
    src_all = grid_indices(n, d)
    sel = np.arange(n ** d) if cols is None else np.asarray(cols, np.int64)
    out = np.empty((len(sel), nv), dtype=np.complex128)
    for c0 in range(0, len(sel), chunk):
        sj = src_all[sel[c0:c0 + chunk]]
        kblk = op.entries(tgt[None, :, :], sj[:, None, :])   # (chunk, n^d)
        out[c0:c0 + chunk] = np.conj(kblk) @ gmat
    if cols is None:
        return out.T.reshape((nv,) + (n,) * d)
    return out.T


def apply_fourier_fft(n: int, d: int, f: np.ndarray) -> np.ndarray:
    """Fourier operator by FFT: u = fftn(f re-indexed by k mod n)."""
    f = _as_batch(f, n, d)
    axes = tuple(range(1, d + 1))
    return np.fft.fftn(np.fft.ifftshift(f, axes=axes), axes=axes)


def adjoint_fourier_fft(n: int, d: int, g: np.ndarray) -> np.ndarray:
    """Adjoint Fourier operator: v_j = n^d ifftn(g)[(j - n/2) mod n]."""
    g = _as_batch(g, n, d)
    axes = tuple(range(1, d + 1))
    return np.fft.fftshift(np.fft.ifftn(g, axes=axes), axes=axes) * float(n) ** d


def apply_dft_fft(op: Operator, f: np.ndarray) -> np.ndarray:
    """Uniform DFT of section 4.3 by FFT: with the grids in natural order
    u = n^d ifftn(f); the bit-reversal ordering permutes each mode of the
    input before and of the output after (the permutation is its own
    inverse)."""
    n, d = op.n, op.d
    f = _as_batch(f, n, d)
    axes = tuple(range(1, d + 1))
    if op.bitrev:
        perm = bit_reverse(np.arange(n), n)
        for ax in axes:
            f = np.take(f, perm, axis=ax)
    u = np.fft.ifftn(f, axes=axes) * float(n) ** d
    if op.bitrev:
        for ax in axes:
            u = np.take(u, perm, axis=ax)
    return u


def adjoint_dft_fft(op: Operator, g: np.ndarray) -> np.ndarray:
    """v_j = sum_i conj(K(i, j)) g_i = fftn of g in natural order."""
    n, d = op.n, op.d
    g = _as_batch(g, n, d)
    axes = tuple(range(1, d + 1))
    if op.bitrev:
        perm = bit_reverse(np.arange(n), n)
        for ax in axes:
            g = np.take(g, perm, axis=ax)
    v = np.fft.fftn(g, axes=axes)
    if op.bitrev:
        for ax in axes:
            v = np.take(v, perm, axis=ax)
    return v


def _helmholtz_difference_kernel(op: Operator) -> np.ndarray:
    """h[delta] = K(x_i, y_j) for delta = i - j in (-n, n)^d, stored on a
    (2n)^d periodic grid (negative offsets wrapped)."""
    n, d = op.n, op.d
    m = 2 * n
    deltas = np.arange(m)
    deltas = np.where(deltas < n, deltas, deltas - m)   # 0..n-1, -n..-1
    axes = np.meshgrid(*([deltas] * d), indexing="ij")
    delta = np.stack(axes, axis=-1).astype(np.int64)
    # K(i, j) depends on i - j only: evaluate it at i = delta, j = 0 (the
    # entry function accepts any integer offsets).
    return op.entries(delta, np.zeros_like(delta))


def apply_helmholtz_fft(op: Operator, f: np.ndarray) -> np.ndarray:
    """Helmholtz operator as a linear convolution u = h * f (zero-padded FFT)."""
    if op.kind != HELMHOLTZ:
        raise ValueError("not a Helmholtz operator")
    n, d = op.n, op.d
    f = _as_batch(f, n, d)
    axes = tuple(range(1, d + 1))
    h = _helmholtz_difference_kernel(op)
    fpad = np.zeros((f.shape[0],) + (2 * n,) * d, dtype=np.complex128)
    fpad[(slice(None),) + (slice(0, n),) * d] = f
    conv = np.fft.ifftn(np.fft.fftn(fpad, axes=axes) * np.fft.fftn(h)[None],
                        axes=axes)
    return conv[(slice(None),) + (slice(0, n),) * d]


def adjoint_helmholtz_fft(op: Operator, g: np.ndarray) -> np.ndarray:
    """v_j = sum_i conj(h[i - j]) g_i: a correlation, done as a convolution
    with hbar[delta] = conj(h[-delta])."""
    n, d = op.n, op.d
    g = _as_batch(g, n, d)
    axes = tuple(range(1, d + 1))
    h = _helmholtz_difference_kernel(op)
    hbar = np.conj(h)
    for ax in range(d):                      # hbar[delta] <- conj(h[-delta])
        hbar = np.roll(np.flip(hbar, axis=ax), 1, axis=ax)
    gpad = np.zeros((g.shape[0],) + (2 * n,) * d, dtype=np.complex128)
    gpad[(slice(None),) + (slice(0, n),) * d] = g
    conv = np.fft.ifftn(np.fft.fftn(gpad, axes=axes) * np.fft.fftn(hbar)[None],
                        axes=axes)
    return conv[(slice(None),) + (slice(0, n),) * d]


def apply_exact(op: Operator, f: np.ndarray) -> np.ndarray:
    """Fastest exact route for the operator: FFT, FFT convolution or brute."""
    if op.kind == FOURIER:
        return apply_fourier_fft(op.n, op.d, f)
    if op.kind == HELMHOLTZ:
        return apply_helmholtz_fft(op, f)
    if op.kind == DFT:
        return apply_dft_fft(op, f)
    return apply_brute(op, f)


def adjoint_exact(op: Operator, g: np.ndarray) -> np.ndarray:
    if op.kind == FOURIER:
        return adjoint_fourier_fft(op.n, op.d, g)
    if op.kind == HELMHOLTZ:
        return adjoint_helmholtz_fft(op, g)
    if op.kind == DFT:
        return adjoint_dft_fft(op, g)
    return adjoint_brute(op, g)


def probe_error(op: Operator, apply_fn, nprobe: int = 16, seed: int = 0):
    """Relative error of the sampled-probe metric of section 4.1.

    F_e has ones at ``nprobe`` random source entries and zeros elsewhere, so
    K F_e is a sum of a few columns of K and is formed entry by entry.
    ``apply_fn`` maps an (1, n, ..., n) input to the approximate output.
    """
    n, d = op.n, op.d
    rng = np.random.default_rng(seed)
    cols = rng.choice(n ** d, size=nprobe, replace=False)
    fe = np.zeros(n ** d, dtype=np.complex128)
    fe[cols] = 1.0
    tgt = grid_indices(n, d)
    src = grid_indices(n, d)[cols]
    exact = op.entries(tgt[:, None, :], src[None, :, :]).sum(axis=1)
    approx = np.asarray(apply_fn(fe.reshape((1,) + (n,) * d))).reshape(-1)
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
