"""Kernel entry functions K(x^i, y^j) of the operators the butterfly compresses.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Every entry is evaluated on demand from integer multi-indices, as section 2
assumes (the operator tensor is never formed; any entry costs O(1)).  All
arithmetic is FP64 / complex128.

Index conventions (one per mode, 0-based):
  target multi-index i in [0, n)^d, source multi-index j in [0, n)^d.

Operators
---------
fourier    K = exp(-2 pi i x.k) with x = i/n (spatial target) and k = j - n/2
           (integer frequency).  This is the uniform DFT of section 4.3 with
           the roles of the two grids swapped and the sign flipped; the phase
           x.k = (i.k)/n is reduced exactly in integers before the
           exponential.
helmholtz  K = exp(+i w rho)/rho, rho = |x - y| (the +i w rho sign throughout).
           d = 3: x = i/n, y = j/n + (2,0,0), two unit cubes whose centres are
           2 apart along x1 (section 4.1, offset along x1).
           d = 2: x = (i/n, 0), y = (j/n, 1), two parallel facing unit
           plates at distance 1 (the example of section 3.2 and the first
           Green's function test of section 4.1).
radon      K = exp(2 pi i phi(x, k)), x = i/n, k = j - n/2 (section 4.2).
           d = 2: phi = x.k + sqrt(c1(x)^2 k1^2 + c2(x)^2 k2^2),
           c1 = (a + b sin(2 pi x1) sin(2 pi x2))/den,
           c2 = (a + b cos(2 pi x1) cos(2 pi x2))/den; the paper uses a=2,
           b=1, den=16, the workloads here den=3 (the default).
           d = 3: phi = x.k + c(x)|k|,
           c = (a + b sin(2 pi x1) sin(2 pi x2) sin(2 pi x3))/den with the
           paper's a=3, b=1, den=100 as the default.
dft        K = exp(2 pi i x.y), the uniform DFT of section 4.3 (any d): x = i,
           y = j/n, with the bit-reversal ordering for each dimension: the
           multi-index i_k stands for the grid point br(i_k), br reversing
           the log2(n) bits (bitrev=False keeps the natural order).  The
           phase br(i).br(j)/n is reduced exactly in integers modulo n.
nudft      K = exp(2 pi i x.y), the type-2 non-uniform DFT of section 4.3:
           y = j/n and x_k = X[k][i_k], with X[k] n given coordinates in
           [0, n - 1] per mode (random in the paper; passed in here, sorted
           so that index blocks are coordinate intervals).  The phase x.y is
           formed in FP64 and reduced modulo 1 before the exponential.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FOURIER = 0
HELMHOLTZ = 1
RADON = 2
NUDFT = 3
DFT = 4

KIND_NAMES = {FOURIER: "fourier", HELMHOLTZ: "helmholtz", RADON: "radon", NUDFT: "nudft",
              DFT: "dft"}


@dataclass(frozen=True)
class Operator:
    """A discretised oscillatory integral operator on an n^d x n^d grid."""

    kind: int
    d: int
    n: int
    omega: float = 0.0          # Helmholtz wavenumber (ignored otherwise)
    radon_a: float | None = None  # Radon constants (ignored otherwise);
    radon_b: float | None = None  # None: (2, 1, 3) for d = 2, (3, 1, 100)
    radon_den: float | None = None  # for d = 3
    nudft_x: tuple | None = None  # NUDFT target coordinates, d tuples of n
    bitrev: bool = True         # DFT: bit-reversal ordering of both grids

    def __post_init__(self):
        if self.nudft_x is not None:
            object.__setattr__(self, "nudft_x",
                               tuple(tuple(float(v) for v in row) for row in self.nudft_x))
        a, b, den = radon_defaults(self.d)
        for name, v in (("radon_a", a), ("radon_b", b), ("radon_den", den)):
            if getattr(self, name) is None:
                object.__setattr__(self, name, v)

    def entries(self, ti: np.ndarray, sj: np.ndarray) -> np.ndarray:
        """K(x^i, y^j) for broadcastable integer arrays of shape (..., d)."""
        ti = np.asarray(ti, dtype=np.int64)
        sj = np.asarray(sj, dtype=np.int64)
        if self.kind == FOURIER:
            return fourier_entries(self.n, ti, sj)
        if self.kind == HELMHOLTZ:
            return helmholtz_entries(self.n, self.omega, ti, sj)
        if self.kind == RADON:
            return radon_entries(self.n, ti, sj, self.radon_a, self.radon_b,
                                 self.radon_den)
        if self.kind == NUDFT:
            return nudft_entries(self.n, np.asarray(self.nudft_x), ti, sj)
        if self.kind == DFT:
            return dft_entries(self.n, ti, sj, self.bitrev)
        raise ValueError(f"unknown kernel kind {self.kind}")


def radon_defaults(d: int) -> tuple:
    """(a, b, den) of the Radon speed function when none are given."""
    return (2.0, 1.0, 3.0) if d == 2 else (3.0, 1.0, 100.0)


def helmholtz_omega(n: int) -> float:
    """Wavenumber giving 4 points per wavelength on a grid of spacing 1/n.

    Section 4.1 fixes 2 pi n / omega = 4, i.e. omega = pi n / 2; each unit
    cube then spans n/4 wavelengths per direction.
    """
    return np.pi * n / 2.0


def fourier_entries(n: int, ti: np.ndarray, sj: np.ndarray) -> np.ndarray:
    # x.k = (i.k)/n with k = j - n/2; exp(-2 pi i x.k) depends on i.k mod n
    # only, so the phase is reduced exactly in integer arithmetic.
    k = sj - n // 2
    p = np.sum(ti * k, axis=-1) % n
    return np.exp(-2j * np.pi * (p.astype(np.float64) / n))


def helmholtz_entries(n: int, omega: float, ti: np.ndarray,
                      sj: np.ndarray) -> np.ndarray:
    d = ti.shape[-1]
    if d == 3:      # cubes: y offset by 2 along x1
        offset = np.array([2.0, 0.0, 0.0])
        gap2 = 0.0
    elif d == 2:    # plates: in-plane coordinates, planes 1 apart
        offset = np.zeros(2)
        gap2 = 1.0
    else:
        raise ValueError("the Helmholtz geometries here are d = 2 (plates) and 3 (cubes)")
    diff = ti.astype(np.float64) / n - (sj.astype(np.float64) / n + offset)
    rho = np.sqrt(np.sum(diff * diff, axis=-1) + gap2)
    return np.exp(1j * omega * rho) / rho


def radon_entries(n: int, ti: np.ndarray, sj: np.ndarray, a: float, b: float,
                  den: float) -> np.ndarray:
    d = ti.shape[-1]
    x = ti.astype(np.float64) / n
    k = (sj - n // 2).astype(np.float64)
    if d == 3:
        c = (a + b * np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1]) *
             np.sin(2 * np.pi * x[..., 2])) / den
        phase = np.sum(x * k, axis=-1) + c * np.sqrt(np.sum(k * k, axis=-1))
        return np.exp(2j * np.pi * phase)
    if d != 2:
        raise ValueError("the Radon operators here are d = 2 and 3")
    s1 = np.sin(2 * np.pi * x[..., 0])
    s2 = np.sin(2 * np.pi * x[..., 1])
    c1 = np.cos(2 * np.pi * x[..., 0])
    c2 = np.cos(2 * np.pi * x[..., 1])
    cc1 = (a + b * s1 * s2) / den
    cc2 = (a + b * c1 * c2) / den
    phase = np.sum(x * k, axis=-1) + np.sqrt(cc1 ** 2 * k[..., 0] ** 2 +
                                             cc2 ** 2 * k[..., 1] ** 2)
    return np.exp(2j * np.pi * phase)


def nudft_entries(n: int, xs: np.ndarray, ti: np.ndarray, sj: np.ndarray) -> np.ndarray:
    # x.y = sum_k X[k][i_k] j_k / n, reduced modulo 1 in FP64
    d = ti.shape[-1]
    if xs.shape != (d, n):
        raise ValueError(f"NUDFT coordinates must have shape ({d}, {n})")
    phase = np.zeros(np.broadcast_shapes(ti.shape[:-1], sj.shape[:-1]))
    for k in range(d):
        phase = phase + xs[k][ti[..., k]] * sj[..., k].astype(np.float64) / n
    return np.exp(2j * np.pi * np.mod(phase, 1.0))


def bit_reverse(i: np.ndarray, n: int) -> np.ndarray:
    """Reverse the log2(n) low bits of each index (n a power of two)."""
    bits = int(n).bit_length() - 1
    if (1 << bits) != n:
        raise ValueError("bit-reversal ordering needs n a power of two")
    i = np.asarray(i, dtype=np.int64)
    out = np.zeros_like(i)
    for b in range(bits):
        out |= ((i >> b) & 1) << (bits - 1 - b)
    return out


def dft_entries(n: int, ti: np.ndarray, sj: np.ndarray, bitrev: bool = True) -> np.ndarray:
    # x = i, y = j/n per mode (after the bit-reversal ordering): the phase
    # x.y = (sum_k x_k y_k n)/n is an integer over n, reduced modulo n
    x = bit_reverse(ti, n) if bitrev else np.asarray(ti, dtype=np.int64)
    y = bit_reverse(sj, n) if bitrev else np.asarray(sj, dtype=np.int64)
    p = np.sum(x * y, axis=-1) % n
    return np.exp(2j * np.pi * (p.astype(np.float64) / n))
