"""Pins of the oracle's kernel entries and dense reference routes.

The operator definitions are fixed by the paper (sections 2, 4.1-4.3 and
the workload definitions).  Each check here compares two independent routes
to the same quantity, or a route to a closed form at special points.
"""
import numpy as np
import pytest

from oracle import dense, kernels
from oracle.kernels import Operator

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("d,n", [(2, 8), (2, 16), (3, 8)])
def test_fourier_fft_equals_brute(d, n):
    op = Operator(kernels.FOURIER, d, n)
    f = _rand((2,) + (n,) * d, 1)
    np.testing.assert_allclose(dense.apply_fourier_fft(n, d, f),
                               dense.apply_brute(op, f), rtol=0, atol=1e-10)
    g = _rand((2,) + (n,) * d, 2)
    np.testing.assert_allclose(dense.adjoint_fourier_fft(n, d, g),
                               dense.adjoint_brute(op, g), rtol=0, atol=1e-10)


def test_fourier_plane_waves():
    # A unit impulse at frequency k0 gives the plane wave exp(-2 pi i x.k0);
    # the conjugate plane wave at x_{i0} gives n^d times an impulse at i0.
    n, d = 16, 2
    j0 = (3, 13)
    k0 = np.array(j0) - n // 2
    f = np.zeros((n, n), complex)
    f[j0] = 1.0
    u = dense.apply_fourier_fft(n, d, f)[0]
    i = dense.grid_indices(n, d).reshape(n, n, d)
    expect = np.exp(-2j * np.pi * (i @ k0) / n)
    np.testing.assert_allclose(u, expect, atol=1e-12)
    i0 = np.array([5, 9])
    k = dense.grid_indices(n, d) - n // 2
    f2 = np.exp(2j * np.pi * (k @ i0) / n).reshape(n, n)
    u2 = dense.apply_brute(Operator(kernels.FOURIER, d, n), f2)[0]
    expect2 = np.zeros((n, n), complex)
    expect2[tuple(i0)] = n ** d
    np.testing.assert_allclose(u2, expect2, atol=1e-9)


def test_fourier_phase_is_periodic_in_k():
    # exp(-2 pi i (i.k)/n) is unchanged by k -> k + n e_m (integer reduction)
    n = 32
    ti = np.array([[7, 30]])
    a = kernels.fourier_entries(n, ti, np.array([[1, 2]]))
    b = kernels.fourier_entries(n, ti, np.array([[1 + n, 2]]))
    np.testing.assert_allclose(a, b, atol=1e-14)


@pytest.mark.parametrize("n", [4, 8])
def test_helmholtz_fft_convolution_equals_brute(n):
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    f = _rand((2, n, n, n), 3)
    np.testing.assert_allclose(dense.apply_helmholtz_fft(op, f),
                               dense.apply_brute(op, f), rtol=0, atol=1e-10)
    g = _rand((2, n, n, n), 4)
    np.testing.assert_allclose(dense.adjoint_helmholtz_fft(op, g),
                               dense.adjoint_brute(op, g), rtol=0, atol=1e-10)


def test_helmholtz_special_values():
    # i = j = 0: rho = 2 exactly (the offset of the second cube).  With n = 8
    # the wavenumber pi n / 2 = 4 pi makes omega rho = 8 pi, so K = 1/2.
    n = 8
    om = kernels.helmholtz_omega(n)
    assert om == pytest.approx(4 * np.pi)
    z = np.zeros((1, 3), np.int64)
    assert kernels.helmholtz_entries(n, om, z, z)[0] == pytest.approx(0.5, abs=1e-14)
    # i = (n, 0, 0)-ish geometry: target x1 = 0, source x1 = 2 + 4/8, rho = 2.5
    ti = np.array([[0, 3, 5]])
    sj = np.array([[4, 3, 5]])
    val = kernels.helmholtz_entries(n, om, ti, sj)[0]
    assert abs(val) == pytest.approx(1 / 2.5, abs=1e-14)
    assert np.angle(val) == pytest.approx(np.angle(np.exp(1j * om * 2.5)), abs=1e-12)
    # omega = 0 is the Newton potential 1/rho (real, positive)
    v0 = kernels.helmholtz_entries(n, 0.0, ti, sj)[0]
    assert v0.imag == 0.0 and v0.real == pytest.approx(0.4, abs=1e-15)


def test_radon_special_points():
    n = 16
    z = np.zeros((1, 2), np.int64)
    # at x = 0: c1 = 2/3, c2 = 1, so K(0, k) = exp(2 pi i sqrt(4/9 k1^2 + k2^2))
    for k2 in (-5, 0, 3, 7):
        sj = np.array([[n // 2, n // 2 + k2]])
        assert kernels.radon_entries(n, z, sj, 2, 1, 3)[0] == pytest.approx(1.0, abs=1e-12)
    for k1 in (-6, 3, 6):   # (2/3)|k1| is an integer when 3 divides k1
        sj = np.array([[n // 2 + k1, n // 2]])
        assert kernels.radon_entries(n, z, sj, 2, 1, 3)[0] == pytest.approx(1.0, abs=1e-12)
    sj = np.array([[n // 2 + 1, n // 2]])
    assert kernels.radon_entries(n, z, sj, 2, 1, 3)[0] == pytest.approx(
        np.exp(2j * np.pi * 2 / 3), abs=1e-12)


def test_radon_without_speed_terms_is_an_inverse_dft():
    # with a = b = 0 both speeds vanish and K = exp(+2 pi i x.k): an inverse
    # DFT of the input re-indexed by k mod n.
    n, d = 16, 2
    op = Operator(kernels.RADON, d, n, radon_a=0.0, radon_b=0.0)
    f = _rand((1, n, n), 5)
    expect = np.fft.ifftn(np.fft.ifftshift(f, axes=(1, 2)), axes=(1, 2)) * n ** d
    np.testing.assert_allclose(dense.apply_brute(op, f), expect, atol=1e-10)


@pytest.mark.parametrize("kind,d,n", [(kernels.FOURIER, 2, 8),
                                      (kernels.HELMHOLTZ, 3, 4),
                                      (kernels.RADON, 2, 8)])
def test_dense_adjoint_identity(kind, d, n):
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    op = Operator(kind, d, n, omega=om)
    f = _rand((1,) + (n,) * d, 6)
    g = _rand((1,) + (n,) * d, 7)
    lhs = np.vdot(g, dense.apply_brute(op, f))
    rhs = np.vdot(dense.adjoint_brute(op, g), f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_probe_error_metric_zero_for_exact_apply():
    n, d = 8, 2
    op = Operator(kernels.FOURIER, d, n)
    err = dense.probe_error(op, lambda fe: dense.apply_fourier_fft(n, d, fe))
    assert err < 1e-13


# ----------------------------------------- parallel plates, 3-D Radon --

@pytest.mark.parametrize("n", [8, 16])
def test_plates_fft_convolution_equals_brute(n):
    # plates (d = 2): K depends on the in-plane offset only, so the FFT
    # convolution route applies; pinned to brute force
    op = Operator(kernels.HELMHOLTZ, 2, n, omega=kernels.helmholtz_omega(n))
    f = _rand((2, n, n), 11)
    np.testing.assert_allclose(dense.apply_helmholtz_fft(op, f),
                               dense.apply_brute(op, f), rtol=0, atol=1e-10)
    g = _rand((2, n, n), 12)
    np.testing.assert_allclose(dense.adjoint_helmholtz_fft(op, g),
                               dense.adjoint_brute(op, g), rtol=0, atol=1e-10)


def test_plates_special_values():
    # facing points (i = j) are the plate distance 1 apart: K = exp(i omega);
    # with n = 8, omega = 4 pi and K = 1.  An in-plane offset of (3, 4)/8
    # gives rho = sqrt(1 + 25/64) = sqrt(89)/8.
    n = 8
    om = kernels.helmholtz_omega(n)
    ti = np.array([[2, 5]])
    assert kernels.helmholtz_entries(n, om, ti, ti)[0] == pytest.approx(1.0, abs=1e-13)
    val = kernels.helmholtz_entries(n, om, np.array([[5, 7]]), np.array([[2, 3]]))[0]
    rho = np.sqrt(89.0) / 8
    assert abs(val) == pytest.approx(1 / rho, abs=1e-14)
    assert np.angle(val) == pytest.approx(np.angle(np.exp(1j * om * rho)), abs=1e-12)
    # translation invariance in the plane
    a = kernels.helmholtz_entries(n, om, np.array([[1, 2]]), np.array([[6, 0]]))
    b = kernels.helmholtz_entries(n, om, np.array([[2, 5]]), np.array([[7, 3]]))
    np.testing.assert_allclose(a, b, atol=1e-14)


def test_radon3_special_points():
    # x = 0: c = a/den = 3/100 and K(0, k) = exp(2 pi i 0.03 |k|); for
    # |k| = 0 it is 1; with x1 = 0 the speed is still 3/100 at any x2, x3
    n = 16
    op = Operator(kernels.RADON, 3, n)
    assert (op.radon_a, op.radon_b, op.radon_den) == (3.0, 1.0, 100.0)
    z = np.zeros((1, 3), np.int64)
    h = n // 2
    assert op.entries(z, np.array([[h, h, h]]))[0] == pytest.approx(1.0, abs=1e-14)
    k = np.array([3, -4, 12])   # |k| = 13
    assert op.entries(z, np.array([h + k]))[0] == pytest.approx(
        np.exp(2j * np.pi * 0.03 * 13), abs=1e-13)
    ti = np.array([[0, 5, 11]])
    x = ti[0] / n
    assert op.entries(ti, np.array([h + k]))[0] == pytest.approx(
        np.exp(2j * np.pi * (x @ k + 0.03 * 13)), abs=1e-12)


def test_radon3_without_speed_term_is_an_inverse_dft():
    n, d = 8, 3
    op = Operator(kernels.RADON, d, n, radon_a=0.0, radon_b=0.0)
    f = _rand((1, n, n, n), 13)
    axes = (1, 2, 3)
    expect = np.fft.ifftn(np.fft.ifftshift(f, axes=axes), axes=axes) * n ** d
    np.testing.assert_allclose(dense.apply_brute(op, f), expect, atol=1e-10)


@pytest.mark.parametrize("kind,d,n", [(kernels.HELMHOLTZ, 2, 8), (kernels.RADON, 3, 4)])
def test_dense_adjoint_identity_new_operators(kind, d, n):
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    op = Operator(kind, d, n, omega=om)
    f = _rand((1,) + (n,) * d, 14)
    g = _rand((1,) + (n,) * d, 15)
    lhs = np.vdot(g, dense.apply_brute(op, f))
    rhs = np.vdot(dense.adjoint_brute(op, g), f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------- non-uniform DFT --
# section 4.3, type 2: K = exp(2 pi i x.y), y = j/n, x_k = X[k][i_k] given

def _nudft(d, n, xs=None, seed=11):
    from paper_2411_03029_amd import inputs
    if xs is None:
        xs = inputs.nudft_points(n, d, seed)
    return Operator(kernels.NUDFT, d, n, nudft_x=xs)


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_nudft_on_integer_points_is_an_inverse_dft(d, n):
    # x_k = i_k exactly: K = exp(2 pi i i.j / n), whose sum is n^d ifftn
    op = _nudft(d, n, xs=np.tile(np.arange(n, dtype=float), (d, 1)))
    f = _rand((1,) + (n,) * d, 16)
    axes = tuple(range(1, d + 1))
    np.testing.assert_allclose(dense.apply_brute(op, f),
                               np.fft.ifftn(f, axes=axes) * n ** d, atol=1e-10)


def test_nudft_shift_of_points_is_a_source_modulation():
    # x -> x + m multiplies K(x, y) by exp(2 pi i m.y): a diagonal on the
    # source side, so K' f = K (e f) with e_j = exp(2 pi i m.j / n)
    d, n = 2, 8
    xs = _nudft(d, n).nudft_x
    m = np.array([3.0, 5.0])
    shifted = _nudft(d, n, xs=np.asarray(xs) + m[:, None])
    f = _rand((1, n, n), 17)
    j = np.stack(np.meshgrid(np.arange(n), np.arange(n), indexing="ij"), axis=-1)
    e = np.exp(2j * np.pi * (j @ m) / n)
    np.testing.assert_allclose(dense.apply_brute(shifted, f),
                               dense.apply_brute(_nudft(d, n), f * e[None]), atol=1e-10)


def test_nudft_special_values():
    # j = 0 gives 1 for every target; a target at the origin gives 1 for every source
    d, n = 3, 4
    xs = np.asarray(_nudft(d, n).nudft_x).copy()
    xs[:, 0] = 0.0
    op = _nudft(d, n, xs=xs)
    ti = np.array([[1, 2, 3], [3, 0, 1]])
    np.testing.assert_allclose(op.entries(ti, np.zeros((2, 3), np.int64)), 1.0, atol=1e-15)
    sj = np.array([[1, 2, 3], [3, 3, 2]])
    np.testing.assert_allclose(op.entries(np.zeros((2, 3), np.int64), sj), 1.0, atol=1e-15)
    # unit modulus everywhere
    kk = op.entries(np.array([[1, 1, 1]]), np.array([[2, 3, 1]]))
    assert abs(abs(kk[0]) - 1.0) < 1e-15


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_nudft_dense_adjoint_identity(d, n):
    op = _nudft(d, n)
    f = _rand((1,) + (n,) * d, 18)
    g = _rand((1,) + (n,) * d, 19)
    lhs = np.vdot(g, dense.apply_brute(op, f))
    rhs = np.vdot(dense.adjoint_brute(op, g), f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------- Radon speed away from x = 0 --
# Section 4.2's speed functions at points where the sin/cos products are
# +-1, 0 or 1/2, so that c1, c2 (d = 2) and c (d = 3) are short fractions
# worked out by hand: every b-term is live, unlike at x = 0.

def _radon2(n, ti, k, a, b, den):
    sj = np.array([[n // 2 + k[0], n // 2 + k[1]]])
    return kernels.radon_entries(n, np.array([ti]), sj, a, b, den)[0]


def test_radon2_speed_at_quarter_points_workload_constants():
    # (a, b, den) = (2, 1, 3).  x = (1/4, 1/4): sin(pi/2)^2 = 1, cos(pi/2) = 0,
    # so c1 = 1 and c2 = 2/3.  k = (3, 6): x.k = 9/4 and
    # sqrt(9 + (2/3)^2 36) = 5, phase 7.25 -> K = exp(i pi/2) = i.
    n = 16
    assert _radon2(n, (4, 4), (3, 6), 2, 1, 3) == pytest.approx(1j, abs=1e-12)
    # k = (4, -3): x.k = 1/4, sqrt(16 + 4) = 2 sqrt 5
    assert _radon2(n, (4, 4), (4, -3), 2, 1, 3) == pytest.approx(
        np.exp(2j * np.pi * (0.25 + 2 * np.sqrt(5.0))), abs=1e-12)
    # x = (3/4, 1/4): sin(3pi/2) sin(pi/2) = -1, so c1 = 1/3, c2 = 2/3.
    # k = (6, 3): x.k = 4.5 + 0.75, sqrt(4 + 4) = 2 sqrt 2
    assert _radon2(n, (12, 4), (6, 3), 2, 1, 3) == pytest.approx(
        np.exp(2j * np.pi * (5.25 + 2 * np.sqrt(2.0))), abs=1e-12)
    # x = (1/8, 1/8): sin^2(pi/4) = cos^2(pi/4) = 1/2, c1 = c2 = 5/6.
    # k = (3, 4): x.k = 7/8, (5/6) |k| = 25/6
    assert _radon2(n, (2, 2), (3, 4), 2, 1, 3) == pytest.approx(
        np.exp(2j * np.pi * (7 / 8 + 25 / 6)), abs=1e-12)
    # x = (0, 1/4): sin 0 = 0, cos 0 cos(pi/2) = 0: c1 = c2 = 2/3 (the b-terms
    # vanish on this line only); k = (3, 0) -> 2, x.k = 0 -> K = 1
    assert _radon2(n, (0, 4), (3, 0), 2, 1, 3) == pytest.approx(1.0, abs=1e-12)


def test_radon2_speed_at_quarter_points_paper_constants():
    # Section 4.2's constants (a, b, den) = (2, 1, 16).  x = (1/4, 1/4):
    # c1 = 3/16, c2 = 1/8.  k = (-16, 24) at n = 64: x.k = 2 and
    # sqrt(9 + 9) = 3 sqrt 2.  x = (1/2, 1/2): sin pi = 0, cos pi cos pi = 1,
    # so c1 = 1/8, c2 = 3/16; k = (16, 16): x.k = 16, sqrt(4 + 9) = sqrt 13.
    n = 64
    assert _radon2(n, (16, 16), (-16, 24), 2, 1, 16) == pytest.approx(
        np.exp(2j * np.pi * (2 + 3 * np.sqrt(2.0))), abs=1e-12)
    assert _radon2(n, (32, 32), (16, 16), 2, 1, 16) == pytest.approx(
        np.exp(2j * np.pi * np.sqrt(13.0)), abs=1e-12)
    # x = (1/4, 3/4): sin(pi/2) sin(3pi/2) = -1, cos(pi/2) cos(3pi/2) = 0,
    # c1 = 1/16, c2 = 1/8; k = (16, 8): x.k = 10, sqrt(1 + 1) = sqrt 2
    assert _radon2(n, (16, 48), (16, 8), 2, 1, 16) == pytest.approx(
        np.exp(2j * np.pi * (10 + np.sqrt(2.0))), abs=1e-12)


def test_radon3_speed_at_quarter_points():
    # (a, b, den) = (3, 1, 100).  x = (1/4, 1/4, 1/4): the sine product is 1,
    # c = 4/100.  k = (3, 4, 12), |k| = 13: phase 19/4 + 0.52.
    n = 16
    op = Operator(kernels.RADON, 3, n)
    h = n // 2
    k = np.array([3, 4, 12])
    assert op.entries(np.array([[4, 4, 4]]), np.array([h + k]))[0] == pytest.approx(
        np.exp(2j * np.pi * (4.75 + 0.52)), abs=1e-12)
    # x = (1/4, 3/4, 1/4): the product is -1, c = 2/100; x.k = 0.75 + 3 + 3
    assert op.entries(np.array([[4, 12, 4]]), np.array([h + k]))[0] == pytest.approx(
        np.exp(2j * np.pi * (6.75 + 0.26)), abs=1e-12)
    # x = (1/8, 1/8, 1/4): product 1/2, c = 3.5/100; k = (0, 6, 8), |k| = 10
    k2 = np.array([0, 6, 8])
    assert op.entries(np.array([[2, 2, 4]]), np.array([h + k2]))[0] == pytest.approx(
        np.exp(2j * np.pi * (0.75 + 2 + 0.35)), abs=1e-12)
    # the workload's own constants (2, 1, 3) at (1/4, 1/4, 1/4): c = 1,
    # phase 4.75 + 13 -> exp(2 pi i 0.75) = -i
    op3 = Operator(kernels.RADON, 3, n, radon_a=2.0, radon_b=1.0, radon_den=3.0)
    assert op3.entries(np.array([[4, 4, 4]]), np.array([h + k]))[0] == pytest.approx(
        -1j, abs=1e-12)


# ------------------------------------------------------- uniform DFT, any d --
# section 4.3: K = exp(2 pi i x.y), x = i, y = j/n, bit-reversal ordering

def test_bit_reversal_values_and_involution():
    np.testing.assert_array_equal(kernels.bit_reverse(np.arange(8), 8), [0, 4, 2, 6, 1, 5, 3, 7])
    for n in (2, 4, 16, 64):
        i = np.arange(n)
        np.testing.assert_array_equal(kernels.bit_reverse(kernels.bit_reverse(i, n), n), i)
    with pytest.raises(ValueError):
        kernels.bit_reverse(np.arange(6), 6)


@pytest.mark.parametrize("d,n,bitrev", [(2, 8, True), (2, 8, False), (3, 4, True), (4, 4, True),
                                        (5, 2, True)])
def test_dft_fft_equals_brute(d, n, bitrev):
    op = Operator(kernels.DFT, d, n, bitrev=bitrev)
    f = _rand((2,) + (n,) * d, 21)
    np.testing.assert_allclose(dense.apply_dft_fft(op, f), dense.apply_brute(op, f),
                               rtol=0, atol=1e-10)
    np.testing.assert_allclose(dense.adjoint_dft_fft(op, f), dense.adjoint_brute(op, f),
                               rtol=0, atol=1e-10)


def test_dft_plane_waves_and_special_values():
    # a unit impulse at source j0 gives exp(2 pi i br(i).br(j0)/n); j0 = 0
    # gives the constant 1; the natural order is the plain n^d ifftn
    n, d = 8, 3
    op = Operator(kernels.DFT, d, n)
    j0 = (1, 6, 3)                      # br = (4, 3, 6)
    f = np.zeros((n,) * d, complex)
    f[j0] = 1.0
    u = dense.apply_dft_fft(op, f)[0]
    i = dense.grid_indices(n, d)
    br = np.array([4, 3, 6])
    expect = np.exp(2j * np.pi * ((kernels.bit_reverse(i, n) @ br) % n) / n).reshape((n,) * d)
    np.testing.assert_allclose(u, expect, atol=1e-12)
    assert op.entries(np.array([[5, 2, 7]]), np.zeros((1, 3), np.int64))[0] == pytest.approx(1.0)
    # at n = 8, br(1) = 4, br(2) = 2, br(6) = 3: the phase br(1) br(2) = 8 is
    # 0 mod 8 (K = 1), br(1) br(6) = 12 is 4 mod 8 (K = exp(i pi) = -1)
    assert op.entries(np.array([[1, 0, 0]]), np.array([[2, 0, 0]]))[0] == pytest.approx(1.0)
    assert op.entries(np.array([[1, 0, 0]]), np.array([[6, 0, 0]]))[0] == pytest.approx(-1.0)
    nat = Operator(kernels.DFT, 2, n, bitrev=False)
    g = _rand((1, n, n), 22)
    np.testing.assert_allclose(dense.apply_dft_fft(nat, g), np.fft.ifftn(g, axes=(1, 2)) * n * n,
                               atol=1e-10)


@pytest.mark.parametrize("d,n", [(2, 8), (4, 4)])
def test_dft_dense_adjoint_identity(d, n):
    op = Operator(kernels.DFT, d, n)
    f = _rand((1,) + (n,) * d, 23)
    g = _rand((1,) + (n,) * d, 24)
    lhs = np.vdot(g, dense.apply_brute(op, f))
    rhs = np.vdot(dense.adjoint_brute(op, g), f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
