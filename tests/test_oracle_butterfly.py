"""Pins of the oracle's tensor butterfly (Algorithms 1 and 2, section 3).

The butterfly is an approximation, so it is pinned against the plain
definition u = K f (FFT / FFT convolution / brute force, themselves pinned in
test_oracle_kernels), against exactness in the full-rank limit, against the
separable structure of the Fourier kernel (section 3.3, DFT paragraph),
against the adjoint identity and against the rank trends of Table 2.
"""
import json
import os

import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import dense, kernels, planio, tucker
from oracle.idqr import column_id
from oracle.kernels import Operator

from .planfile import PlanFile

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def fourier64():
    """The small Fourier workload: d = 2, n = 64, tol 1e-6, leaf 8."""
    return bf.construct(Operator(kernels.FOURIER, 2, 64), 1e-6)


@pytest.fixture(scope="module")
def helm32():
    n = 32
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    return bf.construct(op, 1e-4)


@pytest.fixture(scope="module")
def radon32():
    return bf.construct(Operator(kernels.RADON, 2, 32), 1e-3)


@pytest.fixture(scope="module")
def plates64():
    """Two parallel facing plates (d = 2), n = 64, tol 1e-6."""
    n = 64
    return bf.construct(Operator(kernels.HELMHOLTZ, 2, n, omega=kernels.helmholtz_omega(n)), 1e-6)


@pytest.fixture(scope="module")
def radon3_16():
    """3-D Radon transform, n = 16, leaf 4, tol 1e-3."""
    return bf.construct(Operator(kernels.RADON, 3, 16), 1e-3, leaf=4)


def test_full_rank_limit_is_exact():
    # proxies = whole nodes and eps ~ 0: every ID is exact, so is the product
    for kind, d, n in [(kernels.FOURIER, 2, 16), (kernels.RADON, 2, 16),
                       (kernels.HELMHOLTZ, 3, 8), (kernels.HELMHOLTZ, 2, 16),
                       (kernels.RADON, 3, 8)]:
        om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
        op = Operator(kind, d, n, omega=om)
        plan = bf.construct(op, 1e-13, leaf=4 if n == 8 else 8, p_pair=0,
                            p_other=0, id_tol_scale=1.0)
        f = _rand((2,) + (n,) * d, 0)
        assert _relerr(bf.apply(plan, f), dense.apply_brute(op, f)) < 1e-10
        assert _relerr(bf.apply_adjoint(plan, f), dense.adjoint_brute(op, f)) < 1e-10


def test_fourier64_meets_tolerance(fourier64):
    f = _rand((2, 64, 64), 1)
    u = bf.apply(fourier64, f)
    assert _relerr(u, dense.apply_fourier_fft(64, 2, f)) <= 1e-6
    v = bf.apply_adjoint(fourier64, f)
    assert _relerr(v, dense.adjoint_fourier_fft(64, 2, f)) <= 1e-6


def test_helmholtz32_meets_tolerance(helm32):
    op = helm32.op
    f = _rand((1, 32, 32, 32), 2)
    assert _relerr(bf.apply(helm32, f), dense.apply_helmholtz_fft(op, f)) <= 1e-4
    assert _relerr(bf.apply_adjoint(helm32, f), dense.adjoint_helmholtz_fft(op, f)) <= 1e-4
    # sampled-probe metric of section 4.1
    assert dense.probe_error(op, lambda fe: bf.apply(helm32, fe)) <= 1e-4
    st = bf.plan_stats(helm32)
    # compression: the cores hold far fewer entries than the dense operator
    assert st["core_entries"] < 0.05 * 32 ** 6


@pytest.fixture(scope="module")
def nudft32():
    """Type-2 non-uniform DFT (section 4.3), d = 2, n = 32, tol 1e-6."""
    from paper_2411_03029_amd import inputs
    return bf.construct(Operator(kernels.NUDFT, 2, 32, nudft_x=inputs.nudft_points(32, 2)), 1e-6)


def test_nudft32_meets_tolerance(nudft32):
    op = nudft32.op
    f = _rand((2, 32, 32), 6)
    assert _relerr(bf.apply(nudft32, f), dense.apply_brute(op, f)) <= 1e-6
    assert _relerr(bf.apply_adjoint(nudft32, f), dense.adjoint_brute(op, f)) <= 1e-6


def test_nudft3_meets_tolerance():
    from paper_2411_03029_amd import inputs
    op = Operator(kernels.NUDFT, 3, 16, nudft_x=inputs.nudft_points(16, 3))
    plan = bf.construct(op, 1e-3, leaf=4)
    f = _rand((1, 16, 16, 16), 7)
    assert _relerr(bf.apply(plan, f), dense.apply_brute(op, f)) <= 1e-3
    assert _relerr(bf.apply_adjoint(plan, f), dense.adjoint_brute(op, f)) <= 1e-3


def test_radon32_meets_tolerance(radon32):
    op = radon32.op
    f = _rand((1, 32, 32), 3)
    assert _relerr(bf.apply(radon32, f), dense.apply_brute(op, f)) <= 1e-3
    assert _relerr(bf.apply_adjoint(radon32, f), dense.adjoint_brute(op, f)) <= 1e-3


def test_plates64_meets_tolerance(plates64):
    op = plates64.op
    f = _rand((2, 64, 64), 4)
    assert _relerr(bf.apply(plates64, f), dense.apply_helmholtz_fft(op, f)) <= 1e-6
    assert _relerr(bf.apply_adjoint(plates64, f), dense.adjoint_helmholtz_fft(op, f)) <= 1e-6


def test_radon3_meets_tolerance(radon3_16):
    op = radon3_16.op
    f = _rand((1, 16, 16, 16), 5)
    assert _relerr(bf.apply(radon3_16, f), dense.apply_brute(op, f)) <= 1e-3
    assert _relerr(bf.apply_adjoint(radon3_16, f), dense.adjoint_brute(op, f)) <= 1e-3


@pytest.mark.parametrize("which", ["fourier64", "helm32", "radon32", "plates64", "radon3_16",
                                   "nudft32"])
def test_adjoint_identity_and_linearity(which, request):
    plan = request.getfixturevalue(which)
    shape = (1,) + (plan.n,) * plan.d
    f, g, h = _rand(shape, 10), _rand(shape, 11), _rand(shape, 12)
    u = bf.apply(plan, f)
    v = bf.apply_adjoint(plan, g)
    lhs, rhs = np.vdot(g, u), np.vdot(v, f)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(g) * np.linalg.norm(u) * 10
    a, b = 0.3 - 1.2j, -2.0 + 0.5j
    np.testing.assert_allclose(bf.apply(plan, a * f + b * h),
                               a * u + b * bf.apply(plan, h), atol=1e-10)
    # several right-hand sides at once equal one at a time
    fb = np.concatenate([f, h], axis=0)
    np.testing.assert_allclose(bf.apply(plan, fb)[1:], bf.apply(plan, h), atol=1e-12)


def test_fourier_factors_equal_one_dimensional_ids(fourier64):
    # Section 3.3: for the Fourier kernel the other modes only scale rows by
    # unit-modulus factors, so every sampled unfolding is a stack of scaled
    # copies of the 1-D block exp(-2 pi i x_k k_k) over the paired-mode
    # proxies; its Gram matrix is a positive multiple of the 1-D one, so the
    # ID (rank, skeleton, X) must equal the 1-D block's ID.
    plan = fourier64
    n, leaf, eps = plan.n, plan.leaf, plan.eps_id
    checked = 0
    for l, lev in enumerate(plan.src):
        for (s_flat, tau_flat), per_k in lev.items():
            tau = bf.unflatten(tau_flat, l, 2)
            for k in range(2):
                for nu, sk in enumerate(per_k[k]):
                    if l == 0:
                        s = bf.unflatten(s_flat, plan.Ls, 2)
                        nu_abs = s[k] * (1 << plan.Lt) + nu
                        cols = np.arange(nu_abs * leaf, (nu_abs + 1) * leaf)
                    else:
                        ptau = bf.flatten([b >> 1 for b in tau], l - 1)
                        par = plan.src[l - 1][(s_flat, ptau)][k]
                        cols = np.concatenate([par[2 * nu].skel, par[2 * nu + 1].skel])
                    lo, ln = bf.node_range(l, tau[k], n)
                    x = bf.proxies(lo, ln, 2 * len(cols))
                    B = np.exp(-2j * np.pi * (np.outer(x, cols - n // 2) % n) / n)
                    ref = column_id(B, eps)
                    assert ref.rank == sk.rank
                    assert list(cols[ref.skel]) == list(sk.skel)
                    np.testing.assert_allclose(ref.X, sk.X, atol=1e-8)
                    checked += 1
    assert checked == sum(len(ids) for lev in plan.src for per_k in lev.values()
                          for ids in per_k)


def test_helmholtz_ranks_follow_table2():
    # Table 2 (cubes, n = 512): max rank 5, 6, 7, 8 at eps = 1e-2..1e-5, i.e.
    # about one more per decade, and independent of n (section 3.3).  At
    # n = 32, leaf 8 and IDs run at eps itself, the oracle matches within 1.
    with open(os.path.join(GOLDEN, "table2_cubes.json")) as fh:
        rows = json.load(fh)["rows"]
    n = 32
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    rmax = []
    for eps, rmin_p, rmax_p, err_p, *_ in rows:
        plan = bf.construct(op, eps, id_tol_scale=1.0)
        r = plan.ranks()
        assert abs(int(r.max()) - rmax_p) <= 1
        rmax.append(int(r.max()))
    assert all(b >= a for a, b in zip(rmax, rmax[1:]))


def test_helmholtz_max_rank_independent_of_n():
    # Section 3.3: at fixed points per wavelength the tensor butterfly rank
    # does not grow with n (both n give even L at leaf 4: L = 2 and 4).
    rmax = []
    for n in (16, 64):
        op = Operator(kernels.HELMHOLTZ, 2, n, omega=kernels.helmholtz_omega(n))
        plan = bf.construct(op, 1e-4, leaf=4, id_tol_scale=1.0)
        rmax.append(int(plan.ranks().max()))
    assert abs(rmax[0] - rmax[1]) <= 1


def test_tucker_id_bound():
    # Section 3.1: ||K - TuckerID(K)||_F <= eps sqrt(2d) ||K||_F for exact
    # per-mode IDs (checked with slack 10, since ID projectors are oblique).
    for kind, d, n in [(kernels.HELMHOLTZ, 2, 8), (kernels.RADON, 2, 8),
                       (kernels.HELMHOLTZ, 3, 4)]:
        om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
        op = Operator(kind, d, n, omega=om)
        g = dense.grid_indices(n, d)
        K = op.entries(g[:, None, :], g[None, :, :]).reshape((n,) * (2 * d))
        for eps in (1e-2, 1e-4, 1e-6):
            skels, mats, core = tucker.tucker_id(K, eps)
            err = np.linalg.norm(tucker.tucker_reconstruct(core, mats) - K)
            assert err <= 10 * eps * np.sqrt(2 * d) * np.linalg.norm(K)


def test_degenerate_single_level_is_a_tucker_id():
    # n = leaf: L = 0, one middle pair (t, s) = (root, root); the butterfly is
    # one Tucker-ID of the whole tensor with proxies
    n = 8
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    plan = bf.construct(op, 1e-6, leaf=8)
    assert plan.L == 0 and len(plan.cores) == 1
    f = _rand((1, n, n, n), 4)
    assert _relerr(bf.apply(plan, f), dense.apply_brute(op, f)) < 1e-5


def test_plan_file_round_trip(helm32, tmp_path):
    path = tmp_path / "p.tbplan"
    planio.save_plan(helm32, str(path))
    pf = PlanFile(str(path))
    assert (pf.kind, pf.d, pf.n, pf.leaf, pf.L, pf.Lt, pf.Ls) == (
        kernels.HELMHOLTZ, 3, 32, 8, helm32.L, helm32.Lt, helm32.Ls)
    for l in range(helm32.Lt + 1):
        for key, per_k in helm32.src[l].items():
            for k in range(3):
                for a, (skel, X) in zip(per_k[k], pf.src[l][key][k]):
                    assert list(a.skel) == list(skel)
                    np.testing.assert_array_equal(a.X, X)
    for key, C in helm32.cores.items():
        np.testing.assert_array_equal(C, pf.cores[key])
    raw = bytearray(path.read_bytes())
    raw[100] ^= 0x40
    with pytest.raises(ValueError):
        PlanFile(bytes(raw))


def test_nudft_plan_file_carries_the_points(nudft32, tmp_path):
    # the target coordinates follow the header; every ID and core after them
    # reads back unchanged
    path = tmp_path / "n.tbplan"
    planio.save_plan(nudft32, str(path))
    pf = PlanFile(str(path))
    assert (pf.kind, pf.d, pf.n) == (kernels.NUDFT, 2, 32)
    np.testing.assert_array_equal(pf.nudft_x, np.asarray(nudft32.op.nudft_x))
    for key, C in nudft32.cores.items():
        np.testing.assert_array_equal(C, pf.cores[key])


def _offsets(paper_rmax, ours):
    return [p - o for p, o in zip(paper_rmax, ours)]


def test_plate_ranks_follow_table2_trend():
    # Table 2 (plates, n = 16384): max rank 8, 10, 11, 12, 13 at eps =
    # 1e-2..1e-6.  The paper's leaf size and proxy rule are not stated, so
    # the absolute ranks are parity unpinned; at n = 32, leaf 8 and IDs at
    # eps, the oracle's max ranks grow with the tolerance as the paper's do:
    # the offset to the paper's column stays constant within 1.
    with open(os.path.join(GOLDEN, "table2_plates.json")) as fh:
        rows = json.load(fh)["rows"]
    n = 32
    op = Operator(kernels.HELMHOLTZ, 2, n, omega=kernels.helmholtz_omega(n))
    ours = [int(bf.construct(op, row[0], id_tol_scale=1.0).ranks().max()) for row in rows]
    off = _offsets([row[2] for row in rows], ours)
    assert max(off) - min(off) <= 1, (ours, off)
    assert all(b >= a for a, b in zip(ours, ours[1:])) and ours[-1] > ours[0]


def test_radon3_ranks_follow_table3_trend():
    # Table 3 (3-D Radon, eq. randon3d with the paper's (3 + ...)/100, n =
    # 128): max rank 6, 8, 9, 11 at eps = 1e-2..1e-5.  At n = 16 with leaf 8
    # and IDs at eps the oracle's max ranks keep a constant offset (within
    # 1) to that column; absolute values are parity unpinned (leaf size and
    # proxies unknown).
    with open(os.path.join(GOLDEN, "table3_radon.json")) as fh:
        rows = json.load(fh)["radon3d_n128"]
    op = Operator(kernels.RADON, 3, 16)
    assert (op.radon_a, op.radon_b, op.radon_den) == (3.0, 1.0, 100.0)
    ours = [int(bf.construct(op, row[0], leaf=8, id_tol_scale=1.0).ranks().max()) for row in rows]
    off = _offsets([row[2] for row in rows], ours)
    assert max(off) - min(off) <= 1, (ours, off)
    assert all(b >= a for a, b in zip(ours, ours[1:])) and ours[-1] > ours[0]


# ----------------------------------------- uniform DFT, d = 4 .. 6 (§4.3) --

@pytest.mark.parametrize("d,n,leaf", [(4, 8, 4), (4, 16, 4), (5, 8, 4), (6, 4, 4)])
def test_highd_dft_butterfly_is_exact(d, n, leaf):
    # With the bit-reversal ordering a node pair of the DFT is a block
    # exp(2 pi i (c + 2^l a)(c' + 2^(L-l) b)/n) whose a-b factor
    # exp(2 pi i a b/C_b) is periodic with period C_b in a and b: every
    # unfolding has rank at most the leaf size, so the IDs are exact and the
    # butterfly reproduces the operator (checked against the FFT route,
    # forward and adjoint), with every rank at most the leaf size.
    op = Operator(kernels.DFT, d, n)
    plan = bf.construct(op, 1e-3, leaf=leaf)
    assert int(plan.ranks().max()) <= leaf
    f = _rand((2,) + (n,) * d, 40)
    assert _relerr(bf.apply(plan, f), dense.apply_dft_fft(op, f)) <= 1e-12
    assert _relerr(bf.apply_adjoint(plan, f), dense.adjoint_dft_fft(op, f)) <= 1e-12


def test_highd_dft_factors_equal_one_dimensional_ids():
    # Section 3.3: separability again; each source-side ID of the d = 4 DFT
    # equals the ID of the 1-D block exp(2 pi i br(x) br(y)/n) over the paired
    # mode's proxies and the ID's columns.
    d, n, leaf = 4, 16, 4
    plan = bf.construct(Operator(kernels.DFT, d, n), 1e-3, leaf=leaf)
    eps = plan.eps_id
    checked = 0
    for l, lev in enumerate(plan.src):
        for (s_flat, tau_flat), per_k in lev.items():
            tau = bf.unflatten(tau_flat, l, d)
            for k in range(d):
                for nu, sk in enumerate(per_k[k]):
                    if l == 0:
                        s = bf.unflatten(s_flat, plan.Ls, d)
                        nu_abs = s[k] * (1 << plan.Lt) + nu
                        cols = np.arange(nu_abs * leaf, (nu_abs + 1) * leaf)
                    else:
                        ptau = bf.flatten([b >> 1 for b in tau], l - 1)
                        par = plan.src[l - 1][(s_flat, ptau)][k]
                        cols = np.concatenate([par[2 * nu].skel, par[2 * nu + 1].skel])
                    lo, ln = bf.node_range(l, tau[k], n)
                    x = kernels.bit_reverse(bf.proxies(lo, ln, 2 * len(cols)), n)
                    y = kernels.bit_reverse(cols, n)
                    B = np.exp(2j * np.pi * (np.outer(x, y) % n) / n)
                    ref = column_id(B, eps)
                    assert ref.rank == sk.rank
                    assert list(cols[ref.skel]) == list(sk.skel)
                    np.testing.assert_allclose(ref.X, sk.X, atol=1e-8)
                    checked += 1
    assert checked > 0
