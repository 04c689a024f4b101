"""GPU parity at the measured workloads' own shapes.

1. The n = 64 Helmholtz cube plan (d = 3, leaf 8, tol 1e-4: L = 3 with two
   source transfer levels, the second reading a workspace parent, and 512
   middle pairs), built by the oracle and applied by the library through the
   plan file: every core precision and the autotuned launches against the
   oracle's own apply of that plan, per right-hand side, in the 2-norm and
   for the worst single output.
2. The 2-D Radon transform at n = 256 (tol 1e-6, complex FP32), built on the
   GPU, against direct summation of the operator's definition on 256 sampled
   target rows (forward) and source columns (adjoint).
3. The Helmholtz cubes at n = 128 with 64 right-hand sides (tol 1e-4,
   complex FP32, matrix-core cores), forward and adjoint, against the exact
   FFT convolution on the first and the last right-hand side; and the same
   with the transfer levels and fan-in leaves forced onto the 4 x 4
   matrix-core forms.

Approximation bounds follow the target of the FP32 apply: relative error at
most tol + 1e-5 against the exact operator.
"""
import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import dense, kernels, planio
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import (assert_parity, relerr, say, to_dev, to_host, torch_gpu, with_bf16_cores,
                        with_q16_cores)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cube64(tmp_path_factory):
    torch_gpu()
    import paper_2411_03029_amd as tb
    n = 64
    say("[gpu] oracle construction: helmholtz cubes n=64 tol=1e-4 leaf 8")
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    ora = bf.construct(op, 1e-4, leaf=8)
    assert (ora.L, ora.Lt, ora.Ls) == (3, 2, 1)
    path = str(tmp_path_factory.mktemp("cube64") / "cube64.tbplan")
    planio.save_plan(ora, path)
    plan = tb.load_plan(path, store=("c128", "c64", "cbf16", "cq16"))
    return ora, plan


@pytest.mark.parametrize("dtype,bound", [("c128", 1e-12), ("c64", 2e-5), ("c64otf", 2e-5),
                                         ("cq16", 2e-5), ("cbf16", 2e-5)])
def test_cube_workload_plan_matches_oracle(cube64, dtype, bound):
    # BF16 and 16-bit cores: against the oracle's apply of the same plan with
    # its cores as they are stored (rounded to BF16, or passed through the
    # 16-bit codec), to the FP32 bound; and against the unrounded plan in the
    # 2-norm to 5e-3 (BF16: 2^-9 per core part, random signs) or 1e-4
    # (16-bit: 2^-16 of each column's largest part)
    torch = torch_gpu()
    ora, plan = cube64
    info = plan.info()
    assert (info["L"], info["Lt"], info["Ls"], info["n_pairs"]) == (3, 2, 1, 512)
    f = inputs.rhs_batch(64, 3, 1, config=2)
    ref = {"cbf16": with_bf16_cores, "cq16": with_q16_cores}.get(dtype, lambda o: o)(ora)
    ue, ve = bf.apply(ref, f), bf.apply_adjoint(ref, f)
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    x = to_dev(f, cdt)
    say(f"[gpu] cube n=64 plan {dtype}")
    u = to_host(plan.apply(x, dtype=dtype))
    v = to_host(plan.apply_adjoint(x, dtype=dtype))
    torch.cuda.synchronize()
    assert_parity(u, ue, bound, f"forward {dtype}")
    assert_parity(v, ve, bound, f"adjoint {dtype}")
    if dtype in ("cbf16", "cq16"):
        loose = 5e-3 if dtype == "cbf16" else 1e-4
        assert relerr(u, bf.apply(ora, f)) <= loose
        assert relerr(v, bf.apply_adjoint(ora, f)) <= loose


def test_cube_workload_plan_tuned(cube64, tmp_path):
    # the launches the benchmark times: autotuned for one right-hand side
    torch = torch_gpu()
    ora, plan = cube64
    f = inputs.rhs_batch(64, 3, 1, config=2)
    say("[gpu] cube n=64 plan autotune c64")
    plan.autotune(1, dtype="c64")
    x = to_dev(f, torch.complex64)
    u = to_host(plan.apply(x))
    v = to_host(plan.apply_adjoint(x))
    torch.cuda.synchronize()
    assert_parity(u, bf.apply(ora, f), 2e-5, "forward tuned")
    assert_parity(v, bf.apply_adjoint(ora, f), 2e-5, "adjoint tuned")


def test_radon256_sampled_rows_against_direct_summation():
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n, tol = 256, 1e-6
    op = Operator(kernels.RADON, 2, n)
    say("[gpu] construct radon n=256 tol=1e-6")
    plan = tb.construct("radon", 2, n, tol, store=("c64",))
    f = inputs.rhs_batch(n, 2, 1, config=3)
    x = to_dev(f, torch.complex64)
    u = to_host(plan.apply(x)).reshape(1, -1)
    v = to_host(plan.apply_adjoint(x)).reshape(1, -1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    rows = np.sort(rng.choice(n * n, 256, replace=False))
    cols = np.sort(rng.choice(n * n, 256, replace=False))
    ue = dense.apply_brute(op, f, rows=rows)
    ve = dense.adjoint_brute(op, f, cols=cols)
    eu, ev = relerr(u[:, rows], ue), relerr(v[:, cols], ve)
    say(f"[gpu]   sampled errors forward {eu:.2e} adjoint {ev:.2e}")
    assert eu <= tol + 1e-5 and ev <= tol + 1e-5


def test_helmholtz128_64rhs_against_fft_convolution():
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n, tol, nrhs = 128, 1e-4, 64
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    say("[gpu] construct helmholtz n=128 tol=1e-4")
    plan = tb.construct("helmholtz", 3, n, tol, store=("c64",))
    f = inputs.rhs_batch(n, 3, nrhs, config=5)
    x = to_dev(f, torch.complex64)
    say("[gpu]   apply 64 rhs")
    u = plan.apply(x)
    v = plan.apply_adjoint(x)
    torch.cuda.synchronize()
    for q in (0, nrhs - 1):
        eu = relerr(to_host(u[q]), dense.apply_exact(op, f[q])[0])
        ev = relerr(to_host(v[q]), dense.adjoint_exact(op, f[q])[0])
        say(f"[gpu]   rhs {q}: forward {eu:.2e} adjoint {ev:.2e}")
        assert eu <= tol + 1e-5 and ev <= tol + 1e-5


def test_helmholtz128_64rhs_matrix_core_stages():
    # the same workload with its transfer levels and fan-in leaves forced
    # onto the 4 x 4 matrix-core forms (ranks 3..8, leaf 8): the transfers
    # give the vector forms' bits (the same products in the same order), and
    # with the matrix-core leaves too the apply meets the same bound against
    # FFT convolution
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n, tol, nrhs = 128, 1e-4, 64
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    say("[gpu] construct helmholtz n=128 tol=1e-4 (matrix-core stages)")
    plan = tb.construct("helmholtz", 3, n, tol, store=("c64",))
    f = inputs.rhs_batch(n, 3, nrhs, config=5)
    x = to_dev(f, torch.complex64)
    slots = plan.launch_slots()
    fanin = ("tgt_transfer", "src_transfer_adj")
    fanout = ("src_transfer", "tgt_transfer_adj")
    leaves = ("tgt_leaf", "src_leaf_adj")

    def run(cfgs):
        for s, st in enumerate(slots):
            for names, cfg in cfgs:
                if st in names:
                    plan.set_launch(nrhs, s, dtype="c64", **cfg)
        u, v = plan.apply(x), plan.apply_adjoint(x)
        torch.cuda.synchronize()
        return u, v

    say("[gpu]   vector transfers and leaves")
    u0, v0 = run([(fanin, dict(rhs_tile=4, fanin_in_turn=2, outputs_per_thread=8)),
                  (fanout, dict(outputs_per_thread=8, rhs_tile=2)),
                  (leaves, dict(fanin_in_turn=1, rhs_tile=8))])
    say("[gpu]   matrix-core transfers")
    u1, v1 = run([(fanin + fanout, dict(transfer_mfma=2))])
    assert torch.equal(u0, u1) and torch.equal(v0, v1)
    say("[gpu]   matrix-core transfers and fan-in leaves")
    u2, v2 = run([(leaves, dict(transfer_mfma=2))])
    for a, b in ((u2, u1), (v2, v1)):
        assert float((a - b).abs().max() / b.abs().max()) <= 1e-5
    for q in (0, nrhs - 1):
        eu = relerr(to_host(u2[q]), dense.apply_exact(op, f[q])[0])
        ev = relerr(to_host(v2[q]), dense.adjoint_exact(op, f[q])[0])
        say(f"[gpu]   rhs {q}: forward {eu:.2e} adjoint {ev:.2e}")
        assert eu <= tol + 1e-5 and ev <= tol + 1e-5
