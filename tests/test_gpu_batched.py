"""The uneven multi-operator form: several operators of different kind, d
and n, each with its own number of right-hand sides, applied in one HIP
graph launch (tb_apply_batched).

The graph runs the same kernels as tb_apply with the same arguments, so each
operator's output must equal its single-operator apply bit for bit, on every
replay of the cached graph (inputs are rewritten in place between replays,
with eager device work and synchronisations in between).  Against the oracle:
the batched outputs of oracle-built plans match the oracle's butterfly apply
to 2e-5 (FP32); on the 12-operator mix of 8 Fourier (d=2, n in
{64,128,256}) and 4 Helmholtz (d=3, n in {32,64}) operators with 16..128
right-hand sides the outputs match the exact operator (FFT / FFT
convolution) to tol + 2e-5 in FP32 and tol + 5e-3 with BF16 cores.
"""
import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import dense, kernels, planio
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import assert_parity, relerr, say, to_dev, to_host, torch_gpu

pytestmark = pytest.mark.gpu

SMALL = [  # (kind, d, n, tol, leaf, nrhs)
    (kernels.FOURIER, 2, 64, 1e-6, 8, 3),
    (kernels.HELMHOLTZ, 3, 32, 1e-4, 8, 17),
    (kernels.RADON, 2, 32, 1e-3, 8, 9),
    (kernels.FOURIER, 3, 16, 1e-4, 4, 1),
]


def _oracle_op(kind, d, n):
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    return Operator(kind, d, n, omega=om)


def test_batched_matches_single_and_oracle_over_replays(tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    ops, plans, xs, outs = [], [], [], []
    for i, (kind, d, n, tol, leaf, nrhs) in enumerate(SMALL):
        op = bf.construct(_oracle_op(kind, d, n), tol, leaf=leaf)
        path = str(tmp_path / f"p{i}.tbplan")
        planio.save_plan(op, path)
        ops.append(op)
        plans.append(tb.load_plan(path, store=("c64",)))
        xs.append(torch.empty((nrhs,) + (n,) * d, dtype=torch.complex64, device="cuda"))
        outs.append(torch.empty_like(xs[-1]))
    tb.batched_reset()
    for adjoint in (False, True):
        for rep in range(3):
            say(f"[gpu] batched small mix adjoint={adjoint} replay {rep}")
            fs = []
            for i, x in enumerate(xs):
                f = inputs.rhs_batch(ops[i].n, ops[i].d, x.shape[0], config=60 + 10 * rep + i)
                x.copy_(to_dev(f, torch.complex64))
                fs.append(f)
            torch.cuda.synchronize()
            tb.apply_batched(plans, xs, outs, adjoint=adjoint)
            torch.cuda.synchronize()
            for i, p in enumerate(plans):
                single = p.apply_adjoint(xs[i]) if adjoint else p.apply(xs[i])
                torch.cuda.synchronize()
                assert torch.equal(single, outs[i]), (adjoint, rep, i)
                ref = bf.apply_adjoint(ops[i], fs[i]) if adjoint else bf.apply(ops[i], fs[i])
                assert_parity(to_host(outs[i]), ref, 2e-5, f"adjoint={adjoint} replay {rep} plan {i}")
            # eager work between replays on the same plans and buffers
            for i, p in enumerate(plans):
                outs[i].zero_()
                p.apply(xs[i])
            torch.cuda.synchronize()


def test_batched_capture_failure_then_success(tmp_path):
    # a launch that does not fit (4 right-hand sides per thread with a tile of
    # 1) fails the capture of the second plan's branch after the first plan's
    # branch and part of the second's were captured; every forked branch is
    # joined back and the capture discarded, so the next call, with that
    # launch restored to the heuristic, captures and replays normally
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    from paper_2411_03029_amd import _lib
    ops, plans, xs, outs = [], [], [], []
    for i, (kind, d, n, tol, leaf, nrhs) in enumerate(SMALL[:3]):
        op = bf.construct(_oracle_op(kind, d, n), tol, leaf=leaf)
        path = str(tmp_path / f"p{i}.tbplan")
        planio.save_plan(op, path)
        ops.append(op)
        plans.append(tb.load_plan(path, store=("c64",)))
        f = inputs.rhs_batch(n, d, nrhs, config=70 + i)
        xs.append(to_dev(f, torch.complex64))
        outs.append(torch.empty_like(xs[-1]))
    tb.batched_reset()
    bad = plans[1].launch_slots().index("core") + 1   # first target transfer
    nrhs1 = xs[1].shape[0]
    plans[1].set_launch(nrhs1, bad, rhs_tile=1, rhs_per_thread=4)
    say("[gpu] batched capture that fails in the second branch")
    with pytest.raises(tb.TBError) as ei:
        tb.apply_batched(plans, xs, outs)
    assert ei.value.status == _lib.TB_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    plans[1].set_launch(nrhs1, bad)   # back to the heuristic
    say("[gpu] batched capture after the failure")
    for rep in range(2):
        tb.apply_batched(plans, xs, outs)
        torch.cuda.synchronize()
        for i, p in enumerate(plans):
            assert torch.equal(p.apply(xs[i]), outs[i]), (rep, i)
            assert_parity(to_host(outs[i]), bf.apply(ops[i], to_host(xs[i])), 2e-5, f"plan {i}")


def test_batched_rejects_bad_arguments(tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    op = bf.construct(_oracle_op(kernels.FOURIER, 2, 32), 1e-6)
    path = str(tmp_path / "f.tbplan")
    planio.save_plan(op, path)
    p = tb.load_plan(path, store=("c64",))
    x = torch.zeros((2, 32, 32), dtype=torch.complex64, device="cuda")
    with pytest.raises(tb.TBError):  # same plan twice
        tb.apply_batched([p, p], [x, x.clone()])
    with pytest.raises(tb.TBError):  # no BF16 cores stored
        tb.apply_batched([p], [x], dtype="cbf16")
    with pytest.raises(ValueError):
        tb.apply_batched([p], [x[:, :16]])


MIX_KINDS = [("fourier", 2, n, 1e-6) for n in (64, 128, 256, 64, 128, 256, 64, 128)] + \
            [("helmholtz", 3, n, 1e-4) for n in (32, 64, 32, 64)]


@pytest.fixture(scope="module")
def mix_plans():
    torch_gpu()
    import paper_2411_03029_amd as tb
    plans = []
    for kind, d, n, tol in MIX_KINDS:
        say(f"[gpu] construct {kind} d={d} n={n} tol={tol}")
        plans.append(tb.construct(kind, d, n, tol, store=("c64", "cbf16")))
    return plans


@pytest.mark.parametrize("dtype,slack", [("c64", 2e-5), ("cbf16", 5e-3)])
def test_uneven_mix_against_exact_operator(mix_plans, dtype, slack):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    counts = inputs.uneven_rhs_counts(len(MIX_KINDS))
    xs, fs = [], []
    for i, ((kind, d, n, tol), m) in enumerate(zip(MIX_KINDS, counts)):
        f = inputs.rhs_batch(n, d, int(m), config=70 + i)
        fs.append(f)
        xs.append(to_dev(f, torch.complex64))
    outs = [torch.empty_like(x) for x in xs]
    for adjoint in (False, True):
        say(f"[gpu] uneven mix of 12 operators {dtype} adjoint={adjoint} counts={list(counts)}")
        for rep in range(2):
            tb.apply_batched(mix_plans, xs, outs, adjoint=adjoint, dtype=dtype)
            torch.cuda.synchronize()
        for i, (kind, d, n, tol) in enumerate(MIX_KINDS):
            single = (mix_plans[i].apply_adjoint(xs[i], dtype=dtype) if adjoint
                      else mix_plans[i].apply(xs[i], dtype=dtype))
            torch.cuda.synchronize()
            assert torch.equal(single, outs[i]), (dtype, adjoint, i)
            # exact operator on the first and last right-hand sides
            op = _oracle_op(kernels.FOURIER if kind == "fourier" else kernels.HELMHOLTZ, d, n)
            sel = [0, fs[i].shape[0] - 1]
            exact = dense.adjoint_exact if adjoint else dense.apply_exact
            ref = exact(op, fs[i][sel])
            err = relerr(to_host(outs[i])[sel], ref)
            assert err <= tol + slack, (dtype, adjoint, kind, n, err)
