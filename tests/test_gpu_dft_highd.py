"""The uniform DFT of section 4.3 at d = 4 .. 6, with the bit-reversal
ordering of every mode (TB_KERNEL_DFT), on the GPU.

Applies with d > 3 run on the kernels generic in the number of modes
(apply_generic.hip).  Same-plan parity: the oracle builds the plan, the
library loads it and applies it; forward and adjoint must match the
oracle's own apply per right-hand side, in the 2-norm and for the worst
single output, FP64 to 1e-12 and FP32 to 2e-5.  The largest plans (d = 5 at
n = 8, d = 6 at n = 4: 3.4e7 and 1.7e7 core entries) travel without their
cores, which the library evaluates on the GPU at the oracle's skeletons;
their parity then also covers that evaluation.  The GPU construction must
give the oracle's ranks and skeletons (the IDs are exact: rank at most the
leaf size) and reproduce the exact operator (FFT route).
"""
import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import dense, kernels, planio
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import assert_parity, relerr, say, to_dev, to_host, torch_gpu
from .planfile import PlanFile

pytestmark = pytest.mark.gpu

CASES = [(4, 8, 4), (4, 16, 4), (5, 8, 4), (6, 4, 4)]
_PLANS = {}


def _oracle(d, n, leaf):
    if (d, n, leaf) not in _PLANS:
        _PLANS[(d, n, leaf)] = bf.construct(Operator(kernels.DFT, d, n), 1e-3, leaf=leaf)
    return _PLANS[(d, n, leaf)]


@pytest.mark.parametrize("d,n,leaf", CASES)
def test_highd_dft_same_plan(d, n, leaf, tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    ora = _oracle(d, n, leaf)
    with_cores = d <= 4
    path = str(tmp_path / "dft.tbplan")
    planio.save_plan(ora, path, with_cores=with_cores)
    say(f"[gpu] uniform DFT d={d} n={n} leaf={leaf}: load (cores {'in file' if with_cores else 'on GPU'})")
    plan = tb.load_plan(path, store=("c128", "c64"), recompute_cores=not with_cores)
    info = plan.info()
    assert (info["d"], info["L"], info["Lt"], info["Ls"]) == (d, ora.L, ora.Lt, ora.Ls)
    f = inputs.rhs_batch(n, d, 2, config=44)
    ue, ve = bf.apply(ora, f), bf.apply_adjoint(ora, f)
    for dt, cdt, bound in (("c128", torch.complex128, 1e-12), ("c64", torch.complex64, 2e-5)):
        say(f"[gpu]   apply {dt}")
        x = to_dev(f, cdt)
        u = to_host(plan.apply(x, dtype=dt))
        v = to_host(plan.apply_adjoint(x, dtype=dt))
        torch.cuda.synchronize()
        assert_parity(u, ue, bound, f"forward {dt}")
        assert_parity(v, ve, bound, f"adjoint {dt}")
    with pytest.raises(tb.TBError):      # one launch shape: nothing to tune
        plan.autotune(1, dtype="c64")


@pytest.mark.parametrize("d,n,leaf", [(4, 16, 4), (5, 8, 4)])
def test_highd_dft_gpu_construction(d, n, leaf, tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    ora = _oracle(d, n, leaf)
    say(f"[gpu] construct uniform DFT d={d} n={n} leaf={leaf}")
    plan = tb.construct("dft", d, n, 1e-3, leaf=leaf, store=("c128",))
    info = plan.info()
    assert info["r_max"] <= leaf
    path = str(tmp_path / "gpu.tbplan")
    plan.save(path)
    pf = PlanFile(path)
    same = total = 0
    for side_o, side_g in ((ora.src, pf.src), (ora.tgt, pf.tgt)):
        for l, lev in enumerate(side_o):
            for key, per_k in lev.items():
                for k in range(d):
                    for sk, (gskel, gX) in zip(per_k[k], side_g[l][key][k]):
                        total += 1
                        if list(sk.skel) == list(gskel):
                            same += 1
                            assert np.abs(sk.X - gX).max() <= 1e-7
    assert same == total, (same, total)
    op = Operator(kernels.DFT, d, n)
    f = inputs.rhs_batch(n, d, 1, config=45)
    x = to_dev(f, torch.complex128)
    u = to_host(plan.apply(x, dtype="c128"))
    v = to_host(plan.apply_adjoint(x, dtype="c128"))
    torch.cuda.synchronize()
    assert relerr(u, dense.apply_dft_fft(op, f)) <= 1e-10
    assert relerr(v, dense.adjoint_dft_fft(op, f)) <= 1e-10


def test_bit_reversed_dft_d2_on_the_tuned_kernels():
    # d = 2 and 3 plans of the same operator run on the tuned kernels
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    for d, n in ((2, 64), (3, 16)):
        say(f"[gpu] construct uniform DFT d={d} n={n}")
        plan = tb.construct("dft", d, n, 1e-6, leaf=8 if d == 2 else 4, store=("c64",))
        op = Operator(kernels.DFT, d, n)
        f = inputs.rhs_batch(n, d, 3, config=46)
        x = to_dev(f, torch.complex64)
        u = to_host(plan.apply(x))
        v = to_host(plan.apply_adjoint(x))
        torch.cuda.synchronize()
        assert relerr(u, dense.apply_dft_fft(op, f)) <= 1e-5
        assert relerr(v, dense.adjoint_dft_fft(op, f)) <= 1e-5
        with pytest.raises(tb.TBError):  # no on-the-fly entries for this kind
            plan.apply(x, dtype="c64otf")
