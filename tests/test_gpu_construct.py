"""GPU construction (Algorithm 1): FP64 entries at proxy indices, IDs by
tall-skinny QR + column-pivoted QR, cores.

Several factorisations are correct when pivots tie or nearly tie, so the GPU
factors are compared with the oracle's where they are unique (ranks and
skeletons agree on the vast majority of IDs) and the GPU butterfly is checked
against the plain definition u = K f (FFT, FFT convolution or brute force)
at the requested tolerance.
"""
import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import dense, kernels
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import relerr, say, to_dev, to_host, torch_gpu
from .planfile import PlanFile

pytestmark = pytest.mark.gpu

KIND = {kernels.FOURIER: "fourier", kernels.HELMHOLTZ: "helmholtz", kernels.RADON: "radon",
        kernels.NUDFT: "nudft"}


def _op(kind, d, n):
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    xs = inputs.nudft_points(n, d) if kind == kernels.NUDFT else None
    return Operator(kind, d, n, omega=om, nudft_x=xs)


def _extra(kind, d, n):
    """Construction options an operator needs beyond (kind, d, n, tol)."""
    return {"nudft_x": inputs.nudft_points(n, d)} if kind == kernels.NUDFT else {}


@pytest.mark.parametrize("kind,d,n,tol,leaf", [
    (kernels.FOURIER, 2, 64, 1e-6, 8),
    (kernels.HELMHOLTZ, 3, 32, 1e-4, 8),
    (kernels.RADON, 2, 32, 1e-3, 8),
    (kernels.HELMHOLTZ, 3, 16, 1e-4, 8),
    (kernels.HELMHOLTZ, 2, 64, 1e-6, 8),   # parallel plates
    (kernels.RADON, 3, 16, 1e-3, 4),       # 3-D Radon
    (kernels.NUDFT, 2, 32, 1e-6, 8),       # type-2 non-uniform DFT
    (kernels.NUDFT, 3, 16, 1e-3, 4),
])
def test_gpu_factors_match_oracle(kind, d, n, tol, leaf, tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    op = _op(kind, d, n)
    ora = bf.construct(op, tol, leaf=leaf)
    say(f"[gpu] construct {KIND[kind]} d={d} n={n} tol={tol}")
    plan = tb.construct(KIND[kind], d, n, tol, leaf=leaf, store=("c128", "c64"), **_extra(kind, d, n))
    info = plan.info()
    assert (info["L"], info["Lt"], info["Ls"]) == (ora.L, ora.Lt, ora.Ls)
    path = str(tmp_path / "gpu.tbplan")
    plan.save(path)
    pf = PlanFile(path)
    same_rank = same_skel = total = 0
    xerr = 0.0
    for side_o, side_g in ((ora.src, pf.src), (ora.tgt, pf.tgt)):
        for l, lev in enumerate(side_o):
            for key, per_k in lev.items():
                for k in range(d):
                    for sk, (gskel, gX) in zip(per_k[k], side_g[l][key][k]):
                        total += 1
                        same_rank += sk.rank == len(gskel)
                        if list(sk.skel) == list(gskel):
                            same_skel += 1
                            xerr = max(xerr, float(np.abs(sk.X - gX).max()))
    say(f"[gpu]   ranks {same_rank}/{total} skeletons {same_skel}/{total} max dX {xerr:.2e}")
    assert same_rank >= 0.95 * total
    assert same_skel >= 0.9 * total
    assert xerr <= 1e-7
    # the GPU butterfly against the plain definition
    f = inputs.rhs_batch(n, d, 2, config=95)
    u = to_host(plan.apply(to_dev(f, torch.complex128), dtype="c128"))
    v = to_host(plan.apply_adjoint(to_dev(f, torch.complex128), dtype="c128"))
    torch.cuda.synchronize()
    assert relerr(u, dense.apply_exact(op, f)) <= tol
    assert relerr(v, dense.adjoint_exact(op, f)) <= tol


def test_gpu_construct_exact_limit():
    # whole nodes as proxies and a tiny tolerance: the butterfly is exact
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    op = _op(kernels.RADON, 2, 16)
    say("[gpu] construct exact limit radon n=16")
    plan = tb.construct("radon", 2, 16, 1e-12, proxy_pair=-1, proxy_other=-1,
                        id_tol_scale=1e-3, store=("c128",))
    f = inputs.rhs_batch(16, 2, 1, config=96)
    u = to_host(plan.apply(to_dev(f, torch.complex128), dtype="c128"))
    assert relerr(u, dense.apply_brute(op, f)) <= 1e-10


def test_gpu_construct_max_rank_and_memory_cap():
    torch_gpu()
    import paper_2411_03029_amd as tb
    from paper_2411_03029_amd import _lib
    say("[gpu] construct max_rank / device cap")
    with pytest.raises(tb.TBError) as ei:
        tb.construct("helmholtz", 3, 32, 1e-6, max_rank=3)
    assert ei.value.status == _lib.TB_ERR_NUMERIC
    with pytest.raises(tb.TBError) as ei:
        tb.construct("helmholtz", 3, 32, 1e-4, max_device_bytes=1 << 16)
    assert ei.value.status == _lib.TB_ERR_OOM


def test_gpu_construct_radon_custom_constants_reduce_to_dft():
    # a = b = 0: no speed term, K = exp(+2 pi i x.k), an inverse DFT
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n = 64
    say("[gpu] construct radon a=b=0")
    plan = tb.construct("radon", 2, n, 1e-6, radon=(0.0, 0.0, 1.0), store=("c128",))
    f = inputs.rhs_batch(n, 2, 1, config=97)
    u = to_host(plan.apply(to_dev(f, torch.complex128), dtype="c128"))
    expect = np.fft.ifftn(np.fft.ifftshift(f, axes=(1, 2)), axes=(1, 2)) * n * n
    assert relerr(u, expect) <= 1e-6


def test_construct_without_stored_cores():
    # a plan built with no stored cores applies with on-the-fly cores and
    # meets tol against the exact operator; it holds less device memory
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n, tol = 32, 1e-4
    say("[gpu] construct helmholtz n=32 without stored cores")
    lean = tb.construct("helmholtz", 3, n, tol, store=("otf",))
    full = tb.construct("helmholtz", 3, n, tol, store=("c64",))
    assert lean.info()["device_bytes"] < full.info()["device_bytes"]
    op = Operator(kernels.HELMHOLTZ, 3, n, omega=kernels.helmholtz_omega(n))
    f = inputs.rhs_batch(n, 3, 2, config=96)
    x = to_dev(f, torch.complex64)
    u = to_host(lean.apply(x, dtype="c64otf"))
    v = to_host(lean.apply_adjoint(x, dtype="c64otf"))
    torch.cuda.synchronize()
    assert relerr(u, dense.apply_exact(op, f)) <= tol
    assert relerr(v, dense.adjoint_exact(op, f)) <= tol


def test_nudft_rejects_bad_points():
    # coordinates outside [0, n - 1] or decreasing within a mode are refused
    torch_gpu()
    import paper_2411_03029_amd as tb
    n = 32
    xs = inputs.nudft_points(n, 2)
    bad = xs.copy()
    bad[0, 3] = n
    with pytest.raises(tb.TBError) as ei:
        tb.construct("nudft", 2, n, 1e-6, nudft_x=bad)
    assert ei.value.status == 1   # TB_ERR_INVALID_ARG
    bad = xs.copy()
    bad[1, 5], bad[1, 6] = bad[1, 6], bad[1, 5] - 0.5
    with pytest.raises(tb.TBError) as ei:
        tb.construct("nudft", 2, n, 1e-6, nudft_x=bad)
    assert ei.value.status == 1
