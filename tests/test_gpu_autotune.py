"""The autotuner (tb_plan_autotune): it times the launch candidates of
every apply kernel and keeps the fastest per (dtype, nrhs).

A tuned apply runs different kernels (right-hand-side tiles, outputs per
thread, slicing, vector or matrix-core cores) on the same plan, so it must
still match the oracle's butterfly apply to the bounds of the untuned one
(FP64 1e-12, FP32 2e-5).  The text cache round-trips: a second plan of the
same shapes finds the line and times nothing, and applies bit-identically.
"""
import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import kernels, planio
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import assert_parity, say, to_dev, to_host, torch_gpu, with_bf16_cores, with_q16_cores

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,d,n,tol,leaf", [(kernels.HELMHOLTZ, 3, 32, 1e-4, 8),
                                               (kernels.RADON, 2, 64, 1e-3, 8)])
def test_tuned_apply_matches_oracle_and_cache_round_trips(kind, d, n, tol, leaf, tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    op = bf.construct(Operator(kind, d, n, omega=om), tol, leaf=leaf)
    path = str(tmp_path / "p.tbplan")
    planio.save_plan(op, path)
    cache = str(tmp_path / "tune.txt")
    plan = tb.load_plan(path, store=("c128", "c64"))
    for dt, nrhs, bound in (("c64", 1, 2e-5), ("c64", 12, 2e-5), ("c128", 3, 1e-12)):
        say(f"[gpu] autotune kind={kind} n={n} {dt} nrhs={nrhs}")
        trials = plan.autotune(nrhs, dtype=dt, cache=cache)
        assert trials > 0
        f = inputs.rhs_batch(n, d, nrhs, config=80)
        cdt = torch.complex128 if dt == "c128" else torch.complex64
        x = to_dev(f, cdt)
        u = plan.apply(x, dtype=dt)
        v = plan.apply_adjoint(x, dtype=dt)
        torch.cuda.synchronize()
        assert_parity(to_host(u), bf.apply(op, f), bound, f"forward tuned {dt}")
        assert_parity(to_host(v), bf.apply_adjoint(op, f), bound, f"adjoint tuned {dt}")
        # a fresh plan of the same shapes reads the cache line
        other = tb.load_plan(path, store=("c128", "c64"))
        assert other.autotune(nrhs, dtype=dt, cache=cache) == 0
        u2 = other.apply(x, dtype=dt)
        v2 = other.apply_adjoint(x, dtype=dt)
        torch.cuda.synchronize()
        assert torch.equal(u, u2) and torch.equal(v, v2)
    lines = open(cache).read().splitlines()
    assert len(lines) == 3 and all(l.startswith("tbtune5 ") for l in lines)


def test_autotune_rejects_missing_precision(tmp_path):
    torch_gpu()
    import paper_2411_03029_amd as tb
    op = bf.construct(Operator(kernels.FOURIER, 2, 32), 1e-6)
    path = str(tmp_path / "f.tbplan")
    planio.save_plan(op, path)
    plan = tb.load_plan(path, store=("c64",))
    with pytest.raises(tb.TBError):
        plan.autotune(4, dtype="c128")
    with pytest.raises(tb.TBError):
        plan.autotune(0, dtype="c64")


def _candidates(stage, nrhs, dtype):
    """Every configuration the autotuner may time for a launch slot."""
    if stage.startswith("core"):
        out = [dict(core_kernel=1)]
        if nrhs >= 2:
            out.append(dict(core_kernel=2))
        if dtype != "c128" and nrhs >= 4:   # FP32 matrix cores, stored or on the fly
            out.append(dict(core_kernel=3))
        if dtype == "cbf16" and nrhs >= 4:
            out += [dict(core_kernel=v) for v in (4, 5, 6, 7)]
        if dtype != "c64otf":   # adjoint with 16-lane column groups (forward slots reject)
            out += [dict(core_kernel=8)] + ([dict(core_kernel=9)] if nrhs >= 2 else [])
        if dtype == "cq16":
            out = [c for c in out if not 3 <= c["core_kernel"] <= 7]
        return out
    fanout = stage in ("src_leaf", "src_transfer", "tgt_leaf_adj", "tgt_transfer_adj")
    out = []
    for qt in (1, 2, 4, 8):
        if qt > 1 and qt > nrhs:
            break
        for g in (1, 8):
            for whole in (0, 1):
                out.append(dict(outputs_per_thread=g, rhs_tile=qt, whole_blocks=whole))
                if qt >= 4:
                    out.append(dict(outputs_per_thread=g, rhs_tile=qt, whole_blocks=whole,
                                    rhs_per_thread=4))
        if not fanout:
            out.append(dict(rhs_tile=qt, fanin_in_turn=1))
            out.append(dict(rhs_tile=qt, fanin_in_turn=2, outputs_per_thread=8))
            if qt >= 4:
                out.append(dict(rhs_tile=qt, fanin_in_turn=2, outputs_per_thread=8, rhs_per_thread=4))
        if dtype != "c128":
            out.append(dict(rhs_tile=qt, transfer_mfma=1))
    if dtype != "c128" and nrhs >= 2:   # 4 x 4 matrix-core blocks (d = 3 transfer levels)
        out.append(dict(transfer_mfma=2))
    if dtype != "c128":   # flat staging, one right-hand side per workgroup
        out += [dict(flat_stage=1), dict(flat_stage=1, whole_blocks=1)]
    if nrhs <= 4:   # register fibers, one right-hand side per workgroup; wave per leaf box
        out += [dict(flat_stage=2), dict(flat_stage=2, whole_blocks=1), dict(flat_stage=3),
                dict(flat_stage=3, whole_blocks=1)]
    return out


@pytest.mark.parametrize("kind,d,n,tol,leaf,nrhs,dtype", [
    (kernels.HELMHOLTZ, 3, 32, 1e-4, 8, 5, "c64"),
    (kernels.HELMHOLTZ, 3, 16, 1e-4, 8, 3, "c128"),
    (kernels.RADON, 2, 32, 1e-3, 8, 9, "c64"),
    (kernels.FOURIER, 2, 64, 1e-6, 8, 1, "c64"),
    (kernels.HELMHOLTZ, 3, 32, 1e-4, 8, 6, "c64otf"),
    (kernels.RADON, 2, 32, 1e-3, 8, 20, "cbf16"),
    (kernels.HELMHOLTZ, 3, 32, 1e-4, 8, 5, "cq16"),
])
def test_every_launch_candidate_matches_oracle(kind, d, n, tol, leaf, nrhs, dtype, tmp_path):
    # each slot in turn runs each of its candidates (the rest keep the
    # heuristic); a candidate that does not fit its launch is rejected with
    # TB_ERR_UNSUPPORTED, every other one must give the oracle's result
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    op = bf.construct(Operator(kind, d, n, omega=om), tol, leaf=leaf)
    path = str(tmp_path / "p.tbplan")
    planio.save_plan(op, path)
    store = {"c128": ("c128",), "c64": ("c64",), "c64otf": ("otf",), "cbf16": ("cbf16",),
             "cq16": ("cq16",)}[dtype]
    # BF16 and 16-bit cores: against the oracle's apply of the cores as they
    # are stored (BF16-rounded, or passed through the 16-bit codec), to the
    # FP32 bound, plus 1e-5 for the hi + lo split of the right-hand sides
    # on the BF16 matrix cores
    bound = {"c128": 1e-12, "cbf16": 3e-5}.get(dtype, 2e-5)
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    f = inputs.rhs_batch(n, d, nrhs, config=81)
    x = to_dev(f, cdt)
    ref_plan = {"cbf16": with_bf16_cores, "cq16": with_q16_cores}.get(dtype, lambda o: o)(op)
    ue, ve = bf.apply(ref_plan, f), bf.apply_adjoint(ref_plan, f)
    ran = rejected = 0
    plan = tb.load_plan(path, store=store)
    slots = plan.launch_slots()
    nfwd = len(slots) // 2
    for s, stage in enumerate(slots):
        say(f"[gpu] candidates kind={kind} n={n} {dtype} nrhs={nrhs} slot {s} ({stage})")
        for cand in _candidates(stage, nrhs, dtype):
            plan.set_launch(nrhs, s, dtype=dtype, **cand)
            try:
                y = plan.apply_adjoint(x, dtype=dtype) if s >= nfwd else plan.apply(x, dtype=dtype)
                torch.cuda.synchronize()
            except tb.TBError as e:
                assert e.status == 2, (stage, cand, str(e))   # TB_ERR_UNSUPPORTED
                rejected += 1
                continue
            ref = ve if s >= nfwd else ue
            assert_parity(to_host(y), ref, bound, f"{stage} {cand}")
            ran += 1
        plan.set_launch(nrhs, s, dtype=dtype)   # back to the heuristic
    say(f"[gpu]   {ran} candidate launches checked, {rejected} rejected as not fitting")
    assert ran > 0
