"""GPU parity of the apply kernels (Algorithm 2 and its adjoint).

The oracle builds a plan and writes it to a plan file; the library loads
the file and applies it with its HIP kernels.  Both sides then contract the
same factorisation, so the GPU result must match the oracle's apply element
by element: FP64 to 1e-12 relative, FP32 to 2e-5 relative, per right-hand
side both in the 2-norm and for the worst single output (``assert_parity``).  (FP32 bound:
each output is a chain of about 2(L+1)d small contractions and one core dot
product of at most a few thousand terms, each rounding at 2^-24 ~ 6e-8;
sqrt(terms) growth gives ~1e-5 at worst.)
"""
import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import kernels, planio
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import (assert_parity, relerr, say, to_dev, to_host, torch_gpu, with_bf16_cores,
                        with_q16_cores)

pytestmark = pytest.mark.gpu

CASES = {
    # name: (kind, d, n, tol, leaf[, target middle level])  -- tiles span
    # several blocks and levels
    "fourier2_n32": (kernels.FOURIER, 2, 32, 1e-6, 8),
    "fourier2_n64": (kernels.FOURIER, 2, 64, 1e-6, 8),
    "fourier3_n16": (kernels.FOURIER, 3, 16, 1e-4, 4),
    "helm3_n16": (kernels.HELMHOLTZ, 3, 16, 1e-4, 8),
    "helm3_n32": (kernels.HELMHOLTZ, 3, 32, 1e-4, 8),
    "radon2_n32": (kernels.RADON, 2, 32, 1e-3, 8),
    "radon2_n64_leaf4": (kernels.RADON, 2, 64, 1e-2, 4),
    "helm3_n8_single": (kernels.HELMHOLTZ, 3, 8, 1e-4, 8),   # L = 0
    "plates2_n64": (kernels.HELMHOLTZ, 2, 64, 1e-6, 8),      # parallel plates
    "radon3_n16": (kernels.RADON, 3, 16, 1e-3, 4),           # 3-D Radon
    "nudft2_n32": (kernels.NUDFT, 2, 32, 1e-6, 8),           # type-2 non-uniform DFT
    "nudft3_n16": (kernels.NUDFT, 3, 16, 1e-3, 4),
    # d = 3 with L = 3 (two source transfer levels, the second reading a
    # workspace parent, 512 middle pairs): the structure of the n = 64 cube
    # workload at a quarter of its points
    "helm3_n32_leaf4": (kernels.HELMHOLTZ, 3, 32, 1e-4, 4),
    # contracted dimensions above the on-the-fly cores' 1024-point staging
    # chunk: R_S up to 3375 (forward chunks), and with the target middle
    # level at 0, R_T up to 3375 (adjoint chunks), with ragged last chunks
    "radon3_n16_leaf8": (kernels.RADON, 3, 16, 1e-4, 8),
    "radon3_n16_leaf8_lt0": (kernels.RADON, 3, 16, 1e-4, 8, 0),
}

_PLANS = {}


def oracle_plan(name):
    if name not in _PLANS:
        spec = CASES[name] if name in CASES else LEAF16[name]
        kind, d, n, tol, leaf = spec[:5]
        lt = spec[5] if len(spec) > 5 else None
        om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
        xs = inputs.nudft_points(n, d) if kind == kernels.NUDFT else None
        _PLANS[name] = bf.construct(Operator(kind, d, n, omega=om, nudft_x=xs), tol, leaf=leaf,
                                    lt=lt)
    return _PLANS[name]


def gpu_plan(name, tmp_path, store=("c128", "c64"), recompute=False):
    import paper_2411_03029_amd as tb
    path = str(tmp_path / f"{name}.tbplan")
    planio.save_plan(oracle_plan(name), path)
    return tb.load_plan(path, store=store, recompute_cores=recompute)


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle_fp64(name, tmp_path):
    torch = torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path)
    n, d = op.n, op.d
    for nrhs in (1, 3):
        f = inputs.rhs_batch(n, d, nrhs, config=90)
        say(f"[gpu] apply fp64 {name} nrhs={nrhs}")
        u = to_host(plan.apply(to_dev(f, torch.complex128), dtype="c128"))
        torch.cuda.synchronize()
        assert_parity(u, bf.apply(op, f), 1e-12, "forward")
        say(f"[gpu] adjoint fp64 {name} nrhs={nrhs}")
        v = to_host(plan.apply_adjoint(to_dev(f, torch.complex128), dtype="c128"))
        torch.cuda.synchronize()
        assert_parity(v, bf.apply_adjoint(op, f), 1e-12, "adjoint")


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle_fp32(name, tmp_path):
    torch = torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path)
    n, d = op.n, op.d
    for nrhs in (1, 5):
        f = inputs.rhs_batch(n, d, nrhs, config=91)
        say(f"[gpu] apply fp32 {name} nrhs={nrhs}")
        u = to_host(plan.apply(to_dev(f, torch.complex64), dtype="c64"))
        v = to_host(plan.apply_adjoint(to_dev(f, torch.complex64), dtype="c64"))
        torch.cuda.synchronize()
        assert_parity(u, bf.apply(op, f), 2e-5, "forward")
        assert_parity(v, bf.apply_adjoint(op, f), 2e-5, "adjoint")


@pytest.mark.parametrize("name", list(CASES))
def test_register_fiber_stages_match_oracle(name, tmp_path):
    # every transfer and leaf launch of both directions on the register-fiber
    # kernels (slices, then whole blocks); a stage whose block does not fit
    # the kernel's LDS is rejected with TB_ERR_UNSUPPORTED, and FP32 must run
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path)
    n, d = op.n, op.d
    slots = [s for s, st in enumerate(plan.launch_slots()) if not st.startswith("core")]
    ran = set()
    for whole in (0, 1):
        for dt, cdt, bound, nrhs in (("c128", torch.complex128, 1e-12, 2), ("c64", torch.complex64, 2e-5, 1),
                                     ("c64", torch.complex64, 2e-5, 3)):
            for s in slots:
                plan.set_launch(nrhs, s, dtype=dt, flat_stage=2, whole_blocks=whole)
            f = inputs.rhs_batch(n, d, nrhs, config=93)
            x = to_dev(f, cdt)
            say(f"[gpu] register fibers {name} {dt} nrhs={nrhs} whole={whole}")
            try:
                u = to_host(plan.apply(x, dtype=dt))
                v = to_host(plan.apply_adjoint(x, dtype=dt))
                torch.cuda.synchronize()
            except tb.TBError as e:
                assert e.status == 2, str(e)   # TB_ERR_UNSUPPORTED: the block exceeds the LDS
                continue
            assert_parity(u, bf.apply(op, f), bound, f"forward {dt} whole={whole}")
            assert_parity(v, bf.apply_adjoint(op, f), bound, f"adjoint {dt} whole={whole}")
            ran.add(dt)
    assert "c64" in ran


@pytest.mark.parametrize("name", [k for k, v in CASES.items() if v[1] == 3 and v[2] >= 16])
@pytest.mark.parametrize("side", ["fanin", "fanout", "both", "leaf"])
def test_matrix_core_transfers_match_oracle(name, side, tmp_path):
    # the transfer launches on the 4 x 4 matrix-core forms: the fan-ins
    # (target side forward, source side adjoint), the fan-outs (source side
    # forward, target side adjoint), all of them, or the fan-in leaves
    # (target leaf, source leaf of the adjoint; leaf size 8); four right-hand
    # sides per workgroup, a ragged last group, and fewer right-hand sides
    # than one group.  A plan whose ranks exceed 8 (or, for the leaves, whose
    # leaf size is not 8) is rejected with TB_ERR_UNSUPPORTED; one within
    # them must run it on every such slot
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path)
    n, d = op.n, op.d
    stages = {"fanin": ("tgt_transfer", "src_transfer_adj"),
              "fanout": ("src_transfer", "tgt_transfer_adj"),
              "leaf": ("tgt_leaf", "src_leaf_adj")}
    want = stages["fanin"] + stages["fanout"] if side == "both" else stages[side]
    slots = [s for s, st in enumerate(plan.launch_slots()) if st in want]
    fits = plan.info()["r_max"] <= 8 and (side != "leaf" or op.leaf == 8)
    for nrhs in (4, 7, 2):
        for s in slots:
            plan.set_launch(nrhs, s, dtype="c64", transfer_mfma=2)
        f = inputs.rhs_batch(n, d, nrhs, config=95)
        x = to_dev(f, torch.complex64)
        say(f"[gpu] matrix-core transfers {name} {side} nrhs={nrhs} slots={slots}")
        try:
            u = to_host(plan.apply(x, dtype="c64"))
            v = to_host(plan.apply_adjoint(x, dtype="c64"))
            torch.cuda.synchronize()
        except tb.TBError as e:
            assert e.status == 2 and not fits, str(e)
            continue
        assert slots, "no transfer level"
        assert_parity(u, bf.apply(op, f), 2e-5, f"forward nrhs={nrhs}")
        assert_parity(v, bf.apply_adjoint(op, f), 2e-5, f"adjoint nrhs={nrhs}")


LEAF16 = {"fourier2_n64_leaf16": (kernels.FOURIER, 2, 64, 1e-6, 16),
          "helm3_n32_leaf16": (kernels.HELMHOLTZ, 3, 32, 1e-4, 16)}


@pytest.mark.parametrize("name", list(CASES) + list(LEAF16))
def test_wave_per_box_leaves_match_oracle(name, tmp_path):
    # the four leaf launches (source and target, both directions) on the
    # box-per-workgroup kernels (one wave or four); leaf sizes 4, 8 and 16
    torch = torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path)
    n, d = op.n, op.d
    slots = [s for s, st in enumerate(plan.launch_slots()) if "leaf" in st]
    assert len(slots) == 4
    for (dt, cdt, bound, nrhs), waves4 in zip(
            (("c128", torch.complex128, 1e-12, 2), ("c64", torch.complex64, 2e-5, 1),
             ("c64", torch.complex64, 2e-5, 3), ("c64", torch.complex64, 2e-5, 2)), (0, 0, 1, 1)):
        for s in slots:   # one wave per box, or four (whole_blocks = 1)
            plan.set_launch(nrhs, s, dtype=dt, flat_stage=3, whole_blocks=waves4)
        f = inputs.rhs_batch(n, d, nrhs, config=94)
        x = to_dev(f, cdt)
        say(f"[gpu] wave-per-box leaves {name} {dt} nrhs={nrhs} four waves={waves4}")
        u = to_host(plan.apply(x, dtype=dt))
        v = to_host(plan.apply_adjoint(x, dtype=dt))
        torch.cuda.synchronize()
        assert_parity(u, bf.apply(op, f), bound, f"forward {dt}")
        assert_parity(v, bf.apply_adjoint(op, f), bound, f"adjoint {dt}")


@pytest.mark.parametrize("name", ["helm3_n32_leaf4", "radon2_n64_leaf4"])
def test_stage_io_entries_follow_the_plan(name, tmp_path):
    # the tensor sizes the bench's per-stage byte counts use, against the
    # oracle plan's ranks: an item tensor holds per mode the concatenated
    # ranks of its blocks
    torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path)

    def entries(level):
        tot = 0
        for per_k in level.values():
            tot += int(np.prod([sum(sk.rank for sk in per_k[k]) for k in range(op.d)]))
        return tot

    nd = op.n ** op.d
    src, tgt = [entries(lv) for lv in op.src], [entries(lv) for lv in op.tgt]
    want = [nd + src[0], sum(src[l - 1] + src[l] for l in range(1, len(src))), src[-1] + tgt[-1],
            sum(tgt[l] + tgt[l - 1] for l in range(1, len(tgt))), tgt[0] + nd]
    assert plan.info()["stage_io_entries"] == want


def test_single_input_shape_and_batched_rhs_consistency(tmp_path):
    torch = torch_gpu()
    name = "helm3_n32"
    plan = gpu_plan(name, tmp_path)
    f = inputs.rhs_batch(32, 3, 4, config=92)
    say("[gpu] batched vs single rhs helm3_n32")
    ub = to_host(plan.apply(to_dev(f, torch.complex128), dtype="c128"))
    for q in range(4):
        u1 = to_host(plan.apply(to_dev(f[q], torch.complex128), dtype="c128"))
        np.testing.assert_allclose(u1, ub[q], rtol=0, atol=1e-13 * np.abs(ub).max())


def test_core_evaluation_matches_oracle(tmp_path):
    # cores recomputed on the GPU (FP64 entry evaluation at the oracle's
    # skeletons) against the oracle's cores
    torch_gpu()
    from .planfile import PlanFile
    for name in ("helm3_n32", "radon2_n32", "fourier2_n64"):
        op = oracle_plan(name)
        say(f"[gpu] core evaluation {name}")
        plan = gpu_plan(name, tmp_path, store=("c128",), recompute=True)
        out = str(tmp_path / f"{name}.gpu.tbplan")
        plan.save(out)
        pf = PlanFile(out)
        worst = 0.0
        for key, C in op.cores.items():
            worst = max(worst, float(np.abs(pf.cores[key] - C).max() / np.abs(C).max()))
        assert worst <= 1e-12, worst


def test_deterministic(tmp_path):
    torch = torch_gpu()
    plan = gpu_plan("helm3_n32", tmp_path)
    f = to_dev(inputs.rhs_batch(32, 3, 2, config=93), torch.complex64)
    say("[gpu] determinism helm3_n32")
    a = plan.apply(f)
    b = plan.apply(f)
    c = plan.apply_adjoint(a)
    e = plan.apply_adjoint(b)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, e)


def test_dtype_without_cores_is_rejected(tmp_path):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    plan = gpu_plan("helm3_n16", tmp_path, store=("c64",))
    f = to_dev(inputs.rhs_batch(16, 3, 1, config=94), torch.complex128)
    with pytest.raises(tb.TBError):
        plan.apply(f, dtype="c128")
    with pytest.raises(ValueError):
        plan.apply(to_dev(inputs.rhs_batch(8, 3, 1, config=94), torch.complex64))


@pytest.mark.parametrize("name,nrhs", [("helm3_n32", 8), ("helm3_n32", 40), ("radon2_n32", 17),
                                       ("fourier2_n64", 33)])
def test_batched_rhs_matrix_cores(name, nrhs, tmp_path):
    # from 8 right-hand sides the core contraction runs on the matrix cores
    # (complex via four real 16x16x4 FP32 MFMAs); BF16 cores accumulate in
    # FP32 with the right-hand sides split into BF16 hi + lo parts (each part
    # within 2^-18 of the FP32 value), so against the oracle's apply of the
    # BF16-rounded cores the FP32 bound holds with 1e-5 for the split;
    # against the unrounded cores the BF16 rounding (2^-9 per core part,
    # random signs) stays within 5e-3 in the 2-norm
    torch = torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path, store=("c64", "cbf16"))
    n, d = op.n, op.d
    f = inputs.rhs_batch(n, d, nrhs, config=98)
    obf = with_bf16_cores(op)
    for dt, ref, tol in (("c64", op, 2e-5), ("cbf16", obf, 3e-5)):
        say(f"[gpu] batched {name} nrhs={nrhs} {dt}")
        x = to_dev(f, torch.complex64)
        u = to_host(plan.apply(x, dtype=dt))
        v = to_host(plan.apply_adjoint(x, dtype=dt))
        torch.cuda.synchronize()
        assert_parity(u, bf.apply(ref, f), tol, f"forward {dt}")
        assert_parity(v, bf.apply_adjoint(ref, f), tol, f"adjoint {dt}")
        if dt == "cbf16":
            assert relerr(u, bf.apply(op, f)) <= 5e-3
            assert relerr(v, bf.apply_adjoint(op, f)) <= 5e-3


@pytest.mark.parametrize("name,nrhs", [("helm3_n32", 70), ("radon2_n32", 130), ("fourier2_n64", 9),
                                       ("radon3_n16", 37)])
def test_bf16_core_forms_agree(name, nrhs, tmp_path):
    # the second form of the BF16 matrix-core cores (three workgroup tiles of
    # 128 or 256 rows and 32 or 64 right-hand sides, padded positions in LDS)
    # takes the same products in the same order per accumulator as the
    # first form, so its outputs equal the first form's bit for bit, over
    # ragged right-hand-side tiles; against the oracle to the BF16 bound
    torch = torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path, store=("cbf16",))
    slots = plan.launch_slots()
    cf, ca = slots.index("core"), slots.index("core_adj")
    f = inputs.rhs_batch(op.n, op.d, nrhs, config=99)
    x = to_dev(f, torch.complex64)
    outs = {}
    for form in (4, 5, 6, 7):
        say(f"[gpu] bf16 core form {form} {name} nrhs={nrhs}")
        plan.set_launch(nrhs, cf, dtype="cbf16", core_kernel=form)
        plan.set_launch(nrhs, ca, dtype="cbf16", core_kernel=form)
        outs[form] = (plan.apply(x, dtype="cbf16"), plan.apply_adjoint(x, dtype="cbf16"))
        torch.cuda.synchronize()
    for form in (5, 6, 7):
        assert torch.equal(outs[form][0], outs[4][0]), ("forward", form)
        assert torch.equal(outs[form][1], outs[4][1]), ("adjoint", form)
    obf = with_bf16_cores(op)
    assert_parity(to_host(outs[6][0]), bf.apply(obf, f), 3e-5, "forward")
    assert_parity(to_host(outs[6][1]), bf.apply_adjoint(obf, f), 3e-5, "adjoint")


@pytest.mark.parametrize("name,nrhs", [("helm3_n32", 13), ("radon2_n32", 11), ("fourier3_n16", 9)])
def test_fanin_forms_agree(name, nrhs, tmp_path):
    # the fan-in with the children in turn and the first mode first sums
    # each output in the order of the all-children fan-in (children outer,
    # contracted index inner), so with the same RHS tile and outputs per
    # thread both give the same bits, over ragged RHS tiles and 1 or 4
    # right-hand sides per thread
    torch = torch_gpu()
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path, store=("c64",))
    slots = plan.launch_slots()
    fanin = [i for i, st in enumerate(slots)
             if st in ("tgt_transfer", "tgt_leaf", "src_transfer_adj", "src_leaf_adj")]
    nfwd = len(slots) // 2
    x = to_dev(inputs.rhs_batch(op.n, op.d, nrhs, config=93), torch.complex64)
    for v in (1, 4):
        outs = []
        for turn in (0, 2):
            say(f"[gpu] fan-in form {turn} {name} nrhs={nrhs} rhs/thread={v}")
            for i in fanin:
                plan.set_launch(nrhs, i, outputs_per_thread=8, rhs_tile=4, fanin_in_turn=turn,
                                rhs_per_thread=v)
            outs.append((plan.apply(x), plan.apply_adjoint(x)))
            torch.cuda.synchronize()
        assert torch.equal(outs[0][0], outs[1][0]), ("forward", v)
        assert torch.equal(outs[0][1], outs[1][1]), ("adjoint", v)
    assert any(i < nfwd for i in fanin) and any(i >= nfwd for i in fanin)


@pytest.mark.parametrize("name", ["helm3_n32", "radon2_n32", "fourier2_n64", "plates2_n64", "radon3_n16"])
def test_q16_cores_match_oracle(name, tmp_path):
    # block-scaled 16-bit cores (one scale per core column, int16 parts),
    # encoded on the host from the oracle's FP64 cores.  Against the oracle's
    # apply of the same cores passed through the codec the kernels meet the
    # FP32 bound, per output.  Against the unrounded cores: per part the
    # error is uniform within half a step, 2^-16 of the column's largest
    # part, independent over entries, so the core stage adds a relative
    # error of about 2^-16 * 0.6 * (column max / rms entry): 1.3e-5 for
    # unit-modulus kernels, below 4e-5 for the Helmholtz cubes (distances
    # 1..3); with the FP32 bound 2e-5 the 2-norm stays below 1e-4, per
    # right-hand side, forward and adjoint
    torch = torch_gpu()
    op = oracle_plan(name)
    oq = with_q16_cores(op)
    plan = gpu_plan(name, tmp_path, store=("cq16",))
    n, d = op.n, op.d
    for nrhs in (1, 6):
        f = inputs.rhs_batch(n, d, nrhs, config=92)
        say(f"[gpu] 16-bit cores {name} nrhs={nrhs}")
        x = to_dev(f, torch.complex64)
        u = to_host(plan.apply(x, dtype="cq16"))
        v = to_host(plan.apply_adjoint(x, dtype="cq16"))
        torch.cuda.synchronize()
        assert_parity(u, bf.apply(oq, f), 2e-5, "forward")
        assert_parity(v, bf.apply_adjoint(oq, f), 2e-5, "adjoint")
        ue, ve = bf.apply(op, f), bf.apply_adjoint(op, f)
        for q in range(nrhs):
            assert relerr(u[q], ue[q]) <= 1e-4 and relerr(v[q], ve[q]) <= 1e-4, q


def test_q16_cores_encoded_on_the_gpu(tmp_path):
    # the device encoder (cores evaluated into a temporary FP32 buffer, then
    # one scale per column) against the host encoder of the same plan's FP64
    # cores: the same scales up to FP32 rounding of the entries, so the two
    # applies agree to the quantization bound; and a plan built with the
    # 16-bit cores alone applies within 1e-4 of the FP64 apply
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    name = "helm3_n32"
    op = oracle_plan(name)
    host = gpu_plan(name, tmp_path, store=("cq16",))
    dev = gpu_plan(name, tmp_path, store=("cq16",), recompute=True)
    ref = gpu_plan(name, tmp_path, store=("c128",))
    f = inputs.rhs_batch(op.n, op.d, 3, config=91)
    x = to_dev(f, torch.complex64)
    for adjoint in (False, True):
        a = host.apply_adjoint(x, dtype="cq16") if adjoint else host.apply(x, dtype="cq16")
        b = dev.apply_adjoint(x, dtype="cq16") if adjoint else dev.apply(x, dtype="cq16")
        e = ref.apply_adjoint(to_dev(f, torch.complex128), dtype="c128") if adjoint else \
            ref.apply(to_dev(f, torch.complex128), dtype="c128")
        torch.cuda.synchronize()
        assert relerr(to_host(b), to_host(a)) <= 1e-4
        assert relerr(to_host(b), to_host(e)) <= 1e-4
    lean = tb.construct("radon", 2, 32, 1e-3, store=("cq16",))
    full = tb.construct("radon", 2, 32, 1e-3, store=("c128",))
    assert lean.info()["device_bytes"] < full.info()["device_bytes"]
    f = inputs.rhs_batch(32, 2, 2, config=90)
    u = to_host(lean.apply(to_dev(f, torch.complex64), dtype="cq16"))
    w = to_host(full.apply(to_dev(f, torch.complex128), dtype="c128"))
    torch.cuda.synchronize()
    assert relerr(u, w) <= 1e-4
    with pytest.raises(tb.TBError):
        lean.apply(to_dev(f, torch.complex64), dtype="c64")


def test_stage_multiply_add_split(tmp_path):
    # the per-stage split of the multiply-add count adds up, and the core
    # share is the sum of R_T R_S over the pairs, i.e. the core entries
    torch_gpu()
    for name in ("helm3_n32", "radon2_n32"):
        info = gpu_plan(name, tmp_path).info()
        assert sum(info["stage_cmacs"]) == info["apply_cmacs"]
        assert info["stage_cmacs"][2] == info["core_entries"]
        assert min(info["stage_cmacs"]) > 0


@pytest.mark.parametrize("name", list(CASES))
def test_on_the_fly_cores_match_oracle(name, tmp_path):
    # the cores K(tbar, sbar) evaluated inside the contraction (phase reduced
    # to a fraction of a turn in FP64, sine and cosine in FP32) from the
    # oracle's skeletons: the oracle's apply to the FP32 bound, per RHS, on a
    # plan that stores no cores at all; from 8 right-hand sides on the FP32
    # matrix cores
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    op = oracle_plan(name)
    plan = gpu_plan(name, tmp_path, store=("otf",))
    n, d = op.n, op.d
    for nrhs in (1, 5, 12):
        f = inputs.rhs_batch(n, d, nrhs, config=95)
        say(f"[gpu] on-the-fly cores {name} nrhs={nrhs}")
        x = to_dev(f, torch.complex64)
        u = to_host(plan.apply(x, dtype="c64otf"))
        v = to_host(plan.apply_adjoint(x, dtype="c64otf"))
        torch.cuda.synchronize()
        assert_parity(u, bf.apply(op, f), 2e-5, "forward")
        assert_parity(v, bf.apply_adjoint(op, f), 2e-5, "adjoint")
    with pytest.raises(tb.TBError):  # no stored FP32 cores
        plan.apply(x, dtype="c64")
