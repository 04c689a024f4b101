"""The allocation-free apply (tb_apply_noalloc) against tb_apply.

tb_apply_noalloc runs the same kernels with the same launch shapes as
tb_apply / tb_apply_adjoint, with the intermediates in the library's static
device scratch array instead of the plan's workspace, so its outputs must
equal theirs bit for bit.  Two calls in a row, the second on a smaller input
(a smaller plan and fewer right-hand sides), check that the scratch left
behind by the first call does not leak into the second; a request beyond the
array's size is refused before any launch; and a plan applied only this way
never gets a workspace of its own.
"""
import ctypes

import numpy as np
import pytest

from oracle import butterfly as bf
from oracle import kernels, planio
from oracle.kernels import Operator
from paper_2411_03029_amd import inputs

from .gpu_util import assert_parity, say, to_dev, to_host, torch_gpu

pytestmark = pytest.mark.gpu


def _noalloc(plan, x, adjoint, dtype):
    """One call through the C ABI, output allocated by the test beforehand."""
    import paper_2411_03029_amd as tb
    from paper_2411_03029_amd import _lib
    torch = torch_gpu()
    out = torch.empty_like(x)
    torch.cuda.synchronize()
    st = _lib.load().tb_apply_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), x.shape[0],
                                      tb.DTYPES[dtype], 1 if adjoint else 0,
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


def _oracle_plan(kind, d, n, tol, leaf, tmp_path, name, store):
    import paper_2411_03029_amd as tb
    om = kernels.helmholtz_omega(n) if kind == kernels.HELMHOLTZ else 0.0
    op = bf.construct(Operator(kind, d, n, omega=om), tol, leaf=leaf)
    path = str(tmp_path / f"{name}.tbplan")
    planio.save_plan(op, path)
    return op, tb.load_plan(path, store=store)


def test_noalloc_matches_tb_apply_over_two_calls(tmp_path):
    torch = torch_gpu()
    from paper_2411_03029_amd import _lib
    big = _oracle_plan(kernels.HELMHOLTZ, 3, 32, 1e-4, 8, tmp_path, "big", ("c64", "c128"))
    small = _oracle_plan(kernels.RADON, 2, 32, 1e-3, 8, tmp_path, "small", ("c64",))
    # a fresh plan holds no workspace; the allocation-free call leaves it so
    for op, plan in (big, small):
        base = plan.info()["device_bytes"]
        x = to_dev(inputs.rhs_batch(op.n, op.d, 2, config=76), torch.complex64)
        st, _ = _noalloc(plan, x, False, "c64")
        torch.cuda.synchronize()
        assert st == _lib.TB_OK, _lib.load().tb_last_error()
        assert plan.info()["device_bytes"] == base
    cases = [(big, 5, "c64", torch.complex64), (small, 2, "c64", torch.complex64),
             (big, 3, "c128", torch.complex128), (small, 1, "c64", torch.complex64)]
    for (op, plan), nrhs, dt, cdt in cases:
        f = inputs.rhs_batch(op.n, op.d, nrhs, config=77)
        x = to_dev(f, cdt)
        for adjoint in (False, True):
            say(f"[gpu] noalloc n={op.n} d={op.d} nrhs={nrhs} {dt} adjoint={adjoint}")
            ref = plan.apply_adjoint(x, dtype=dt) if adjoint else plan.apply(x, dtype=dt)
            torch.cuda.synchronize()
            ws0 = plan.info()["device_bytes"]
            st, out = _noalloc(plan, x, adjoint, dt)
            torch.cuda.synchronize()
            assert st == _lib.TB_OK, _lib.load().tb_last_error()
            assert plan.info()["device_bytes"] == ws0
            assert torch.equal(out, ref), (op.n, nrhs, dt, adjoint)
            oref = bf.apply_adjoint(op, f) if adjoint else bf.apply(op, f)
            assert_parity(to_host(out), oref, 1e-12 if dt == "c128" else 2e-5, "noalloc")


def test_noalloc_refuses_requests_beyond_the_scratch(tmp_path):
    torch = torch_gpu()
    from paper_2411_03029_amd import _lib
    op, plan = _oracle_plan(kernels.HELMHOLTZ, 3, 32, 1e-4, 8, tmp_path, "p", ("c64",))
    # the workspace of one right-hand side, from the plan's memory before and
    # after its first apply; twice the array's size in right-hand sides
    base = plan.info()["device_bytes"]
    x1 = to_dev(inputs.rhs_batch(32, 3, 1, config=78), torch.complex64)
    plan.apply(x1)
    torch.cuda.synchronize()
    ws1 = plan.info()["device_bytes"] - base
    assert ws1 > 0
    nrhs = 2 * (256 << 20) // ws1 + 1
    big = torch.zeros((nrhs,) + (32,) * 3, dtype=torch.complex64, device="cuda")
    say(f"[gpu] noalloc beyond the scratch size: {nrhs} right-hand sides")
    st, _ = _noalloc(plan, big, False, "c64")
    torch.cuda.synchronize()
    assert st == _lib.TB_ERR_OOM
    assert b"scratch" in _lib.load().tb_last_error()
    # a normal call afterwards still works
    st, out = _noalloc(plan, x1, False, "c64")
    torch.cuda.synchronize()
    assert st == _lib.TB_OK and torch.equal(out, plan.apply(x1))
