"""Differentiation through the butterfly: TBApply (torch.autograd.Function)
whose backward is the library's adjoint kernels.

For a real loss of u = K f PyTorch returns grad_f = K^H grad_u, so the
directional derivative along v is Re<grad_f, v>.  Checked by
torch.autograd.gradcheck in FP64 and by central finite differences of
L(f) = ||K f - b||^2 on 32 seeded directions for the 2-D Radon operator at
n = 256 (65536 points), with FP64 and FP32 plans.  L is exactly quadratic
in f, so central differences have no truncation error and the step is taken
large (h = 0.1 ||f|| / ||v||) to keep rounding in the FP32 losses small.
"""
import numpy as np
import pytest

from paper_2411_03029_amd import inputs

from .gpu_util import say, torch_gpu

pytestmark = pytest.mark.gpu


def test_gradcheck_fp64_small():
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    say("[gpu] gradcheck radon n=16 / helmholtz n=8")
    for kind, d, n in (("radon", 2, 16), ("helmholtz", 3, 8)):
        plan = tb.construct(kind, d, n, 1e-8, store=("c128",))
        f = torch.from_numpy(inputs.rhs_batch(n, d, 1, config=30)).to("cuda")
        f.requires_grad_(True)
        assert torch.autograd.gradcheck(lambda x: tb.TBApply.apply(x, plan, "c128"), (f,),
                                        eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)


@pytest.fixture(scope="module")
def radon256():
    torch_gpu()
    import paper_2411_03029_amd as tb
    say("[gpu] construct radon n=256 tol=1e-6 (FP64 + FP32 cores)")
    return tb.construct("radon", 2, 256, 1e-6, store=("c128", "c64"))


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-8), ("c64", 1e-3)])
def test_finite_differences_radon256(radon256, dtype, tol):
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n = 256
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    f0 = torch.from_numpy(inputs.rhs_batch(n, 2, 1, config=3)).to("cuda", cdt)
    ftrue = torch.from_numpy(inputs.rhs_batch(n, 2, 1, config=31)).to("cuda", cdt)
    b = radon256.apply(ftrue, dtype=dtype)
    b = b + 1e-3 * b.abs().mean() * torch.from_numpy(
        inputs.complex_normal(tuple(b.shape), 32) / np.sqrt(2)).to("cuda", cdt)

    def loss(f):
        r = tb.TBApply.apply(f, radon256, dtype) - b
        return (r.real.double() ** 2 + r.imag.double() ** 2).sum()

    f = f0.clone().requires_grad_(True)
    say(f"[gpu] FD radon n=256 {dtype}")
    L = loss(f)
    L.backward()
    g = f.grad.detach().to(torch.complex128)
    worst = 0.0
    for m in range(32):
        v = torch.from_numpy(inputs.complex_normal((1, n, n), 3200 + m)).to("cuda", cdt)
        h = 0.1 * float(f0.abs().norm() / v.abs().norm())
        with torch.no_grad():
            fd = (loss(f0 + h * v) - loss(f0 - h * v)).item() / (2 * h)
        an = float(torch.real(torch.vdot(g.reshape(-1), v.to(torch.complex128).reshape(-1))))
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-30))
    say(f"[gpu]   worst relative FD mismatch {worst:.2e} (bound {tol})")
    assert worst <= tol


def test_least_squares_descent_decreases_loss():
    # gradient descent on ||K f - b||^2 with the hand-written adjoint gradient
    torch = torch_gpu()
    import paper_2411_03029_amd as tb
    n = 32
    say("[gpu] least-squares descent helmholtz n=32")
    plan = tb.construct("helmholtz", 3, n, 1e-4)
    ftrue = torch.from_numpy(inputs.gaussian_bumps(n, 16, 50)[None]).to("cuda", torch.complex64)
    b = plan.apply(ftrue)
    f = torch.zeros_like(ftrue, requires_grad=True)
    losses = []
    # step from the operator norm estimate (power iteration on K^H K)
    x = torch.ones_like(ftrue)
    for _ in range(10):
        x = plan.apply_adjoint(plan.apply(x))
        x = x / x.abs().norm()
    lam = float(plan.apply(x).abs().norm() ** 2)
    for _ in range(20):
        if f.grad is not None:
            f.grad = None
        r = tb.TBApply.apply(f, plan, "c64") - b
        L = (r.abs() ** 2).sum()
        L.backward()
        losses.append(float(L))
        with torch.no_grad():
            f -= (0.5 / lam) * f.grad
    assert losses[-1] < 0.5 * losses[0]
    assert all(b2 <= a2 * (1 + 1e-5) for a2, b2 in zip(losses, losses[1:]))
