"""Helpers shared by the GPU tests (test code only)."""
from __future__ import annotations

import sys

import numpy as np
import pytest


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(x: np.ndarray, dtype):
    torch = torch_gpu()
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype=dtype, device="cuda")


def to_host(t) -> np.ndarray:
    return t.detach().to("cpu").numpy().astype(np.complex128)


def relerr(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def elemerr(a, b) -> float:
    """Worst single output: max |a - b| / max |b|."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def assert_parity(u, ue, bound: float, what: str = "") -> tuple:
    """Same-plan parity of a GPU result u with the oracle's ue.

    Both carry the right-hand sides on the leading axis.  For every
    right-hand side q, the relative 2-norm ||u_q - ue_q|| / ||ue_q|| and the
    worst single output max_i |u_qi - ue_qi| / max_i |ue_qi| must both stay
    within ``bound``.  The second one catches a few wrong outputs that the
    norm would average away (at 32768 outputs a single output wrong by
    bound * sqrt(N) of the RMS output still passes a norm bound).
    Returns the largest (norm, element) errors seen."""
    u, ue = np.asarray(u), np.asarray(ue)
    assert u.shape == ue.shape, (what, u.shape, ue.shape)
    worst = (0.0, 0.0)
    for q in range(u.shape[0]):
        en, ee = relerr(u[q], ue[q]), elemerr(u[q], ue[q])
        assert en <= bound, (what, "rhs", q, "norm", en, bound)
        assert ee <= bound, (what, "rhs", q, "element", ee, bound)
        worst = (max(worst[0], en), max(worst[1], ee))
    return worst


def bf16_round(c: np.ndarray) -> np.ndarray:
    """Each real and imaginary part rounded as BF16 cores are stored: FP64 to
    FP32 (round to nearest), then to BF16 (round to nearest even, the upper
    16 bits of the FP32 word).  Returned as complex128."""
    c32 = np.ascontiguousarray(np.asarray(c, dtype=np.complex64))
    w = c32.view(np.uint32).astype(np.uint64)
    w = (w + 0x7FFF + ((w >> 16) & 1)) & 0xFFFF0000
    return w.astype(np.uint32).view(np.float32).view(np.complex64).astype(np.complex128)


def with_bf16_cores(plan):
    """The oracle's plan with BF16-rounded cores: the factorisation a BF16
    apply contracts.  Against it the BF16 kernels meet FP32 bounds, which
    separates kernel errors from the rounding of the stored cores."""
    import dataclasses
    return dataclasses.replace(plan, cores={k: bf16_round(C) for k, C in plan.cores.items()})


def q16_round(C: np.ndarray) -> np.ndarray:
    """A core as 16-bit cores store it: per column (source index), the scale
    s = FP32(largest real or imaginary magnitude / 32767) and every part
    rounded to the nearest integer multiple of s, within +-32767 s (the
    documented codec); returned as the decoded complex128 values q s."""
    C = np.asarray(C, dtype=np.complex128)
    mx = np.maximum(np.abs(C.real), np.abs(C.imag)).max(axis=0)
    s = (mx / 32767.0).astype(np.float32).astype(np.float64)
    safe = np.where(s > 0, s, 1.0)
    qr = np.clip(np.rint(C.real / safe), -32767, 32767)
    qi = np.clip(np.rint(C.imag / safe), -32767, 32767)
    return np.where(s > 0, (qr + 1j * qi) * s, 0.0)


def with_q16_cores(plan):
    """The oracle's plan with its cores passed through the 16-bit codec: the
    factorisation a 16-bit-core apply contracts."""
    import dataclasses
    return dataclasses.replace(plan, cores={k: q16_round(C) for k, C in plan.cores.items()})


def say(msg: str) -> None:
    """Name the case on stdout before a GPU step (flushed)."""
    print(msg, flush=True)
    sys.stderr.flush()
