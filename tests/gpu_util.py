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


def say(msg: str) -> None:
    """Name the case on stdout before a GPU step (flushed)."""
    print(msg, flush=True)
    sys.stderr.flush()
