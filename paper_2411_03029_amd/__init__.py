"""MI355X tensor butterfly: construct and apply compressed oscillatory
integral operators (arXiv 2411.03029) through libtb.so.

PyTorch supplies device memory and the current stream; every computation
runs in the library's HIP kernels.

    import paper_2411_03029_amd as tb
    plan = tb.construct("helmholtz", d=3, n=64, tol=1e-4)
    u = plan.apply(f)              # f: complex64 cuda tensor (nrhs, n, n, n)
    v = plan.apply_adjoint(u)
    u = tb.TBApply.apply(f, plan)  # autograd: backward = K^H grad
"""
from __future__ import annotations

import ctypes
import math

from . import _lib
from ._lib import TBError

KINDS = {"fourier": _lib.TB_KERNEL_FOURIER, "helmholtz": _lib.TB_KERNEL_HELMHOLTZ,
         "radon": _lib.TB_KERNEL_RADON, "nudft": _lib.TB_KERNEL_NUDFT, "dft": _lib.TB_KERNEL_DFT}
DTYPES = {"c128": _lib.TB_C128, "c64": _lib.TB_C64, "cbf16": _lib.TB_CBF16,
          "c64otf": _lib.TB_C64_OTF, "cq16": _lib.TB_CQ16}
STORE = {"c128": _lib.TB_STORE_C128, "c64": _lib.TB_STORE_C64,
         "cbf16": _lib.TB_STORE_CBF16, "otf": _lib.TB_STORE_OTF, "cq16": _lib.TB_STORE_CQ16}

__all__ = ["construct", "load_plan", "Plan", "TBApply", "TBError",
           "helmholtz_omega"]


def helmholtz_omega(n: int) -> float:
    """Wavenumber with 4 points per wavelength (2 pi n / omega = 4)."""
    return math.pi * n / 2.0


def _options(leaf=0, lt=None, proxy_pair=0, proxy_other=0, id_tol_scale=0.0,
             store=("c64",), max_rank=0, max_device_bytes=0, radon=None):
    o = _lib.TbOptions()
    o.leaf_size = leaf
    o.lt_override = 0 if lt is None else lt + 1
    o.proxy_pair = proxy_pair
    o.proxy_other = proxy_other
    o.id_tol_scale = id_tol_scale
    mask = 0
    for s in store:
        mask |= STORE[s]
    o.store_mask = mask
    o.max_rank = max_rank
    o.max_device_bytes = max_device_bytes
    if radon is not None:
        o.radon_custom = 1
        o.radon_a, o.radon_b, o.radon_den = radon
    return o


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


class Plan:
    """A tensor butterfly factorisation held on the GPU by libtb."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:  # modules may be gone at interpreter exit
            _lib.load().tb_destroy(h)
            self._h = None

    def close(self):
        self.__del__()

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        info = _lib.TbPlanInfo()
        _lib.check(_lib.load().tb_plan_info(self._h, ctypes.byref(info)))
        out = {name: getattr(info, name) for name, _ in info._fields_}
        out["stage_cmacs"] = list(out["stage_cmacs"])
        out["stage_io_entries"] = list(out["stage_io_entries"])
        return out

    @property
    def n(self) -> int:
        return self.info()["n"]

    @property
    def d(self) -> int:
        return self.info()["d"]

    def _run(self, fn, x, out, dtype):
        import torch
        info = self.info()
        n, d = info["n"], info["d"]
        if not x.is_cuda:
            raise ValueError("input must be a CUDA (HIP) tensor")
        squeeze = x.dim() == d
        xb = x.unsqueeze(0) if squeeze else x
        if tuple(xb.shape[1:]) != (n,) * d:
            raise ValueError(f"expected shape (nrhs, {n}^{d}), got {tuple(x.shape)}")
        want = torch.complex128 if dtype == "c128" else torch.complex64
        if xb.dtype != want:
            raise TypeError(f"dtype {dtype} needs {want} input, got {xb.dtype}")
        xb = xb.contiguous()
        if out is None:
            out = torch.empty_like(xb)
        elif out.shape != xb.shape or out.dtype != want or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor shaped like the input")
        _lib.check(fn(self._h, ctypes.c_void_p(xb.data_ptr()),
                      ctypes.c_void_p(out.data_ptr()), xb.shape[0], DTYPES[dtype],
                      _stream_handle(None)))
        return out.squeeze(0) if squeeze else out

    def apply(self, f, out=None, dtype="c64"):
        """u = K_BF f (Algorithm 2)."""
        return self._run(_lib.load().tb_apply, f, out, dtype)

    def apply_adjoint(self, g, out=None, dtype="c64"):
        """v = K_BF^H g."""
        return self._run(_lib.load().tb_apply_adjoint, g, out, dtype)

    def apply_noalloc(self, x, out=None, adjoint: bool = False, dtype="c64"):
        """K_BF x (or K_BF^H x) through tb_apply_noalloc: the intermediates
        live in the library's fixed device scratch array, no allocation; calls
        overlapping on one GPU race (see tb_apply_noalloc)."""
        lib = _lib.load()
        fn = lambda h, i, o, q, io, st: lib.tb_apply_noalloc(h, i, o, q, io, 1 if adjoint else 0, st)
        return self._run(fn, x, out, dtype)

    def autotune(self, nrhs: int, dtype: str = "c64", cache: str | None = None,
                 stream=None) -> int:
        """Time the launch candidates of every apply kernel for ``nrhs``
        right-hand sides and keep the fastest (see tb_plan_autotune).
        Returns the number of configurations timed (0 on a cache hit)."""
        trials = ctypes.c_int(0)
        _lib.check(_lib.load().tb_plan_autotune(
            self._h, int(nrhs), DTYPES[dtype], cache.encode() if cache else None,
            _stream_handle(stream), ctypes.byref(trials)))
        return trials.value

    def set_launch(self, nrhs: int, slot: int, dtype: str = "c64", outputs_per_thread=0,
                   rhs_tile=0, whole_blocks=0, core_kernel=0, fanin_in_turn=0,
                   transfer_mfma=0, rhs_per_thread=0, flat_stage=0) -> None:
        """Force the configuration of one launch slot (see tb_plan_set_launch)."""
        c = _lib.TbLaunchCfg(outputs_per_thread, rhs_tile, whole_blocks, core_kernel,
                             fanin_in_turn, transfer_mfma, rhs_per_thread, flat_stage)
        _lib.check(_lib.load().tb_plan_set_launch(self._h, int(nrhs), DTYPES[dtype], int(slot),
                                                  ctypes.byref(c)))

    def launch_slots(self) -> list:
        """Stage names of the launch slots, forward sequence then adjoint."""
        i = self.info()
        Lt, Ls = i["Lt"], i["Ls"]
        fwd = (["src_leaf"] + ["src_transfer"] * Lt + ["core"] + ["tgt_transfer"] * Ls +
               ["tgt_leaf"])
        adj = (["tgt_leaf_adj"] + ["tgt_transfer_adj"] * Ls + ["core_adj"] +
               ["src_transfer_adj"] * Lt + ["src_leaf_adj"])
        return fwd + adj

    def set_timing(self, enable: bool = True) -> None:
        """Record HIP events around every apply kernel (per-stage timing)."""
        _lib.check(_lib.load().tb_plan_set_timing(self._h, 1 if enable else 0))

    def stage_times(self) -> dict:
        """{stage: (total ms, launches)} recorded since the last call."""
        ms = (ctypes.c_double * len(_lib.STAGES))()
        cnt = (ctypes.c_longlong * len(_lib.STAGES))()
        _lib.check(_lib.load().tb_plan_stage_times(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.STAGES)}

    def save(self, path: str) -> None:
        _lib.check(_lib.load().tb_plan_save(self._h, path.encode()))


def apply_batched(plans, xs, outs=None, adjoint: bool = False, dtype: str = "c64",
                  stream=None):
    """Apply several plans (of any n, d and RHS count) in one HIP graph launch.

    ``xs[i]`` has shape (nrhs_i, n_i, ..) or (n_i, ..); ``outs`` (optional)
    are contiguous tensors of the same shapes.  The graph is cached on the
    argument pointers, so a loop that reuses the same ``xs``/``outs`` pays the
    capture once and then one launch per call.
    """
    import torch
    if len(plans) != len(xs) or (outs is not None and len(outs) != len(xs)):
        raise ValueError("plans, xs and outs must have the same length")
    want = torch.complex128 if dtype == "c128" else torch.complex64
    ins, res, counts = [], [], []
    for i, (p, x) in enumerate(zip(plans, xs)):
        info = p.info()
        n, d = info["n"], info["d"]
        if not x.is_cuda or x.dtype != want or not x.is_contiguous():
            raise ValueError(f"xs[{i}] must be a contiguous CUDA {want} tensor")
        xb = x.unsqueeze(0) if x.dim() == d else x
        if tuple(xb.shape[1:]) != (n,) * d:
            raise ValueError(f"xs[{i}]: expected (nrhs, {n}^{d}), got {tuple(x.shape)}")
        o = torch.empty_like(x) if outs is None else outs[i]
        if o.shape != x.shape or o.dtype != want or not o.is_contiguous():
            raise ValueError(f"outs[{i}] must be a contiguous tensor shaped like xs[{i}]")
        ins.append(xb.data_ptr())
        res.append(o)
        counts.append(xb.shape[0])
    m = len(plans)
    P = ctypes.c_void_p
    hs = (P * m)(*[p.handle for p in plans])
    ip = (P * m)(*ins)
    op = (P * m)(*[o.data_ptr() for o in res])
    nr = (ctypes.c_longlong * m)(*counts)
    _lib.check(_lib.load().tb_apply_batched(m, hs, ip, op, nr, 1 if adjoint else 0,
                                            DTYPES[dtype], _stream_handle(stream)))
    return res


def batched_reset() -> None:
    """Drop the cached graphs of apply_batched."""
    _lib.check(_lib.load().tb_batched_reset())


def construct(kind, d: int, n: int, tol: float, omega: float | None = None,
              stream=None, **opts) -> Plan:
    """Build the butterfly of operator ``kind`` on the GPU (Algorithm 1).

    ``kind``: "fourier", "helmholtz", "radon", "nudft" or "dft" (the uniform
    DFT with the bit-reversal ordering, d = 2 .. 6).  ``omega`` defaults
    to 4 points per wavelength for Helmholtz.  Options: leaf, lt, proxy_pair,
    proxy_other, id_tol_scale, store (tuple of "c128"/"c64"/"cbf16"/"cq16"/
    "otf"), max_rank, max_device_bytes, radon=(a, b, den), nudft_x (the
    NUDFT's (d, n) target coordinates).
    """
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    if omega is None:
        omega = helmholtz_omega(n) if k == _lib.TB_KERNEL_HELMHOLTZ else 0.0
    xs = opts.pop("nudft_x", None)
    o = _options(**opts)
    if xs is not None:
        import numpy as np
        xs = np.ascontiguousarray(xs, dtype=np.float64)
        if xs.shape != (d, n):
            raise ValueError(f"nudft_x must have shape ({d}, {n})")
        o.nudft_x = xs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    _lib.check(_lib.load().tb_construct(k, d, n, float(omega), float(tol), ctypes.byref(o),
                                        _stream_handle(stream), ctypes.byref(h)))
    return Plan(h)


def load_plan(path: str, store=("c64",), recompute_cores: bool = False,
              max_device_bytes: int = 0, stream=None) -> Plan:
    """Load a plan file (format in include/tb.h)."""
    o = _options(store=store, max_device_bytes=max_device_bytes)
    h = ctypes.c_void_p()
    _lib.check(_lib.load().tb_plan_load(path.encode(), ctypes.byref(o),
                                        1 if recompute_cores else 0,
                                        _stream_handle(stream), ctypes.byref(h)))
    return Plan(h)


def __getattr__(name):
    if name == "TBApply":
        from .autograd import TBApply
        return TBApply
    raise AttributeError(name)
