"""Writer for the plan file (tensor butterfly factorisation on disk).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  The GPU library reads
and writes the same documented format with its own code; this module is the
oracle's side of that interface and holds no code shared with it.

Format, version 1 (little endian, no padding between fields)
-------------------------------------------------------------
  char[8]   magic "TBPLAN01"
  int32[8]  kind, d, n, leaf, L, Lt, Ls, has_cores
  float64[5] omega, tol, radon_a, radon_b, radon_den
  float64[d][n] target coordinates X[k][i] (kind 3, the NUDFT, only)
  source IDs: for l = 0..Lt, s_flat, tau_flat (at level l), k = 0..d-1,
              nu = 0..2^(Lt-l)-1:
      int32 r, int32 c, int32 skel[r], complex128 X[r][c]
  target IDs: for l = 0..Ls, t_flat, nu_flat (at level l), k, tau:
      int32 r, int32 c, int32 skel[r], complex128 X[r][c]
  cores (if has_cores): for t_flat, s_flat: complex128 C[R_T][R_S]
      (R_T = prod_k r of the top target IDs, R_S likewise, rows and columns
      row-major over the modes in skeleton order)
  uint32 crc32 (zlib/IEEE polynomial) of every preceding byte, uint32 0

``skel`` holds global per-mode indices in pivot order; X's columns follow
the ID's columns: the leaf's C_b indices in increasing order (l = 0) or the
first child's skeleton followed by the second child's (l > 0).
"""
from __future__ import annotations

import struct
import zlib

import numpy as np

from .butterfly import Plan

MAGIC = b"TBPLAN01"


def _id_bytes(sk) -> bytes:
    r, c = sk.X.shape
    return (struct.pack("<ii", r, c) + np.asarray(sk.skel, "<i4").tobytes() +
            np.ascontiguousarray(sk.X, dtype="<c16").tobytes())


def plan_bytes(plan: Plan, with_cores: bool = True) -> bytes:
    op = plan.op
    d = op.d
    parts = [MAGIC,
             struct.pack("<8i", op.kind, d, op.n, plan.leaf, plan.L, plan.Lt,
                         plan.Ls, 1 if with_cores else 0),
             struct.pack("<5d", op.omega, plan.tol, op.radon_a, op.radon_b,
                         op.radon_den)]
    if op.nudft_x is not None:
        parts.append(np.asarray(op.nudft_x, dtype="<f8").tobytes())
    for l in range(plan.Lt + 1):
        for s_flat in range(1 << (d * plan.Ls)):
            for tau_flat in range(1 << (d * l)):
                for ids in plan.src[l][(s_flat, tau_flat)]:
                    parts.extend(_id_bytes(sk) for sk in ids)
    for l in range(plan.Ls + 1):
        for t_flat in range(1 << (d * plan.Lt)):
            for nu_flat in range(1 << (d * l)):
                for ids in plan.tgt[l][(t_flat, nu_flat)]:
                    parts.extend(_id_bytes(sk) for sk in ids)
    if with_cores:
        for t_flat in range(1 << (d * plan.Lt)):
            for s_flat in range(1 << (d * plan.Ls)):
                parts.append(np.ascontiguousarray(plan.cores[(t_flat, s_flat)],
                                                  dtype="<c16").tobytes())
    body = b"".join(parts)
    return body + struct.pack("<II", zlib.crc32(body) & 0xFFFFFFFF, 0)


def save_plan(plan: Plan, path: str, with_cores: bool = True) -> None:
    with open(path, "wb") as fh:
        fh.write(plan_bytes(plan, with_cores))
