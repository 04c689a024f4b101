"""Test-side reader for the plan file (format documented in include/tb.h).

Used to inspect plans the GPU library writes and to check the oracle's
writer; it is test code, not part of the oracle or of the product path.
"""
from __future__ import annotations

import struct
import zlib

import numpy as np


class PlanFile:
    def __init__(self, path_or_bytes):
        if isinstance(path_or_bytes, (bytes, bytearray)):
            buf = bytes(path_or_bytes)
        else:
            with open(path_or_bytes, "rb") as fh:
                buf = fh.read()
        if buf[:8] != b"TBPLAN01":
            raise ValueError("bad magic")
        crc, zero = struct.unpack_from("<II", buf, len(buf) - 8)
        if zlib.crc32(buf[:-8]) & 0xFFFFFFFF != crc or zero != 0:
            raise ValueError("checksum mismatch")
        (self.kind, self.d, self.n, self.leaf, self.L, self.Lt, self.Ls,
         self.has_cores) = struct.unpack_from("<8i", buf, 8)
        (self.omega, self.tol, self.radon_a, self.radon_b,
         self.radon_den) = struct.unpack_from("<5d", buf, 40)
        self._buf = buf
        self._pos = 80
        d = self.d
        self.nudft_x = None
        if self.kind == 3:   # NUDFT: the target coordinates follow the header
            self.nudft_x = np.frombuffer(buf, "<f8", d * self.n, self._pos).reshape(d, self.n)
            self._pos += 8 * d * self.n
        self.src = []
        for l in range(self.Lt + 1):
            lev = {}
            for s_flat in range(1 << (d * self.Ls)):
                for tau_flat in range(1 << (d * l)):
                    lev[(s_flat, tau_flat)] = [
                        [self._read_id() for _ in range(1 << (self.Lt - l))]
                        for _ in range(d)]
            self.src.append(lev)
        self.tgt = []
        for l in range(self.Ls + 1):
            lev = {}
            for t_flat in range(1 << (d * self.Lt)):
                for nu_flat in range(1 << (d * l)):
                    lev[(t_flat, nu_flat)] = [
                        [self._read_id() for _ in range(1 << (self.Ls - l))]
                        for _ in range(d)]
            self.tgt.append(lev)
        self.cores = {}
        if self.has_cores:
            for t_flat in range(1 << (d * self.Lt)):
                for s_flat in range(1 << (d * self.Ls)):
                    rt = int(np.prod([self.tgt[self.Ls][(t_flat, s_flat)][k][0][0].size
                                      for k in range(d)]))
                    rs = int(np.prod([self.src[self.Lt][(s_flat, t_flat)][k][0][0].size
                                      for k in range(d)]))
                    nbytes = rt * rs * 16
                    arr = np.frombuffer(buf, "<c16", rt * rs, self._pos).reshape(rt, rs)
                    self._pos += nbytes
                    self.cores[(t_flat, s_flat)] = arr
        if self._pos != len(buf) - 8:
            raise ValueError("trailing bytes in plan file")

    def _read_id(self):
        r, c = struct.unpack_from("<ii", self._buf, self._pos)
        self._pos += 8
        skel = np.frombuffer(self._buf, "<i4", r, self._pos).astype(np.int64)
        self._pos += 4 * r
        X = np.frombuffer(self._buf, "<c16", r * c, self._pos).reshape(r, c)
        self._pos += 16 * r * c
        return skel, X
