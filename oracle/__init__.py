"""CPU FP64 oracle for per-pixel TDM-MIMO beat-cube synthesis.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The GPU library
never links, loads or calls it, and this package never imports the GPU
library: the two share nothing except the seeded input generator.

The arithmetic lives in `oracle.c` (plain C + OpenMP, built with
-ffp-contract=off -fno-fast-math).  This module builds it with gcc, loads it
with ctypes and converts NumPy inputs.  `brute` holds the 50-digit mpmath
brute-force sums used to pin the C code on tiny inputs.

Functions follow Sec. II: eq. (1) read per virtual channel c = m*N + r and
summed over pixels as in eq. (2), with exact per-channel ranges.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build(src: str = SRC, out: str = LIB, extra: Sequence[str] = ()) -> str:
    """Compile the oracle with gcc; returns the library path."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp", "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + res.stderr)
    os.replace(out + ".tmp", out)
    return out


class _Radar(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("Ns", ctypes.c_int32),
                ("L", ctypes.c_int32), ("fc", ctypes.c_double), ("mu", ctypes.c_double),
                ("Fs", ctypes.c_double), ("Tb", ctypes.c_double), ("c0", ctypes.c_double),
                ("tx", ctypes.POINTER(ctypes.c_double)), ("rx", ctypes.POINTER(ctypes.c_double)),
                ("carrier_phase", ctypes.c_int32), ("model", ctypes.c_int32)]


class _Pixels(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64)] + [
        (f, ctypes.POINTER(ctypes.c_float)) for f in ("x", "y", "z", "amp", "vr")]


def _f64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Oracle:
    """ctypes front end of one built oracle library."""

    def __init__(self, lib_path: Optional[str] = None):
        path = lib_path or LIB
        if lib_path is None and (not os.path.exists(LIB) or
                                 os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        self.path = path
        self.lib = ctypes.CDLL(path)
        for name in ("orc_cube", "orc_marginal_n", "orc_marginal_l"):
            fn = getattr(self.lib, name)
            fn.argtypes = [ctypes.POINTER(_Radar), ctypes.POINTER(_Pixels),
                           ctypes.POINTER(ctypes.c_double), ctypes.c_int]
            fn.restype = ctypes.c_int
        self.lib.orc_entries.argtypes = [
            ctypes.POINTER(_Radar), ctypes.POINTER(_Pixels), ctypes.c_int64,
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        self.lib.orc_entries.restype = ctypes.c_int
        self.lib.orc_chan_args.argtypes = [ctypes.POINTER(_Radar), ctypes.POINTER(_Pixels), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        self.lib.orc_chan_args.restype = ctypes.c_int
        self.lib.orc_max_threads.argtypes = [ctypes.c_int]
        self.lib.orc_max_threads.restype = ctypes.c_int

    # -- argument marshalling -------------------------------------------------
    @staticmethod
    def _radar(r):
        tx = np.ascontiguousarray(r.tx, dtype=np.float64).reshape(r.M, 3)
        rx = np.ascontiguousarray(r.rx, dtype=np.float64).reshape(r.N, 3)
        s = _Radar(int(r.M), int(r.N), int(r.Ns), int(r.L), float(r.fc), float(r.mu),
                   float(r.Fs), float(r.Tb), float(r.c0), _f64p(tx), _f64p(rx),
                   int(r.carrier_phase), int(getattr(r, "model", 0)))
        return s, (tx, rx)

    @staticmethod
    def _pixels(px, radar):
        """Strengths are [P], or [L][P] (block l's strengths in row l) when the
        radar's model has the block-strength flag (16)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in
                (px.x, px.y, px.z, px.amp, px.vr)]
        P = int(arrs[0].shape[0])
        for i, a in enumerate(arrs):
            want = (int(radar.L), P) if i == 3 and int(getattr(radar, "model", 0)) & 16 else (P,)
            if a.shape != want:
                raise ValueError(f"pixel array {i} has shape {a.shape}, expected {want}")
        return _Pixels(P, *[_f32p(a) for a in arrs]), arrs

    # -- computations -----------------------------------------------------------
    def cube(self, radar, px, threads: int = 0) -> np.ndarray:
        """Full cube Y[C][L][Ns] (complex128) by the direct sum."""
        rs, keep_r = self._radar(radar)
        ps, keep_p = self._pixels(px, radar)
        out = np.empty((radar.M * radar.N, radar.L, radar.Ns, 2), dtype=np.float64)
        if self.lib.orc_cube(ctypes.byref(rs), ctypes.byref(ps), _f64p(out), threads):
            raise ValueError("oracle rejected the arguments")
        return out.view(np.complex128)[..., 0]

    def entries(self, radar, px, c, l, n, threads: int = 0) -> np.ndarray:
        """Selected entries Y[c_k][l_k][n_k] (complex128) by the direct sum."""
        c = np.ascontiguousarray(c, dtype=np.int32)
        l = np.ascontiguousarray(l, dtype=np.int32)
        n = np.ascontiguousarray(n, dtype=np.int32)
        K = int(c.shape[0])
        rs, keep_r = self._radar(radar)
        ps, keep_p = self._pixels(px, radar)
        out = np.empty((K, 2), dtype=np.float64)
        ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if self.lib.orc_entries(ctypes.byref(rs), ctypes.byref(ps), K, ip(c), ip(l), ip(n),
                                _f64p(out), threads):
            raise ValueError("oracle rejected the arguments")
        return out.view(np.complex128)[:, 0]

    def marginal_n(self, radar, px, threads: int = 0) -> np.ndarray:
        """Closed-form sum over fast time, S[C][L] = sum_n Y[c][l][n]."""
        rs, keep_r = self._radar(radar)
        ps, keep_p = self._pixels(px, radar)
        out = np.empty((radar.M * radar.N, radar.L, 2), dtype=np.float64)
        if self.lib.orc_marginal_n(ctypes.byref(rs), ctypes.byref(ps), _f64p(out), threads):
            raise ValueError("oracle rejected the arguments")
        return out.view(np.complex128)[..., 0]

    def marginal_l(self, radar, px, threads: int = 0) -> np.ndarray:
        """Closed-form sum over slow time, S[C][Ns] = sum_l Y[c][l][n]."""
        rs, keep_r = self._radar(radar)
        ps, keep_p = self._pixels(px, radar)
        out = np.empty((radar.M * radar.N, radar.Ns, 2), dtype=np.float64)
        if self.lib.orc_marginal_l(ctypes.byref(rs), ctypes.byref(ps), _f64p(out), threads):
            raise ValueError("oracle rejected the arguments")
        return out.view(np.complex128)[..., 0]

    def chan_args(self, radar, px, c: int):
        """(psi, b, beta) of every pixel in channel c, float64 arrays [P]."""
        rs, keep_r = self._radar(radar)
        ps, keep_p = self._pixels(px, radar)
        out = [np.empty(px.P, dtype=np.float64) for _ in range(3)]
        if self.lib.orc_chan_args(ctypes.byref(rs), ctypes.byref(ps), int(c), *[_f64p(a) for a in out]):
            raise ValueError("oracle rejected the arguments")
        return tuple(out)

    def max_threads(self, threads: int = 0) -> int:
        return int(self.lib.orc_max_threads(threads))


_default: Optional[Oracle] = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def cube(radar, px, threads: int = 0):
    return default().cube(radar, px, threads)


def entries(radar, px, c, l, n, threads: int = 0):
    return default().entries(radar, px, c, l, n, threads)


def marginal_n(radar, px, threads: int = 0):
    return default().marginal_n(radar, px, threads)


def marginal_l(radar, px, threads: int = 0):
    return default().marginal_l(radar, px, threads)
