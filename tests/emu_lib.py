"""Build/load helpers for the CPU workgroup emulator of the HIP kernel bodies.

The emulator (tests/native/emu.cpp) compiles the GPU kernel bodies as host
code and runs each workgroup on host threads.  Arrays are passed with NaN
guard zones on both sides: an out-of-bounds read poisons the result with NaN
and an out-of-bounds write changes a guard, so both are caught on the CPU.
"""
from __future__ import annotations

import ctypes
import glob
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "emu.cpp")
OUT_DIR = os.path.join(HERE, "native", "_build")
LIB = os.path.join(OUT_DIR, "libbltt_emu.so")
HEADERS = glob.glob(os.path.join(ROOT, "paper_2307_07749_amd", "csrc", "*.hpp"))

GUARD = 4096
_lib = None


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in [SRC, *HEADERS])


def build() -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-fPIC", "-shared",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2307_07749_amd", "csrc"),
           SRC, "-o", LIB + ".tmp", "-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stdout)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        args = [ctypes.c_int, P, P, ctypes.c_int64, ctypes.c_double, P, P]
        for t in ("f64", "f32"):
            getattr(L, f"emu_space_{t}").argtypes = args + [P, P]
            getattr(L, f"emu_time_{t}").argtypes = args + [P]
            getattr(L, f"emu_precond_{t}").argtypes = args + [P, P]
            getattr(L, f"emu_sym_{t}").argtypes = args + [P, P, ctypes.c_int]
            getattr(L, f"emu_sym_{t}").restype = ctypes.c_double
            getattr(L, f"emu_sym_nostencil_{t}").argtypes = args + [P, P, ctypes.c_int]
            getattr(L, f"emu_sym_nostencil_{t}").restype = ctypes.c_double
            getattr(L, f"emu_vupd_stencil_{t}").argtypes = args + [P, P, P]
            getattr(L, f"emu_time_aux_{t}").argtypes = args + [P]
            getattr(L, f"emu_time_aux_{t}").restype = ctypes.c_double
        L.emu_resid_f64.argtypes = args + [P, P, P]
        L.emu_resid_f64.restype = ctypes.c_double
        L.emu_error.restype = ctypes.c_int
        _lib = L
    return _lib


class Guarded:
    """A 1-D array with NaN guard zones; `.ptr` points at the interior."""

    def __init__(self, values: np.ndarray, dtype):
        n = values.size
        self.buf = np.full(n + 2 * GUARD, np.nan, dtype=dtype)
        self.buf[GUARD:GUARD + n] = values.ravel()
        self.n = n

    @property
    def ptr(self):
        return self.buf.ctypes.data + GUARD * self.buf.itemsize

    @property
    def data(self) -> np.ndarray:
        return self.buf[GUARD:GUARD + self.n]

    def guards_intact(self) -> bool:
        return bool(np.all(np.isnan(self.buf[:GUARD])) and np.all(np.isnan(self.buf[GUARD + self.n:])))


def _common(prob):
    m = (ctypes.c_int * 3)(*(list(prob.m) + [1] * (3 - prob.dim)))
    h = (ctypes.c_double * 3)(*(list(prob.h) + [1.0] * (3 - prob.dim)))
    p = np.ascontiguousarray(prob.p, dtype=np.float64)
    q = np.ascontiguousarray(prob.q, dtype=np.float64)
    return [prob.dim, ctypes.cast(m, ctypes.c_void_p), ctypes.cast(h, ctypes.c_void_p), prob.N,
            float(prob.alpha), p.ctypes.data, q.ctypes.data], (m, h, p, q)


def _tag(dtype):
    return "f64" if np.dtype(dtype) == np.float64 else "f32"


def _check(*arrs):
    L = lib()
    if L.emu_error() != 0:
        raise AssertionError(f"emulator reported error {L.emu_error()} (LDS guard or bad size)")
    for a in arrs:
        if not a.guards_intact():
            raise AssertionError("kernel wrote outside its buffer")


def space(prob, x, dtype=np.float64):
    args, keep = _common(prob)
    gx = Guarded(x, dtype)
    gy = Guarded(np.zeros(x.size), dtype)
    getattr(lib(), f"emu_space_{_tag(dtype)}")(*args, gx.ptr, gy.ptr)
    _check(gx, gy)
    return gy.data.copy()


def time_pass(prob, x, dtype=np.float64):
    args, keep = _common(prob)
    gx = Guarded(x, dtype)
    getattr(lib(), f"emu_time_{_tag(dtype)}")(*args, gx.ptr)
    _check(gx)
    return gx.data.copy()


def precond(prob, x, dtype=np.float64):
    args, keep = _common(prob)
    gx = Guarded(x, dtype)
    gy = Guarded(np.zeros(x.size), dtype)
    getattr(lib(), f"emu_precond_{_tag(dtype)}")(*args, gx.ptr, gy.ptr)
    _check(gx, gy)
    return gy.data.copy()


def sym(prob, x, dtype=np.float64, force_fft=False):
    args, keep = _common(prob)
    gx = Guarded(x, dtype)
    gy = Guarded(np.zeros(x.size), dtype)
    dot = getattr(lib(), f"emu_sym_{_tag(dtype)}")(*args, gx.ptr, gy.ptr, int(force_fft))
    _check(gx, gy)
    return gy.data.copy(), dot


def sym_nostencil(prob, x, dtype=np.float64, force_fft=False):
    args, keep = _common(prob)
    gx = Guarded(x, dtype)
    gy = Guarded(np.zeros(x.size), dtype)
    dot = getattr(lib(), f"emu_sym_nostencil_{_tag(dtype)}")(*args, gx.ptr, gy.ptr, int(force_fft))
    _check(gx, gy)
    return gy.data.copy(), dot


def vupd_stencil(prob, q1, z, dtype=np.float64):
    args, keep = _common(prob)
    gq = Guarded(q1, dtype)
    gz = Guarded(z, dtype)
    gv = Guarded(np.zeros(q1.size), dtype)
    getattr(lib(), f"emu_vupd_stencil_{_tag(dtype)}")(*args, gq.ptr, gz.ptr, gv.ptr)
    _check(gq, gz, gv)
    return gv.data.copy()


def time_aux(prob, x, dtype=np.float64):
    args, keep = _common(prob)
    gx = Guarded(x, dtype)
    s = getattr(lib(), f"emu_time_aux_{_tag(dtype)}")(*args, gx.ptr)
    _check(gx)
    return gx.data.copy(), s


def resid(prob, u, f):
    args, keep = _common(prob)
    gu = Guarded(u, np.float64)
    gf = Guarded(f, np.float64)
    gr = Guarded(np.zeros(u.size), np.float64)
    s = lib().emu_resid_f64(*args, gu.ptr, gf.ptr, gr.ptr)
    _check(gu, gf, gr)
    return gr.data.copy(), s
