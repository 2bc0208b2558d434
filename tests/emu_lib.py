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
        for t in ("f64", "f32"):
            getattr(L, f"emu_time_upd_{t}").argtypes = args + [P, P, P, P, P, P, ctypes.c_int]
            getattr(L, f"emu_time_upd_{t}").restype = ctypes.c_double
            getattr(L, f"emu_sym_spec_{t}").argtypes = args + [P, P, ctypes.c_int]
            getattr(L, f"emu_sym_spec_{t}").restype = ctypes.c_double
            getattr(L, f"emu_wx_{t}").argtypes = [P, P, P, P, ctypes.c_int64, P]
        L.emu_time_upd_mixed.argtypes = args + [P, P, P, P, ctypes.c_int]
        L.emu_time_upd_mixed.restype = ctypes.c_double
        L.emu_resid_spec_f64.argtypes = args + [P, P, P, ctypes.c_int]
        L.emu_resid_spec_f64.restype = ctypes.c_double
        L.emu_resid_upd_f64.argtypes = args + [P, P, P, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                               ctypes.c_int]
        L.emu_resid_upd_f64.restype = ctypes.c_double
        L.emu_resid_upd_r32_f64.argtypes = args + [P, P, P, ctypes.c_double, P, ctypes.c_int, P, ctypes.c_double,
                                                   ctypes.c_int]
        L.emu_resid_upd_r32_f64.restype = ctypes.c_double
        L.emu_state_size.restype = ctypes.c_int64
        L.emu_transpose_f64.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
        L.emu_mode_pairs.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64, P, P]
        L.emu_set_faces.argtypes = [P, P, P]
        L.emu_resid_full_f64.argtypes = args + [P, P, P, ctypes.c_int]
        L.emu_resid_full_f64.restype = ctypes.c_double
        L.emu_sine_io.argtypes = args + [P, P, ctypes.c_int]
        L.emu_sine_io.restype = ctypes.c_double
        L.emu_state_offsets.argtypes = [P]
        L.emu_scalar.argtypes = [ctypes.c_int, P, P, ctypes.c_int64, P, P, P, ctypes.c_int]
        L.emu_combine_f32.argtypes = [P, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int64]
        L.emu_resid_f64.argtypes = args + [P, P, P]
        L.emu_resid_f64.restype = ctypes.c_double
        L.emu_error.restype = ctypes.c_int
        L.emu_set_plan.argtypes = [ctypes.c_int]
        L.emu_set_cs_blocks.argtypes = [ctypes.c_int]
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


class faces:
    """Context manager: the emulated kernels use the variable-coefficient
    stencil with these face arrays (one per dimension) while active."""

    def __init__(self, arrays):
        self.arrays = [np.ascontiguousarray(a, dtype=np.float64) for a in arrays]

    def __enter__(self):
        ptrs = [a.ctypes.data for a in self.arrays] + [None] * (3 - len(self.arrays))
        lib().emu_set_faces(*ptrs)
        return self

    def __exit__(self, *exc):
        lib().emu_set_faces(None, None, None)
        return False


def resid_full(prob, u, f, force_fft=False):
    """r = Y (f - A u) with the stencil inside the time-line pass; returns (r, ||r||^2)."""
    args, keep = _common(prob)
    gu = Guarded(u, np.float64)
    gf = Guarded(f, np.float64)
    gr = Guarded(np.zeros(prob.n), np.float64)
    s = lib().emu_resid_full_f64(*args, gu.ptr, gf.ptr, gr.ptr, int(force_fft))
    _check(gu, gf, gr)
    return gr.data.copy(), s


def sine_io(prob, x, direction):
    """The sine-basis transforms in and out: direction 0 takes a time-major x
    to (I x U) x mode-major (and returns the reported ||x||^2), direction 1 a
    mode-major x to (I x U) x time-major."""
    args, keep = _common(prob)
    gx = Guarded(x, np.float64)
    gy = Guarded(np.zeros(x.size), np.float64)
    s = lib().emu_sine_io(*args, gx.ptr, gy.ptr, int(direction))
    _check(gx, gy)
    return gy.data.copy(), s


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


def _ptr(g):
    return None if g is None else g.ptr


def time_upd(prob, Q, V1, V2, coef, full, dtype=np.float64, write_v=True, qrev=False):
    """vhat = c0 Q (+ c1 V1 + c2 V2), zhat = P^{-1} vhat in sine coordinates
    (qrev, start only: vhat = c0 Y Q); returns (vhat as stored or None, zhat,
    <vhat, zhat>)."""
    args, keep = _common(prob)
    gq = Guarded(Q, dtype)
    g1 = Guarded(V1, dtype) if V1 is not None else None
    g2 = Guarded(V2, dtype) if V2 is not None else None
    gv = Guarded(np.zeros(prob.n), dtype) if write_v else None
    gz = Guarded(np.zeros(prob.n), dtype)
    c = np.ascontiguousarray(coef, dtype=np.float64)
    dot = getattr(lib(), f"emu_time_upd_{_tag(dtype)}")(*args, gq.ptr, _ptr(g1), _ptr(g2), _ptr(gv), gz.ptr,
                                                        c.ctypes.data, 2 if qrev else int(full))
    _check(*[g for g in (gq, g1, g2, gv, gz) if g is not None])
    return (gv.data.copy() if gv is not None else None), gz.data.copy(), dot


def time_upd_mixed(prob, Q64, coef, qrev=False):
    """FP32 pass on an FP64 right-hand side scaled by coef[0] (qrev: on Y Q64)."""
    args, keep = _common(prob)
    gq = Guarded(Q64, np.float64)
    gv = Guarded(np.zeros(prob.n), np.float32)
    gz = Guarded(np.zeros(prob.n), np.float32)
    c = np.ascontiguousarray(coef, dtype=np.float64)
    dot = lib().emu_time_upd_mixed(*args, gq.ptr, gv.ptr, gz.ptr, c.ctypes.data, int(qrev))
    _check(gq, gv, gz)
    return gv.data.copy(), gz.data.copy(), dot


FORMS = {"direct": 0, "cs": 1, "2n": 2}


def sym_spec(prob, z, dtype=np.float64, force_fft=False, form=None):
    """form: 'direct' (short p), 'cs' (N-point), '2n' (2N-point); force_fft=True means 'cs'."""
    args, keep = _common(prob)
    gz = Guarded(z, dtype)
    go = Guarded(np.zeros(z.size), dtype)
    f = FORMS[form] if form else (1 if force_fft else 0)
    dot = getattr(lib(), f"emu_sym_spec_{_tag(dtype)}")(*args, gz.ptr, go.ptr, f)
    _check(gz, go)
    return go.data.copy(), dot


def resid_spec(prob, u, f, force_fft=False, form=None):
    args, keep = _common(prob)
    gu = Guarded(u, np.float64)
    gf = Guarded(f, np.float64)
    gr = Guarded(np.zeros(u.size), np.float64)
    fm = FORMS[form] if form else (1 if force_fft else 0)
    s = lib().emu_resid_spec_f64(*args, gu.ptr, gf.ptr, gr.ptr, fm)
    _check(gu, gf, gr)
    return gr.data.copy(), s


class State:
    """The solver's device-resident scalar state, on the host."""

    SC_NORM, SC_START, SC_DELTA, SC_BETA = 0, 1, 2, 3

    def __init__(self):
        L = lib()
        self.buf = np.zeros(int(L.emu_state_size()), dtype=np.uint8)
        off = np.zeros(8, dtype=np.int64)
        L.emu_state_offsets(off.ctypes.data)
        self.off = [int(o) for o in off]

    @property
    def ptr(self):
        return self.buf.ctypes.data

    def coef_v_ptr(self):
        return self.ptr + self.off[0]

    def coef_w_ptr(self):
        return self.ptr + self.off[1]

    def f64(self, k):
        return float(np.frombuffer(self.buf, dtype=np.float64, count=1, offset=self.off[k])[0])

    @property
    def eta(self):
        return self.f64(2)

    @property
    def eta0(self):
        return self.f64(3)

    @property
    def status(self):
        return int(np.frombuffer(self.buf, dtype=np.int32, count=1, offset=self.off[4])[0])

    def coef_v(self):
        return np.frombuffer(self.buf, dtype=np.float64, count=3, offset=self.off[0]).copy()

    def scalar(self, phase, total, hist=None, zb=None):
        """zb: (om, y) float64 arrays of lengths 2K and K for the stored-basis iterate."""
        part = np.array([total], dtype=np.float64)
        om, y, K = (None, None, 0) if zb is None else (zb[0].ctypes.data, zb[1].ctypes.data, zb[1].size)
        lib().emu_scalar(phase, self.ptr, part.ctypes.data, 1, None if hist is None else hist.ctypes.data, om, y, K)


def wx(Z, Wa, Wb, X, coef_ptr):
    """Wa <- c0 Z + c1 Wa + c2 Wb; X += c3 Wa (in place on numpy arrays)."""
    tag = "f64" if Z.dtype == np.float64 else "f32"
    getattr(lib(), f"emu_wx_{tag}")(Z.ctypes.data, Wa.ctypes.data, Wb.ctypes.data, X.ctypes.data, Z.size, coef_ptr)


def transpose(x, R, C, rev=False):
    """out (C x R) = x (R x C)^T through the library's tiled transpose."""
    gi = Guarded(x, np.float64)
    go = Guarded(np.zeros(x.size), np.float64)
    lib().emu_transpose_f64(gi.ptr, go.ptr, R, C, int(rev))
    _check(gi, go)
    return go.data.copy()


def mode_pairs(M, mx, count):
    """(ia, ib) of complex lines 0..count-1 as the sine-basis kernels pair modes."""
    ia, ib = np.zeros(count, np.int64), np.zeros(count, np.int64)
    lib().emu_mode_pairs(M, mx, count, ia.ctypes.data, ib.ctypes.data)
    return ia, ib


def combine_f32(u, Zs, y, s):
    """u += s * sum_i y[i] Zs[i] (u float64, Zs float32 rows), in place on a copy."""
    k = len(Zs)
    zs = np.ascontiguousarray(np.stack(Zs).astype(np.float32))
    out = np.ascontiguousarray(u, dtype=np.float64).copy()
    yy = np.ascontiguousarray(y, dtype=np.float64)
    lib().emu_combine_f32(out.ctypes.data, zs.ctypes.data, k, yy.ctypes.data, float(s), out.size)
    return out


def resid_upd(prob, u, f, Zs, y, s, u_zero, two_n=False):
    """(u_new, r, ||r||^2): u_new = (0 if u_zero else u) + s sum y_i Zs[i]; r = Y(f - A u_new)."""
    args, keep = _common(prob)
    gu = Guarded(u, np.float64)
    gf = Guarded(f, np.float64)
    gr = Guarded(np.zeros(u.size), np.float64)
    zs = np.ascontiguousarray(np.stack(Zs).astype(np.float32))
    yy = np.ascontiguousarray(y, dtype=np.float64)
    ss = lib().emu_resid_upd_f64(*args, gu.ptr, gf.ptr, gr.ptr, zs.ctypes.data, len(Zs), yy.ctypes.data, float(s),
                                 int(u_zero), int(two_n))
    _check(gu, gf, gr)
    return gu.data.copy(), gr.data.copy(), ss


def resid_upd_r32(prob, u, f, Zs, y, s, u_zero, r32_scale):
    """As resid_upd in the 2N-point form, with the residual returned as FP32, times r32_scale."""
    args, keep = _common(prob)
    gu = Guarded(u, np.float64)
    gf = Guarded(f, np.float64)
    gr = Guarded(np.zeros(u.size), np.float32)
    zs = np.ascontiguousarray(np.stack(Zs).astype(np.float32))
    yy = np.ascontiguousarray(y, dtype=np.float64)
    ss = lib().emu_resid_upd_r32_f64(*args, gu.ptr, gf.ptr, gr.ptr, float(r32_scale), zs.ctypes.data, len(Zs),
                                     yy.ctypes.data, float(s), int(u_zero))
    _check(gu, gf, gr)
    return gu.data.copy(), gr.data.copy(), ss


class radix_plan:
    """with radix_plan(1): the emulated FP32 time pass and N-point matvec use
    the alternative radix plan (16*16*4 at N = 1024, 16*4*8 at N = 512)."""

    def __init__(self, plan):
        self.plan = plan

    def __enter__(self):
        lib().emu_set_plan(self.plan)

    def __exit__(self, *exc):
        lib().emu_set_plan(0)


class cs_blocks:
    """with cs_blocks(n): the emulated N-point matvec runs on n persistent
    workgroups (each looping over tiles of mode pairs) instead of one per tile."""

    def __init__(self, blocks):
        self.blocks = blocks

    def __enter__(self):
        lib().emu_set_cs_blocks(self.blocks)

    def __exit__(self, *exc):
        lib().emu_set_cs_blocks(0)
