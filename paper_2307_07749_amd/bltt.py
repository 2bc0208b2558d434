"""Python binding of libbltt.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/bltt.h; all
arithmetic of the solver runs in the library's HIP kernels.  PyTorch supplies
device memory (tensors) and the current HIP stream.  If the library is not
built, importing works but constructing a `Solver` raises `BlttUnavailable`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbltt.so")

FP64, MIXED, FP32 = 0, 1, 2
SINE, PHYSICAL = 0, 1  # Krylov basis (bltt_basis)
PRECOND_ABAC, PRECOND_NONE = 0, 1  # bltt_precond
PLAN_AUTO, PLAN_BASE, PLAN_ALT = 0, 1, 2  # bltt_fft_plan
PLAN_SOURCES = {0: "default", 1: "timed", 2: "cache", 3: "forced"}
KERNEL_CLASSES = ["matvec", "dst_x_vupd", "dst_strided", "time_prec", "dst_x_dot", "wx_update", "resid64", "other",
                  "time_start"]
OK, NOCONV = 0, 1
STATUS = {0: "BLTT_OK", 1: "BLTT_NOCONV", -1: "BLTT_EINVAL", -2: "BLTT_EASSUMPTION", -3: "BLTT_ENAN",
          -4: "BLTT_EBREAKDOWN", -5: "BLTT_ENOMEM", -6: "BLTT_EHIP", -7: "BLTT_EUNSUPPORTED"}


class BlttUnavailable(RuntimeError):
    """libbltt.so is missing or cannot be loaded."""


class BlttError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Blocks(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("m", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3),
                ("p", ctypes.POINTER(ctypes.c_double)), ("q", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("check_factor", ctypes.c_double), ("basis", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("initial_guess", ctypes.c_int32), ("plan_cache", ctypes.c_char_p), ("fft_plan", ctypes.c_int32),
                ("eager", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters_inner", ctypes.c_int32), ("iters_outer", ctypes.c_int32), ("true_relres", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double), ("c0", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load() -> ctypes.CDLL:
    """Load libbltt.so from the package directory (raises BlttUnavailable)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BlttUnavailable(f"{LIB_PATH} not built; run python -m paper_2307_07749_amd.build_lib")
    try:
        L = ctypes.CDLL(LIB_PATH)
    except OSError as e:  # pragma: no cover - depends on the machine
        raise BlttUnavailable(str(e)) from e
    P = ctypes.c_void_p
    L.bltt_setup.argtypes = [ctypes.POINTER(Blocks), ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                             ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    L.bltt_setup.restype = ctypes.c_int
    L.bltt_setup_varcoef.argtypes = [ctypes.POINTER(Blocks), ctypes.POINTER(P), ctypes.c_double, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_double, ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    L.bltt_setup_varcoef.restype = ctypes.c_int
    L.bltt_pminres.argtypes = [P, P, ctypes.c_double, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Info)]
    L.bltt_pminres.restype = ctypes.c_int
    for name in ("bltt_apply_sym", "bltt_apply_precond", "bltt_apply_space"):
        fn = getattr(L, name)
        fn.argtypes = [P, ctypes.c_int32, P, P]
        fn.restype = ctypes.c_int
    D = ctypes.POINTER(ctypes.c_double)
    L.bltt_modes_forward.argtypes = [P, P, P, D]
    L.bltt_modes_backward.argtypes = [P, P, P]
    L.bltt_modes_sym.argtypes = [P, ctypes.c_int32, P, P, D]
    L.bltt_modes_lanczos.argtypes = [P, ctypes.c_int32, P, P, P, D, P, P, D]
    L.bltt_modes_lanczos_noalloc.argtypes = [P, ctypes.c_int32, P, P, P, D, P, P, D]
    L.bltt_modes_resid.argtypes = [P, P, P, P, ctypes.POINTER(P), D, ctypes.c_int32, ctypes.c_double, D]
    for name in ("bltt_modes_forward", "bltt_modes_backward", "bltt_modes_sym", "bltt_modes_lanczos",
                 "bltt_modes_lanczos_noalloc", "bltt_modes_resid"):
        getattr(L, name).restype = ctypes.c_int
    L.bltt_profile_enable.argtypes = [P, ctypes.c_int32]
    L.bltt_profile_enable.restype = ctypes.c_int
    L.bltt_profile_read.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.bltt_profile_read.restype = ctypes.c_int
    L.bltt_plan_info.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int32)]
    L.bltt_plan_info.restype = ctypes.c_int
    L.bltt_batch_plans.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    L.bltt_batch_plans.restype = ctypes.c_int
    L.bltt_destroy.argtypes = [P]
    L.bltt_destroy.restype = None
    L.bltt_setup_batched.argtypes = [ctypes.POINTER(Blocks), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                     ctypes.c_int32, ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    L.bltt_setup_batched.restype = ctypes.c_int
    L.bltt_pminres_batched.argtypes = [P, ctypes.POINTER(P), ctypes.c_double, ctypes.c_int32, ctypes.POINTER(P),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(Info)]
    L.bltt_pminres_batched.restype = ctypes.c_int
    L.bltt_batch_classes.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.bltt_batch_classes.restype = ctypes.c_int
    L.bltt_destroy_batched.argtypes = [P]
    L.bltt_destroy_batched.restype = None
    L.bltt_strerror.argtypes = [ctypes.c_int]
    L.bltt_strerror.restype = ctypes.c_char_p
    L.bltt_version.restype = ctypes.c_char_p
    _lib = L
    return L


def strerror(code: int) -> str:
    return load().bltt_strerror(code).decode()


def _check(rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        raise BlttError(rc, strerror(rc))
    return rc


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Solver:
    """One BLTT instance on the GPU (wraps a bltt_handle).

    Blocks are ``p[k] I + q[k] L_h`` on a ``dim``-dimensional grid with ``m``
    interior points and spacing ``h`` per dimension (x first).  With ``face``
    (one array per dimension, the layout of bltt_setup_varcoef) the blocks are
    ``p[k] I + q[k] L_{a,h}`` and ``abar`` is the coefficient of the
    mean-coefficient system the preconditioner is built from."""

    def __init__(self, dim: int, m, h, p, q, alpha: float, precision: int = FP64, inner_tol: float = 0.0,
                 max_refine: int = 0, check_factor: float = 0.0, basis: int = 0, precond: int = 0, stream=None,
                 face=None, abar: float = 1.0, initial_guess: bool = False, plan_cache: str | None = None,
                 fft_plan: int = PLAN_AUTO, eager: bool = False):
        L = load()
        self._L = L
        m = list(m)
        h = list(h)
        self.dim = dim
        self.m = tuple(m)
        self.N = len(p)
        self.M = int(np.prod(m))
        self.n = self.N * self.M
        self.precision = precision
        self._p = np.ascontiguousarray(p, dtype=np.float64)
        self._q = np.ascontiguousarray(q, dtype=np.float64)
        blk = Blocks()
        blk.dim = dim
        for d in range(3):
            blk.m[d] = m[d] if d < dim else 1
            blk.h[d] = h[d] if d < dim else 1.0
        blk.p = self._p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        blk.q = self._q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.initial_guess = bool(initial_guess)
        self._plan_cache = plan_cache.encode() if plan_cache else None
        opt = Options(precision, inner_tol, max_refine, check_factor, basis, precond, int(bool(initial_guess)),
                      self._plan_cache, int(fft_plan), int(bool(eager)))
        self.stream = stream
        handle = ctypes.c_void_p()
        if face is None:
            rc = L.bltt_setup(ctypes.byref(blk), self.N, self.M, float(alpha), ctypes.byref(opt),
                              ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(handle))
        else:
            self._face = [np.ascontiguousarray(a, dtype=np.float64) for a in face]
            ptrs = (ctypes.c_void_p * 3)(*([a.ctypes.data for a in self._face] + [None] * (3 - len(self._face))))
            rc = L.bltt_setup_varcoef(ctypes.byref(blk), ptrs, float(abar), self.N, self.M, float(alpha),
                                      ctypes.byref(opt), ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(handle))
        _check(rc)
        self._h = handle

    @classmethod
    def from_problem(cls, prob, **kw) -> "Solver":
        return cls(prob.dim, prob.m, prob.h, prob.p, prob.q, prob.alpha, **kw)

    def close(self):
        if getattr(self, "_h", None):
            self._L.bltt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x, dtype):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dtype and x.is_contiguous()
                and x.numel() == self.n):
            raise ValueError(f"expected a contiguous CUDA tensor of {self.n} {dtype}")
        return ctypes.c_void_p(x.data_ptr())

    def pminres(self, f, tol: float, maxit: int, u=None):
        """Solve A u = f.  Returns (u, iters, hist, info, status).  A handle
        set up with initial_guess=True starts from the u passed in."""
        import torch
        fp = self._vec(f, torch.float64)
        if u is None:
            if self.initial_guess:
                raise ValueError("this solver starts from the u passed in (initial_guess=True)")
            u = torch.empty_like(f)
        up = self._vec(u, torch.float64)
        iters = ctypes.c_int32(0)
        hist = np.zeros(maxit + 2, dtype=np.float64)
        info = Info()
        rc = self._L.bltt_pminres(self._h, fp, float(tol), int(maxit), up, ctypes.byref(iters),
                                  hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(info))
        _check(rc, allow=(OK, NOCONV))
        return u, int(iters.value), hist[: iters.value + 1].copy(), info.as_dict(), rc

    def _apply(self, name, x, y=None):
        import torch
        prec = FP64 if x.dtype == torch.float64 else FP32
        xp = self._vec(x, x.dtype)
        if y is None:
            y = torch.empty_like(x)
        yp = self._vec(y, x.dtype)
        _check(getattr(self._L, name)(self._h, prec, xp, yp))
        return y

    def apply_sym(self, x, y=None):
        """y = Y A x (float64 -> FP64 kernels, float32 -> FP32 kernels)."""
        return self._apply("bltt_apply_sym", x, y)

    def apply_precond(self, x, y=None):
        """y = P_alpha^{-1} x."""
        return self._apply("bltt_apply_precond", x, y)

    def profile(self, enable: bool):
        """Start (clearing counters) or stop per-kernel event timing."""
        _check(self._L.bltt_profile_enable(self._h, int(bool(enable))))

    def profile_read(self) -> dict:
        """{class: {"launches", "ms", "bytes"}} for every kernel class."""
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            n = ctypes.c_int64(0)
            ms = ctypes.c_double(0.0)
            by = ctypes.c_double(0.0)
            _check(self._L.bltt_profile_read(self._h, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
            out[name] = {"launches": int(n.value), "ms": float(ms.value), "bytes": float(by.value)}
        return out

    def plan_info(self) -> dict:
        """Kernel plans of the FP32 sine-basis iteration (bltt_plan_info)."""
        tp, cp, src = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        blocks, cs_blocks = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(self._L.bltt_plan_info(self._h, ctypes.byref(tp), ctypes.byref(cp), ctypes.byref(blocks),
                                      ctypes.byref(cs_blocks), ctypes.byref(src)))
        return {"time_plan": tp.value, "cs_plan": cp.value, "time_blocks": blocks.value,
                "cs_blocks": cs_blocks.value, "source": PLAN_SOURCES.get(src.value, src.value)}

    def apply_space(self, x, y=None):
        """y = (I_N (x) U) x, the orthonormal sine transform of every time slice."""
        return self._apply("bltt_apply_space", x, y)

    # ---- sine-coordinate steps (mode-major vectors: element (i, n) at i*N + n)
    def modes_forward(self, x, xhat=None):
        """xhat = (I_N (x) U) x in mode-major order; returns (xhat, ||x||^2)."""
        import torch
        xp = self._vec(x, torch.float64)
        if xhat is None:
            xhat = torch.empty_like(x)
        nrm = ctypes.c_double(0.0)
        _check(self._L.bltt_modes_forward(self._h, xp, self._vec(xhat, torch.float64), ctypes.byref(nrm)))
        return xhat, float(nrm.value)

    def modes_backward(self, xhat, x=None):
        """x = (I_N (x) U) xhat in time-major order (xhat is overwritten)."""
        import torch
        xh = self._vec(xhat, torch.float64)
        if x is None:
            x = torch.empty_like(xhat)
        _check(self._L.bltt_modes_backward(self._h, xh, self._vec(x, torch.float64)))
        return x

    def modes_sym(self, z, q=None):
        """q = Y T z per sine mode; returns (q, <q, z>)."""
        import torch
        prec = FP64 if z.dtype == torch.float64 else FP32
        zp = self._vec(z, z.dtype)
        if q is None:
            q = torch.empty_like(z)
        dot = ctypes.c_double(0.0)
        _check(self._L.bltt_modes_sym(self._h, prec, zp, self._vec(q, z.dtype), ctypes.byref(dot)))
        return q, float(dot.value)

    def modes_lanczos(self, q, v1=None, v2=None, coef=(1.0, 0.0, 0.0), z=None, want_v=False, dtype=None,
                      noalloc=False, v=None):
        """vhat = coef[0] q + coef[1] v1 + coef[2] v2, z = P^{-1} vhat per mode.
        dtype: precision of v1/v2/outputs (default q's; float32 with a
        float64 q is the mixed sweep start).  noalloc: through
        bltt_modes_lanczos_noalloc (outputs z and, with want_v, v must then be
        passed in).  Returns (z, vhat or None, <vhat, z>)."""
        import torch
        if noalloc:
            if z is None or (want_v and v is None):
                raise ValueError("the no-alloc entry point takes its output tensors from the caller")
            return self._modes_lanczos_call("bltt_modes_lanczos_noalloc", q, v1, v2, coef, z, v if want_v else None,
                                            dtype)
        dt = dtype or q.dtype
        if z is None:
            z = torch.empty(q.numel(), dtype=dt, device=q.device)
        if want_v and v is None:
            v = torch.empty(q.numel(), dtype=dt, device=q.device)
        return self._modes_lanczos_call("bltt_modes_lanczos", q, v1, v2, coef, z, v if want_v else None, dtype)

    def _modes_lanczos_call(self, name, q, v1, v2, coef, z, v, dtype):
        import torch
        dt = dtype or q.dtype
        prec = FP64 if dt == torch.float64 else (MIXED if q.dtype == torch.float64 else FP32)
        qp = self._vec(q, q.dtype)
        v1p = self._vec(v1, dt) if v1 is not None else None
        v2p = self._vec(v2, dt) if v2 is not None else None
        c = (ctypes.c_double * 4)(*[float(x) for x in coef], 0.0)
        dot = ctypes.c_double(0.0)
        _check(getattr(self._L, name)(self._h, prec, qp, v1p, v2p, c, self._vec(v, dt) if v is not None else None,
                                      self._vec(z, dt), ctypes.byref(dot)))
        return z, v, float(dot.value)

    def modes_resid(self, fhat, u, r=None, zs=(), y=(), scale=1.0):
        """u += scale * sum_j y[j] zs[j] (FP32 zs), then r = Y (fhat - T u).
        Returns (r, ||r||^2); u is updated in place."""
        import torch
        fp = self._vec(fhat, torch.float64)
        up = self._vec(u, torch.float64)
        if r is None:
            r = torch.empty_like(fhat)
        k = len(zs)
        zp = (ctypes.c_void_p * max(k, 1))(*[self._vec(zz, torch.float32).value for zz in zs])
        yy = (ctypes.c_double * max(k, 1))(*[float(v) for v in y])
        nrm = ctypes.c_double(0.0)
        _check(self._L.bltt_modes_resid(self._h, fp, up, self._vec(r, torch.float64), zp if k else None,
                                        yy if k else None, k, float(scale), ctypes.byref(nrm)))
        return r, float(nrm.value)


class Batch:
    """Many independent instances (uneven N, grid, blocks, alpha), each with
    ``nrhs`` right-hand sides, solved together (wraps a bltt_batch).

    ``problems``: objects with dim, m, h, p, q, alpha (like workloads.Problem).
    System ``g = i*nrhs + r`` is instance i with right-hand side r."""

    def __init__(self, problems, nrhs: int = 1, inner_tol: float = 0.0, max_refine: int = 0, stream=None,
                 plan_cache: str | None = None, fft_plan: int = PLAN_AUTO):
        L = load()
        self._L = L
        self.count = len(problems)
        self.nrhs = int(nrhs)
        self.sizes = []
        blks = (Blocks * self.count)()
        self._keep = []
        N = (ctypes.c_int64 * self.count)()
        M = (ctypes.c_int64 * self.count)()
        A = (ctypes.c_double * self.count)()
        for i, pr in enumerate(problems):
            p = np.ascontiguousarray(pr.p, dtype=np.float64)
            q = np.ascontiguousarray(pr.q, dtype=np.float64)
            self._keep += [p, q]
            b = blks[i]
            b.dim = pr.dim
            for d in range(3):
                b.m[d] = pr.m[d] if d < pr.dim else 1
                b.h[d] = pr.h[d] if d < pr.dim else 1.0
            b.p = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            b.q = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            N[i] = len(p)
            M[i] = int(np.prod(pr.m))
            A[i] = float(pr.alpha)
            self.sizes += [N[i] * M[i]] * self.nrhs
        self._plan_cache = plan_cache.encode() if plan_cache else None
        opt = Options(MIXED, inner_tol, max_refine, 0.0, SINE, PRECOND_ABAC, 0, self._plan_cache, int(fft_plan))
        handle = ctypes.c_void_p()
        rc = L.bltt_setup_batched(blks, N, M, A, self.count, self.nrhs, ctypes.byref(opt),
                                  ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(handle))
        _check(rc)
        self._h = handle

    def classes(self):
        """Workgroup size the setup chose for each shape class."""
        n = ctypes.c_int32(0)
        _check(self._L.bltt_batch_classes(self._h, ctypes.byref(n), None))
        t = (ctypes.c_int32 * max(n.value, 1))()
        _check(self._L.bltt_batch_classes(self._h, ctypes.byref(n), t))
        return [int(t[i]) for i in range(n.value)]

    def plans(self):
        """Radix plan the setup chose for each shape class (with classes())."""
        n = ctypes.c_int32(0)
        _check(self._L.bltt_batch_classes(self._h, ctypes.byref(n), None))
        t = (ctypes.c_int32 * max(n.value, 1))()
        _check(self._L.bltt_batch_plans(self._h, t))
        return [int(t[i]) for i in range(n.value)]

    def pminres(self, fs, tol: float, maxit: int, us=None):
        """fs: list of count*nrhs float64 CUDA tensors.  Returns
        (us, iters, hists, infos, status)."""
        import torch
        nsys = self.count * self.nrhs
        if len(fs) != nsys:
            raise ValueError(f"expected {nsys} right-hand sides")
        if us is None:
            us = [torch.empty_like(f) for f in fs]
        for f, u, n in zip(fs, us, self.sizes):
            for x in (f, u):
                if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64
                        and x.is_contiguous() and x.numel() == n):
                    raise ValueError(f"expected contiguous CUDA float64 tensors of {n} elements")
        Pa = ctypes.c_void_p * nsys
        fp = Pa(*[f.data_ptr() for f in fs])
        up = Pa(*[u.data_ptr() for u in us])
        iters = (ctypes.c_int32 * nsys)()
        hist = np.zeros((nsys, maxit + 1), dtype=np.float64)
        infos = (Info * nsys)()
        rc = self._L.bltt_pminres_batched(self._h, fp, float(tol), int(maxit), up, iters,
                                          hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), infos)
        _check(rc, allow=(OK, NOCONV))
        it = [int(iters[g]) for g in range(nsys)]
        return us, it, [hist[g, : it[g] + 1].copy() for g in range(nsys)], [infos[g].as_dict() for g in range(nsys)], rc

    def close(self):
        if getattr(self, "_h", None):
            self._L.bltt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
