"""C-ABI checks that need no GPU: the library loads, exports every function
include/bltt.h declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(bltt.LIB_PATH), reason="libbltt.so not built")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bltt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bltt_[a-z_]+)\s*\(", text)))


def test_header_functions_are_exported():
    L = bltt.load()
    names = declared_functions()
    assert "bltt_setup" in names and "bltt_pminres" in names
    for name in names:
        assert hasattr(L, name), name


def test_version_and_strerror():
    L = bltt.load()
    assert L.bltt_version().startswith(b"bltt")
    for code in bltt.STATUS:
        assert len(bltt.strerror(code)) > 1
    assert bltt.strerror(12345) == "unknown status"


def _setup(prob, N=None, M=None, alpha=None, dim=None, m=None, precision=bltt.FP64, eager=0):
    L = bltt.load()
    blk = bltt.Blocks()
    blk.dim = prob.dim if dim is None else dim
    mm = list(prob.m) if m is None else list(m)
    for d in range(3):
        blk.m[d] = mm[d] if d < len(mm) else 1
        blk.h[d] = prob.h[0]
    p = np.ascontiguousarray(prob.p)
    q = np.ascontiguousarray(prob.q)
    blk.p = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    blk.q = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    opt = bltt.Options(precision, 0.0, 0, 0.0)
    opt.eager = eager
    h = ctypes.c_void_p()
    rc = L.bltt_setup(ctypes.byref(blk), prob.N if N is None else N, prob.M if M is None else M,
                      prob.alpha if alpha is None else alpha, ctypes.byref(opt), None, ctypes.byref(h))
    return rc, h


def test_invalid_arguments_rejected_on_host():
    prob = W.fractional_l1(2, 7, 16, 0.5, 0.01)
    assert _setup(prob, alpha=0.0)[0] == -1
    assert _setup(prob, alpha=1.5)[0] == -1
    assert _setup(prob, M=prob.M + 1)[0] == -1
    assert _setup(prob, dim=4)[0] == -1
    assert _setup(prob, precision=7)[0] == -1
    assert _setup(prob, eager=2)[0] == -1
    L = bltt.load()
    assert L.bltt_setup(None, 16, 49, 0.1, None, None, None) == -1
    assert L.bltt_pminres(None, None, 1e-8, 10, None, None, None, None) == -1
    L.bltt_destroy(None)


def test_unsupported_sizes_rejected_on_host():
    prob = W.fractional_l1(1, 6, 16, 0.5, 0.01)        # m + 1 = 7: not a power of two
    assert _setup(prob)[0] == -7
    prob = W.fractional_l1(1, 7, 24, 0.5, 0.01)        # N = 24
    assert _setup(prob)[0] == -7
    prob = W.fractional_l1(1, 7, 4096, 0.5, 0.01)      # N too large
    assert _setup(prob)[0] == -7
    prob = W.heat_cn(1, 7, 16, 0.1)
    prob.q[:] = 0.1                                     # q with more than 4 taps
    assert _setup(prob)[0] == -7


def test_single_block_limits_rejected_on_host():
    """N = 1 is supported for constant-coefficient ABAC handles only."""
    prob = W.heat_bdf(1, 7, 1, 0.1)
    L = bltt.load()
    blk = bltt.Blocks()
    blk.dim = 1
    blk.m[0], blk.m[1], blk.m[2] = 7, 1, 1
    blk.h[0] = blk.h[1] = blk.h[2] = prob.h[0]
    p = np.ascontiguousarray(prob.p)
    q = np.ascontiguousarray(prob.q)
    blk.p = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    blk.q = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    none = bltt.Options(bltt.FP64, 0.0, 0, 0.0, bltt.SINE, bltt.PRECOND_NONE)
    assert L.bltt_setup(ctypes.byref(blk), 1, 7, 0.1, ctypes.byref(none), None, ctypes.byref(h)) == -7
    face = np.ones(8)
    faces = (ctypes.c_void_p * 3)(face.ctypes.data, None, None)
    assert L.bltt_setup_varcoef(ctypes.byref(blk), faces, 1.0, 1, 7, 0.1, None, None, ctypes.byref(h)) == -7


def test_assumption_violation_rejected_on_host():
    prob = W.heat_bdf(1, 7, 8, 0.1)
    prob.p[1] = -4.0 * prob.p[0]                        # |A_1| dominates A_0 on low modes
    assert _setup(prob)[0] == -2
