"""Variable-coefficient blocks p_k I + q_k L_{a,h} (Section 5.2, the heat
equation with a variable coefficient): the oracle's operator pinned to the
mathematics and to the paper's Table 3, the kernel source (run in the CPU
workgroup emulator) against the oracle, and the C entry point's argument
checks.  No GPU needed."""
import ctypes
import json
import math
import os

import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt

from tests import emu_lib as E
from tests import paper_examples as PE

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_iteration_counts.json")


def coef_2d(x1, x2):
    return (20.0 + x1 ** 2) * (20.0 + x2 ** 2)


def coef_3d(x1, x2, x3):
    return 1.0 + x1 + 2.0 * x2 * x2 + np.sin(3.0 * x3)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def grid(ms, lo=0.0, hi=1.0):
    hs = tuple((hi - lo) / (m + 1) for m in ms)
    return ms, hs


CASES = [((7,), coef_2d), ((5, 7), coef_2d), ((3, 4, 5), coef_3d)]


def _coef(ms, fn):
    if len(ms) == 1:
        return lambda x: fn(x, 0.3)
    return fn


# ---------------------------------------------------------------------------
# the oracle's L_{a,h}, pinned
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ms", [(7,), (5, 6), (3, 4, 5)])
def test_constant_coefficient_is_the_plain_laplacian(ms):
    ms, hs = grid(ms)
    ones = PE.face_samples(lambda *x: np.ones_like(x[0]), ms, hs, 0.0)
    v = np.random.default_rng(1).standard_normal((3, int(np.prod(ms))))
    assert np.allclose(O.laplacian_apply(v, ms, hs, ones), O.laplacian_apply(v, ms, hs), rtol=0, atol=1e-10)


@pytest.mark.parametrize("ms,fn", CASES)
def test_matrix_free_and_assembled_agree(ms, fn):
    ms, hs = grid(ms)
    faces = PE.face_samples(_coef(ms, fn), ms, hs, 0.0)
    v = np.random.default_rng(2).standard_normal((2, int(np.prod(ms))))
    L = O.laplacian_matrix(ms, hs, faces)
    assert np.allclose(O.laplacian_apply(v, ms, hs, faces), (L @ v.T).T, rtol=1e-13, atol=1e-9)
    # symmetric and positive definite
    Ld = L.toarray()
    assert np.allclose(Ld, Ld.T)
    assert np.linalg.eigvalsh(Ld).min() > 0


@pytest.mark.parametrize("ms,fn", CASES)
def test_energy_identity(ms, fn):
    """<v, L_{a,h} v> = sum over faces of a_f (jump of v across f)^2 / h^2,
    with v = 0 outside the grid (summation by parts of the central scheme)."""
    ms, hs = grid(ms)
    faces = PE.face_samples(_coef(ms, fn), ms, hs, 0.0)
    v = np.random.default_rng(3).standard_normal(int(np.prod(ms)))
    lhs = float(v @ O.laplacian_apply(v[None, :], ms, hs, faces)[0])
    g = v.reshape(tuple(reversed(ms)))
    energy = 0.0
    for d in range(len(ms)):
        ax = g.ndim - 1 - d
        shape = list(g.shape)
        shape[ax] += 1
        a = faces[d].reshape(shape)
        pad = [(0, 0)] * g.ndim
        pad[ax] = (1, 1)
        jump = np.diff(np.pad(g, pad), axis=ax)
        energy += float(np.sum(a * jump ** 2)) / hs[d] ** 2
    assert abs(lhs - energy) <= 1e-12 * abs(energy)


def test_second_order_consistency():
    """For smooth u and a, L_{a,h} u at the grid points approaches
    -div(a grad u) like h^2 (central differences)."""
    def u(x, y):
        return np.sin(math.pi * x) * np.sin(2 * math.pi * y)

    def minus_div(x, y):
        ux = math.pi * np.cos(math.pi * x) * np.sin(2 * math.pi * y)
        uy = 2 * math.pi * np.sin(math.pi * x) * np.cos(2 * math.pi * y)
        uxx = -math.pi ** 2 * u(x, y)
        uyy = -4 * math.pi ** 2 * u(x, y)
        a = coef_2d(x, y)
        ax = 2 * x * (20 + y ** 2)
        ay = 2 * y * (20 + x ** 2)
        return -(ax * ux + a * uxx + ay * uy + a * uyy)

    errs = []
    for mp1 in (16, 32, 64):
        ms, hs = grid((mp1 - 1, mp1 - 1))
        x = hs[0] * np.arange(1, mp1)
        X = np.tile(x, mp1 - 1)
        Y = np.repeat(x, mp1 - 1)
        faces = PE.face_samples(coef_2d, ms, hs, 0.0)
        got = O.laplacian_apply(u(X, Y)[None, :], ms, hs, faces)[0]
        errs.append(np.max(np.abs(got - minus_div(X, Y))))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def _var_system(ms, fn, N, alpha, kind="cn"):
    ms, hs = grid(ms)
    faces = PE.face_samples(_coef(ms, fn), ms, hs, 0.0)
    abar = PE.grid_mean(_coef(ms, fn), ms, hs, 0.0)
    tau = 1.0 / N
    p = np.zeros(N)
    q = np.zeros(N)
    if kind == "cn":
        p[0], p[1], q[0], q[1] = 1 / tau, -1 / tau, 0.5, 0.5
    else:
        k = np.arange(N)
        p = tau ** -0.5 / math.gamma(1.5) * np.where(
            k == 0, 1.0, (k + 1.0) ** 0.5 - 2 * k ** 0.5 + np.abs(k - 1.0) ** 0.5)
        q[0] = 1.0
    return O.System(ms, hs, p, q, alpha, faces, abar)


@pytest.mark.parametrize("ms,fn", CASES)
def test_exact_solve_matches_dense_lu(ms, fn):
    sysm = _var_system(ms, fn, 4, 0.1)
    n = sysm.N * sysm.M
    f = np.random.default_rng(4).standard_normal(n)
    A = np.column_stack([O.bltt_apply(sysm, e).ravel() for e in np.eye(n)])
    assert rel(O.exact_solve(sysm, f), np.linalg.solve(A, f)) < 1e-12
    # Y A is symmetric for the variable coefficient too (symmetric blocks, eq. (4))
    K = np.column_stack([O.sym_apply(sysm, e).ravel() for e in np.eye(n)])
    assert np.allclose(K, K.T, atol=1e-10 * np.abs(K).max())


@pytest.mark.parametrize("kind", ["cn", "frac"])
def test_pminres_solves_the_variable_system(kind):
    sysm = _var_system((7, 7), coef_2d, 16, 0.01, kind)
    f = np.random.default_rng(5).standard_normal(sysm.N * sysm.M)
    res = O.pminres(sysm, f, 1e-10, 200)
    assert rel(res.x, O.exact_solve(sysm, f)) < 1e-8
    assert res.iters <= 20


@pytest.mark.parametrize("row", json.load(open(GOLDEN))["example2_heat_varcoef_cn"]["rows"])
def test_paper_table3_counts(row):
    sysm, f, _, _ = PE.example2_system_and_rhs(row["N"], row["m_plus_1"], 1e-8)
    assert O.pminres(sysm, f, 1e-6, 100).iters == row["P_alpha"]
    if row["m_plus_1"] <= 32:
        sysm.alpha = 1.0
        it = O.pminres(sysm, f, 1e-6, 1000).iters
        assert abs(it - row["P_1"]) <= 0.03 * row["P_1"], it


@pytest.mark.parametrize("row", json.load(open(GOLDEN))["example4_fractional_varcoef"]["rows"])
def test_paper_tables7to9_counts(row):
    sysm, f, _, _, _ = PE.example4_system_and_rhs(row["gamma"], row["N"], row["m_plus_1"], 1e-8)
    assert O.pminres(sysm, f, 1e-6, 100).iters == row["P_alpha"]
    sysm.alpha = 1.0
    assert O.pminres(sysm, f, 1e-6, 100).iters == row["P_1"]


# ---------------------------------------------------------------------------
# kernel source (CPU workgroup emulator) against the oracle
# ---------------------------------------------------------------------------

class _Prob:
    """The duck-typed problem the emulator wrappers take."""

    def __init__(self, sysm):
        self.dim = len(sysm.ms)
        self.m = list(sysm.ms)
        self.h = list(sysm.hs)
        self.N = sysm.N
        self.M = sysm.M
        self.n = sysm.N * sysm.M
        self.alpha = sysm.alpha
        self.p = sysm.p
        self.q = sysm.q


@pytest.mark.parametrize("force_fft", [False, True])
@pytest.mark.parametrize("ms,fn", CASES)
def test_emulated_matvec_and_residual(ms, fn, force_fft):
    sysm = _var_system(ms, fn, 16, 0.05)
    prob = _Prob(sysm)
    rng = np.random.default_rng(6)
    z = rng.standard_normal(prob.n)
    f = rng.standard_normal(prob.n)
    with E.faces(sysm.faces):
        y, dot = E.sym(prob, z, np.float64, force_fft=force_fft)
        y32, dot32 = E.sym(prob, z, np.float32, force_fft=force_fft)
        r, rr = E.resid_full(prob, z, f, force_fft=force_fft)
    ref = O.sym_apply(sysm, z).ravel()
    assert rel(y, ref) < 1e-12
    assert abs(dot - ref @ z) <= 1e-11 * np.linalg.norm(ref) * np.linalg.norm(z)
    assert rel(y32, ref) < 1e-5
    rref = O.time_reverse((f.reshape(sysm.N, -1) - O.bltt_apply(sysm, z))).ravel()
    assert rel(r, rref) < 1e-12
    assert abs(rr - rref @ rref) <= 1e-11 * (rref @ rref)


# ---------------------------------------------------------------------------
# C entry point: arguments checked on the host
# ---------------------------------------------------------------------------

@pytest.mark.skipif(not os.path.exists(bltt.LIB_PATH), reason="libbltt.so not built")
def test_varcoef_setup_rejects_bad_arguments_on_host():
    L = bltt.load()
    sysm = _var_system((7, 7), coef_2d, 8, 0.1)
    blk = bltt.Blocks()
    blk.dim = 2
    for d in range(3):
        blk.m[d] = 7 if d < 2 else 1
        blk.h[d] = sysm.hs[0]
    p = np.ascontiguousarray(sysm.p)
    q = np.ascontiguousarray(sysm.q)
    blk.p = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    blk.q = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    faces = [np.ascontiguousarray(a) for a in sysm.faces]
    h = ctypes.c_void_p()

    def call(fs, abar=sysm.abar, opt=None):
        ptrs = (ctypes.c_void_p * 3)(*([a.ctypes.data if a is not None else None for a in fs] + [None]))
        return L.bltt_setup_varcoef(ctypes.byref(blk), ptrs, abar, 8, 49, 0.1,
                                    ctypes.byref(opt) if opt else None, None, ctypes.byref(h))

    assert L.bltt_setup_varcoef(ctypes.byref(blk), None, 1.0, 8, 49, 0.1, None, None, ctypes.byref(h)) == -1
    assert call([faces[0], None]) == -1
    bad = faces[1].copy()
    bad[3] = -1.0
    assert call([faces[0], bad]) == -1
    bad[3] = np.nan
    assert call([faces[0], bad]) == -1
    assert call(faces, abar=0.0) == -1
    none = bltt.Options(bltt.FP64, 0.0, 0, 0.0, bltt.SINE, bltt.PRECOND_NONE)
    assert call(faces, opt=none) == -7
