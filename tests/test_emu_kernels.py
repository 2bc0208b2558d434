"""CPU emulation of the HIP kernel bodies against the oracle.

The same __host__ __device__ kernel code that runs on the MI355X is executed
workgroup by workgroup on host threads (tests/native/emu.cpp), with NaN guard
zones around every buffer.  Sizes span several workgroups and ragged tails.
"""
import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import workloads as W
from tests import emu_lib as E

TOL = {np.float64: 1e-12, np.float32: 2e-5}


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def prob_of(kind, dim, m, N, alpha=0.05, gamma=0.4):
    if kind == "frac":
        return W.fractional_l1(dim, m, N, gamma, alpha)
    if kind == "heat":
        return W.heat_bdf(dim, m, N, alpha)
    if kind == "cn":
        return W.heat_cn(dim, m, N, alpha)
    raise ValueError(kind)


SPACE_CASES = [(1, 1, 2), (1, 7, 4), (1, 31, 8), (2, 3, 4), (2, 7, 2), (2, 15, 4), (3, 3, 4), (3, 7, 2),
               (1, 255, 2), (2, 63, 2)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("dim,m,N", SPACE_CASES)
def test_space_transform(dim, m, N, dtype):
    prob = prob_of("frac", dim, m, N)
    x = np.random.default_rng(dim * 100 + m).standard_normal(prob.n)
    got = E.space(prob, x, dtype)
    ref = O.space_transform(x.reshape(N, -1), prob.m).ravel()
    assert rel(got, ref) < TOL[dtype] * 10


TIME_CASES = [("frac", 1, 7, 2), ("frac", 1, 7, 4), ("frac", 1, 5, 8), ("frac", 1, 9, 16), ("heat", 2, 3, 32),
              ("frac", 2, 7, 64), ("cn", 1, 15, 128), ("frac", 1, 3, 256), ("frac", 1, 3, 512),
              ("frac", 1, 1, 1024), ("heat", 1, 3, 2048)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kind,dim,m,N", TIME_CASES)
def test_time_pass(kind, dim, m, N, dtype):
    prob = prob_of(kind, dim, m, N, alpha=0.05)
    sysm = O.from_problem(prob)
    P = O.precond_setup(sysm)
    x = np.random.default_rng(N + m).standard_normal(prob.n)
    got = E.time_pass(prob, x, dtype)
    # time part alone: U P^{-1} U (U symmetric orthogonal)
    ref = O.space_transform(O.precond_apply(P, O.space_transform(x.reshape(N, -1), prob.m)), prob.m).ravel()
    tol = TOL[dtype] * (100 if dtype == np.float32 else 1e3)
    assert rel(got, ref) < tol


PRE_CASES = [("frac", 1, 31, 32, 0.01), ("heat", 2, 7, 16, 0.01), ("frac", 2, 15, 8, 0.1), ("cn", 2, 3, 4, 0.5),
             ("frac", 3, 3, 8, 0.05), ("frac", 1, 63, 64, 0.001)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kind,dim,m,N,alpha", PRE_CASES)
def test_precond(kind, dim, m, N, alpha, dtype):
    prob = prob_of(kind, dim, m, N, alpha=alpha)
    P = O.precond_setup(O.from_problem(prob))
    x = np.random.default_rng(7).standard_normal(prob.n)
    got = E.precond(prob, x, dtype)
    ref = O.precond_apply(P, x.reshape(N, -1)).ravel()
    tol = 1e-11 if dtype == np.float64 else 5e-5 / alpha ** 0.5
    assert rel(got, ref) < tol


SYM_CASES = [("frac", 1, 31, 32), ("heat", 2, 7, 16), ("cn", 2, 5, 8), ("frac", 3, 3, 8), ("frac", 2, 15, 64), ("frac", 1, 3, 2048),
             ("heat", 1, 3, 2), ("frac", 1, 5, 256)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("force_fft", [False, True])
@pytest.mark.parametrize("kind,dim,m,N", SYM_CASES)
def test_sym_matvec(kind, dim, m, N, force_fft, dtype):
    prob = prob_of(kind, dim, m, N)
    sysm = O.from_problem(prob)
    z = np.random.default_rng(3).standard_normal(prob.n)
    got, dot = E.sym(prob, z, dtype, force_fft)
    ref = O.sym_apply(sysm, z.reshape(N, -1)).ravel()
    assert rel(got, ref) < TOL[dtype] * 50
    zz = z.astype(dtype).astype(np.float64)
    assert abs(dot - np.dot(ref, zz)) <= TOL[dtype] * 50 * np.linalg.norm(ref) * np.linalg.norm(zz)


SPLIT_CASES = [("frac", 1, 31, 32), ("heat", 2, 7, 16), ("cn", 2, 7, 8), ("frac", 3, 3, 8), ("cn", 3, 3, 4),
               ("frac", 2, 15, 64)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kind,dim,m,N", SPLIT_CASES)
def test_split_matvec_equals_full(kind, dim, m, N, dtype):
    """Inside MINRES the time-line matvec forms Y (p * z) only; the x-line pass
    adds Y L_h (q * z); the sum must be Y A z."""
    prob = prob_of(kind, dim, m, N)
    sysm = O.from_problem(prob)
    z = np.random.default_rng(13).standard_normal(prob.n)
    q1, dot1 = E.sym_nostencil(prob, z, dtype, force_fft=True)
    v = E.vupd_stencil(prob, q1, z, dtype)
    ref = O.sym_apply(sysm, z.reshape(N, -1)).ravel()
    assert rel(v, ref) < TOL[dtype] * 50
    # the time-line part alone: blocks p_k I only
    psys = O.System(sysm.ms, sysm.hs, sysm.p, np.zeros_like(sysm.q), sysm.alpha)
    refp = O.sym_apply(psys, z.reshape(N, -1)).ravel()
    assert rel(q1, refp) < TOL[dtype] * 50
    zz = z.astype(dtype).astype(np.float64)
    assert abs(dot1 - np.dot(refp, zz)) <= TOL[dtype] * 50 * np.linalg.norm(refp) * np.linalg.norm(zz)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kind,dim,m,N", SPLIT_CASES)
def test_time_pass_spatial_dot(kind, dim, m, N, dtype):
    """The time pass output t is z in sine coordinates (z = U t); its side
    output must equal <Y L_h (q * z), z>."""
    prob = prob_of(kind, dim, m, N)
    sysm = O.from_problem(prob)
    x = np.random.default_rng(17).standard_normal(prob.n)
    t, s = E.time_aux(prob, x, dtype)
    z = O.space_transform(t.reshape(N, -1), prob.m)
    qsys = O.System(sysm.ms, sysm.hs, np.zeros_like(sysm.p), sysm.q, sysm.alpha)
    ref = float(np.vdot(O.sym_apply(qsys, z).ravel(), z.ravel()))
    scale = np.linalg.norm(O.sym_apply(qsys, z)) * np.linalg.norm(z)
    assert abs(s - ref) <= TOL[dtype] * 100 * scale


@pytest.mark.parametrize("kind,dim,m,N", SPLIT_CASES[:-1] + [("frac", 2, 15, 16)])
def test_split_residual(kind, dim, m, N):
    """r = Y (f - A u): time-line FFT pass without the stencil, then the x-line
    stencil pass with ||r||^2 (dense-p path of the FP64 residual)."""
    prob = prob_of(kind, dim, m, N)
    sysm = O.from_problem(prob)
    rng = np.random.default_rng(23)
    u = rng.standard_normal(prob.n)
    f = rng.standard_normal(prob.n)
    r, s = E.resid(prob, u, f)
    ref = O.time_reverse(f.reshape(N, -1) - O.bltt_apply(sysm, u)).ravel()
    assert rel(r, ref) < 1e-12
    assert abs(s - np.dot(ref, ref)) < 1e-10 * np.dot(ref, ref)


def test_scalar_kernel_flags_breakdown_and_nan():
    """The scalar kernel's checks that bltt_pminres turns into BLTT_EBREAKDOWN
    (status -4: <b, P^{-1} b> <= 0 at the start, <vhat, P^{-1} vhat> < 0 later,
    i.e. P not SPD in floating point) and BLTT_ENAN (status -3), forced from
    the host with the partial sums the reduction would have produced."""
    SC_START, SC_DELTA, SC_BETA = E.State.SC_START, E.State.SC_DELTA, E.State.SC_BETA
    st = E.State()
    st.scalar(SC_START, -1.0)
    assert st.status == -4
    st = E.State()
    st.scalar(SC_START, 0.0)
    assert st.status == -4
    st = E.State()
    st.scalar(SC_START, 4.0)
    assert st.status == 0 and st.eta0 == 2.0
    st.scalar(SC_DELTA, 0.5)
    assert st.status == 0
    st.scalar(SC_BETA, -1e-3)
    assert st.status == -4
    st = E.State()
    st.scalar(SC_START, float("nan"))
    assert st.status == -3
    st = E.State()
    st.scalar(SC_START, 1.0)
    st.scalar(SC_DELTA, float("nan"))
    assert st.status == -3
    # a zero beta is the happy breakdown: exact convergence, status 1
    st = E.State()
    st.scalar(SC_START, 1.0)
    st.scalar(SC_DELTA, 1.0)
    st.scalar(SC_BETA, 0.0)
    assert st.status == 1
