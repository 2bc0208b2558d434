"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Step-level operators (sine transform, preconditioner, symmetrised matvec) are
compared element by element at sizes spanning several workgroups with ragged
tails; full solves are compared with the oracle's exact solution u* = A^{-1} f
and with its MINRES history.  The full-size workloads are checked on sampled
outputs: projections of u onto selected sine modes, which the oracle solves
one by one.
"""
import math

import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W
from tests.mode_checks import mode_errors, worst

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def prob_of(kind, dim, m, N, alpha=0.05, gamma=0.4):
    return {"frac": lambda: W.fractional_l1(dim, m, N, gamma, alpha),
            "heat": lambda: W.heat_bdf(dim, m, N, alpha),
            "cn": lambda: W.heat_cn(dim, m, N, alpha)}[kind]()


def cuda(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


STEP_CASES = [("frac", 1, 31, 32, 0.01), ("heat", 2, 7, 16, 0.01), ("frac", 2, 15, 64, 0.05),
              ("cn", 2, 7, 32, 0.2), ("frac", 3, 7, 8, 0.05), ("frac", 1, 63, 1024, 0.01),
              ("heat", 1, 3, 2048, 0.01), ("frac", 2, 31, 128, 0.001), ("frac", 1, 1, 2, 0.5),
              ("frac", 1, 3, 2048, 0.01)]


@pytest.mark.parametrize("kind,dim,m,N,alpha", STEP_CASES)
def test_step_operators(kind, dim, m, N, alpha):
    prob = prob_of(kind, dim, m, N, alpha)
    print(f"[step] {kind} dim={dim} m={m} N={N} alpha={alpha}", flush=True)
    sysm = O.from_problem(prob)
    P = O.precond_setup(sysm)
    x = np.random.default_rng(m + N).standard_normal(prob.n)
    ref_space = O.space_transform(x.reshape(N, -1), prob.m).ravel()
    ref_pre = O.precond_apply(P, x.reshape(N, -1)).ravel()
    ref_sym = O.sym_apply(sysm, x.reshape(N, -1)).ravel()
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64)
    try:
        for dt, tol_s, tol_p in ((torch.float64, 1e-12, 1e-9), (torch.float32, 2e-5, 2e-4 / math.sqrt(alpha))):
            xt = cuda(x, dt)
            got = s.apply_space(xt).cpu().double().numpy()
            assert rel(got, ref_space) < tol_s * 10, ("space", dt)
            got = s.apply_precond(xt).cpu().double().numpy()
            assert rel(got, ref_pre) < tol_p, ("precond", dt, rel(got, ref_pre))
            got = s.apply_sym(xt).cpu().double().numpy()
            assert rel(got, ref_sym) < tol_s * 50, ("sym", dt, rel(got, ref_sym))
    finally:
        s.close()


SOLVE_CASES = [("frac", 1, 31, 32, 0.01, 1e-10), ("heat", 2, 15, 32, 0.01, 1e-10),
               ("frac", 2, 31, 64, 0.01, 1e-10), ("cn", 2, 15, 16, 0.05, 1e-10), ("frac", 3, 7, 16, 0.01, 1e-10)]


BASES = [bltt.SINE, bltt.PHYSICAL]


# accuracy targets of the two paths: relative 2-norm error against u* = A^{-1} f
ERR_FP64, ERR_MIXED = 1e-10, 1e-8


@pytest.mark.parametrize("basis", BASES)
@pytest.mark.parametrize("kind,dim,m,N,alpha,tol", SOLVE_CASES)
def test_fp64_solve_matches_oracle(kind, dim, m, N, alpha, tol, basis):
    prob = prob_of(kind, dim, m, N, alpha, gamma=0.5)
    print(f"[fp64 solve] {kind} dim={dim} m={m} N={N} basis={basis}", flush=True)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, 11)
    ustar = O.exact_solve(sysm, f).ravel()
    ores = O.pminres(sysm, f, tol, 100)
    # the explicit residual after every iteration (check_factor beyond any
    # |eta| ratio), which is the oracle's stopping test: same iteration count
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64, basis=basis, check_factor=1e30)
    try:
        ft = cuda(f, torch.float64)
        u, iters, hist, info, rc = s.pminres(ft, tol, 100)
        # the reported residual against the physical-space operator applied to the returned u
        phys = relnorm(s.apply_sym(u).cpu().numpy(), O.time_reverse(f.reshape(N, -1)).ravel())
    finally:
        s.close()
    u = u.cpu().numpy()
    assert rc == bltt.OK
    assert info["true_relres"] <= tol
    # the sine basis reports the residual of the transformed system: the two
    # differ by the FP64 rounding of the sine transforms, amplified by at most
    # cond(A) (~1e3 here)
    assert abs(phys - info["true_relres"]) < 1e-11
    # same Krylov iteration: identical residual-estimate history
    k = min(len(hist), len(ores.eta_hist))
    assert np.allclose(hist[:k], ores.eta_hist[:k], rtol=1e-6, atol=1e-13)
    assert iters == ores.iters, (iters, ores.iters)
    err = relnorm(u, ustar)
    print(f"  iters={iters} relres={info['true_relres']:.2e} err={err:.2e}", flush=True)
    assert err <= ERR_FP64


# N = 2048: the FP32 N-point matvec reads its tables from global memory (too
# large to stage in LDS), the other cases stage them
MIXED_CASES = [("frac", 2, 31, 64, 0.01), ("heat", 2, 31, 32, 0.01), ("frac", 1, 63, 256, 0.01),
               ("frac", 3, 7, 32, 0.01), ("frac", 1, 15, 2048, 0.01)]


@pytest.mark.parametrize("basis", BASES)
@pytest.mark.parametrize("kind,dim,m,N,alpha", MIXED_CASES)
def test_mixed_solve_matches_exact(kind, dim, m, N, alpha, basis):
    prob = prob_of(kind, dim, m, N, alpha, gamma=0.3)
    print(f"[mixed solve] {kind} dim={dim} m={m} N={N} basis={basis}", flush=True)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, 5)
    ustar = O.exact_solve(sysm, f).ravel()
    s = bltt.Solver.from_problem(prob, precision=bltt.MIXED, basis=basis)
    try:
        u, iters, hist, info, rc = s.pminres(cuda(f, torch.float64), 1e-8, 200)
    finally:
        s.close()
    u = u.cpu().numpy()
    assert rc == bltt.OK, info
    assert info["true_relres"] <= 1e-8
    assert info["iters_outer"] >= 1
    err = relnorm(u, ustar)
    print(f"  iters={iters} outer={info['iters_outer']} relres={info['true_relres']:.2e} err={err:.2e}", flush=True)
    assert err <= ERR_MIXED


@pytest.mark.parametrize("basis", BASES)
def test_zero_rhs_and_noconv(basis):
    prob = prob_of("frac", 2, 7, 16, 0.01)
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64, basis=basis)
    try:
        u, iters, hist, info, rc = s.pminres(torch.zeros(prob.n, dtype=torch.float64, device="cuda"), 1e-10, 10)
        assert rc == bltt.OK and iters == 0 and float(u.abs().max()) == 0.0
        f = W.rhs_normal(prob, 1)
        u, iters, hist, info, rc = s.pminres(cuda(f, torch.float64), 1e-14, 1)
        assert rc == bltt.NOCONV and iters == 1
        assert np.all(np.isfinite(u.cpu().numpy()))
        f[3] = np.nan
        with pytest.raises(bltt.BlttError) as ei:
            s.pminres(cuda(f, torch.float64), 1e-10, 10)
        assert ei.value.code == -3
    finally:
        s.close()


@pytest.mark.parametrize("name", ["frac1d_m31_n32", "heat2d_m255_n256"])
def test_named_workloads_fp64(name):
    prob, seed = W.workload(name)
    print(f"[workload] {name}", flush=True)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, seed)
    ustar = O.exact_solve(sysm, f).ravel()
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64)
    try:
        u, iters, hist, info, rc = s.pminres(cuda(f, torch.float64), 1e-10, 100)
    finally:
        s.close()
    u = u.cpu().numpy()
    err = relnorm(u, ustar)
    print(f"  iters={iters} relres={info['true_relres']:.3e} err={err:.3e}", flush=True)
    assert rc == bltt.OK
    assert err <= ERR_FP64


FULL_CASES = [("frac2d_m511_n1024_g03", bltt.MIXED, bltt.SINE), ("frac2d_m511_n1024_g03", bltt.FP64, bltt.SINE),
              ("frac2d_m511_n1024_g07", bltt.MIXED, bltt.SINE), ("frac3d_m127_n256", bltt.MIXED, bltt.SINE),
              ("frac2d_m511_n1024_g03", bltt.MIXED, bltt.PHYSICAL), ("frac3d_m127_n256", bltt.MIXED, bltt.PHYSICAL)]


@pytest.mark.parametrize("name,precision,basis", FULL_CASES)
def test_full_size_sampled(name, precision, basis):
    """Full-size workloads (2D: M = 511^2, N = 1024, gamma 0.3 / 0.7; 3D:
    M = 127^3, N = 256, gamma 0.5): sampled sine-mode projections of u
    against the oracle's per-mode exact solution, each mode's error relative
    to that mode's own exact norm.  Mixed solves run to 1e-8 and are held to
    1e-8; FP64 solves run to 1e-10 and are held to 1e-10."""
    tol = 1e-8 if precision == bltt.MIXED else 1e-10
    bar = ERR_MIXED if precision == bltt.MIXED else ERR_FP64
    prob, seed = W.workload(name)
    print(f"[full size] {name} precision={precision} basis={basis}", flush=True)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, seed)
    s = bltt.Solver.from_problem(prob, precision=precision, basis=basis)
    try:
        ft = cuda(f, torch.float64)
        u, iters, hist, info, rc = s.pminres(ft, tol, 200)
        del ft
    finally:
        s.close()
    assert rc == bltt.OK, info
    assert info["true_relres"] <= tol
    u = u.cpu().numpy()
    rng = np.random.default_rng(0)
    modes = [0, 1, 511, prob.M - 1] + list(rng.integers(0, prob.M, 4))
    errs, floor = mode_errors(sysm, u, f, modes)
    print(f"  iters={iters} outer={info['iters_outer']} relres={info['true_relres']:.3e} "
          f"per-mode err max={errs.max():.3e} (modes {modes}: {np.array2string(errs, precision=2)}; "
          f"floors {np.array2string(floor, precision=1)}) solve_ms={info['solve_ms']:.1f}", flush=True)
    assert worst(errs, floor, bar) <= 1.0


@pytest.mark.parametrize("basis", BASES)
@pytest.mark.parametrize("precision", [bltt.FP64, bltt.MIXED])
def test_initial_guess(basis, precision):
    """bltt_pminres from a caller's initial guess (opt.initial_guess = 1): the
    exact solution needs no iteration; a perturbed one converges to the oracle's
    u*, in FP64 with the oracle's own iteration count from the same guess."""
    prob = prob_of("frac", 2, 15, 64, 0.01, gamma=0.3)
    print(f"[initial guess] precision={precision} basis={basis}", flush=True)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, 21)
    ustar = O.exact_solve(sysm, f).ravel()
    tol, bar = (1e-10, ERR_FP64) if precision == bltt.FP64 else (1e-8, ERR_MIXED)
    s = bltt.Solver.from_problem(prob, precision=precision, basis=basis, initial_guess=True, check_factor=1e30)
    s0 = bltt.Solver.from_problem(prob, precision=precision, basis=basis, check_factor=1e30)
    try:
        ft = cuda(f, torch.float64)
        u, iters, hist, info, rc = s.pminres(ft, tol, 100, cuda(ustar, torch.float64))
        assert rc == bltt.OK and iters == 0 and info["true_relres"] <= tol
        assert relnorm(u.cpu().numpy(), ustar) <= 1e-12
        guess = ustar + 1e-3 * np.linalg.norm(ustar) / math.sqrt(prob.n) * \
            np.random.default_rng(2).standard_normal(prob.n)
        u, iters, hist, info, rc = s.pminres(ft, tol, 100, cuda(guess, torch.float64))
        err = relnorm(u.cpu().numpy(), ustar)
        _, iters0, _, _, _ = s0.pminres(ft, tol, 100)
        print(f"  from the guess: iters={iters} err={err:.2e}; from zero: iters={iters0}", flush=True)
        assert rc == bltt.OK and info["true_relres"] <= tol and err <= bar
        assert iters <= iters0
        if precision == bltt.FP64:
            ores = O.pminres(sysm, f, tol, 100, x0=guess)
            assert iters == ores.iters
        # f = 0 returns u = 0 whatever the guess
        z = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        u, iters, _, _, rc = s.pminres(z, tol, 100, cuda(guess, torch.float64))
        assert rc == bltt.OK and iters == 0 and float(u.abs().max()) == 0.0
    finally:
        s.close()
        s0.close()


@pytest.mark.parametrize("basis", BASES)
def test_aliased_f_and_u_rejected(basis):
    prob = prob_of("frac", 2, 7, 16, 0.01)
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64, basis=basis)
    try:
        buf = torch.zeros(2 * prob.n, dtype=torch.float64, device="cuda")
        f = buf[: prob.n]
        for u in (f, buf[prob.n // 2: prob.n // 2 + prob.n]):
            with pytest.raises(bltt.BlttError) as ei:
                s.pminres(f, 1e-8, 10, u)
            assert ei.value.code == -1
        # disjoint halves are fine
        _, _, _, _, rc = s.pminres(f, 1e-8, 10, buf[prob.n:])
        assert rc == bltt.OK
    finally:
        s.close()
