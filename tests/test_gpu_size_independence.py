"""Size independence on the GPU (Theorem 1, Lemma 11): preconditioned MINRES
on the 3D time-fractional workload (L1 scheme, gamma = 0.5, 7-point
Laplacian, M = 127^3, alpha = 0.01, f ~ N(0,1) seeded) at N = 64, 128 and 256
(up to 524 M unknowns).  The eigenvalues of P_alpha^{-1} Y A cluster in
[-1 - alpha mu, -1 + alpha mu] u [1 - alpha mu, 1 + alpha mu] whatever N, so the
FP64 iteration count must not grow with N; the mixed path's counts are
reported beside it.  Each solution is checked on sampled sine modes against
the oracle's per-mode exact solution, every mode against its own norm.

The FP64 leg solves to 1e-13 for its 1e-10 per-mode target: the stopping test
is the global relative residual, which weighs each mode's residual by its share
of ||f|| (about 1/sqrt(M) for a random f) and is dominated by the high modes,
while the low modes converge last; at tolerances 1e-10 and 1e-12 the solve
stops after 6 iterations with the global residual at 2.8e-13 and mode 0 of the
N = 128 grid measured at 1.01e-10.  The mixed leg runs at the workload's 1e-8."""
import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W
from tests.mode_checks import mode_errors, worst

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NS = (64, 128, 256)


@pytest.fixture(scope="module")
def runs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    out = {}
    for N in NS:
        prob = W.fractional_l1(3, 127, N, 0.5, 0.01)
        sysm = O.from_problem(prob)
        print(f"[size independence] 3D m=127 N={N}: n={prob.n}", flush=True)
        f = W.rhs_normal(prob, 5)
        ft = torch.from_numpy(f).cuda()
        rng = np.random.default_rng(N)
        modes = sorted(set([0, 1, 126, 127, prob.M // 2, prob.M - 1] + [int(i) for i in rng.integers(0, prob.M, 6)]))
        for prec, tol, target in ((bltt.FP64, 1e-13, 1e-10), (bltt.MIXED, 1e-8, 1e-8)):
            s = bltt.Solver.from_problem(prob, precision=prec)
            try:
                u, iters, hist, info, rc = s.pminres(ft, tol, 200)
            finally:
                s.close()
            errs, floor = mode_errors(sysm, u.cpu().numpy(), f, modes)
            del u
            name = "fp64" if prec == bltt.FP64 else "mixed"
            out[(name, N)] = {"iters": iters, "outer": info["iters_outer"], "relres": info["true_relres"],
                              "err": float(errs.max()), "ratio": worst(errs, floor, target), "rc": rc,
                              "solve_ms": info["solve_ms"]}
            print(f"  {name}: iters={iters} outer={info['iters_outer']} relres={info['true_relres']:.2e} "
                  f"per-mode err max={errs.max():.2e} (floor at that mode {floor[errs.argmax()]:.1e}) "
                  f"solve={info['solve_ms']:.1f} ms", flush=True)
        del ft
    torch.cuda.synchronize()
    return out


def test_fp64_iterations_flat_in_N(runs):
    its = [runs[("fp64", N)]["iters"] for N in NS]
    assert all(runs[("fp64", N)]["rc"] == bltt.OK for N in NS)
    assert max(its) - min(its) <= 1, its


def test_mixed_converges_with_flat_sweeps(runs):
    its = [runs[("mixed", N)]["iters"] for N in NS]
    outer = [runs[("mixed", N)]["outer"] for N in NS]
    print(f"  mixed FP32 iterations {its}, refinement sweeps {outer} for N = {NS}", flush=True)
    assert all(runs[("mixed", N)]["rc"] == bltt.OK for N in NS)
    assert max(outer) - min(outer) <= 1, outer


def test_solutions_match_oracle(runs):
    """Per-mode errors within the targets (FP64 1e-10, mixed 1e-8) plus the
    rounding floor of an FP64 physical-space solution (tests/mode_checks.py)."""
    for N in NS:
        assert runs[("fp64", N)]["ratio"] <= 1.0, (N, runs[("fp64", N)])
        assert runs[("mixed", N)]["ratio"] <= 1.0, (N, runs[("mixed", N)])
