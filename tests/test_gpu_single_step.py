"""N = 1 on the GPU (Section 3 with a single block): P_alpha = |A_(0)| = A_(0),
so MINRES ends after one iteration at u = A_(0)^{-1} f.  Checked against the
oracle's exact solve (dense per-mode division, itself pinned to a dense LU on
the CPU), in both precisions and every dimension, with an initial guess, and
the step entry points that need N >= 2 refusing the handle."""
import ctypes

import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


CASES = [("frac", 1, 31), ("heat", 2, 63), ("cn", 2, 255), ("frac", 3, 15), ("frac", 2, 511)]


def _problem(kind, dim, m):
    if kind == "frac":
        return W.fractional_l1(dim, m, 1, 0.5, 0.01)
    if kind == "heat":
        return W.heat_bdf(dim, m, 1, 0.01)
    return W.heat_cn(dim, m, 1, 0.01)


@pytest.mark.parametrize("prec", [bltt.FP64, bltt.MIXED])
@pytest.mark.parametrize("case", CASES)
def test_single_block_solve(case, prec):
    prob = _problem(*case)
    print(f"[N=1] {case} prec={prec}", flush=True)
    f = W.rhs_normal(prob, 21)
    ustar = O.exact_solve(O.from_problem(prob), f).ravel()
    s = bltt.Solver.from_problem(prob, precision=prec)
    try:
        u, it, hist, info, rc = s.pminres(torch.from_numpy(f).cuda(), 1e-10, 10)
    finally:
        s.close()
    err = float(np.linalg.norm(u.cpu().numpy() - ustar) / np.linalg.norm(ustar))
    print(f"  iters {it} relres {info['true_relres']:.2e} err {err:.2e}", flush=True)
    assert rc == bltt.OK and it == 1 and info["iters_outer"] == 1
    assert info["true_relres"] <= 1e-13 and err <= 1e-12
    assert hist[0] == 1.0 and hist[1] == pytest.approx(info["true_relres"])


def test_single_block_initial_guess_and_limits():
    prob = _problem("heat", 2, 31)
    f = W.rhs_normal(prob, 4)
    ft = torch.from_numpy(f).cuda()
    ustar = O.exact_solve(O.from_problem(prob), f).ravel()
    s = bltt.Solver.from_problem(prob, initial_guess=True)
    try:
        # a guess at the solution: zero iterations, u returned as given
        u0 = torch.from_numpy(ustar.copy()).cuda()
        u, it, _, info, rc = s.pminres(ft, 1e-10, 10, u=u0)
        assert rc == bltt.OK and it == 0 and info["true_relres"] <= 1e-10
        # a poor guess: one iteration to the solution
        u1 = torch.from_numpy(ustar + np.random.default_rng(2).standard_normal(ustar.size)).cuda()
        u, it, _, info, rc = s.pminres(ft, 1e-10, 10, u=u1)
        err = float(np.linalg.norm(u.cpu().numpy() - ustar) / np.linalg.norm(ustar))
        assert rc == bltt.OK and it == 1 and err <= 1e-12
        # the step entry points that apply a time operator need N >= 2
        L = bltt.load()
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        y = torch.zeros_like(x)
        P = ctypes.c_void_p
        for name in ("bltt_apply_sym", "bltt_apply_precond"):
            assert getattr(L, name)(s._h, bltt.FP64, P(x.data_ptr()), P(y.data_ptr())) == -7
        with pytest.raises(bltt.BlttError):
            s.modes_sym(x)
    finally:
        s.close()
