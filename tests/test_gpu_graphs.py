"""Graph replay of the sine-basis MINRES loop on the GPU.

By default each iteration position of the loop is captured once as a HIP graph
and replayed, and the host learns the scalar state from a host-mapped copy the
scalar kernel publishes instead of synchronising the stream.  The same handle
options with eager launches must give bit-identical iterates, iteration counts
and residual histories: the graphs hold the same kernels with the same
arguments.  Checked over repeated solves on one handle (every replay after the
first capture), a solve that needs a longer history buffer (the graphs are
rebuilt), warm starts, and both precisions."""
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


def _solves(prob, prec, rhs, maxits, eager, tol=1e-10):
    s = bltt.Solver.from_problem(prob, precision=prec, eager=eager)
    out = []
    try:
        for f, maxit in zip(rhs, maxits):
            u, it, hist, info, rc = s.pminres(torch.from_numpy(f).cuda(), tol, maxit)
            out.append((u.cpu().numpy(), it, np.asarray(hist), info["iters_outer"], rc))
    finally:
        s.close()
    return out


@pytest.mark.parametrize("prec,tol", [(bltt.FP64, 1e-10), (bltt.MIXED, 1e-8)])
@pytest.mark.parametrize("case", [("frac", 1, 31, 32), ("frac", 2, 31, 256), ("heat", 2, 15, 64)])
def test_graph_replay_matches_eager(case, prec, tol):
    kind, dim, m, N = case
    prob = W.fractional_l1(dim, m, N, 0.5, 0.01) if kind == "frac" else W.heat_bdf(dim, m, N, 0.01)
    rhs = [W.rhs_normal(prob, 11 + k) for k in range(4)]
    # the third solve asks for a longer history than the first two: new graphs
    maxits = [60, 60, 400, 60]
    print(f"[graphs] {case} prec={prec}", flush=True)
    a = _solves(prob, prec, rhs, maxits, eager=True, tol=tol)
    b = _solves(prob, prec, rhs, maxits, eager=False, tol=tol)
    sysm = O.from_problem(prob)
    for k, ((ua, ia, ha, oa, ra), (ub, ib, hb, ob, rb)) in enumerate(zip(a, b)):
        assert ra == rb == bltt.OK, (k, ra, rb)
        assert ia == ib and oa == ob, (k, ia, ib, oa, ob)
        assert np.array_equal(ha, hb), k
        assert np.array_equal(ua, ub), (k, float(np.abs(ua - ub).max()))
    # and the answer is the oracle's
    ustar = O.exact_solve(sysm, rhs[0]).ravel()
    err = float(np.linalg.norm(b[0][0] - ustar) / np.linalg.norm(ustar))
    print(f"  iters {[r[1] for r in b]} err vs oracle {err:.2e}", flush=True)
    assert err <= 1e-7


def test_graph_replay_with_initial_guess():
    prob = W.fractional_l1(2, 15, 128, 0.4, 0.01)
    f = W.rhs_normal(prob, 3)
    ft = torch.from_numpy(f).cuda()
    res = []
    for eager in (True, False):
        s = bltt.Solver.from_problem(prob, precision=bltt.FP64, initial_guess=True, eager=eager)
        try:
            u = torch.zeros_like(ft)
            its = []
            for tol in (1e-4, 1e-8, 1e-11):
                u, it, hist, info, rc = s.pminres(ft, tol, 200, u=u)
                assert rc == bltt.OK
                its.append(it)
            res.append((u.cpu().numpy(), its))
        finally:
            s.close()
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])

