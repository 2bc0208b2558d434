"""The paper's printed iteration counts reproduced by the GPU solver (FP64,
sine basis): Example 3 (Tables 4-6: P_alpha with alpha = 1e-8 and the P_1
comparator, alpha = 1) and Example 1 (Table 1: P_alpha and the unpreconditioned
MINRES-I comparator), stop at relative residual 1e-6 with the residual checked
every iteration."""
import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from tests.paper_examples import example1_system_and_rhs, example3_system_and_rhs, example_problem, golden_counts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def gpu_solve(prob, f, tol, maxit, precond=bltt.PRECOND_ABAC):
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64, precond=precond, check_factor=1e12)
    try:
        u, iters, hist, info, rc = s.pminres(torch.from_numpy(np.ascontiguousarray(f.ravel())).cuda(), tol, maxit)
    finally:
        s.close()
    return u.cpu().numpy(), iters, info, rc


@pytest.mark.parametrize("row", golden_counts()["example3_fractional"]["rows"])
def test_table4to6_counts_on_gpu(row):
    g, N, mp1 = row["gamma"], row["N"], row["m_plus_1"]
    print(f"[example 3] gamma={g} N={N} m+1={mp1}", flush=True)
    sysm, f = example3_system_and_rhs(g, N, mp1, 1e-8)
    u, it, info, rc = gpu_solve(example_problem("example3", N, mp1, 1e-8, g), f, 1e-6, 100)
    assert rc == bltt.OK and it == row["P_alpha"]
    ustar = O.exact_solve(sysm, f).ravel()
    assert np.linalg.norm(u - ustar) <= 1e-4 * np.linalg.norm(ustar)
    _, it1, _, rc1 = gpu_solve(example_problem("example3", N, mp1, 1.0, g), f, 1e-6, 100)
    assert rc1 == bltt.OK and it1 == row["P_1"]


@pytest.mark.parametrize("row", golden_counts()["example1_heat_bdf"]["rows"])
def test_table1_counts_on_gpu(row):
    N, mp1 = row["N"], row["m_plus_1"]
    print(f"[example 1] N={N} m+1={mp1}", flush=True)
    sysm, f = example1_system_and_rhs(N, mp1, 1e-8)
    prob = example_problem("example1", N, mp1, 1e-8)
    _, it, _, rc = gpu_solve(prob, f, 1e-6, 100)
    assert rc == bltt.OK and it == row["P_alpha"]
    _, itI, _, rcI = gpu_solve(prob, f, 1e-6, 200, precond=bltt.PRECOND_NONE)
    assert rcI == bltt.OK and itI == row["I"]
