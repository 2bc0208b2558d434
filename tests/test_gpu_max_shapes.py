"""The largest shapes of the ABI's limits on the GPU: the longest sine
transform (2(m + 1) = 2048, 2D m = 1023), the longest time line (N = 2048,
whose FP64 residual runs 4096-point transforms) and the largest vector of the
suite (3D m = 255, N = 64: 1.06e9 unknowns, about 120 GB of device memory on
the mixed path).  Sampled sine-mode projections of u against the oracle's
per-mode exact solution, each mode's error relative to that mode's own norm
(mixed solves to 1e-8 held to 1e-8, FP64 solves to 1e-10 held to 1e-10)."""
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


# dim, m, N, gamma, precision
CASES = [(2, 1023, 64, 0.5, bltt.MIXED), (2, 1023, 64, 0.5, bltt.FP64), (2, 255, 2048, 0.4, bltt.MIXED),
         (3, 255, 64, 0.6, bltt.MIXED)]


@pytest.mark.parametrize("dim,m,N,gamma,precision", CASES)
def test_max_shapes_sampled(dim, m, N, gamma, precision):
    prob = W.fractional_l1(dim, m, N, gamma, 0.01)
    tol = 1e-8 if precision == bltt.MIXED else 1e-10
    print(f"[max shape] dim={dim} m={m} N={N} n={prob.n} precision={precision}", flush=True)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, 40 + dim)
    s = bltt.Solver.from_problem(prob, precision=precision)
    try:
        ft = torch.from_numpy(f).cuda()
        u, iters, _, info, rc = s.pminres(ft, tol, 200)
        del ft
        u = u.cpu().numpy()
    finally:
        s.close()
    torch.cuda.empty_cache()
    assert rc == bltt.OK, info
    assert info["true_relres"] <= tol
    rng = np.random.default_rng(1)
    modes = [0, 1, m - 1, prob.M - 1] + list(rng.integers(0, prob.M, 4))
    errs, floor = mode_errors(sysm, u, f, modes)
    print(f"  iters={iters} outer={info['iters_outer']} relres={info['true_relres']:.3e} solve_ms={info['solve_ms']:.1f} "
          f"per-mode err {np.array2string(errs, precision=2)}", flush=True)
    assert worst(errs, floor, tol) <= 1.0
