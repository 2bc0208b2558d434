"""Small alpha (Section 3: P_alpha approaches |T| as alpha -> 0, so the paper
runs alpha down to 1e-8).  The FP64 path applies alpha as given; everything
that applies the preconditioner in FP32 uses alpha' = max(alpha, 1e-4)
(an FP32 time pass amplifies its rounding by about 1/alpha).  Checked: mixed
solves at alpha = 1e-6 and 1e-8 converge to the oracle's solution in the
iterations alpha' = 1e-4 takes; the FP32 step entry point applies P_alpha'
(against the oracle's P at 1e-4) while the FP64 one applies P_alpha."""
import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W
from tests.mode_checks import pair_err, tol_time

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("alpha", [1e-6, 1e-8])
@pytest.mark.parametrize("dim,m,N", [(2, 63, 256), (1, 255, 1024)])
def test_mixed_small_alpha(dim, m, N, alpha):
    prob = W.fractional_l1(dim, m, N, 0.5, alpha)
    ref = W.fractional_l1(dim, m, N, 0.5, 1e-4)
    print(f"[small alpha] dim={dim} m={m} N={N} alpha={alpha}", flush=True)
    f = W.rhs_normal(prob, 3)
    ustar = O.exact_solve(O.from_problem(prob), f).ravel()
    ft = torch.from_numpy(f).cuda()
    out = {}
    for name, pr in (("given", prob), ("1e-4", ref)):
        s = bltt.Solver.from_problem(pr, precision=bltt.MIXED, fft_plan=bltt.PLAN_BASE)
        try:
            out[name] = s.pminres(ft, 1e-8, 200)
        finally:
            s.close()
    u, iters, _, info, rc = out["given"]
    err = float(np.linalg.norm(u.cpu().numpy() - ustar) / np.linalg.norm(ustar))
    print(f"  iters={iters} outer={info['iters_outer']} relres={info['true_relres']:.2e} err={err:.2e}", flush=True)
    assert rc == bltt.OK and info["true_relres"] <= 1e-8
    assert err <= 1e-8
    # the same FP32 sweeps as alpha = 1e-4 (the blocks do not depend on alpha)
    assert iters == out["1e-4"][1]
    assert torch.equal(u, out["1e-4"][0])


def test_step_precond_alpha_floor():
    dim, m, N, alpha = 2, 15, 256, 1e-6
    prob = W.fractional_l1(dim, m, N, 0.5, alpha)
    sysm = O.from_problem(prob)
    sys4 = O.from_problem(W.fractional_l1(dim, m, N, 0.5, 1e-4))
    M = prob.M
    modes = np.arange(M)
    v = np.random.default_rng(5).standard_normal((M, N))
    s = bltt.Solver.from_problem(prob, precision=bltt.MIXED)
    try:
        z64 = s.modes_lanczos(torch.from_numpy(v.ravel()).cuda(), coef=(1.0, 0.0, 0.0))[0].cpu().numpy()
        v32 = v.astype(np.float32)
        z32 = s.modes_lanczos(torch.from_numpy(v32.ravel()).cuda(), coef=(1.0, 0.0, 0.0))[0].cpu().numpy()
    finally:
        s.close()
    v32 = v32.astype(np.float64)
    e64 = pair_err(z64, O.mode_precond_apply(sysm, v, modes), v, sysm, modes, M)
    e32 = pair_err(z32, O.mode_precond_apply(sys4, v32, modes), v32, sys4, modes, M)
    print(f"[alpha floor] FP64 step at alpha={alpha}: {e64:.2e}; FP32 step against P at 1e-4: {e32:.2e}", flush=True)
    assert e64 < tol_time(torch.float64, N, alpha)
    assert e32 < tol_time(torch.float32, N, 1e-4)
