"""The setup autotuner and its kernel plans on the GPU.

The FP32 time pass and N-point matvec of the mixed path come in two radix
plans at N = 512 and 1024 (16*8*4 / 16*4*8, 16*8*8 / 16*16*4) and the time
pass runs on 2, 4 or 8 persistent workgroups per compute unit.  Checked here:
each forced plan against the oracle (step kernels, element by element, and
whole mixed solves); the autotuner's choice, written to and read back from a
plan cache; and batched solves under each plan against the single-system
solver and the oracle."""
import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W
from tests.mode_checks import TOL_MV, line_err, pair_err, tol_time

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("N", [512, 1024])
@pytest.mark.parametrize("plan", [bltt.PLAN_BASE, bltt.PLAN_ALT])
def test_forced_plan_step_kernels(N, plan):
    prob = W.fractional_l1(2, 15, N, 0.4, 0.01)          # M = 225: ragged last mode pair
    sysm = O.from_problem(prob)
    M = prob.M
    modes = np.arange(M)
    print(f"[plan step] N={N} plan={plan}", flush=True)
    s = bltt.Solver.from_problem(prob, precision=bltt.MIXED, fft_plan=plan)
    try:
        info = s.plan_info()
        want = 1 if plan == bltt.PLAN_ALT else 0
        assert info["time_plan"] == want and info["cs_plan"] == want and info["source"] == "forced"
        rng = np.random.default_rng(N + plan)
        f32 = lambda a: a.astype(np.float32).astype(np.float64)
        z = f32(rng.standard_normal((M, N)))
        q, _ = s.modes_sym(torch.from_numpy(z.ravel()).float().cuda())
        assert line_err(q.cpu().numpy(), O.mode_sym_apply(sysm, z, modes)) < TOL_MV["float32"]
        qv, v1, v2 = (f32(rng.standard_normal((M, N))) for _ in range(3))
        coef = (0.7, -1.3, 0.4)
        t = lambda a: torch.from_numpy(a.ravel()).float().cuda()
        zz, _, _ = s.modes_lanczos(t(qv), t(v1), t(v2), coef)
        vhat = coef[0] * qv + coef[1] * v1 + coef[2] * v2
        err = pair_err(zz.cpu().numpy(), O.mode_precond_apply(sysm, vhat, modes), vhat, sysm, modes, M)
        print(f"  time pass pair err {err:.2e}", flush=True)
        assert err < tol_time("float32", N, prob.alpha)
    finally:
        s.close()


def test_mixed_solves_agree_under_both_plans():
    prob = W.fractional_l1(2, 31, 1024, 0.3, 0.01)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, 8)
    ustar = O.exact_solve(sysm, f).ravel()
    ft = torch.from_numpy(f).cuda()
    us = []
    for plan in (bltt.PLAN_BASE, bltt.PLAN_ALT):
        s = bltt.Solver.from_problem(prob, precision=bltt.MIXED, fft_plan=plan)
        try:
            u, it, _, info, rc = s.pminres(ft, 1e-8, 200)
        finally:
            s.close()
        err = relnorm(u.cpu().numpy(), ustar)
        print(f"[plan solve] plan={plan}: iters {it} outer {info['iters_outer']} err {err:.2e}", flush=True)
        assert rc == bltt.OK and info["true_relres"] <= 1e-8 and err <= 1e-8
        us.append(u.cpu().numpy())
    assert relnorm(us[1], us[0]) <= 2e-8


def test_autotuner_writes_and_reads_plan_cache(tmp_path):
    cache = str(tmp_path / "plans.txt")
    prob = W.fractional_l1(2, 63, 1024, 0.3, 0.01)
    s = bltt.Solver.from_problem(prob, precision=bltt.MIXED, plan_cache=cache)
    try:
        first = s.plan_info()
    finally:
        s.close()
    print(f"[autotune] chose {first}", flush=True)
    assert first["source"] == "timed"
    assert first["time_plan"] in (0, 1) and first["cs_plan"] in (0, 1)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert first["time_blocks"] in (2 * cus, 4 * cus, 8 * cus)
    assert first["cs_blocks"] in (0, 2 * cus, 4 * cus, 8 * cus)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and "N=1024" in lines[0] and "M=3969" in lines[0]
    s = bltt.Solver.from_problem(prob, precision=bltt.MIXED, plan_cache=cache)
    try:
        second = s.plan_info()
        f = torch.from_numpy(W.rhs_normal(prob, 2)).cuda()
        _, _, _, info, rc = s.pminres(f, 1e-8, 200)
    finally:
        s.close()
    assert second["source"] == "cache"
    assert {k: second[k] for k in ("time_plan", "cs_plan", "time_blocks", "cs_blocks")} == \
        {k: first[k] for k in ("time_plan", "cs_plan", "time_blocks", "cs_blocks")}
    assert rc == bltt.OK and info["true_relres"] <= 1e-8
    assert len(open(cache).read().splitlines()) == 1
    # an FP64 handle runs no FP32 kernels: nothing to tune
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64)
    try:
        assert s.plan_info()["source"] == "default"
    finally:
        s.close()


@pytest.mark.parametrize("plan", [bltt.PLAN_AUTO, bltt.PLAN_BASE, bltt.PLAN_ALT])
def test_batched_under_each_plan(plan, tmp_path):
    probs = [W.fractional_l1(2, 15, 1024, 0.3, 0.01), W.fractional_l1(2, 7, 512, 0.6, 0.05),
             W.fractional_l1(2, 15, 1024, 0.5, 0.003), W.fractional_l1(1, 31, 64, 0.4, 0.01)]
    fs, refs = [], []
    for i, pr in enumerate(probs):
        f = W.rhs_normal(pr, 500 + i)
        fs.append(torch.from_numpy(f).cuda())
        refs.append(O.exact_solve(O.from_problem(pr), f).ravel())
    cache = str(tmp_path / "batch_plans.txt")
    b = bltt.Batch(probs, 1, plan_cache=cache, fft_plan=plan)
    try:
        plans, tpbs = b.plans(), b.classes()
        us, iters, _, infos, rc = b.pminres(fs, 1e-8, 200)
    finally:
        b.close()
    print(f"[batched plans] fft_plan={plan}: classes tpb {tpbs} plans {plans}", flush=True)
    assert rc == bltt.OK
    if plan == bltt.PLAN_ALT:
        assert plans.count(1) == 2          # the N = 512 and N = 1024 classes
    if plan == bltt.PLAN_BASE:
        assert plans == [0] * len(plans)
    for g, pr in enumerate(probs):
        u = us[g].cpu().numpy()
        assert relnorm(u, refs[g]) <= 1e-8, (g, relnorm(u, refs[g]))
        s = bltt.Solver.from_problem(pr, precision=bltt.MIXED, fft_plan=plan)
        try:
            u1, _, _, _, rc1 = s.pminres(fs[g], 1e-8, 200)
        finally:
            s.close()
        assert rc1 == bltt.OK and relnorm(u, u1.cpu().numpy()) <= 2e-8
    if plan == bltt.PLAN_AUTO:
        # the classes' choices are in the cache; a second setup reads them
        assert len(open(cache).read().splitlines()) == len(plans)
        b = bltt.Batch(probs, 1, plan_cache=cache)
        try:
            assert b.plans() == plans and b.classes() == tpbs
        finally:
            b.close()
        assert len(open(cache).read().splitlines()) == len(plans)
