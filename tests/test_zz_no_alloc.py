"""bltt_modes_lanczos_noalloc (the entry point for callers that cannot
allocate) against bltt_modes_lanczos through the C ABI: same kernels, so the
outputs must agree exactly, on two calls in a row on one GPU (the second on a
smaller system, reusing the scratch the first one left), in every precision;
and its documented refusals (tables not built yet, too many partial sums)."""
import numpy as np
import pytest

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


def inputs(n, seed, dt_q, dt):
    rng = np.random.default_rng(seed)
    q = torch.from_numpy(rng.standard_normal(n)).to(dt_q).cuda()
    v1 = torch.from_numpy(rng.standard_normal(n)).to(dt).cuda()
    v2 = torch.from_numpy(rng.standard_normal(n)).to(dt).cuda()
    return q, v1, v2


def compare(s, n, seed, dt_q, dt, full):
    q, v1, v2 = inputs(n, seed, dt_q, dt)
    coef = (0.8, -1.1, 0.3) if full else (1.7, 0.0, 0.0)
    a1, a2 = (v1, v2) if full else (None, None)
    z_ref, v_ref, d_ref = s.modes_lanczos(q, a1, a2, coef, want_v=True, dtype=dt)
    z = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    v = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    z2, v2o, d2 = s.modes_lanczos(q, a1, a2, coef, z=z, want_v=True, v=v, dtype=dt, noalloc=True)
    assert z2.data_ptr() == z.data_ptr() and v2o.data_ptr() == v.data_ptr()
    assert torch.equal(z, z_ref) and torch.equal(v, v_ref)
    assert d2 == d_ref and np.isfinite(d2) and d2 > 0


@pytest.mark.parametrize("dt_q,dt", [(torch.float32, torch.float32), (torch.float64, torch.float32),
                                     (torch.float64, torch.float64)])
def test_noalloc_matches_allocating_entry_point(dt_q, dt):
    big = W.fractional_l1(2, 63, 1024, 0.3, 0.01)       # M = 3969, N = 1024
    small = W.fractional_l1(2, 15, 64, 0.6, 0.05)       # M = 225, N = 64 (ragged last mode pair)
    prec = bltt.FP64 if dt == torch.float64 else bltt.MIXED
    sb = bltt.Solver.from_problem(big, precision=prec)
    ss = bltt.Solver.from_problem(small, precision=prec)
    try:
        full = dt_q == dt
        print(f"[noalloc] q {dt_q} out {dt}: big system then small", flush=True)
        compare(sb, big.n, 1, dt_q, dt, full)
        compare(ss, small.n, 2, dt_q, dt, full)
        if full:
            # the start form (no v1, v2) on the small system, after the full form
            compare(ss, small.n, 3, dt_q, dt, False)
    finally:
        sb.close()
        ss.close()


def test_noalloc_refusals():
    prob = W.fractional_l1(2, 15, 64, 0.5, 0.01)
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64)
    try:
        q, v1, v2 = inputs(prob.n, 4, torch.float32, torch.float32)
        z = torch.empty(prob.n, dtype=torch.float32, device="cuda")
        # an FP64 handle has no FP32 tables yet: building them would allocate
        with pytest.raises(bltt.BlttError) as ei:
            s.modes_lanczos(q, coef=(1.0, 0.0, 0.0), z=z, noalloc=True)
        assert ei.value.code == -1
        # after the allocating entry point has built them, the no-alloc one runs
        z_ref, _, d_ref = s.modes_lanczos(q, coef=(1.0, 0.0, 0.0))
        _, _, d = s.modes_lanczos(q, coef=(1.0, 0.0, 0.0), z=z, noalloc=True)
        assert torch.equal(z, z_ref) and d == d_ref
    finally:
        s.close()
    # FP64 at M = 511^2, N = 1024: 32641 partial sums, beyond the 16384 the scratch holds
    prob, _ = W.workload("frac2d_m511_n1024_g03")
    s = bltt.Solver.from_problem(prob, precision=bltt.FP64)
    try:
        q = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        z = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        with pytest.raises(bltt.BlttError) as ei:
            s.modes_lanczos(q, coef=(1.0, 0.0, 0.0), z=z, noalloc=True)
        assert ei.value.code == -7
    finally:
        s.close()
