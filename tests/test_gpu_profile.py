"""Per-class kernel profiling (bltt_profile_enable / bltt_profile_read) on a
mixed sine-basis solve: each launch lands in its class, the launch counts
follow the sweep structure, the algorithmic bytes follow the streams each
kernel moves, and a profiled solve (direct launches) returns the same answer,
bit for bit, as an unprofiled one (graph replay)."""
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


@pytest.mark.parametrize("dim,m,N", [(2, 63, 256), (3, 15, 128)])
def test_profile_classes_follow_the_sweeps(dim, m, N):
    prob = W.fractional_l1(dim, m, N, 0.5, 0.01)
    print(f"[profile] dim={dim} m={m} N={N} n={prob.n}", flush=True)
    f = torch.from_numpy(W.rhs_normal(prob, 5)).cuda()
    s = bltt.Solver.from_problem(prob, precision=bltt.MIXED)
    try:
        u0, it0, _, info0, rc0 = s.pminres(f, 1e-8, 100)
        s.profile(True)
        u1, it1, _, info1, rc1 = s.pminres(f, 1e-8, 100)
        p = s.profile_read()
        s.profile(False)
        # reading resets nothing; disabling and solving again adds nothing
        s.pminres(f, 1e-8, 100)
        p2 = s.profile_read()
    finally:
        s.close()
    torch.cuda.synchronize()
    assert rc0 == rc1 == bltt.OK and it0 == it1
    assert torch.equal(u0, u1)
    assert p2 == p
    sweeps, n = info1["iters_outer"], prob.n
    assert sweeps >= 2 and it1 >= sweeps
    launches = {k: v["launches"] for k, v in p.items()}
    print(f"  iters {it1} sweeps {sweeps} launches {launches}", flush=True)
    # one start pass and one FP64 residual per sweep; a matvec and a time pass per iteration
    assert launches["time_start"] == sweeps
    assert launches["resid64"] == sweeps
    assert launches["time_prec"] == it1
    assert launches["matvec"] == it1
    # transforms in and out: x (fused with the layout move) once each way, y and z in place
    assert launches["dst_x_vupd"] == 2
    assert launches["dst_strided"] == 2 * (dim - 1)
    assert launches["dst_x_dot"] == 0 and launches["wx_update"] == 0
    # algorithmic bytes per element: FP32 time pass 16 on a sweep's first
    # iteration (Q, V_1 in; V_2, Z_2 out) and 20 after (V_{j-1} in as well);
    # matvec 8; start pass 16 on the first sweep (FHAT in FP64; V_1, Z_1
    # out) and 8 after (the FP32 residual in; Z_1 out); FP64 residual
    # 28 + 4 k (U in and out, F in, R out in FP32, k stored Z in), less the
    # 8 of reading U on the first sweep, whose iterate starts at zero
    assert p["time_prec"]["bytes"] == pytest.approx((16 * sweeps + 20 * (it1 - sweeps)) * n)
    assert p["matvec"]["bytes"] == pytest.approx(8 * it1 * n)
    assert p["time_start"]["bytes"] == pytest.approx((16 + 8 * (sweeps - 1)) * n)
    assert p["resid64"]["bytes"] == pytest.approx((28 * sweeps + 4 * it1 - 8) * n)
    for k, v in p.items():
        assert v["ms"] >= 0.0
        if v["launches"]:
            assert v["ms"] > 0.0, k
