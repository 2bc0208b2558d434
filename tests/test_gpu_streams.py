"""Handles bound to caller streams other than the default one: every device
operation of a handle is ordered on its stream (the ABI's stream argument),
so solves on side streams, with inputs produced on those streams, return the
same answers bit for bit as on the default stream, in both precisions, with
graph replay and with direct launches, and two handles on two streams used
alternately do not disturb each other.  The radix plan and workgroup counts
are fixed (BLTT_PLAN_BASE): timed choices could differ between handles, and
the workgroup count sets the order of the partial sums."""
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


TOL = {bltt.FP64: 1e-10, bltt.MIXED: 1e-8}


@pytest.mark.parametrize("eager", [False, True])
def test_side_streams_match_default(eager):
    prob = W.fractional_l1(2, 31, 64, 0.4, 0.01)
    f = torch.from_numpy(W.rhs_normal(prob, 8)).cuda()
    ref = {}
    for prec in (bltt.FP64, bltt.MIXED):
        s = bltt.Solver.from_problem(prob, precision=prec, eager=eager, fft_plan=bltt.PLAN_BASE)
        try:
            ref[prec] = s.pminres(f, TOL[prec], 200)[0].clone()
        finally:
            s.close()
    torch.cuda.synchronize()
    streams = {bltt.FP64: torch.cuda.Stream(), bltt.MIXED: torch.cuda.Stream()}
    solvers = {}
    try:
        for prec, st in streams.items():
            with torch.cuda.stream(st):
                solvers[prec] = bltt.Solver.from_problem(prob, precision=prec, eager=eager, stream=st,
                                                         fft_plan=bltt.PLAN_BASE)
        # alternate the two handles, each on its own stream, inputs made on that stream
        for rep in range(2):
            for prec, st in streams.items():
                with torch.cuda.stream(st):
                    fs = f.clone()
                    u = solvers[prec].pminres(fs, TOL[prec], 200)[0]
                    st.synchronize()
                    print(f"[streams] eager={eager} rep={rep} prec={prec}", flush=True)
                    assert torch.equal(u, ref[prec])
    finally:
        for s in solvers.values():
            s.close()
    torch.cuda.synchronize()
