"""GPU parity of the batched solver (many instances of uneven shape, several
right-hand sides each) against the CPU oracle and against the single-system
solver of the same instance."""
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


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_batch():
    # uneven shapes, blocks and alpha; two instances share each 2D shape; the
    # N = 2048 class's matvec reads its tables from global memory (too large
    # to stage in LDS beside the exchange lines), the others stage them
    return [W.fractional_l1(2, 7, 16, 0.3, 0.01), W.fractional_l1(2, 7, 16, 0.7, 0.05),
            W.fractional_l1(2, 15, 32, 0.5, 0.003), W.heat_bdf(2, 15, 32, 0.02),
            W.fractional_l1(1, 31, 64, 0.4, 0.01), W.heat_cn(2, 7, 8, 0.1),
            W.fractional_l1(1, 15, 2048, 0.5, 0.01)]


def test_batched_matches_oracle_and_single():
    probs = small_batch()
    nrhs = 2
    print(f"[batched] {len(probs)} instances x {nrhs} rhs", flush=True)
    fs, refs = [], []
    for i, pr in enumerate(probs):
        sysm = O.from_problem(pr)
        for r in range(nrhs):
            f = W.rhs_normal(pr, 4000 + 4 * i + r)
            fs.append(torch.from_numpy(f).cuda())
            refs.append((sysm, f, O.exact_solve(sysm, f).ravel()))
    b = bltt.Batch(probs, nrhs)
    try:
        assert all(t in (256, 512) for t in b.classes())
        us, iters, hists, infos, rc = b.pminres(fs, 1e-8, 200)
        # a second call on the same handle (cached graphs) gives the same answer
        us2, iters2, _, _, rc2 = b.pminres(fs, 1e-8, 200)
    finally:
        b.close()
    assert rc == bltt.OK and rc2 == bltt.OK
    for g, (sysm, f, ustar) in enumerate(refs):
        u = us[g].cpu().numpy()
        assert infos[g]["true_relres"] <= 1e-8, (g, infos[g])
        assert relnorm(u, ustar) <= 1e-8, (g, relnorm(u, ustar))
        assert np.array_equal(u, us2[g].cpu().numpy()) and iters[g] == iters2[g]
        assert hists[g][0] == 1.0 and np.all(np.isfinite(hists[g]))
    # the same instance solved alone by the single-system mixed path
    for g in (0, 5, 9):
        i = g // nrhs
        s = bltt.Solver.from_problem(probs[i], precision=bltt.MIXED)
        try:
            u1, it1, _, info1, rc1 = s.pminres(fs[g], 1e-8, 200)
        finally:
            s.close()
        assert rc1 == bltt.OK
        assert relnorm(us[g].cpu().numpy(), u1.cpu().numpy()) < 2e-8
        print(f"  system {g}: batched iters {iters[g]} single {it1}", flush=True)


def test_batched_zero_rhs():
    probs = [W.fractional_l1(2, 7, 16, 0.5, 0.01), W.fractional_l1(2, 15, 16, 0.5, 0.01)]
    fs = [torch.zeros(pr.n, dtype=torch.float64, device="cuda") for pr in probs]
    fs[1] = torch.from_numpy(W.rhs_normal(probs[1], 3)).cuda()
    b = bltt.Batch(probs, 1)
    try:
        us = [torch.full_like(f, 7.0) for f in fs]
        us, iters, hists, infos, rc = b.pminres(fs, 1e-8, 100, us)
    finally:
        b.close()
    assert rc == bltt.OK
    assert iters[0] == 0 and float(us[0].abs().max()) == 0.0
    sysm = O.from_problem(probs[1])
    ref = O.exact_solve(sysm, fs[1].cpu().numpy()).ravel()
    assert relnorm(us[1].cpu().numpy(), ref) <= 1e-8


def test_batched_uneven_full_size():
    """The uneven batched workload: 64 2D fractional instances, M from
    {63^2, 127^2, 255^2}, N from {64, 256, 1024}, gamma ~ U(0.2, 0.8),
    alpha ~ logU(1e-3, 1e-1), 4 right-hand sides each, tol 1e-8.  Every system
    must reach the tolerance; one system per shape class is checked on sampled
    sine modes against the oracle's per-mode exact solution."""
    params = W.batched_instances(64, 4)
    probs = [W.fractional_l1(2, m, N, g, a) for (m, N, g, a) in params]
    nrhs = 4
    fs = []
    for i, pr in enumerate(probs):
        for r in range(nrhs):
            fs.append(torch.from_numpy(W.rhs_normal(pr, 4000 + 4 * i + r)).cuda())
        if i % 16 == 15:
            print(f"  right-hand sides of {i + 1} instances on the device", flush=True)
    print(f"[batched full] {len(fs)} systems, {sum(f.numel() for f in fs) / 1e9:.2f} G unknowns", flush=True)
    b = bltt.Batch(probs, nrhs)
    try:
        us, iters, hists, infos, rc = b.pminres(fs, 1e-8, 200)
        print(f"  classes {len(b.classes())}, solve {infos[0]['solve_ms']:.0f} ms, iters "
              f"{min(iters)}..{max(iters)}", flush=True)
    finally:
        b.close()
    assert rc == bltt.OK
    assert max(inf["true_relres"] for inf in infos) <= 1e-8
    seen = set()
    rng = np.random.default_rng(1)
    for i, (m, N, g, a) in enumerate(params):
        if (m, N) in seen:
            continue
        seen.add((m, N))
        gsys = i * nrhs + int(rng.integers(0, nrhs))
        sysm = O.from_problem(probs[i])
        f = fs[gsys].cpu().numpy()
        u = us[gsys].cpu().numpy()
        modes = [0, probs[i].M - 1] + list(rng.integers(0, probs[i].M, 3))
        got = O.project_modes(sysm, u, modes)
        ref = O.exact_modes(sysm, f, modes)
        # each sampled mode against its own exact norm
        err = float((np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())
        print(f"  class m={m} N={N} system {gsys}: per-mode err max {err:.2e}", flush=True)
        assert err <= 1e-8, ((m, N), err)


def test_batched_rejects_aliased_outputs():
    probs = [W.fractional_l1(2, 7, 16, 0.5, 0.01), W.fractional_l1(2, 15, 16, 0.5, 0.01)]
    fs = [torch.from_numpy(W.rhs_normal(pr, 3)).cuda() for pr in probs]
    b = bltt.Batch(probs, 1)
    try:
        # u equal to an f, u overlapping another system's f, two systems sharing one u
        big = torch.empty(probs[1].n, dtype=torch.float64, device="cuda")
        cases = [[fs[0], torch.empty_like(fs[1])],
                 [torch.empty_like(fs[0]), fs[1]],
                 [big[: probs[0].n], big]]
        for us in cases:
            with pytest.raises(bltt.BlttError) as ei:
                b.pminres(fs, 1e-8, 50, us)
            assert ei.value.code == -1
        us = [torch.empty_like(f) for f in fs]
        _, _, _, _, rc = b.pminres(fs, 1e-8, 50, us)
        assert rc == bltt.OK
    finally:
        b.close()


def test_one_destroy_for_both_handle_types():
    """bltt_destroy releases a batch as well as a single-system handle (each
    keeps a type tag as its first member); the batch alias does the same."""
    probs = [W.fractional_l1(2, 7, 64, 0.4, 0.01), W.fractional_l1(1, 15, 32, 0.6, 0.05)]
    L = bltt.load()
    for _ in range(2):
        b = bltt.Batch(probs, 1)
        L.bltt_destroy(b._h)          # the batch through the common entry point
        b._h = None
        s = bltt.Solver.from_problem(probs[0], precision=bltt.MIXED)
        L.bltt_destroy(s._h)
        s._h = None
    b = bltt.Batch(probs, 2)
    fs = [torch.from_numpy(W.rhs_normal(p, 7 + k)).cuda() for p in probs for k in range(2)]
    _, _, _, _, rc = b.pminres(fs, 1e-8, 200)
    L.bltt_destroy_batched(b._h)
    b._h = None
    assert rc == bltt.OK
