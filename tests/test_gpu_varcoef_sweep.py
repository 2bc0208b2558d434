"""Seeded random variable-coefficient problems (Section 5.2: blocks
p_k I + q_k L_{a,h} with the mean-coefficient preconditioner) across 1D to
3D and N from 2 to 1024, with a smooth positive coefficient
a(x) = c0 prod_d (1 + e_d sin(k_d pi x_d + phi_d)), e_d <= 0.3 (the paper's
examples vary a by a few percent; a larger spread only lengthens the
iteration).  Each answer has its residual re-formed by the oracle's operator
and is compared with the oracle's exact solve (sparse LU of the first block,
then forward substitution)."""
import numpy as np
import pytest

from oracle import bltt_oracle as O
from paper_2307_07749_amd import bltt
from paper_2307_07749_amd import workloads as W
from tests import paper_examples as PE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _case(seed):
    rng = np.random.default_rng(seed)
    dim = int(rng.integers(1, 4))
    m = 2 ** int(rng.integers(1, {1: 9, 2: 6, 3: 4}[dim] + 1)) - 1
    logn = min(10, int(np.floor(np.log2(max(4.0, 5e4 / m ** dim)))))
    N = 2 ** int(rng.integers(1, logn + 1))
    kind = ("frac", "heat", "cn")[int(rng.integers(0, 3))]
    alpha = float(10 ** rng.uniform(-3, np.log10(0.3)))
    gamma = float(rng.uniform(0.1, 0.9))
    prec = (bltt.FP64, bltt.MIXED)[int(rng.integers(0, 2))]
    c0 = float(10 ** rng.uniform(-1, 1.5))
    eps, kk, ph = rng.uniform(0.0, 0.3, 3), rng.integers(1, 4, 3), rng.uniform(0, 2 * np.pi, 3)
    return dim, m, N, kind, alpha, gamma, prec, c0, eps, kk, ph


@pytest.mark.parametrize("seed", range(500, 516))
def test_random_varcoef(seed):
    dim, m, N, kind, alpha, gamma, prec, c0, eps, kk, ph = _case(seed)

    def a(*xs):
        v = c0
        for d, x in enumerate(xs):
            v = v * (1.0 + eps[d] * np.sin(kk[d] * np.pi * x + ph[d]))
        return v

    if kind == "frac":
        prob = W.fractional_l1(dim, m, N, gamma, alpha)
    elif kind == "heat":
        prob = W.heat_bdf(dim, m, N, alpha)
    else:
        prob = W.heat_cn(dim, m, N, alpha)
    ms, hs = tuple(prob.m), tuple(prob.h)
    faces = PE.face_samples(a, ms, hs, 0.0)
    abar = PE.grid_mean(a, ms, hs, 0.0)
    sysm = O.System(ms, hs, np.asarray(prob.p, np.float64), np.asarray(prob.q, np.float64), alpha, faces, abar)
    tol = 1e-10 if prec == bltt.FP64 else 1e-8
    print(f"[varcoef {seed}] {kind} dim={dim} m={m} N={N} alpha={alpha:.3g} c0={c0:.3g} eps={np.round(eps, 2)} "
          f"prec={'fp64' if prec == bltt.FP64 else 'mixed'}", flush=True)
    f = W.rhs_normal(prob, 700 + seed)
    ustar = O.exact_solve(sysm, f).ravel()
    s = bltt.Solver(dim, ms, hs, sysm.p, sysm.q, alpha, precision=prec, face=faces, abar=abar)
    try:
        u, iters, _, info, rc = s.pminres(torch.from_numpy(f).cuda(), tol, 600)
    finally:
        s.close()
    u = u.cpu().numpy()
    relres = float(np.linalg.norm(f - O.bltt_apply(sysm, u).ravel()) / np.linalg.norm(f))
    err = float(np.linalg.norm(u - ustar) / np.linalg.norm(ustar))
    print(f"  rc={rc} iters={iters} outer={info['iters_outer']} reported={info['true_relres']:.2e} "
          f"oracle residual={relres:.2e} err={err:.2e}", flush=True)
    assert rc == bltt.OK
    assert info["true_relres"] <= tol
    # physical-space residual in FP64 on both sides
    assert relres <= tol * (1 + 1e-3) + 1e-13
    assert err <= 30 * tol
