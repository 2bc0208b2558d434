"""Seeded synthetic workloads for the BLTT all-at-once systems.

This module only *describes problems*: block coefficients of the BLTT matrix
and seeded right-hand sides.  It holds none of the solver's arithmetic, imports
nothing from the solver or from the CPU oracle, and is the one module both of
them read inputs from.

Block model (Section 5, examples): every block is ``A_(k) = p[k] I + q[k] L_h``
with ``L_h = -Delta_h`` the zero-Dirichlet central-difference negative
Laplacian on a uniform grid of ``m`` interior points per dimension,
``h = (b - a)/(m + 1)``.  Unknowns are time-major, ``u[n*M + i]``, with the
spatial index ``i`` lexicographic and x fastest.

Problems:
  * heat equation, backward Euler (Example 1, BDF system): ``A_(0) = I/tau + L_h``,
    ``A_(1) = -I/tau``;
  * heat equation, Crank-Nicolson (Example 1, CN system, scaled by 1/tau):
    ``A_(0) = I/tau + L_h/2``, ``A_(1) = -I/tau + L_h/2``;
  * time-fractional sub-diffusion, L1 scheme (Section 5.3, eq. for T and the
    weights l_k): ``A_(0) = l_0 tau^-gamma I + L_h``, ``A_(k) = l_k tau^-gamma I``
    with ``l_0 = 1/Gamma(2-gamma)`` and
    ``l_k = [(k+1)^(1-gamma) - 2 k^(1-gamma) + (k-1)^(1-gamma)] / Gamma(2-gamma)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One BLTT instance: grid, time steps, block coefficients and alpha."""

    name: str
    dim: int
    m: tuple            # interior points per dimension (len == dim)
    h: tuple            # grid spacing per dimension
    N: int              # number of time steps (blocks)
    p: np.ndarray       # float64[N], identity coefficients
    q: np.ndarray       # float64[N], Laplacian coefficients
    alpha: float
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(np.prod(self.m))

    @property
    def n(self) -> int:
        return self.M * self.N


def heat_bdf(dim: int, m: int, N: int, alpha: float, T: float = 1.0,
             length: float = 1.0, diffusion: float = 1.0) -> Problem:
    """Backward-Euler heat equation blocks (Example 1, BDF system)."""
    tau = T / N
    h = length / (m + 1)
    p = np.zeros(N)
    q = np.zeros(N)
    p[0] = 1.0 / tau
    if N > 1:
        p[1] = -1.0 / tau
    q[0] = diffusion
    return Problem("heat_bdf", dim, (m,) * dim, (h,) * dim, N, p, q, alpha,
                   {"tau": tau, "diffusion": diffusion})


def heat_cn(dim: int, m: int, N: int, alpha: float, T: float = 1.0,
            length: float = 1.0, diffusion: float = 1.0) -> Problem:
    """Crank-Nicolson heat equation blocks (Example 1, CN system)."""
    tau = T / N
    h = length / (m + 1)
    p = np.zeros(N)
    q = np.zeros(N)
    p[0] = 1.0 / tau
    q[0] = 0.5 * diffusion
    if N > 1:
        p[1] = -1.0 / tau
        q[1] = 0.5 * diffusion
    return Problem("heat_cn", dim, (m,) * dim, (h,) * dim, N, p, q, alpha,
                   {"tau": tau, "diffusion": diffusion})


def l1_weights(gamma: float, N: int) -> np.ndarray:
    """L1-scheme weights l_0..l_{N-1} (Section 5.3)."""
    g = 1.0 - gamma
    k = np.arange(N, dtype=np.float64)
    w = np.empty(N)
    w[0] = 1.0
    if N > 1:
        kk = k[1:]
        w[1:] = (kk + 1.0) ** g - 2.0 * kk ** g + (kk - 1.0) ** g
    return w / math.gamma(2.0 - gamma)


def fractional_l1(dim: int, m: int, N: int, gamma: float, alpha: float,
                  T: float = 1.0, length: float = 1.0) -> Problem:
    """Time-fractional sub-diffusion, L1 scheme (Section 5.3)."""
    tau = T / N
    h = length / (m + 1)
    p = l1_weights(gamma, N) * tau ** (-gamma)
    q = np.zeros(N)
    q[0] = 1.0
    return Problem("fractional_l1", dim, (m,) * dim, (h,) * dim, N, p, q, alpha,
                   {"tau": tau, "gamma": gamma})


def rhs_normal(prob: Problem, seed: int, nrhs: int = 1) -> np.ndarray:
    """f ~ N(0,1) i.i.d., float64, time-major, shape (n,) or (nrhs, n)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nrhs, prob.n))
    return f[0] if nrhs == 1 else f


# --- the named workloads -----------------------------------------------------

def workload(name: str) -> tuple[Problem, int]:
    """Return (problem, seed) for a named synthetic workload.

    Names:
      ``frac1d_m31_n32``      1D L1 gamma=0.5, m=31, N=32, alpha=0.01 (FP64, tol 1e-10)
      ``heat2d_m255_n256``    2D heat BDF, m=255, N=256, alpha=0.01 (FP64, tol 1e-10)
      ``frac2d_m511_n1024_g03`` / ``_g07``  2D L1, m=511, N=1024, alpha=0.01
      ``frac3d_m127_n256``    3D L1 gamma=0.5, m=127, N=256, alpha=0.01
    """
    if name == "frac1d_m31_n32":
        return fractional_l1(1, 31, 32, 0.5, 0.01), 1
    if name == "heat2d_m255_n256":
        return heat_bdf(2, 255, 256, 0.01), 2
    if name == "frac2d_m511_n1024_g03":
        return fractional_l1(2, 511, 1024, 0.3, 0.01), 3
    if name == "frac2d_m511_n1024_g07":
        return fractional_l1(2, 511, 1024, 0.7, 0.01), 33
    if name == "frac3d_m127_n256":
        return fractional_l1(3, 127, 256, 0.5, 0.01), 5
    raise KeyError(name)


def batched_instances(count: int = 64, seed: int = 4):
    """Parameters of the uneven batched workload: M from {63^2,127^2,255^2},
    N from {64,256,1024}, gamma ~ U(0.2,0.8), alpha ~ logU(1e-3,1e-1).
    Right-hand side r of instance i is drawn from seed 4000 + 4 i + r."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.choice([63, 127, 255]))
        N = int(rng.choice([64, 256, 1024]))
        gamma = float(rng.uniform(0.2, 0.8))
        alpha = float(10.0 ** rng.uniform(-3.0, -1.0))
        out.append((m, N, gamma, alpha))
    return out
