"""The paper's analytic examples as test problems (Section 5): the block
coefficients and right-hand sides of Example 1 (heat, backward Euler) and
Example 3 (time-fractional L1 scheme), and the iteration counts the paper
prints for them (tests/golden/paper_iteration_counts.json)."""
import json
import math
import os

import numpy as np

from oracle import bltt_oracle as O
from paper_2307_07749_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_counts():
    with open(os.path.join(GOLDEN, "paper_iteration_counts.json")) as fh:
        return json.load(fh)


def example_problem(kind, N, mp1, alpha, gamma=None):
    """The workloads.Problem behind an example (for the GPU solver)."""
    if kind == "example3":
        return W.fractional_l1(2, mp1 - 1, N, gamma, alpha, length=math.pi)
    return W.heat_bdf(2, mp1 - 1, N, alpha, diffusion=1e-6)


def example3_system_and_rhs(gamma, N, mp1, alpha):
    """Example 3: (0,pi)^2, T=1, u = sin x sin y t^2, u0 = 0,
    f = sin x sin y [2 t^{2-gamma}/Gamma(3-gamma) + 2 t^2]."""
    prob = W.fractional_l1(2, mp1 - 1, N, gamma, alpha, length=math.pi)
    sysm = O.from_problem(prob)
    h = math.pi / mp1
    x = h * np.arange(1, mp1)
    S = np.outer(np.sin(x), np.sin(x)).ravel()           # y slow, x fast
    t = (np.arange(1, N + 1) / N)[:, None]
    f = S[None, :] * (2 * t ** (2 - gamma) / math.gamma(3 - gamma) + 2 * t ** 2)
    return sysm, f


def example1_system_and_rhs(N, mp1, alpha):
    """Example 1 (BDF), read with diffusion 1e-6 and first block + u0/tau."""
    eps = 1e-6
    prob = W.heat_bdf(2, mp1 - 1, N, alpha, diffusion=eps)
    sysm = O.from_problem(prob)
    h = 1.0 / mp1
    x = h * np.arange(1, mp1)
    X1 = np.tile(x, mp1 - 1)        # x fastest
    X2 = np.repeat(x, mp1 - 1)
    g = X1 * (X1 - 1) * X2 * (X2 - 1)
    t = (np.arange(1, N + 1) / N)[:, None]
    f = np.exp(t) * (g[None, :] - 2 * eps * (X1 * (X1 - 1) + X2 * (X2 - 1))[None, :])
    f[0] += g * N                    # + u0 / tau
    return sysm, f


