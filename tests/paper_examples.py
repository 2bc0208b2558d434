"""The paper's analytic examples as test problems (Section 5): the block
coefficients and right-hand sides of Example 1 (heat, backward Euler),
Example 2 (heat with a variable coefficient, Crank-Nicolson), Example 3
(time-fractional L1 scheme) and Example 4 (L1 scheme, variable coefficient), and the iteration counts the paper prints for
them (tests/golden/paper_iteration_counts.json).  Sampling a coefficient
function at grid points and faces is input generation, shared by the oracle
tests and the GPU tests."""
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
    if kind == "example1cn":
        return W.heat_cn(2, mp1 - 1, N, alpha, diffusion=1e-6)
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




def example1cn_system_and_rhs(N, mp1, alpha):
    """Example 1 with Crank-Nicolson: blocks (I + tau eps L_h / 2) / tau and
    (-I + tau eps L_h / 2) / tau, L_h = -Delta_h, diffusion eps = 1e-6 (the
    reading that reproduces Table 1); right-hand side f at the half steps
    (n - 1/2) tau, and the first one plus (I - tau eps L_h / 2) u0 / tau, the
    initial-value term of the first equation moved to the right."""
    eps = 1e-6
    prob = W.heat_cn(2, mp1 - 1, N, alpha, diffusion=eps)
    sysm = O.from_problem(prob)
    h = 1.0 / mp1
    x = h * np.arange(1, mp1)
    X1 = np.tile(x, mp1 - 1)        # x fastest
    X2 = np.repeat(x, mp1 - 1)
    g = X1 * (X1 - 1) * X2 * (X2 - 1)
    t = ((np.arange(1, N + 1) - 0.5) / N)[:, None]
    f = np.exp(t) * (g[None, :] - 2 * eps * (X1 * (X1 - 1) + X2 * (X2 - 1))[None, :])
    Lu0 = O.laplacian_apply(g[None, :], sysm.ms, sysm.hs)[0]
    f[0] += g * N - 0.5 * eps * Lu0
    return sysm, f


def face_samples(a, ms, hs, lo):
    """a(x) at the faces of every dimension, in the layout of bltt_setup_varcoef
    (and of the oracle's laplacian_apply): grid points x_i = lo + (i+1) h, the
    faces along d at lo + (j + 1/2) h_d, j = 0..m_d, other coordinates at the
    grid points; x fastest."""
    faces = []
    for d in range(len(ms)):
        axes = []
        for e, (m, h) in enumerate(zip(ms, hs)):
            if e == d:
                axes.append(lo + (np.arange(m + 1) + 0.5) * h)
            else:
                axes.append(lo + (np.arange(m) + 1.0) * h)
        grids = np.meshgrid(*reversed(axes), indexing="ij")   # slowest dimension first
        faces.append(np.asarray(a(*reversed(grids)), dtype=np.float64).ravel())
    return tuple(faces)


def grid_mean(a, ms, hs, lo) -> float:
    """Mean of a(x) over the grid points."""
    axes = [lo + (np.arange(m) + 1.0) * h for m, h in zip(ms, hs)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return float(np.mean(a(*reversed(grids))))


def example2_coefficient(x1, x2):
    """Example 2: a(x) = (20 + x1^2)(20 + x2^2) on (0,1)^2."""
    return (20.0 + x1 ** 2) * (20.0 + x2 ** 2)


def example2_system_and_rhs(N, mp1, alpha):
    """Example 2 with Crank-Nicolson: blocks (I + tau/2 L_a)/tau and
    (-I + tau/2 L_a)/tau (p = (1/tau, -1/tau), q = (1/2, 1/2)), L_a = -Delta_{a,h};
    u = exp(t) x1(1-x1) x2(1-x2), f(x, t) = u_t - div(a grad u) sampled at
    t_{k-1/2}; first block + u0/tau - (1/2) L_a u0.  The printed f carries
    (20 + x2^2) in its second derivative term, where differentiating a gives
    (20 + x1^2); the derived form is used.  Returns (system, f, faces, abar)."""
    m = mp1 - 1
    h = 1.0 / mp1
    tau = 1.0 / N
    ms, hs = (m, m), (h, h)
    p = np.zeros(N)
    q = np.zeros(N)
    p[0], p[1] = 1.0 / tau, -1.0 / tau
    q[0], q[1] = 0.5, 0.5
    faces = face_samples(example2_coefficient, ms, hs, 0.0)
    abar = grid_mean(example2_coefficient, ms, hs, 0.0)
    sysm = O.System(ms, hs, p, q, alpha, faces, abar)
    x = h * np.arange(1, mp1)
    X1 = np.tile(x, m)
    X2 = np.repeat(x, m)
    g = X1 * (1 - X1) * X2 * (1 - X2)
    A = example2_coefficient(X1, X2)
    fx = (g - 2 * X1 * (20 + X2 ** 2) * (1 - 2 * X1) * X2 * (1 - X2)
          - 2 * X2 * (20 + X1 ** 2) * (1 - 2 * X2) * X1 * (1 - X1)
          + 2 * A * (X1 * (1 - X1) + X2 * (1 - X2)))
    t = ((np.arange(1, N + 1) - 0.5) / N)[:, None]
    f = np.exp(t) * fx[None, :]
    Lu0 = O.laplacian_apply(g[None, :], ms, hs, faces)[0]
    f[0] += g / tau - 0.5 * Lu0
    return sysm, f, faces, abar


def example4_coefficient(x, y):
    """Example 4: a(x, y) = 35 + x^3.5 + y^3.5 on (0,1)^2."""
    return 35.0 + x ** 3.5 + y ** 3.5


def example4_system_and_rhs(gamma, N, mp1, alpha):
    """Example 4: L1 scheme for the time-fractional equation with
    -div(a grad u), u = sin(pi x) sin(pi y) t^2 (u0 = 0), f = u's fractional
    derivative - div(a grad u) at t_n = n tau (the printed f writes alpha for
    gamma).  Returns (system, f, faces, abar, problem)."""
    m = mp1 - 1
    h = 1.0 / mp1
    ms, hs = (m, m), (h, h)
    prob = W.fractional_l1(2, m, N, gamma, alpha)
    faces = face_samples(example4_coefficient, ms, hs, 0.0)
    abar = grid_mean(example4_coefficient, ms, hs, 0.0)
    sysm = O.System(ms, hs, np.asarray(prob.p, np.float64), np.asarray(prob.q, np.float64), alpha, faces, abar)
    x = h * np.arange(1, mp1)
    X = np.tile(x, m)
    Y = np.repeat(x, m)
    S = np.sin(math.pi * X) * np.sin(math.pi * Y)
    ax = 3.5 * X ** 2.5
    ay = 3.5 * Y ** 2.5
    t = (np.arange(1, N + 1) / N)[:, None]
    f = (S[None, :] * (2 * t ** (2 - gamma) / math.gamma(3 - gamma) + 2 * math.pi ** 2 * example4_coefficient(X, Y)[None, :] * t ** 2)
         - math.pi * t ** 2 * (ax * np.cos(math.pi * X) * np.sin(math.pi * Y)
                               + ay * np.sin(math.pi * X) * np.cos(math.pi * Y))[None, :])
    return sysm, f, faces, abar, prob
