"""Per-mode accuracy of a physical-space solution at full size, on sampled
sine modes, against the oracle's per-mode exact solution (test helper).

Each sampled mode's error is taken relative to that mode's own exact norm.
A solution held in FP64 in physical space cannot carry a small mode more
accurately than its own rounding allows: projecting u onto one orthonormal
sine vector is a dot product whose rounding is about eps ||u|| per time step,
and the solve's two log-depth sine transforms add about 2 log2(2(m+1)) times
that.  A mode whose exact norm is a fraction r of ||u|| therefore has a floor
of about 2 log2(2(m+1)) eps / r; the check allows the target plus this floor
(with a margin of 4), which matters only for FP64 targets and for modes many
orders of magnitude below the whole solution."""
import math

import numpy as np

from oracle import bltt_oracle as O

EPS64 = 2.2e-16


def mode_errors(sysm, u, f, modes):
    """(per-mode relative errors, per-mode floors) for the sampled modes."""
    got = O.project_modes(sysm, u, modes)
    ref = O.exact_modes(sysm, f, modes)
    nref = np.linalg.norm(ref, axis=0)
    errs = np.linalg.norm(got - ref, axis=0) / nref
    depth = 2.0 * math.log2(2 * (max(sysm.ms) + 1))
    floor = 4.0 * depth * EPS64 * np.linalg.norm(u) / nref
    return errs, floor


def worst(errs, floor, target):
    """The largest ratio of a mode's error to what it is allowed (<= 1 passes)."""
    return float(np.max(errs / (target + floor)))
