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


# ---------------------------------------------------------------------------
# step-kernel error metrics (sine-coordinate lines, element by element)
# ---------------------------------------------------------------------------

def _is64(dtype) -> bool:
    return "64" in str(dtype)


def line_err(got, ref):
    """max over lines of max|got - ref| / max|ref| within the line (rows)."""
    got = np.asarray(got, np.float64).reshape(ref.shape)
    den = np.maximum(np.abs(ref).max(axis=1), 1e-300)
    return float((np.abs(got - ref).max(axis=1) / den).max())


def pair_partner(i, M, mx):
    """The sine mode that shares mode i's complex line in the sine-basis
    kernels.  Modes are numbered x fastest in rows of mx (odd); within a row
    modes 2j and 2j+1 of the row pair up, and the last modes of rows r and
    r+1 (r even) pair with each other; a lone last mode is its own partner.
    (With mx = 1 this is i ^ 1.)"""
    r, x = divmod(int(i), int(mx))
    if x < mx - 1:
        return r * mx + (x ^ 1)
    rr = r ^ 1
    return rr * mx + mx - 1 if rr < M // mx else int(i)


def pair_err(got, ref, inp, sysm, modes, M):
    """Time-pass error of each line, normwise over its packed pair.  The kernel
    transforms two sine modes (pair_partner) as the real and imaginary parts
    of one complex line, so its rounding is relative to that complex line: it
    scales with the larger input of the pair times the larger multiplier
    either mode applies, max_k |lambda_{i,k}|^{-1} (eq. (9)).  When one mode's
    input or output is much larger than its partner's, the smaller one's
    relative error grows by that ratio (cross-talk of the two-for-one split),
    which is why the kernels pair modes of neighbouring x frequency."""
    got = np.asarray(got, np.float64).reshape(ref.shape)
    row = {int(i): k for k, i in enumerate(modes)}
    pn = (1.0 / np.abs(O.mode_precond(sysm, modes).lam)).max(axis=0)
    im = np.abs(np.asarray(inp, np.float64)).max(axis=1)
    part = [row[pair_partner(i, M, sysm.ms[0])] for i in modes]
    scale = np.maximum(im, im[part]) * np.maximum(pn, pn[part])
    return float((np.abs(got - ref).max(axis=1) / np.maximum(scale, 1e-300)).max())


def tol_time(dtype, N, alpha):
    """Rounding of the time pass on a packed pair (normwise, see pair_err):
    four N-point transforms
    (eps log2 N each) between alpha^{-n/N} scalings that amplify it by up to
    1/alpha, with a margin of two: 2 eps log2(2N) / alpha (FP32).  In FP64 the
    oracle's own dense N x N Fourier products dominate (error growing like
    eps N / alpha): 4 eps (N + 16) / alpha."""
    if _is64(dtype):
        return 4 * 1.1e-16 * (N + 16) / alpha
    return 2 * 6e-8 * math.log2(2 * N) / alpha


TOL_MV = {"float64": 1e-12, "float32": 2e-5}
