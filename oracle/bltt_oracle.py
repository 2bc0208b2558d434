"""CPU FP64 oracle for preconditioned MINRES on symmetrised BLTT systems.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
GPU path is checked against.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import it; the solver itself never does.
It shares no code with the GPU path: transforms are dense matrices applied by
matrix products, the Toeplitz matvec is a dense lower-triangular Toeplitz
product, and MINRES is written out from its recurrences.

Notation follows Li, Lin, Hon, Wu, "A preconditioned MINRES method for block
lower triangular Toeplitz systems" (arXiv 2307.07749):

* BLTT matrix A with symmetric blocks A_(k) (Section 1, eqs. (1)-(2)); every
  block here is ``p[k] I + q[k] L_h`` with L_h = -Delta_h (Section 5).
* Time-reversal Y = Y_N (x) I_M; Y A is symmetric (Section 2, eq. (4)).
* Block alpha-circulant C_alpha (Section 3, eq. (5)), diagonalised by the
  spatial sine transform U, the scaling D_alpha = diag(alpha^{j/N}) and the
  unitary Fourier matrix F = N^{-1/2}[theta^{jk}], theta = exp(2 pi i/N)
  (eqs. (8)-(10)); eigenvalues lambda_i^{(k,alpha)} from eq. (9).
* ABAC preconditioner P_alpha = |C_alpha| = (C^{1/2})^* C^{1/2}
  (Definitions 2-3, eqs. (11)-(13)); P^{-1} y = C^{-1/2} (C^{-1/2})^* y applied
  as two three-step procedures (Section 5.1).

Readings where the paper is silent or ambiguous:
  * MINRES is not printed; the standard preconditioned MINRES of Paige-Saunders
    in the Elman-Silvester-Wathen form is used, zero initial guess.
  * The stopping test is the relative, unpreconditioned 2-norm of the
    symmetrised residual ||Y(f - A u_k)||_2 / ||Y f||_2 <= tol.
  * D_alpha is 0-based: alpha^{j/N}, j = 0..N-1.
  * U is the orthonormal DST-I, x fastest in the lexicographic order.

All arrays are float64 / complex128.  Vectors are time-major 2-D arrays of
shape (N, M) internally; public functions accept flat length-MN vectors too.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ---------------------------------------------------------------------------
# spatial operators
# ---------------------------------------------------------------------------

def dst1_matrix(m: int) -> np.ndarray:
    """Orthonormal DST-I matrix U[j,k] = sqrt(2/(m+1)) sin(pi (j+1)(k+1)/(m+1)).

    U is the orthogonal matrix that diagonalises every block (Remark 1 and the
    fast sine transforms of Section 5.1).  U is symmetric and U U = I.
    """
    j = np.arange(1, m + 1, dtype=np.float64)
    return math.sqrt(2.0 / (m + 1)) * np.sin(np.pi * np.outer(j, j) / (m + 1))


def laplacian_eigs_1d(m: int, h: float) -> np.ndarray:
    """Eigenvalues of the 1-D negative Laplacian h^-2 tridiag(-1, 2, -1),
    in DST-I mode order k = 1..m: 4 h^-2 sin^2(k pi / (2(m+1)))."""
    k = np.arange(1, m + 1, dtype=np.float64)
    return 4.0 / (h * h) * np.sin(k * np.pi / (2.0 * (m + 1))) ** 2


def laplacian_eigs(ms, hs) -> np.ndarray:
    """Eigenvalues mu_i of L_h on the tensor grid, lexicographic, x fastest."""
    mu = np.zeros(1)
    for m, h in zip(ms, hs):
        # the new (slower) dimension is the outer index
        mu = (laplacian_eigs_1d(m, h)[:, None] + mu[None, :]).ravel()
    return mu


def _as_grid(v: np.ndarray, N: int, ms) -> np.ndarray:
    """(N, M) -> (N, m_{d-1}, ..., m_1, m_0) with x = m_0 fastest."""
    return v.reshape((N,) + tuple(reversed(ms)))


def laplacian_apply(v: np.ndarray, ms, hs, faces=None) -> np.ndarray:
    """L_h v for every time slice: 2d/h^2 on the diagonal, -1/h^2 on each
    neighbour, zero Dirichlet boundary (central differences, Section 5).

    With ``faces`` it is L_{a,h} = -Delta_{a,h}, the central-difference form of
    -div(a grad) (Section 5.2): per dimension d, faces[d] holds a at the points
    halfway between neighbours along d (grid shape with m_d + 1 entries along
    d; entry j sits between points j-1 and j, the outer two on the boundary),
    and (L_{a,h} v)_i = sum_d [a_{j=i+1} (v_i - v_{i+1}) + a_{j=i} (v_i - v_{i-1})] / h_d^2
    with v = 0 outside the grid."""
    N = v.shape[0]
    g = _as_grid(v, N, ms)
    out = np.zeros_like(g)
    dim = len(ms)
    for d in range(dim):
        ax = g.ndim - 1 - d          # axis of dimension d (x is last)
        inv_h2 = 1.0 / (hs[d] * hs[d])
        if faces is None:
            out += 2.0 * inv_h2 * g
            lo = [slice(None)] * g.ndim
            hi = [slice(None)] * g.ndim
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            out[tuple(lo)] -= inv_h2 * g[tuple(hi)]
            out[tuple(hi)] -= inv_h2 * g[tuple(lo)]
        else:
            # flux through face j: a_j (v_j - v_{j-1}), with zero ghost values
            pad = [(0, 0)] * g.ndim
            pad[ax] = (1, 1)
            gp = np.pad(g, pad)
            a = faces[d].reshape(tuple(reversed([m + (1 if e == d else 0) for e, m in enumerate(ms)])))
            flux = a[None] * np.diff(gp, axis=ax)
            lo = [slice(None)] * g.ndim
            hi = [slice(None)] * g.ndim
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            out += inv_h2 * (flux[tuple(lo)] - flux[tuple(hi)])
    return out.reshape(N, -1)


def space_transform(v: np.ndarray, ms) -> np.ndarray:
    """(I_N (x) U) v with U = U_{d-1} (x) ... (x) U_0, each a dense DST-I.

    U is symmetric and orthogonal, so this one routine applies both U and
    U^T (Steps 1 and 3 of Section 5.1)."""
    N = v.shape[0]
    g = _as_grid(v, N, ms)
    for d, m in enumerate(ms):
        ax = g.ndim - 1 - d
        U = dst1_matrix(m)
        g = np.moveaxis(np.tensordot(g, U, axes=([ax], [0])), -1, ax)
    return g.reshape(N, -1)


# ---------------------------------------------------------------------------
# the BLTT operator
# ---------------------------------------------------------------------------

@dataclass
class System:
    """A BLTT system A u = f with blocks p[k] I + q[k] L_h and parameter alpha.

    With ``faces`` (see laplacian_apply) the blocks are p[k] I + q[k] L_{a,h};
    the preconditioner is then the one of the mean-coefficient system, blocks
    p[k] I + q[k] abar L_h (Section 5.2)."""

    ms: tuple
    hs: tuple
    p: np.ndarray
    q: np.ndarray
    alpha: float
    faces: tuple | None = None
    abar: float = 1.0

    @property
    def N(self) -> int:
        return len(self.p)

    @property
    def M(self) -> int:
        return int(np.prod(self.ms))


def lower_toeplitz(c: np.ndarray) -> np.ndarray:
    """Dense N x N lower-triangular Toeplitz matrix with first column c,
    i.e. sum_k c_k H_0^{(k)} (eq. (3)), H_0^{(0)} = I."""
    N = len(c)
    i, j = np.indices((N, N))
    T = np.zeros((N, N))
    mask = i >= j
    T[mask] = c[(i - j)[mask]]
    return T


def bltt_apply(sys: System, v: np.ndarray) -> np.ndarray:
    """A v from the tensor form of eq. (3) with A_(k) = p_k I + q_k L_h:
    (A v)_n = sum_{k=0}^{n} (p_k v_{n-k} + q_k L_h v_{n-k}).
    The sums over k are one dense lower-triangular Toeplitz product each."""
    N = sys.N
    V = v.reshape(N, -1)
    out = lower_toeplitz(sys.p) @ V
    if np.any(sys.q != 0.0):
        out += lower_toeplitz(sys.q) @ laplacian_apply(V, sys.ms, sys.hs, sys.faces)
    return out


def time_reverse(v: np.ndarray) -> np.ndarray:
    """Y v with Y = Y_N (x) I_M, Y_N the anti-identity (Section 2)."""
    return v[::-1].copy()


def sym_apply(sys: System, v: np.ndarray) -> np.ndarray:
    """K v = Y A v, the symmetrised operator of eq. (4)."""
    return time_reverse(bltt_apply(sys, v))


# ---------------------------------------------------------------------------
# the ABAC preconditioner
# ---------------------------------------------------------------------------

def fourier_unitary(N: int) -> np.ndarray:
    """F = N^{-1/2} [theta^{jk}], theta = exp(2 pi i / N) (eq. (8))."""
    j = np.arange(N)
    return np.exp(2j * np.pi * np.outer(j, j) / N) / math.sqrt(N)


def alpha_scaling(N: int, alpha: float) -> np.ndarray:
    """Diagonal of D_alpha, alpha^{j/N} for j = 0..N-1 (eq. (8))."""
    return alpha ** (np.arange(N, dtype=np.float64) / N)


def alpha_eigenvalues(sys: System) -> np.ndarray:
    """lambda[k, i] = sum_j lambda_i^{(j)} alpha^{j/N} theta^{-k j} (eq. (9)),
    with lambda_i^{(j)} = p_j + q_j mu_i the eigenvalues of block j in mode i
    (mu scaled by abar for a variable-coefficient system: the eigenvalues of
    its mean-coefficient system).

    Written as sqrt(N) F^* D_alpha c_i, the right-hand form of eq. (9)."""
    N = sys.N
    mu = sys.abar * laplacian_eigs(sys.ms, sys.hs)
    cols = sys.p[:, None] + sys.q[:, None] * mu[None, :]          # (N, M)
    F = fourier_unitary(N)
    return math.sqrt(N) * (F.conj().T @ (alpha_scaling(N, sys.alpha)[:, None] * cols))


def principal_sqrt(lam: np.ndarray) -> np.ndarray:
    """Principal branch of the complex square root (Definition 2)."""
    return np.sqrt(lam.astype(np.complex128))


@dataclass
class Precond:
    sys: System
    lam: np.ndarray          # (N, M) complex eigenvalues
    sq: np.ndarray           # (N, M) principal square roots
    F: np.ndarray
    d: np.ndarray            # alpha^{j/N}


def precond_setup(sys: System) -> Precond:
    lam = alpha_eigenvalues(sys)
    if np.any(lam.real <= 0.0):
        raise ValueError("alpha-circulant eigenvalue with non-positive real part; "
                         "Assumption 1(ii) violated")
    return Precond(sys, lam, principal_sqrt(lam), fourier_unitary(sys.N),
                   alpha_scaling(sys.N, sys.alpha))


def _time_sandwich(P: Precond, t: np.ndarray, diag: np.ndarray,
                   pre: np.ndarray, post: np.ndarray) -> np.ndarray:
    """Per spatial mode i: diag(post) F diag(diag[:, i]) F^* diag(pre) t_i.
    Returns the real part, after checking the imaginary part is roundoff
    (Lemma 3(b): the half-preconditioners are real)."""
    F = P.F
    s = pre[:, None] * t
    s = F.conj().T @ s
    s = diag * s
    s = F @ s
    s = post[:, None] * s
    # roundoff in the imaginary part is amplified by D_alpha^{-1} (up to 1/alpha)
    scale = max(1e-300, float(np.max(np.abs(s.real))))
    bound = max(1e-8, 64.0 * len(pre) * np.finfo(np.float64).eps / P.sys.alpha)
    assert float(np.max(np.abs(s.imag))) <= bound * scale, "half-preconditioner not real"
    return s.real


def precond_half_adjoint(P: Precond, y: np.ndarray) -> np.ndarray:
    """(C^{-1/2})^* y via Steps 1-3 of Section 5.1:
    U^T, then D F conj(Lambda)^{-1/2} F^* D^{-1} per mode, then U."""
    ms = P.sys.ms
    yt = space_transform(y.reshape(P.sys.N, -1), ms)
    zt = _time_sandwich(P, yt, 1.0 / P.sq.conj(), 1.0 / P.d, P.d)
    return space_transform(zt, ms)


def precond_half(P: Precond, y: np.ndarray) -> np.ndarray:
    """C^{-1/2} y with C^{1/2} from eq. (13): U^T, then
    D^{-1} F Lambda^{-1/2} F^* D per mode, then U."""
    ms = P.sys.ms
    yt = space_transform(y.reshape(P.sys.N, -1), ms)
    zt = _time_sandwich(P, yt, 1.0 / P.sq, P.d, 1.0 / P.d)
    return space_transform(zt, ms)


def precond_apply(P: Precond, y: np.ndarray) -> np.ndarray:
    """P_alpha^{-1} y = C^{-1/2} (C^{-1/2})^* y (Section 5.1)."""
    return precond_half(P, precond_half_adjoint(P, y))


# ---------------------------------------------------------------------------
# preconditioned MINRES
# ---------------------------------------------------------------------------

@dataclass
class MinresResult:
    x: np.ndarray            # (N, M) solution of A x = f
    iters: int
    eta_hist: list           # |eta_j| / eta_0, j = 0..iters
    relres_hist: list        # ||Y(f - A x_j)|| / ||Y f||, j = 0..iters
    converged: bool


def pminres(sys: System, f: np.ndarray, tol: float, maxit: int,
            precond: str = "abac", x0: np.ndarray | None = None) -> MinresResult:
    """Preconditioned MINRES on K u = b, K = Y A, b = Y f (eq. (4)).

    ``precond``: "abac" (P_alpha of eq. (13)), or "none" (MINRES-I).  MINRES-P_1
    is "abac" with alpha = 1.

    Recurrences (Lanczos vectors normalised so <v_j, z_j> = 1, z_j = P^{-1} v_j):
        q = K z_j;  delta = <q, z_j>
        vhat = q - delta v_j - beta_j v_{j-1};  zhat = P^{-1} vhat
        beta_{j+1} = sqrt(<vhat, zhat>)
        a0 = c_j delta - c_{j-1} s_j beta_j;  a1 = hypot(a0, beta_{j+1})
        a2 = s_j delta + c_{j-1} c_j beta_j;   a3 = s_{j-1} beta_j
        c_{j+1} = a0 / a1;  s_{j+1} = beta_{j+1} / a1
        w_j = (z_j - a3 w_{j-2} - a2 w_{j-1}) / a1
        x_j = x_{j-1} + c_{j+1} eta w_j;  eta <- -s_{j+1} eta
    Stops when the relative symmetrised residual ||b - K x_j|| / ||b|| <= tol.
    """
    N = sys.N
    b = time_reverse(f.reshape(N, -1).astype(np.float64))
    if precond == "abac":
        P = precond_setup(sys)
        Pinv = lambda y: precond_apply(P, y)
    elif precond == "none":
        Pinv = lambda y: y.copy()
    else:
        raise ValueError(precond)
    K = lambda v: sym_apply(sys, v)
    dot = lambda a, c: float(np.vdot(a.ravel(), c.ravel()))

    bnorm = math.sqrt(dot(b, b))
    x = np.zeros_like(b) if x0 is None else x0.reshape(N, -1).astype(np.float64).copy()
    r0 = b - K(x) if x0 is not None else b.copy()
    if bnorm == 0.0:
        return MinresResult(x, 0, [1.0], [0.0], True)
    relres0 = math.sqrt(dot(r0, r0)) / bnorm
    if relres0 <= tol:
        return MinresResult(x, 0, [1.0], [relres0], True)

    z = Pinv(r0)
    beta = math.sqrt(dot(r0, z))
    v = r0 / beta
    z = z / beta
    v_prev = np.zeros_like(b)
    w_prev = np.zeros_like(b)      # w_{j-1}
    w_prev2 = np.zeros_like(b)     # w_{j-2}
    eta = beta
    eta0 = beta
    c_prev, c = 1.0, 1.0           # c_{j-1}, c_j
    s_prev, s = 0.0, 0.0           # s_{j-1}, s_j
    beta_j = 0.0                   # beta_j (beta_1 enters only via v_1, z_1)
    eta_hist = [1.0]
    relres_hist = [relres0]
    converged = False
    j = 0
    for j in range(1, maxit + 1):
        qv = K(z)
        delta = dot(qv, z)
        vhat = qv - delta * v - beta_j * v_prev
        zhat = Pinv(vhat)
        bsq = dot(vhat, zhat)
        if bsq < 0.0:
            raise FloatingPointError("preconditioner not SPD in floating point")
        beta_next = math.sqrt(bsq)
        a0 = c * delta - c_prev * s * beta_j
        a1 = math.hypot(a0, beta_next)
        a2 = s * delta + c_prev * c * beta_j
        a3 = s_prev * beta_j
        c_next = a0 / a1
        s_next = beta_next / a1
        w = (z - a3 * w_prev2 - a2 * w_prev) / a1
        x = x + c_next * eta * w
        eta = -s_next * eta
        res = b - K(x)
        relres = math.sqrt(dot(res, res)) / bnorm
        eta_hist.append(abs(eta) / eta0)
        relres_hist.append(relres)
        if relres <= tol or beta_next == 0.0:
            converged = relres <= tol or beta_next == 0.0
            break
        # shift the recurrence
        v_prev, v = v, vhat / beta_next
        z = zhat / beta_next
        w_prev2, w_prev = w_prev, w
        c_prev, c = c, c_next
        s_prev, s = s, s_next
        beta_j = beta_next
    return MinresResult(x, j, eta_hist, relres_hist, converged)


# ---------------------------------------------------------------------------
# exact solution
# ---------------------------------------------------------------------------

def laplacian_matrix(ms, hs, faces=None):
    """L_h (or L_{a,h} with faces) as a scipy.sparse matrix, assembled face by
    face: each interior face between lexicographic points i and i' adds
    a_f/h^2 to (i,i) and (i',i') and -a_f/h^2 to (i,i') and (i',i); each
    boundary face adds a_f/h^2 to the diagonal of its one point."""
    import scipy.sparse as sp
    M = int(np.prod(ms))
    rows, cols, vals = [], [], []
    idx = np.arange(M).reshape(tuple(reversed(ms)))
    for d, m in enumerate(ms):
        ax = idx.ndim - 1 - d
        shape = list(reversed([mm + (1 if e == d else 0) for e, mm in enumerate(ms)]))
        a = np.ones(shape) if faces is None else faces[d].reshape(shape)
        w = a / (hs[d] * hs[d])
        for j in range(m + 1):
            wj = np.take(w, j, axis=ax).ravel()
            if j > 0:
                left = np.take(idx, j - 1, axis=ax).ravel()
                rows.append(left); cols.append(left); vals.append(wj)
            if j < m:
                right = np.take(idx, j, axis=ax).ravel()
                rows.append(right); cols.append(right); vals.append(wj)
            if 0 < j < m:
                rows += [left, right]; cols += [right, left]; vals += [-wj, -wj]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(M, M))


def exact_solve(sys: System, f: np.ndarray) -> np.ndarray:
    """u* = A^{-1} f by block forward substitution in sine-transform
    coordinates (physical coordinates and a sparse LU of the first block for
    a variable-coefficient system).  Every block is diagonal there with entries
    p_k + q_k mu_i (Remark 1), so each time step is a pointwise division:
        ut_n = (ft_n - sum_{k=1}^{n} (p_k + q_k mu) ut_{n-k}) / (p_0 + q_0 mu).
    """
    N = sys.N
    if sys.faces is not None:
        # not sine-diagonal: forward substitution with a sparse LU of A_(0) = p_0 I + q_0 L_{a,h}
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        L = laplacian_matrix(sys.ms, sys.hs, sys.faces)
        lu = spla.splu((sys.p[0] * sp.identity(sys.M) + sys.q[0] * L).tocsc())
        F = f.reshape(N, -1).astype(np.float64)
        U = np.zeros_like(F)
        for n in range(N):
            rhs = F[n].copy()
            for k in range(1, n + 1):
                if sys.p[k] != 0.0:
                    rhs -= sys.p[k] * U[n - k]
                if sys.q[k] != 0.0:
                    rhs -= sys.q[k] * (L @ U[n - k])
            U[n] = lu.solve(rhs)
        return U
    mu = laplacian_eigs(sys.ms, sys.hs)
    ft = space_transform(f.reshape(N, -1).astype(np.float64), sys.ms)
    lam = sys.p[:, None] + sys.q[:, None] * mu[None, :]
    ut = np.zeros_like(ft)
    for n in range(N):
        acc = ft[n] - np.einsum("km,km->m", lam[1:n + 1], ut[n - 1::-1][:n]) if n else ft[n]
        ut[n] = acc / lam[0]
    return space_transform(ut, sys.ms)


def assumption_margin(sys: System) -> float:
    """min_i (lambda_i^{(0)} - sum_{k>=1} |lambda_i^{(k)}|) (Proposition 1)."""
    mu = laplacian_eigs(sys.ms, sys.hs)
    lam = sys.p[:, None] + sys.q[:, None] * mu[None, :]
    return float(np.min(lam[0] - np.sum(np.abs(lam[1:]), axis=0)))


def from_problem(prob) -> System:
    """Build a System from a workload description (duck-typed)."""
    return System(tuple(prob.m), tuple(prob.h), np.asarray(prob.p, np.float64),
                  np.asarray(prob.q, np.float64), float(prob.alpha))


# ---------------------------------------------------------------------------
# sampled outputs at sizes where the full oracle is too slow
# ---------------------------------------------------------------------------

def mode_vectors(sys: System, modes) -> np.ndarray:
    """Rows of U (the orthonormal sine basis, Remark 1) for the given
    lexicographic mode indices: shape (len(modes), M)."""
    rows = []
    Us = [dst1_matrix(m) for m in sys.ms]
    for i in modes:
        vec = np.ones(1)
        rest = int(i)
        ks = []
        for m in sys.ms:
            ks.append(rest % m)
            rest //= m
        for d, m in enumerate(sys.ms):
            # dimension d is slower than all previous ones: outer factor
            vec = np.outer(Us[d][ks[d]], vec).ravel()
        rows.append(vec)
    return np.array(rows)


def project_modes(sys: System, v: np.ndarray, modes) -> np.ndarray:
    """(U^T v_n)_i for every time step n and each mode i: shape (N, len(modes))."""
    B = mode_vectors(sys, modes)
    return v.reshape(sys.N, -1) @ B.T


def exact_modes(sys: System, f: np.ndarray, modes) -> np.ndarray:
    """(U^T u*)_i, u* = A^{-1} f, for the given modes only.  In sine
    coordinates each mode is an independent lower-triangular Toeplitz system
    with entries p_k + q_k mu_i (Remark 1), solved by forward substitution."""
    mu = laplacian_eigs(sys.ms, sys.hs)[list(modes)]
    ft = project_modes(sys, f, modes)                       # (N, K)
    lam = sys.p[:, None] + sys.q[:, None] * mu[None, :]     # (N, K)
    ut = np.zeros_like(ft)
    for n in range(sys.N):
        acc = ft[n] - (np.einsum("kj,kj->j", lam[1:n + 1], ut[n - 1::-1][:n]) if n else 0.0)
        ut[n] = acc / lam[0]
    return ut


# ---------------------------------------------------------------------------
# sine coordinates, mode by mode (Remark 1)
# ---------------------------------------------------------------------------
# Every block p_k I + q_k L_h is diagonal in the orthonormal sine basis: mode i
# sees the scalar lower-triangular Toeplitz matrix T_i = sum_k (p_k + q_k mu_i)
# H_0^{(k)} (eq. (3) with M = 1), and the block alpha-circulant C_alpha the
# scalar alpha-circulant with the same first column (eqs. (5)-(7)).  These
# functions act on the time lines of selected modes only, so that single
# lines of a full-size vector can be checked.  Rows of Z are time lines.

def mode_columns(sys: System, modes) -> np.ndarray:
    """First columns p + mu_i q of T_i for the given modes: shape (N, K)."""
    mu = laplacian_eigs(sys.ms, sys.hs)[np.asarray(modes, dtype=np.int64)]
    return sys.p[:, None] + sys.q[:, None] * mu[None, :]


def _mode_toeplitz(cols: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Rows t_i = T_i z_i, (T_i z)_n = sum_{k<=n} cols[k, i] z_{n-k} (eq. (3))."""
    Z = np.asarray(Z, np.float64)
    out = np.zeros_like(Z)
    N = Z.shape[1]
    for k in range(N):
        out[:, k:] += cols[k][:, None] * Z[:, :N - k]
    return out


def mode_sym_apply(sys: System, Z: np.ndarray, modes) -> np.ndarray:
    """Y_N T_i z_i for each listed mode (rows of Z), the symmetrised operator
    of eq. (4) in sine coordinates."""
    return _mode_toeplitz(mode_columns(sys, modes), Z)[:, ::-1].copy()


def mode_precond(sys: System, modes) -> Precond:
    """The per-mode eigenvalues of eq. (9), lambda_i^{(k,alpha)} =
    sum_j (p_j + mu_i q_j) alpha^{j/N} theta^{-kj}, for the listed modes only
    (columns), with their principal square roots."""
    N = sys.N
    F = fourier_unitary(N)
    d = alpha_scaling(N, sys.alpha)
    lam = math.sqrt(N) * (F.conj().T @ (d[:, None] * mode_columns(sys, modes)))
    if np.any(lam.real <= 0.0):
        raise ValueError("alpha-circulant eigenvalue with non-positive real part")
    return Precond(sys, lam, principal_sqrt(lam), F, d)


def mode_precond_apply(sys: System, Z: np.ndarray, modes) -> np.ndarray:
    """P_alpha^{-1} on the listed modes' time lines: the two half-solves of
    Section 5.1 Step 2, (C^{-1/2})^* = D F conj(Lambda)^{-1/2} F^* D^{-1} first,
    then C^{-1/2} = D^{-1} F Lambda^{-1/2} F^* D (eqs. (8)-(13))."""
    P = mode_precond(sys, modes)
    t = _time_sandwich(P, np.asarray(Z, np.float64).T, 1.0 / P.sq.conj(), 1.0 / P.d, P.d)
    t = _time_sandwich(P, t, 1.0 / P.sq, P.d, 1.0 / P.d)
    return t.T.copy()


def mode_residual(sys: System, Fh: np.ndarray, Uh: np.ndarray, modes) -> np.ndarray:
    """Y_N (fhat_i - T_i uhat_i) for each listed mode (rows of Fh, Uh)."""
    return (np.asarray(Fh, np.float64) - _mode_toeplitz(mode_columns(sys, modes), Uh))[:, ::-1].copy()
