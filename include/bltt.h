/*
 * bltt.h -- C ABI of the MI355X PMINRES solver for symmetrised block lower
 * triangular Toeplitz (BLTT) all-at-once systems.
 *
 * Method: Li, Lin, Hon, Wu, "A preconditioned MINRES method for block lower
 * triangular Toeplitz systems" (arXiv 2307.07749).  The solver runs MINRES on
 * Y A u = Y f (Section 2, eq. (4)) preconditioned by the absolute-value block
 * alpha-circulant matrix P_alpha = |C_alpha| (Section 3, eqs. (5)-(13)),
 * applied as in Section 5.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Vectors are time-major: element (n, i) of an MN-vector sits at n*M + i,
 *    n = 0..N-1 the time step, i the lexicographic spatial index with x
 *    fastest (i = x + m0*(y + m1*z)).
 *  - Blocks are A_(k) = p[k] I + q[k] L_h, where L_h is the zero-Dirichlet
 *    central-difference negative Laplacian (Section 5): h_d^-2 (2 on the
 *    diagonal, -1 on each neighbour) summed over the dimensions.  Every block
 *    is then diagonalised by the orthonormal sine transform (Remark 1).
 *  - Device pointers ("_dev") are HIP device memory owned by the caller; the
 *    library never frees them.  Host pointers are read during the call only.
 *  - The stream argument is a hipStream_t passed as void*; NULL is the null
 *    stream.  All device work of a handle is enqueued on that stream.
 *  - Return codes: BLTT_OK (0) on success, BLTT_NOCONV (> 0) when the
 *    iteration limit was reached (outputs are still valid), a negative
 *    BLTT_E* code on error (outputs untouched unless stated).
 *  - Size limits: N and every m_d + 1 must be powers of two with
 *    1 <= N <= 2048 and 2 <= 2(m_d + 1) <= 2048; p may be dense; q may have at
 *    most 4 leading non-zero taps (q[k] = 0 for k >= 4).  Other inputs give
 *    BLTT_EUNSUPPORTED.
 *  - N = 1 (a single block, Section 3): the alpha-circulant of one block is
 *    the block itself, so P_alpha = |A_(0)| = A_(0) and MINRES ends after one
 *    iteration at u = A_(0)^{-1} f; bltt_pminres forms that iterate per sine
 *    mode in FP64 in either precision.  At N = 1 the variable-coefficient
 *    setup, BLTT_PRECOND_NONE, the batched setup and the step entry points
 *    that apply a time operator (bltt_apply_sym, bltt_apply_precond,
 *    bltt_modes_sym, bltt_modes_lanczos*, bltt_modes_resid) give
 *    BLTT_EUNSUPPORTED.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef BLTT_H
#define BLTT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bltt_status {
  BLTT_OK = 0,
  BLTT_NOCONV = 1,          /* maxit reached before tol; u, iters, hist valid   */
  BLTT_EINVAL = -1,         /* bad argument (null pointer, size, alpha, tol)     */
  BLTT_EASSUMPTION = -2,    /* Assumption 1(ii) fails: min_i(l_i^(0) -
                               sum_k |l_i^(k)|) <= 0 (Section 2, Prop. 1)        */
  BLTT_ENAN = -3,           /* non-finite value met in the input or iteration    */
  BLTT_EBREAKDOWN = -4,     /* <v, P^{-1} v> < 0: preconditioner not SPD in
                               floating point                                   */
  BLTT_ENOMEM = -5,         /* device allocation failed                          */
  BLTT_EHIP = -6,           /* a HIP runtime call failed                         */
  BLTT_EUNSUPPORTED = -7    /* size or block structure outside the limits above  */
};

enum bltt_precision {
  BLTT_FP64 = 0,            /* every step in FP64                                 */
  BLTT_MIXED = 1,           /* FP32 transforms/matvec/Krylov vectors inside an
                               FP64 iterative-refinement loop                     */
  BLTT_FP32 = 2             /* step-level entry points only: FP32 arithmetic      */
};

/* Basis the Krylov iteration runs in (both give the same iterates up to the
 * change of basis, in exact arithmetic). */
enum bltt_basis {
  BLTT_BASIS_SINE = 0,      /* default: f is sine-transformed once (I_N (x) U),
                               MINRES runs on the mode-decoupled system, where
                               L_h = diag(mu) (Remark 1) and P_alpha^{-1} is the
                               time pass alone; u is transformed back once      */
  BLTT_BASIS_PHYSICAL = 1   /* every iteration in physical space: stencil
                               matvec, and sine transforms inside each
                               preconditioner application (Section 5.1)        */
};

/* Preconditioner.  BLTT_PRECOND_NONE runs plain MINRES on Y A u = Y f (the
 * MINRES-I comparator of Section 5); it is supported with BLTT_FP64 and the
 * sine basis.  The P_1 comparator of Section 5 is BLTT_PRECOND_ABAC with
 * alpha = 1. */
enum bltt_precond {
  BLTT_PRECOND_ABAC = 0,    /* P_alpha = |C_alpha| (default)                       */
  BLTT_PRECOND_NONE = 1     /* identity                                          */
};

/* Kernel plans of the FP32 sine-basis iteration (the mixed path's time pass and
 * N-point matvec): the radix plan of their N-point transforms and the number of
 * workgroups of the persistent time pass.  BLTT_PLAN_AUTO times the variants
 * on the handle's own buffers at setup and keeps the fastest (or reads an
 * earlier choice from opt->plan_cache); the others force a radix plan.  Radix
 * plans differ only for N = 512 (16*8*4 or 16*4*8) and N = 1024 (16*8*8 or
 * 16*16*4); both compute the same transform. */
enum bltt_fft_plan {
  BLTT_PLAN_AUTO = 0,       /* default: autotuned at setup                         */
  BLTT_PLAN_BASE = 1,       /* radix plan 0, default workgroup count               */
  BLTT_PLAN_ALT = 2         /* radix plan 1 where it exists, default workgroups    */
};
enum bltt_plan_source {
  BLTT_PLAN_SOURCE_DEFAULT = 0,  /* defaults (FP64 handle, or nothing to tune)      */
  BLTT_PLAN_SOURCE_TIMED = 1,    /* timed at setup                                  */
  BLTT_PLAN_SOURCE_CACHE = 2,    /* read from the plan cache                        */
  BLTT_PLAN_SOURCE_FORCED = 3    /* opt->fft_plan                                   */
};

/* Block description.  dim in {1,2,3}; m[d] interior points and h[d] spacing of
 * dimension d (d = 0 is x, the fastest); p and q are host arrays of length N
 * (copied during bltt_setup). */
typedef struct {
  int32_t dim;
  int32_t m[3];
  double h[3];
  const double *p;
  const double *q;
} bltt_blocks;

/* Solver options.  Pass NULL for the defaults. */
typedef struct {
  int32_t precision;      /* BLTT_FP64 (default) or BLTT_MIXED                    */
  double inner_tol;       /* MIXED: relative tolerance of each FP32 inner solve
                             on its own right-hand side (default 1e-4)            */
  int32_t max_refine;     /* MIXED: maximum refinement sweeps (default 20)        */
  double check_factor;    /* FP64: compute the true residual once the MINRES
                             estimate |eta_j|/eta_0 <= check_factor*tol
                             (default 10)                                         */
  int32_t basis;          /* BLTT_BASIS_SINE (default) or BLTT_BASIS_PHYSICAL     */
  int32_t precond;        /* BLTT_PRECOND_ABAC (default) or BLTT_PRECOND_NONE     */
  int32_t initial_guess;  /* 0 (default): MINRES starts from u = 0 (Section 5);
                             1: bltt_pminres reads its initial guess from u_dev
                             and iterates on the residual Y(f - A u0)           */
  const char *plan_cache; /* NULL, or a text file of kernel plans chosen by the
                             setup autotuner: read when it holds an entry for
                             this shape, appended to when the tuner had to run  */
  int32_t fft_plan;       /* BLTT_PLAN_AUTO (default), _BASE or _ALT           */
  int32_t eager;          /* 0 (default): the sine-basis MINRES loop captures
                             each iteration's kernels once as a HIP graph (one
                             per iteration position: 7 in FP64, one per stored
                             vector in a MIXED sweep) and replays it; 1: every
                             kernel is launched directly.  Both give identical
                             results; with profiling on the loop is eager.   */
} bltt_options;

/* Per-solve report. */
typedef struct {
  int32_t iters_inner;    /* MINRES iterations (all inner sweeps in MIXED)        */
  int32_t iters_outer;    /* refinement sweeps (MIXED), 1 for FP64                */
  double true_relres;     /* ||Y(f - A u)||_2 / ||Y f||_2, computed in FP64 (in
                             the sine basis: of the transformed system, equal
                             to the physical one up to the FP64 rounding of the
                             two sine transforms)                                 */
  double setup_ms;        /* wall time of bltt_setup                              */
  double solve_ms;        /* wall time of the bltt_pminres call                   */
  double c0;              /* Assumption 1(ii) margin of the blocks                */
} bltt_info;

typedef struct bltt_handle bltt_handle;

/*
 * bltt_setup -- validate the blocks, check Assumption 1(ii) (Section 2,
 * Proposition 1) and build the device tables the iteration needs: Laplacian
 * eigenvalues mu_i of every sine mode, the DFTs of alpha^{j/N} p_j and
 * alpha^{j/N} q_j that give the alpha-circulant eigenvalues
 * lambda_i^{(k,alpha)} = sigma_k + mu_i rho_k (eq. (9)), the matvec spectra
 * and the FFT twiddles.  Allocates the Krylov workspace for opt->precision
 * (MIXED also allocates the FP64 refinement vectors).
 *   blk    block description (N entries of p and q)
 *   N      number of time steps (blocks); M must equal m[0]*...*m[dim-1]
 *   alpha  in (0, 1]; the FP64 preconditioner uses it as given.  Everything
 *          that applies the preconditioner in FP32 (the sweeps of BLTT_MIXED,
 *          the FP32 step entry points, the batched sweeps) uses
 *          alpha' = max(alpha, 1e-4) instead: an FP32 time pass scales its
 *          lines by up to 1/alpha around its transforms, so its rounding
 *          grows like eps_32/alpha, and below 1e-4 the sweeps slow down
 *          (and fail to converge at 1e-8).  P_alpha' is an SPD preconditioner
 *          of the same system, and the FP64 refinement solves that system.
 *   opt    options or NULL
 *   stream hipStream_t (void*) for all work of this handle
 *   out    receives the new handle; untouched on error
 * Errors: BLTT_EINVAL, BLTT_EUNSUPPORTED, BLTT_EASSUMPTION, BLTT_ENOMEM,
 * BLTT_EHIP.
 */
int bltt_setup(const bltt_blocks *blk, int64_t N, int64_t M, double alpha,
               const bltt_options *opt, void *stream, bltt_handle **out);

/*
 * bltt_setup_varcoef -- as bltt_setup, for blocks p_k I + q_k L_{a,h} with a
 * variable coefficient a(x) > 0: L_{a,h} = -Delta_{a,h} is the central-
 * difference form of -div(a grad) with zero Dirichlet boundary (Section 5.2,
 * the heat equation with variable coefficients):
 *   (L_{a,h} v)_i = sum_d [a_{d,hi}(i) (v_i - v_{i+e_d}) + a_{d,lo}(i) (v_i - v_{i-e_d})] / h_d^2.
 * The preconditioner is P_alpha of the mean-coefficient system, blocks
 * p_k I + q_k abar L_h (Section 5.2): abar is the constant the caller takes
 * for a (the paper uses the mean of a over the grid points).
 *   face   face[d], d < dim: host arrays of a at the faces along dimension d,
 *          lexicographic with x fastest, extents m_e for e != d and m_d + 1
 *          along d; entry j along d lies between grid points j-1 and j (j = 0
 *          and j = m_d are the boundary faces).  Copied at setup; every
 *          entry must be finite and > 0.
 *   abar   > 0
 * The operator is not diagonalised by the sine transform, so the solver runs
 * in the physical basis whatever opt->basis says (FP64 or MIXED precision);
 * opt->precond must be BLTT_PRECOND_ABAC.  Assumption 1(ii) is checked for
 * the mean-coefficient system.
 * Errors: as bltt_setup; BLTT_EINVAL for a null face array or a coefficient
 * that is not finite and positive.
 */
int bltt_setup_varcoef(const bltt_blocks *blk, const double *const *face, double abar, int64_t N,
                       int64_t M, double alpha, const bltt_options *opt, void *stream,
                       bltt_handle **out);

/*
 * bltt_pminres -- solve A u = f by preconditioned MINRES on Y A u = Y f, from
 * a zero initial guess (Section 5) or, when the handle was set up with
 * opt->initial_guess = 1, from the u_dev passed in.  Stops when
 * ||Y(f - A u)||_2 / ||Y f||_2 <= tol (an initial guess that already meets it
 * returns with zero iterations).
 *   f_dev   FP64 device vector of length N*M (not modified)
 *   tol     relative residual target, > 0
 *   maxit   iteration cap (>= 1); in MIXED it caps the total inner iterations
 *   u_dev   FP64 device vector of length N*M receiving the solution (and
 *           holding the initial guess on entry when so set up); must not
 *           overlap f_dev
 *   iters   host, receives the number of MINRES iterations (may be NULL)
 *   hist    host array of length maxit+1 or NULL; receives |eta_j|/eta_0, the
 *           P^{-1}-norm residual estimate MINRES carries (hist[0] = 1); in
 *           MIXED the inner histories are concatenated, each relative to its
 *           own sweep's start
 *   info    host, receives the report (may be NULL)
 * f = 0 returns BLTT_OK with u = 0 and zero iterations.
 * Errors: BLTT_EINVAL, BLTT_ENAN, BLTT_EBREAKDOWN, BLTT_EHIP; BLTT_NOCONV
 * when maxit is reached.
 */
int bltt_pminres(bltt_handle *h, const double *f_dev, double tol, int32_t maxit,
                 double *u_dev, int32_t *iters, double *hist, bltt_info *info);

/*
 * Step-level entry points: one application of a hot-path operator on device
 * vectors of length N*M, in the precision given (BLTT_FP64: double*,
 * BLTT_FP32: float*).  x_dev and y_dev must not overlap.  They use the
 * handle's workspace for that precision (allocated on first use).
 *
 * bltt_apply_sym:     y = Y A x (Section 2, eq. (4); Section 5.1: FFT
 *                     Toeplitz product along time plus the spatial stencil,
 *                     then the time reversal).
 * bltt_apply_precond: y = P_alpha^{-1} x = C^{-1/2} (C^{-1/2})^* x (Section
 *                     5.1, Steps 1-3 twice: sine transform in space, per mode
 *                     the alpha-scaled Fourier sandwich in time, inverse sine
 *                     transform).
 * bltt_apply_space:   y = (I_N (x) U) x, the orthonormal sine transform of
 *                     every time slice (Steps 1 and 3 of Section 5.1).
 * Errors: BLTT_EINVAL, BLTT_ENOMEM, BLTT_EHIP.
 */
int bltt_apply_sym(bltt_handle *h, int32_t precision, const void *x_dev, void *y_dev);
int bltt_apply_precond(bltt_handle *h, int32_t precision, const void *x_dev, void *y_dev);
int bltt_apply_space(bltt_handle *h, int32_t precision, const void *x_dev, void *y_dev);

/*
 * Sine-coordinate step entry points: one application of a kernel of the
 * default (sine-basis) solve.  Every block p_k I + q_k L_h is diagonal in the
 * orthonormal sine basis (Remark 1): sine mode i sees the scalar lower
 * triangular Toeplitz matrix T_i with first column p + mu_i q, mu_i the
 * eigenvalue of L_h for mode i, and P_alpha^{-1} acts on each mode's time
 * line alone (Section 5.1, Step 2).  These entry points take mode-major
 * vectors: element (i, n) of a sine-coordinate vector sits at i*N + n.
 * Device buffers belong to the caller; outputs must not overlap inputs.  The
 * handle's tables for the precision used are built on first use.  Scalar
 * results are reduced in FP64 on the device and returned through host
 * pointers (each may be NULL).  Variable-coefficient handles
 * (bltt_setup_varcoef) are not sine-diagonal: BLTT_EUNSUPPORTED.
 *
 * bltt_modes_forward:  xhat = (I_N (x) U) x, x time-major FP64 (the ABI
 *                      layout), xhat mode-major FP64; *norm2 = ||x||^2.
 * bltt_modes_backward: x = (I_N (x) U) xhat back to time-major; xhat is
 *                      used as scratch and overwritten.
 * bltt_modes_sym:      q = Y T z per mode (Section 2, eq. (4), in sine
 *                      coordinates); *dot = <q, z>.  precision BLTT_FP64
 *                      (double*) or BLTT_FP32 (float*).
 * bltt_modes_lanczos:  vhat = coef[0] q + coef[1] v1 + coef[2] v2 (a NULL v1
 *                      or v2 drops its term; coef NULL means 1, 0, 0),
 *                      zout = P_alpha^{-1} vhat (eqs. (8)-(13), both
 *                      half-solves), vout = vhat when vout is non-NULL, and
 *                      *dot = <vhat, zout>: the fused Lanczos update and
 *                      preconditioner of one MINRES iteration.  precision
 *                      BLTT_FP64 (all double*), BLTT_FP32 (all float*), or
 *                      BLTT_MIXED (q double*, vout/zout float*, v1 = v2 =
 *                      NULL: the start of an FP32 refinement sweep).
 * bltt_modes_resid:    FP64 refinement residual: first u += scale *
 *                      sum_{j<k} y[j] z[j] (k FP32 mode-major vectors z[j],
 *                      a host array of device pointers, and k host weights y;
 *                      k = 0 skips it, at most 32), then r = Y (fhat - T u)
 *                      and *norm2 = ||r||^2.  u is updated in place.
 * Errors: BLTT_EINVAL, BLTT_EUNSUPPORTED, BLTT_ENOMEM, BLTT_EHIP.
 */
int bltt_modes_forward(bltt_handle *h, const double *x_dev, double *xhat_dev, double *norm2);
int bltt_modes_backward(bltt_handle *h, double *xhat_dev, double *x_dev);
int bltt_modes_sym(bltt_handle *h, int32_t precision, const void *z_dev, void *q_dev, double *dot);
int bltt_modes_lanczos(bltt_handle *h, int32_t precision, const void *q_dev, const void *v1_dev,
                       const void *v2_dev, const double *coef, void *vout_dev, void *zout_dev, double *dot);
int bltt_modes_resid(bltt_handle *h, const double *fhat_dev, double *u_dev, double *r_dev,
                     const float *const *z_dev, const double *y, int32_t k, double scale, double *norm2);

/*
 * bltt_modes_lanczos_noalloc -- bltt_modes_lanczos for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments, same kernels, same
 * results, and no hipMalloc, hipFree or other allocating call.  Its partial
 * sums, their reduction, the coefficients and the reduced <vhat, zout> live in
 * a static device array of the library, one per GPU (about 130 KiB, held
 * until the process ends); the caller passes inputs and outputs.
 *   - The handle must already hold the tables of `precision` (built by
 *     bltt_setup for its own precision, FP64 tables always; or by one call of
 *     bltt_modes_lanczos): otherwise BLTT_EINVAL.
 *   - At most 16384 partial sums per launch: FP32 and mixed always fit (one
 *     per persistent workgroup); FP64 fits when ceil(M / (2 NL)) <= 16384,
 *     NL = 256 / (N / min(N, 16)) mode-line pairs per workgroup (e.g. M up to
 *     131072 at N = 1024).  Larger systems give BLTT_EUNSUPPORTED.
 *   - Every call on one GPU uses that GPU's array, whatever the handle; calls
 *     that overlap in time on one GPU (other host threads, other streams) race
 *     and must be serialised by the caller.  Nothing in the array needs to
 *     start at zero: each call writes what it reads.
 * Errors: as bltt_modes_lanczos.
 */
int bltt_modes_lanczos_noalloc(bltt_handle *h, int32_t precision, const void *q_dev, const void *v1_dev,
                               const void *v2_dev, const double *coef, void *vout_dev, void *zout_dev,
                               double *dot);

/*
 * Per-kernel timing of the hot path.  While enabled, every kernel launch the
 * handle makes is bracketed by HIP events on the handle's stream and its
 * algorithmic traffic (bytes the step must read and write at least once,
 * e.g. 2*N*M*sizeof(real) for the time pass) is accumulated per kernel class.
 * bltt_profile_enable(h, 1) clears the counters and starts recording;
 * bltt_profile_enable(h, 0) stops.  bltt_profile_read synchronises the
 * stream and returns, for one kernel class, the number of launches, their
 * summed duration in milliseconds and the summed algorithmic bytes (any
 * output pointer may be NULL).
 * Errors: BLTT_EINVAL (null handle, class out of range), BLTT_EHIP.
 */
enum bltt_kernel_class {
  BLTT_K_MATVEC = 0,        /* q = Y A z, FFT or direct form                     */
  BLTT_K_DST_X_VUPD = 1,    /* Lanczos update + sine transform along x           */
  BLTT_K_DST_STRIDED = 2,   /* sine transform along y / z                        */
  BLTT_K_TIME = 3,          /* alpha-circulant time pass of the preconditioner   */
  BLTT_K_DST_X_DOT = 4,     /* inverse sine transform along x + dot product      */
  BLTT_K_WX = 5,            /* MINRES direction and iterate update               */
  BLTT_K_RESID64 = 6,       /* FP64 residual Y(f - A u)                          */
  BLTT_K_OTHER = 7,         /* right-hand side, casts, fills, scalar kernels     */
  BLTT_K_TIME_START = 8,    /* time pass of a Krylov start (z_1 = P^{-1} b, sine
                               basis); BLTT_K_TIME counts the iterations' passes */
  BLTT_K_COUNT = 9
};
int bltt_profile_enable(bltt_handle *h, int32_t enable);
int bltt_profile_read(bltt_handle *h, int32_t kernel_class, int64_t *launches, double *total_ms,
                      double *bytes);

/*
 * Batched solves: many independent instances of uneven size and blocks, each
 * with nrhs right-hand sides, solved together (mixed precision, sine basis:
 * the BLTT_MIXED path of bltt_pminres).  Instances with the same N, dim, m and
 * h form a shape class whose systems share every launch of a phase (per-
 * instance tables, one partial sum per tile and system); classes run on
 * streams of their own.  Each MINRES iteration of a class is replayed from a
 * HIP graph captured once per position in the sweep; at setup a few timed
 * launches choose each class's workgroup size and radix plan (or the plan
 * cache supplies them).  An FP32 sweep stops after at
 * most 5 iterations (the refinement loop continues with a new sweep).
 *
 * bltt_setup_batched -- validate and prepare count instances.
 *   blk[i], N[i], M[i], alpha[i]   instance i, as for bltt_setup (p and q
 *                                  copied; N[i] and 2(m_d+1) powers of two)
 *   nrhs                           right-hand sides per instance (>= 1)
 *   opt                            NULL or precision BLTT_MIXED, basis
 *                                  BLTT_BASIS_SINE (others: BLTT_EUNSUPPORTED);
 *                                  inner_tol, max_refine, plan_cache and
 *                                  fft_plan as for bltt_setup (each class's
 *                                  workgroup size and radix plan are tuned
 *                                  together)
 *   stream                         hipStream_t the solves are ordered on
 *   out                            receives the batch handle
 * Errors: as bltt_setup; BLTT_ENOMEM when the workspace of all classes does
 * not fit (split the batch).
 *
 * bltt_pminres_batched -- solve all count*nrhs systems to tol.  System
 * g = i*nrhs + r is instance i with right-hand side r:
 *   f_dev[g], u_dev[g]   FP64 device vectors of length N[i]*M[i] (host
 *                        arrays of device pointers); u_dev[g] receives the
 *                        solution and must not overlap any f_dev
 *   iters[g]             host, may be NULL: inner iterations of system g
 *   hist                 host, may be NULL: count*nrhs rows of maxit+1
 *                        residual estimates, as bltt_pminres
 *   info[g]              host, may be NULL: per-system report (solve_ms is
 *                        the wall time of the whole batched call)
 * Returns BLTT_OK when every system reached tol, BLTT_NOCONV if one did not,
 * or the first error.
 *
 * bltt_batch_classes -- number of shape classes and (tpb, may be NULL, room
 * for that many) the workgroup size the setup chose for each.
 */
typedef struct bltt_batch bltt_batch;
int bltt_setup_batched(const bltt_blocks *blk, const int64_t *N, const int64_t *M, const double *alpha,
                       int32_t count, int32_t nrhs, const bltt_options *opt, void *stream, bltt_batch **out);
int bltt_pminres_batched(bltt_batch *b, const double *const *f_dev, double tol, int32_t maxit,
                         double *const *u_dev, int32_t *iters, double *hist, bltt_info *info);
int bltt_batch_classes(const bltt_batch *b, int32_t *nclasses, int32_t *tpb);
void bltt_destroy_batched(bltt_batch *b);  /* the same as bltt_destroy on a batch */

/*
 * bltt_plan_info -- the kernel plans a handle runs with: radix plans of the
 * FP32 time pass and N-point matvec (0 or 1), workgroups of the persistent
 * FP32 time pass, workgroups of the FP32 N-point matvec (0: one per tile of
 * modes, else that many persistent ones), and where they came from
 * (bltt_plan_source).  Any output pointer may be NULL.  Errors: BLTT_EINVAL.
 * bltt_batch_plans -- per shape class of a batch: the radix plan (0 or 1) the
 * setup chose with the workgroup size of bltt_batch_classes (room for that
 * many classes; NULL allowed).  Errors: BLTT_EINVAL.
 */
int bltt_plan_info(const bltt_handle *h, int32_t *time_plan, int32_t *cs_plan, int64_t *time_blocks,
                   int64_t *cs_blocks, int32_t *source);
int bltt_batch_plans(const bltt_batch *b, int32_t *plans);

/* Release all device memory, tables, graphs and streams of a handle from
 * bltt_setup, bltt_setup_varcoef or bltt_setup_batched (the handle types are
 * told apart by a tag the library keeps in each); NULL is a no-op.  The
 * handle must not be used afterwards. */
void bltt_destroy(void *handle);

/* Static message for a status code. */
const char *bltt_strerror(int code);

/* Library version string. */
const char *bltt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLTT_H */
