// Streaming kernels (right-hand side, MINRES direction/iterate update,
// refinement casts) and the single-workgroup scalar kernel.
#include <mutex>

#include "launchers.hpp"

namespace bltt {

template <typename TO>
__global__ __launch_bounds__(TPB_EW) void k_rhs(const double* __restrict__ f, TO* __restrict__ b, int64_t N,
                                                int64_t M, double scale, double* __restrict__ partials) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  rhs_body<TO>(ctx, red, f, b, N, M, scale, partials);
}

template <typename T, typename TX>
__global__ __launch_bounds__(TPB_EW) void k_wx(const T* __restrict__ Z, T* __restrict__ Wa, const T* __restrict__ Wb,
                                               TX* __restrict__ X, int64_t n, const double* __restrict__ coef) {
  DevCtx ctx = make_ctx();
  wx_body<T, TX>(ctx, Z, Wa, Wb, X, n, coef);
}

template <typename T>
__global__ __launch_bounds__(TPB_EW) void k_fill(T* __restrict__ x, int64_t n, T val) {
  DevCtx ctx = make_ctx();
  fill_body<T>(ctx, x, n, val);
}

template <typename TI, typename TO>
__global__ __launch_bounds__(TPB_EW) void k_scale_cast(const TI* __restrict__ x, TO* __restrict__ y, int64_t n,
                                                       const double* __restrict__ sptr, int invert) {
  DevCtx ctx = make_ctx();
  scale_cast_body<TI, TO>(ctx, x, y, n, sptr, invert);
}

template <typename TD>
__global__ __launch_bounds__(TPB_EW) void k_axpy64(double* __restrict__ u, const TD* __restrict__ d, int64_t n,
                                                   const double* __restrict__ sptr) {
  DevCtx ctx = make_ctx();
  axpy64_body<TD>(ctx, u, d, n, sptr);
}

template <typename T, bool Q1>
__global__ __launch_bounds__(TPB_EW) void k_resid_stencil(T* __restrict__ r, VupdStencil<T> st,
                                                          double* __restrict__ partials) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  resid_stencil_body<T, Q1>(ctx, red, r, st, partials);
}

__global__ __launch_bounds__(TPB_EW) void k_reduce(const double* __restrict__ in, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  reduce_chunk_body(ctx, red, in, n, out);
}

// mirror: null, or the host-mapped pinned copy of the state that the host
// polls instead of synchronising the stream.  Thread 0 (which made every
// write to *st) copies the state, then, after a system-scope fence, bumps
// st->seq and stores it into mirror->seq last, so a host that sees the new
// sequence number sees the whole state.
__global__ __launch_bounds__(TPB_EW) void k_scalar(int phase, SolverState* __restrict__ st,
                                                   const double* __restrict__ partials, int64_t np,
                                                   const double* __restrict__ aux, int64_t naux,
                                                   double* __restrict__ hist, ZBasis zb, SolverState* mirror) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  scalar_body(ctx, red, phase, st, partials, np, aux, naux, hist, zb);
  if (mirror && ctx.tid == 0) {
    const int32_t seq = st->seq + 1;
    st->seq = seq;
    SolverState copy = *st;
    copy.seq = seq - 1;  // the mirror's current number, unchanged until the fence below
    *mirror = copy;
    __threadfence_system();
    __hip_atomic_store(&mirror->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// One time step (N = 1): A = A_(0) = p_0 I + q_0 L_h is diagonal in sine
// coordinates, lambda_i = p_0 + q_0 mu_i.  solve: uhat = fhat / lambda (the
// single-block system, Section 3 with N = 1); then r = fhat - lambda uhat and
// one partial sum of ||r||^2 per workgroup.
__global__ __launch_bounds__(TPB_EW) void k_single_step(const double* __restrict__ fhat, double* __restrict__ uhat,
                                                        int64_t M, const double* __restrict__ mu, double p0,
                                                        double q0, int solve, double* __restrict__ partials) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  double part = 0.0;
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t i = (int64_t)ctx.bid * TPB_EW + ctx.tid; i < M; i += stride) {
    const double lam = p0 + q0 * mu[i];
    double u;
    if (solve) {
      u = fhat[i] / lam;
      uhat[i] = u;
    } else {
      u = uhat[i];
    }
    const double r = fhat[i] - lam * u;
    part += r * r;
  }
  const double sum = block_sum<TPB_EW>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

hipError_t launch_single_step(const double* fhat, double* uhat, int64_t M, const double* mu, double p0, double q0,
                              int solve, double* partials, int64_t* nparts, hipStream_t s) {
  const int64_t blocks = ew_blocks(M);
  if (nparts) *nparts = blocks;
  hipLaunchKernelGGL(k_single_step, dim3((unsigned)blocks), dim3(TPB_EW), 0, s, fhat, uhat, M, mu, p0, q0, solve,
                     partials);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(TPB_EW) void k_combine(double* __restrict__ u, ZList<T> zl,
                                                    const double* __restrict__ y, const double* __restrict__ sptr,
                                                    int64_t n) {
  DevCtx ctx = make_ctx();
  combine_body<T>(ctx, u, zl, y, sptr, n);
}

template <typename T>
hipError_t launch_combine(double* u, const ZList<T>& zl, const double* y, const double* sptr, int64_t n,
                          hipStream_t s) {
  if (zl.k < 0 || zl.k > ZB_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_combine<T>, dim3((unsigned)ew_blocks(n)), dim3(TPB_EW), 0, s, u, zl, y, sptr, n);
  return hipGetLastError();
}
template hipError_t launch_combine<float>(double*, const ZList<float>&, const double*, const double*, int64_t,
                                          hipStream_t);

template <typename T>
hipError_t launch_resid_stencil(T* r, const VupdStencil<T>& st, int64_t nlines, double* partials, int64_t* nparts,
                                hipStream_t s) {
  if (nlines > 2147483647LL) return hipErrorInvalidValue;
  if (nparts) *nparts = nlines;
  if (st.qtaps <= 1)
    hipLaunchKernelGGL((k_resid_stencil<T, true>), dim3((unsigned)nlines), dim3(TPB_EW), 0, s, r, st, partials);
  else
    hipLaunchKernelGGL((k_resid_stencil<T, false>), dim3((unsigned)nlines), dim3(TPB_EW), 0, s, r, st, partials);
  return hipGetLastError();
}
template hipError_t launch_resid_stencil<float>(float*, const VupdStencil<float>&, int64_t, double*, int64_t*,
                                                hipStream_t);
template hipError_t launch_resid_stencil<double>(double*, const VupdStencil<double>&, int64_t, double*, int64_t*,
                                                 hipStream_t);

template <typename TO>
hipError_t launch_rhs(const double* f, TO* b, int64_t N, int64_t M, double scale, double* partials,
                      int64_t* nparts, hipStream_t s) {
  const int64_t blocks = ew_blocks(N * M);
  if (nparts) *nparts = blocks;
  hipLaunchKernelGGL((k_rhs<TO>), dim3((unsigned)blocks), dim3(TPB_EW), 0, s, f, b, N, M, scale, partials);
  return hipGetLastError();
}
template <typename T, typename TX>
hipError_t launch_wx(const T* Z, T* Wa, const T* Wb, TX* X, int64_t n, const double* coef, hipStream_t s) {
  hipLaunchKernelGGL((k_wx<T, TX>), dim3((unsigned)ew_blocks(n)), dim3(TPB_EW), 0, s, Z, Wa, Wb, X, n, coef);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(T* x, int64_t n, T val, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)ew_blocks(n)), dim3(TPB_EW), 0, s, x, n, val);
  return hipGetLastError();
}
template <typename TI, typename TO>
hipError_t launch_scale_cast(const TI* x, TO* y, int64_t n, const double* sptr, int invert, hipStream_t s) {
  hipLaunchKernelGGL((k_scale_cast<TI, TO>), dim3((unsigned)ew_blocks(n)), dim3(TPB_EW), 0, s, x, y, n, sptr,
                     invert);
  return hipGetLastError();
}
template <typename TD>
hipError_t launch_axpy64(double* u, const TD* d, int64_t n, const double* sptr, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy64<TD>), dim3((unsigned)ew_blocks(n)), dim3(TPB_EW), 0, s, u, d, n, sptr);
  return hipGetLastError();
}
hipError_t launch_scalar(int phase, SolverState* st, const double* partials, int64_t np, const double* aux,
                         int64_t naux, double* hist, double* scratch, int64_t scratch_half, ZBasis zb,
                         hipStream_t s, SolverState* mirror) {
  // long partial-sum arrays go through one wide first stage (into scratch,
  // aux at scratch + scratch_half)
  if (np > RED_CHUNK) {
    const int64_t nb = (np + RED_CHUNK - 1) / RED_CHUNK;
    if (nb > scratch_half) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)nb), dim3(TPB_EW), 0, s, partials, np, scratch);
    partials = scratch;
    np = nb;
  }
  if (aux && naux > RED_CHUNK) {
    const int64_t nb = (naux + RED_CHUNK - 1) / RED_CHUNK;
    if (nb > scratch_half) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)nb), dim3(TPB_EW), 0, s, aux, naux, scratch + scratch_half);
    aux = scratch + scratch_half;
    naux = nb;
  }
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(TPB_EW), 0, s, phase, st, partials, np, aux, naux, hist, zb, mirror);
  return hipGetLastError();
}

template hipError_t launch_rhs<float>(const double*, float*, int64_t, int64_t, double, double*, int64_t*,
                                      hipStream_t);
template hipError_t launch_rhs<double>(const double*, double*, int64_t, int64_t, double, double*, int64_t*,
                                       hipStream_t);
template hipError_t launch_wx<float, float>(const float*, float*, const float*, float*, int64_t, const double*,
                                            hipStream_t);
template hipError_t launch_wx<double, double>(const double*, double*, const double*, double*, int64_t,
                                              const double*, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_scale_cast<double, float>(const double*, float*, int64_t, const double*, int,
                                                     hipStream_t);
template hipError_t launch_scale_cast<double, double>(const double*, double*, int64_t, const double*, int,
                                                      hipStream_t);
template hipError_t launch_axpy64<float>(double*, const float*, int64_t, const double*, hipStream_t);
template hipError_t launch_axpy64<double>(double*, const double*, int64_t, const double*, hipStream_t);

hipError_t configure_time_kernels();
hipError_t configure_matvec_kernels();
hipError_t configure_dst_kernels();
hipError_t configure_spec_kernels();
hipError_t configure_cs_kernels();
hipError_t configure_batch_kernels();

hipError_t configure_kernels_once() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] { err = configure_kernels(); });
  return err;
}

hipError_t configure_kernels() {
  hipError_t e;
  if ((e = configure_time_kernels()) != hipSuccess) return e;
  if ((e = configure_matvec_kernels()) != hipSuccess) return e;
  if ((e = configure_dst_kernels()) != hipSuccess) return e;
  if ((e = configure_spec_kernels()) != hipSuccess) return e;
  if ((e = configure_cs_kernels()) != hipSuccess) return e;
  return configure_batch_kernels();
}

}  // namespace bltt
