// Batched sine-basis kernels (bodies in bltt_kernels.hpp): many systems of
// one shape (N, grid) whose mode-major vectors sit back to back; one launch
// covers the tiles of every system.
#include <algorithm>

#include "launchers.hpp"

namespace bltt {

template <int L, typename TQ, bool FULL, int TPB, int PLAN>
__global__ __attribute__((amdgpu_waves_per_eu(1, max_waves_fft<float>()))) __launch_bounds__(TPB, 1) void k_bt_upd(
    const TQ* __restrict__ Q, const float* __restrict__ V1, const float* __restrict__ V2, float* __restrict__ Vout,
    float* __restrict__ Zout, BatchVec bv, BatchTabs bt, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  DevCtx ctx = make_ctx();
  bt_upd_body<L, TQ, FULL, TPB, PLAN>(ctx, smem, Q, V1, V2, Vout, Zout, bv, bt, partials);
}

template <int L, int TPB, int PLAN>
__global__ __attribute__((amdgpu_waves_per_eu(1, max_waves_fft<float>()))) __launch_bounds__(TPB, 1) void k_bt_cs(
    const float* __restrict__ Z, float* __restrict__ Q, BatchVec bv, BatchTabs bt, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  DevCtx ctx = make_ctx();
  bt_cs_body<L, TPB, PLAN>(ctx, smem, Z, Q, bv, bt, partials);
}

template <int L2, bool R32 = false>
__global__ __attribute__((amdgpu_waves_per_eu(2, max_waves_fft<double>()))) __launch_bounds__((tpb_fft<double, fk_mv<true, L2>()>()), 1) void k_bt_resid(
    double* const* __restrict__ u, double* __restrict__ R, const double* __restrict__ Fh, BatchVec bv, BatchTabs bt,
    IterUpd pool, const double* __restrict__ zb, int K, int64_t T2, double* __restrict__ partials,
    float* __restrict__ r32) {
  extern __shared__ __align__(16) unsigned char smem[];
  DevCtx ctx = make_ctx();
  bt_resid_body<L2, R32>(ctx, smem, u, R, Fh, bv, bt, pool, zb, K, T2, partials, r32);
}

__global__ __launch_bounds__(TPB_EW) void k_bt_scalar(int phase, SolverState* __restrict__ states,
                                                      const double* __restrict__ partials, int64_t T,
                                                      double* __restrict__ hist, int64_t hist_stride,
                                                      double* __restrict__ zb, int K, double inner_tol, int cap,
                                                      const int* __restrict__ active,
                                                      const double* __restrict__ etol) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  batch_scalar_body(ctx, red, phase, states, partials, T, hist, hist_stride, zb, K, inner_tol, cap, active, etol);
}

__global__ __launch_bounds__(TPB_EW) void k_bt_rhs(const double* __restrict__ f, double* __restrict__ b, int log2N,
                                                   int64_t n, int64_t BPS, double* __restrict__ partials) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  bt_rhs_body(ctx, red, f, b, log2N, n, BPS, partials);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int L, int TPB, int PLAN>
static hipError_t go_bt(int which, const void* Q, const float* V1, const float* V2, float* Vout, float* Z,
                        float* Qout, const BatchVec& bv, const BatchTabs& bt, double* partials, hipStream_t s) {
  const int64_t blocks = bv.T * bv.S;
  const size_t lds = bt_upd_lds<L, TPB>(), lds_cs = bt_cs_lds<L, TPB>();
  switch (which) {
    case BT_START:
      hipLaunchKernelGGL((k_bt_upd<L, double, false, TPB, PLAN>), dim3((unsigned)blocks), dim3(TPB), lds, s,
                         (const double*)Q, V1, V2, Vout, Z, bv, bt, partials);
      break;
    case BT_UPD:
      hipLaunchKernelGGL((k_bt_upd<L, float, true, TPB, PLAN>), dim3((unsigned)blocks), dim3(TPB), lds, s, (const float*)Q,
                         V1, V2, Vout, Z, bv, bt, partials);
      break;
    case BT_START32:
      hipLaunchKernelGGL((k_bt_upd<L, float, false, TPB, PLAN>), dim3((unsigned)blocks), dim3(TPB), lds, s,
                         (const float*)Q, V1, V2, Vout, Z, bv, bt, partials);
      break;
    case BT_MATVEC:
      hipLaunchKernelGGL((k_bt_cs<L, TPB, PLAN>), dim3((unsigned)blocks), dim3(TPB), lds_cs, s,
                         (const float*)Z, Qout, bv, bt, partials);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bt(int which, int L, int tpb, int plan, const void* Q, const float* V1, const float* V2,
                     float* Vout, float* Z, float* Qout, const BatchVec& bv, const BatchTabs& bt, double* partials,
                     hipStream_t s) {
  if (plan != 0 && (plan != 1 || !fft_plan_alt(L))) return hipErrorInvalidValue;
#define BLTT_CASE(LL)                                                                                       \
  case LL:                                                                                                  \
    if constexpr (fft_plan_alt(LL)) {                                                                       \
      if (plan == 1 && tpb == 256) return go_bt<LL, 256, 1>(which, Q, V1, V2, Vout, Z, Qout, bv, bt, partials, s); \
      if (plan == 1 && tpb == 512) return go_bt<LL, 512, 1>(which, Q, V1, V2, Vout, Z, Qout, bv, bt, partials, s); \
    }                                                                                                       \
    if (tpb == 256) return go_bt<LL, 256, 0>(which, Q, V1, V2, Vout, Z, Qout, bv, bt, partials, s);       \
    if constexpr (LL >= 32)                                                                                 \
      if (tpb == 512) return go_bt<LL, 512, 0>(which, Q, V1, V2, Vout, Z, Qout, bv, bt, partials, s);     \
    return hipErrorInvalidValue;
  switch (L) {
    BLTT_CASE(2) BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64)
    BLTT_CASE(128) BLTT_CASE(256) BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
  }
#undef BLTT_CASE
  return hipErrorInvalidValue;
}

int64_t bt_tiles(int L, int tpb, int64_t M) {
  const int64_t nl = tpb / (L / (L < 16 ? L : 16));
  return (M + 2 * nl - 1) / (2 * nl);
}

template <int L2>
static hipError_t go_bt_resid(double* const* u, double* R, const double* Fh, const BatchVec& bv, const BatchTabs& bt,
                              const ZPool& pool, const double* zb, int K, int u_zero, double* partials,
                              int64_t* T2out, float* r32, hipStream_t s) {
  if (r32 && !bv.bscale) return hipErrorInvalidValue;
  IterUpd up{};
  for (int i = 0; i < ZB_MAX; ++i) up.z[i] = i < K ? pool.z[i] : nullptr;
  up.k = 0;
  up.u_zero = u_zero;
  constexpr int FK = fk_mv<true, L2>();
  const int64_t T2 = fft_tiles<double, FK>(L2, bv.M);
  if (T2out) *T2out = T2;
  const size_t lds = fft_lds_bytes<double, FK>(L2);
  if (r32)
    hipLaunchKernelGGL((k_bt_resid<L2, true>), dim3((unsigned)(T2 * bv.S)), dim3(tpb_fft<double, FK>()), lds, s, u, R,
                       Fh, bv, bt, up, zb, K, T2, partials, r32);
  else
    hipLaunchKernelGGL((k_bt_resid<L2>), dim3((unsigned)(T2 * bv.S)), dim3(tpb_fft<double, FK>()), lds, s, u, R, Fh,
                       bv, bt, up, zb, K, T2, partials, nullptr);
  return hipGetLastError();
}

hipError_t launch_bt_resid(int L2, double* const* u, double* R, const double* Fh, const BatchVec& bv,
                           const BatchTabs& bt, const ZPool& pool, const double* zb, int K, int u_zero,
                           double* partials, int64_t* T2, float* r32, hipStream_t s) {
  switch (L2) {
#define BLTT_CASE(LL) \
  case LL: return go_bt_resid<LL>(u, R, Fh, bv, bt, pool, zb, K, u_zero, partials, T2, r32, s);
    BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64) BLTT_CASE(128)
    BLTT_CASE(256) BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048) BLTT_CASE(4096)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bt_scalar(int phase, const BatchVec& bv, const double* partials, int64_t T, double* hist,
                            int64_t hist_stride, double* zb, int K, double inner_tol, int cap, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_scalar, dim3((unsigned)bv.S), dim3(TPB_EW), 0, s, phase, bv.states, partials, T, hist,
                     hist_stride, zb, K, inner_tol, cap, bv.active, bv.etol);
  return hipGetLastError();
}

hipError_t launch_bt_rhs(const double* f, double* b, int64_t N, const BatchVec& bv, double* partials, int64_t* BPS,
                         hipStream_t s) {
  int log2N = 0;
  while (((int64_t)1 << log2N) < N) ++log2N;
  if (((int64_t)1 << log2N) != N) return hipErrorInvalidValue;
  const int64_t bps = std::min<int64_t>(ew_blocks(bv.n), 1024);
  if (BPS) *BPS = bps;
  hipLaunchKernelGGL(k_bt_rhs, dim3((unsigned)(bps * bv.S)), dim3(TPB_EW), 0, s, f, b, log2N, bv.n, bps, partials);
  return hipGetLastError();
}

template <int L, int TPB, int PLAN = 0>
static hipError_t attr_bt() {
  const int bytes = (int)bt_upd_lds<L, TPB>();
  hipError_t e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_upd<L, double, false, TPB, PLAN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_upd<L, float, true, TPB, PLAN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_upd<L, float, false, TPB, PLAN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_cs<L, TPB, PLAN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bt_cs_lds<L, TPB>())) != hipSuccess)
    return e;
  if constexpr (PLAN == 0 && fft_plan_alt(L)) return attr_bt<L, TPB, 1>();
  return hipSuccess;
}
template <int L2>
static hipError_t attr_bt_resid() {
  const int bytes = (int)fft_lds_bytes<double, fk_mv<true, L2>()>(L2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_resid<L2>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_resid<L2, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t configure_batch_kernels() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR(L)                                                   \
  if ((e = attr_bt<L, 256>()) != hipSuccess) return e;                 \
  if constexpr (L >= 32)                                               \
    if ((e = attr_bt<L, 512>()) != hipSuccess) return e;
  BLTT_ATTR(2) BLTT_ATTR(4) BLTT_ATTR(8) BLTT_ATTR(16) BLTT_ATTR(32) BLTT_ATTR(64)
  BLTT_ATTR(128) BLTT_ATTR(256) BLTT_ATTR(512) BLTT_ATTR(1024) BLTT_ATTR(2048)
#undef BLTT_ATTR
#define BLTT_ATTR2(L) \
  if ((e = attr_bt_resid<L>()) != hipSuccess) return e;
  BLTT_ATTR2(4) BLTT_ATTR2(8) BLTT_ATTR2(16) BLTT_ATTR2(32) BLTT_ATTR2(64) BLTT_ATTR2(128)
  BLTT_ATTR2(256) BLTT_ATTR2(512) BLTT_ATTR2(1024) BLTT_ATTR2(2048) BLTT_ATTR2(4096)
#undef BLTT_ATTR2
  return e;
}

}  // namespace bltt
