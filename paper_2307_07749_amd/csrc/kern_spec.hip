// Lanczos update fused with the time pass of the preconditioner, for MINRES in
// sine coordinates (mode-major vectors): one workgroup per 2*NL sine modes.
#include <algorithm>

#include "launchers.hpp"

namespace bltt {

// exchange lines + reduction slots (+ the LDS twiddle table of the FP32 pass)
template <typename T, int L>
constexpr size_t upd_lds_bytes() { return fft_lds_bytes<T, FK_SPEC>(L) + upd_twl_bytes<T, L>(); }
static_assert(2 * upd_lds_bytes<float, 1024>() <= 160 * 1024, "two workgroups per CU");

template <typename T, int L, typename TQ, bool FULL, bool PREC, int PLAN>
__global__ __attribute__((amdgpu_waves_per_eu(min_waves_upd<T>(), max_waves_fft<T>()))) __launch_bounds__((tpb_fft<T, FK_SPEC>()), waves_fft<T>()) void k_time_upd(
    const TQ* __restrict__ Q, const T* __restrict__ V1, const T* __restrict__ V2, T* __restrict__ Vout,
    T* __restrict__ Zout, int64_t M, TimeTables<T> tb, const double* __restrict__ coef,
    double* __restrict__ partials, int qrev) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = tpb_fft<T, FK_SPEC>() / (L / fft_V(L));
  using F = LineFft<T, L, NL, false, LAST_PAIRED>;
  DevCtx ctx = make_ctx();
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  time_upd_body<T, L, TQ, FULL, true, PREC, PLAN>(ctx, reinterpret_cast<cx<T>*>(smem), red, Q, V1, V2, Vout, Zout, M, tb,
                                            coef, partials, qrev != 0);
}

template <typename T, typename TQ, int L, int PLAN = 0>
static hipError_t go_upd(bool full, bool prec, bool qrev, const TQ* Q, const T* V1, const T* V2, T* Vout, T* Zout, int64_t M,
                         const TimeTables<T>& tb, const double* coef, double* partials, int64_t max_blocks,
                         int64_t* nparts, hipStream_t s) {
  const int64_t blocks = upd_blocks<T>(L, M, max_blocks);
  const size_t lds = upd_lds_bytes<T, L>();
  if (nparts) *nparts = blocks;
  if (!prec) {
    // no preconditioner (MINRES-I): FP64 only
    if constexpr (sizeof(T) == 8) {
      if (full)
        hipLaunchKernelGGL((k_time_upd<T, L, TQ, true, false, 0>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_SPEC>()),
                           lds, s, Q, V1, V2, Vout, Zout, M, tb, coef, partials, qrev ? 1 : 0);
      else
        hipLaunchKernelGGL((k_time_upd<T, L, TQ, false, false, 0>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_SPEC>()),
                           lds, s, Q, V1, V2, Vout, Zout, M, tb, coef, partials, qrev ? 1 : 0);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (full)
    hipLaunchKernelGGL((k_time_upd<T, L, TQ, true, true, PLAN>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_SPEC>()),
                       lds, s, Q, V1, V2, Vout, Zout, M, tb, coef, partials, qrev ? 1 : 0);
  else
    hipLaunchKernelGGL((k_time_upd<T, L, TQ, false, true, PLAN>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_SPEC>()),
                       lds, s, Q, V1, V2, Vout, Zout, M, tb, coef, partials, qrev ? 1 : 0);
  return hipGetLastError();
}

template <typename T, typename TQ>
hipError_t launch_time_upd(int L, bool full, bool prec, const TQ* Q, const T* V1, const T* V2, T* Vout, T* Zout, int64_t M,
                           const TimeTables<T>& tb, const double* coef, double* partials, int64_t max_blocks,
                           int64_t* nparts, hipStream_t s, bool qrev, int plan) {
  if (full && (!V1 || !V2)) return hipErrorInvalidValue;
  if (full && qrev) return hipErrorInvalidValue;
  // the alternative radix plan exists for the preconditioned FP32 pass at L = 512, 1024
  if (plan != 0 && (plan != 1 || sizeof(T) != 4 || !prec || !fft_plan_alt(L))) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 4) {
    if (plan == 1 && L == 512)
      return go_upd<T, TQ, 512, 1>(full, prec, qrev, Q, V1, V2, Vout, Zout, M, tb, coef, partials, max_blocks, nparts, s);
    if (plan == 1 && L == 1024)
      return go_upd<T, TQ, 1024, 1>(full, prec, qrev, Q, V1, V2, Vout, Zout, M, tb, coef, partials, max_blocks, nparts,
                                    s);
  }
  switch (L) {
#define BLTT_CASE(LL) \
  case LL: return go_upd<T, TQ, LL>(full, prec, qrev, Q, V1, V2, Vout, Zout, M, tb, coef, partials, max_blocks, nparts, s);
    BLTT_CASE(2) BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64)
    BLTT_CASE(128) BLTT_CASE(256) BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}

#define BLTT_INST(T, TQ)                                                                                      \
  template hipError_t launch_time_upd<T, TQ>(int, bool, bool, const TQ*, const T*, const T*, T*, T*, int64_t,      \
                                             const TimeTables<T>&, const double*, double*, int64_t, int64_t*,  \
                                             hipStream_t, bool, int);
BLTT_INST(float, float)
BLTT_INST(float, double)
BLTT_INST(double, double)
#undef BLTT_INST

template <typename T, typename TQ, int L>
static hipError_t attr_upd() {
  const int bytes = (int)upd_lds_bytes<T, L>();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_upd<T, L, TQ, true, true, 0>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_upd<T, L, TQ, false, true, 0>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  if constexpr (sizeof(T) == 4 && fft_plan_alt(L)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_upd<T, L, TQ, true, true, 1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_upd<T, L, TQ, false, true, 1>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  }
  if (sizeof(T) != 8) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_upd<T, L, TQ, true, false, 0>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_upd<T, L, TQ, false, false, 0>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t configure_spec_kernels() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR(L)                                                  \
  if ((e = attr_upd<float, float, L>()) != hipSuccess) return e;     \
  if ((e = attr_upd<float, double, L>()) != hipSuccess) return e;    \
  if ((e = attr_upd<double, double, L>()) != hipSuccess) return e;
  BLTT_ATTR(2) BLTT_ATTR(4) BLTT_ATTR(8) BLTT_ATTR(16) BLTT_ATTR(32) BLTT_ATTR(64)
  BLTT_ATTR(128) BLTT_ATTR(256) BLTT_ATTR(512) BLTT_ATTR(1024) BLTT_ATTR(2048)
#undef BLTT_ATTR
  return e;
}

}  // namespace bltt
