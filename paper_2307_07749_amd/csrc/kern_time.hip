// Time pass of the ABAC preconditioner: one workgroup per 2*NL sine modes.
#include "launchers.hpp"

namespace bltt {

template <typename T, int L>
__global__ __attribute__((amdgpu_waves_per_eu(1, max_waves_fft<T>()))) __launch_bounds__((tpb_fft<T, FK_TIME>()), waves_fft<T>()) void k_time_prec(T* __restrict__ x, int64_t M, TimeTables<T> tb) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = tpb_fft<T, FK_TIME>() / (L / fft_V(L));
  using F = LineFft<T, L, NL, true, LAST_PAIRED>;
  DevCtx ctx = make_ctx();
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  time_prec_body<T, L>(ctx, reinterpret_cast<cx<T>*>(smem), red, x, M, tb);
}

template <typename T, int L>
static hipError_t go_time(T* x, int64_t M, const TimeTables<T>& tb, hipStream_t s) {
  const int64_t blocks = fft_blocks<T, FK_TIME>(L, M);
  const size_t lds = fft_lds_bytes<T, FK_TIME>(L);
  hipLaunchKernelGGL((k_time_prec<T, L>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_TIME>()), lds, s, x, M, tb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_time_prec(int L, T* x, int64_t M, const TimeTables<T>& tb, hipStream_t s) {
  switch (L) {
    case 2: return go_time<T, 2>(x, M, tb, s);
    case 4: return go_time<T, 4>(x, M, tb, s);
    case 8: return go_time<T, 8>(x, M, tb, s);
    case 16: return go_time<T, 16>(x, M, tb, s);
    case 32: return go_time<T, 32>(x, M, tb, s);
    case 64: return go_time<T, 64>(x, M, tb, s);
    case 128: return go_time<T, 128>(x, M, tb, s);
    case 256: return go_time<T, 256>(x, M, tb, s);
    case 512: return go_time<T, 512>(x, M, tb, s);
    case 1024: return go_time<T, 1024>(x, M, tb, s);
    case 2048: return go_time<T, 2048>(x, M, tb, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_time_prec<float>(int, float*, int64_t, const TimeTables<float>&, hipStream_t);
template hipError_t launch_time_prec<double>(int, double*, int64_t, const TimeTables<double>&, hipStream_t);

template <typename T, int L>
static hipError_t attr_time() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_time_prec<T, L>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)fft_lds_bytes<T, FK_TIME>(L));
}

hipError_t configure_time_kernels() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR(L)                                           \
  if ((e = attr_time<float, L>()) != hipSuccess) return e;    \
  if ((e = attr_time<double, L>()) != hipSuccess) return e;
  BLTT_ATTR(2) BLTT_ATTR(4) BLTT_ATTR(8) BLTT_ATTR(16) BLTT_ATTR(32) BLTT_ATTR(64)
  BLTT_ATTR(128) BLTT_ATTR(256) BLTT_ATTR(512) BLTT_ATTR(1024) BLTT_ATTR(2048)
#undef BLTT_ATTR
  return e;
}

}  // namespace bltt
