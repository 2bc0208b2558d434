// Sine-coordinate matvec (mode-major vectors) with N-point circulant and
// skew-circulant transforms; the FP64 residual variant also folds in the
// refinement update of the iterate.  The four N-entry tables (stage
// twiddles, the two spectra, e^{i pi n/N}) are staged in LDS when they fit
// beside the exchange buffers.
#include <algorithm>

#include "launchers.hpp"

namespace bltt {

template <typename T, int L, int MODE, int PLAN>
__global__ __attribute__((amdgpu_waves_per_eu(MODE == MV_DOT ? min_waves_upd<T>() : 1, max_waves_fft<T>()))) __launch_bounds__((tpb_fft<T, FK_SPEC>()), waves_fft<T>()) void k_matvec_cs(
    T* z, T* __restrict__ out, const T* __restrict__ fin, int64_t M, MatvecCSTables<T> tb, IterUpd up,
    double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = tpb_fft<T, FK_SPEC>() / (L / fft_V(L));
  using F = LineFft<T, L, NL, false, LAST_DEFAULT>;
  DevCtx ctx = make_ctx();
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  cx<T>* tabs = reinterpret_cast<cx<T>*>(smem + cs_lds_base<T, L>());
  matvec_cs_body<T, L, MODE, PLAN>(ctx, reinterpret_cast<cx<T>*>(smem), red, tabs, z, out, fin, M, tb, up, partials);
}

template <typename T, int L, int PLAN = 0>
static hipError_t go_cs(int mode, T* z, T* out, const T* fin, int64_t M, const MatvecCSTables<T>& tb,
                        const IterUpd& up, double* partials, int64_t max_blocks, int64_t* nparts, hipStream_t s) {
  // max_blocks > 0: at most that many workgroups, each looping over tiles;
  // 0: one tile per workgroup
  const int64_t tiles = fft_tiles<T, FK_SPEC>(L, M);
  const int64_t blocks = max_blocks > 0 ? std::min(tiles, max_blocks) : tiles;
  const size_t lds = cs_lds_bytes<T, L>();
  if (nparts) *nparts = blocks;
  if (mode == MV_DOT)
    hipLaunchKernelGGL((k_matvec_cs<T, L, MV_DOT, PLAN>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_SPEC>()), lds, s, z,
                       out, fin, M, tb, up, partials);
  else
    hipLaunchKernelGGL((k_matvec_cs<T, L, MV_RESID, PLAN>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_SPEC>()), lds, s, z,
                       out, fin, M, tb, up, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_matvec_cs(int L, int mode, T* z, T* out, const T* fin, int64_t M, const MatvecCSTables<T>& tb,
                            const IterUpd& up, double* partials, int64_t max_blocks, int64_t* nparts,
                            hipStream_t s, int plan) {
  if (up.k < 0 || up.k > ZB_MAX || (up.k > 0 && mode != MV_RESID)) return hipErrorInvalidValue;
  // the alternative radix plan exists for the FP32 form at L = 512, 1024
  if (plan != 0 && (plan != 1 || sizeof(T) != 4 || !fft_plan_alt(L))) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 4) {
    if (plan == 1 && L == 512) return go_cs<T, 512, 1>(mode, z, out, fin, M, tb, up, partials, max_blocks, nparts, s);
    if (plan == 1 && L == 1024) return go_cs<T, 1024, 1>(mode, z, out, fin, M, tb, up, partials, max_blocks, nparts, s);
  }
  switch (L) {
#define BLTT_CASE(LL) \
  case LL: return go_cs<T, LL>(mode, z, out, fin, M, tb, up, partials, max_blocks, nparts, s);
    BLTT_CASE(2) BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64)
    BLTT_CASE(128) BLTT_CASE(256) BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_matvec_cs<float>(int, int, float*, float*, const float*, int64_t,
                                            const MatvecCSTables<float>&, const IterUpd&, double*, int64_t, int64_t*,
                                            hipStream_t, int);
template hipError_t launch_matvec_cs<double>(int, int, double*, double*, const double*, int64_t,
                                             const MatvecCSTables<double>&, const IterUpd&, double*, int64_t,
                                             int64_t*, hipStream_t, int);

template <typename T, int L, int PLAN = 0>
static hipError_t attr_cs() {
  const int bytes = (int)cs_lds_bytes<T, L>();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_matvec_cs<T, L, MV_DOT, PLAN>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_matvec_cs<T, L, MV_RESID, PLAN>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  if constexpr (PLAN == 0 && sizeof(T) == 4 && fft_plan_alt(L)) return attr_cs<T, L, 1>();
  return hipSuccess;
}

hipError_t configure_cs_kernels() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR(L)                                        \
  if ((e = attr_cs<float, L>()) != hipSuccess) return e;   \
  if ((e = attr_cs<double, L>()) != hipSuccess) return e;
  BLTT_ATTR(2) BLTT_ATTR(4) BLTT_ATTR(8) BLTT_ATTR(16) BLTT_ATTR(32) BLTT_ATTR(64)
  BLTT_ATTR(128) BLTT_ATTR(256) BLTT_ATTR(512) BLTT_ATTR(1024) BLTT_ATTR(2048)
#undef BLTT_ATTR
  return e;
}

}  // namespace bltt
