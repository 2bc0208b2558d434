// Sine-transform passes: contiguous x-lines (with the fused Lanczos update or
// the fused dot product), x-lines fused with the move to or from the
// mode-major layout, and strided y/z-lines (in place).
#include "launchers.hpp"

namespace bltt {

template <typename T, int L, int KIND, bool FULL, bool Q1, bool STEN = FULL>
__global__ __attribute__((amdgpu_waves_per_eu(1, max_waves_fft<T>()))) __launch_bounds__((tpb_fft<T, FK_DSTX>()), waves_fft<T>()) void k_dst_x(const T* in, const T* __restrict__ v1,
                                                        const T* __restrict__ v2, T* __restrict__ vout,
                                                        const T* __restrict__ vdot, T* out,
                                                        int64_t nlines, DstTables<T> tb,
                                                        const double* __restrict__ coef,
                                                        double* __restrict__ partials, VupdStencil<T> sten) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = tpb_fft<T, FK_DSTX>() / (L / fft_V(L));
  using F = LineFft<T, L, NL, false, LAST_LINEAR>;
  DevCtx ctx = make_ctx();
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  dst_x_body<T, L, KIND, FULL, Q1, STEN>(ctx, reinterpret_cast<cx<T>*>(smem), red, in, v1, v2, vout, vdot, out, nlines, tb, coef,
                         partials, sten);
}

template <typename T, int L>
constexpr size_t dstxt_lds_bytes() {
  const size_t slots = (size_t)(DSTXT_TPB / (L / fft_V(L))) * (size_t)fft_padded(L);
  return (dst_split<T>() ? (slots + 1) / 2 : slots) * sizeof(cx<T>) + DSTXT_TPB * sizeof(double);
}
// waves per SIMD the FP64 sine transforms ask for: the split exchange leaves
// LDS for three, and their registers fit three (at most 168 VGPRs)
template <typename T>
constexpr int dst_min_waves() { return dst_split<T>() ? 3 : 1; }
template <typename T>
constexpr int dst_max_waves() { return dst_split<T>() ? 4 : max_waves_fft<T>(); }

template <typename T, int L, bool PAIRED>
__global__ __attribute__((amdgpu_waves_per_eu(dst_min_waves<T>(), dst_max_waves<T>()))) __launch_bounds__((tpb_fft<T, FK_DSTS>()), waves_fft<T>()) void k_dst_strided(T* __restrict__ x, int64_t nlines, int64_t S,
                                                              DstTables<T> tb) {
  extern __shared__ __align__(16) unsigned char smem[];
  DevCtx ctx = make_ctx();
  dst_strided_body<T, L, PAIRED>(ctx, reinterpret_cast<cx<T>*>(smem), x, nlines, S, tb);
}

template <typename T, int L, int DIR>
__global__ __attribute__((amdgpu_waves_per_eu(dst_min_waves<T>(), dst_max_waves<T>()))) __launch_bounds__(DSTXT_TPB) void k_dst_xt(const T* __restrict__ in, T* __restrict__ out, int64_t N,
                                                      int64_t M, DstTables<T> tb, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = DSTXT_TPB / (L / fft_V(L));
  using F = LineFft<T, L, NL, false, LAST_LINEAR, false, 0, dst_split<T>()>;
  DevCtx ctx = make_ctx();
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  dst_xt_body<T, L, DIR>(ctx, reinterpret_cast<cx<T>*>(smem), red, in, out, N, M, tb, partials);
}

// The same pass for S systems of one shape at once: workgroup b works on
// system b / bps (bps workgroups each, the single-system grid); each side is
// a pointer per system (p) or a base with stride n (b).
template <typename T, int L, int DIR>
__global__ __attribute__((amdgpu_waves_per_eu(dst_min_waves<T>(), dst_max_waves<T>()))) __launch_bounds__(DSTXT_TPB) void k_bt_dst_xt(
    const T* const* __restrict__ in_p, const T* __restrict__ in_b, T* const* __restrict__ out_p,
    T* __restrict__ out_b, int64_t n, int64_t N, int64_t M, DstTables<T> tb, int bps) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = DSTXT_TPB / (L / fft_V(L));
  using F = LineFft<T, L, NL, false, LAST_LINEAR, false, 0, dst_split<T>()>;
  DevCtx ctx = make_ctx();
  const int s = ctx.bid / bps;
  ctx.bid -= s * bps;
  ctx.nbx = bps;
  const T* in = in_p ? in_p[s] : in_b + (int64_t)s * n;
  T* out = out_p ? out_p[s] : out_b + (int64_t)s * n;
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  dst_xt_body<T, L, DIR>(ctx, reinterpret_cast<cx<T>*>(smem), red, in, out, N, M, tb, nullptr);
}

template <typename T, int L>
static hipError_t go_bt_dxt(int dir, const T* const* in_p, const T* in_b, T* const* out_p, T* out_b, int64_t n,
                            int64_t N, int64_t M, int S, const DstTables<T>& tb, hipStream_t s) {
  constexpr int m = L / 2 - 1;
  if (M % m != 0 || n != N * M || S < 1 || (!in_p && !in_b) || (!out_p && !out_b)) return hipErrorInvalidValue;
  const int64_t bps = dstxt_blocks(M / m, N, dstxt_lines<T, L>());
  if (bps < 1 || bps * S > 2147483647LL) return hipErrorInvalidValue;
  const size_t lds = dstxt_lds_bytes<T, L>();
  const dim3 grid((unsigned)(bps * S)), block(DSTXT_TPB);
  if (dir == 0)
    hipLaunchKernelGGL((k_bt_dst_xt<T, L, 0>), grid, block, lds, s, in_p, in_b, out_p, out_b, n, N, M, tb, (int)bps);
  else
    hipLaunchKernelGGL((k_bt_dst_xt<T, L, 1>), grid, block, lds, s, in_p, in_b, out_p, out_b, n, N, M, tb, (int)bps);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bt_dst_xt(int L, int dir, const T* const* in_p, const T* in_b, T* const* out_p, T* out_b,
                            int64_t n, int64_t N, int64_t M, int S, const DstTables<T>& tb, hipStream_t s) {
  switch (L) {
#define BLTT_CASE(LL) \
  case LL: return go_bt_dxt<T, LL>(dir, in_p, in_b, out_p, out_b, n, N, M, S, tb, s);
    BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64) BLTT_CASE(128) BLTT_CASE(256)
    BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_bt_dst_xt<double>(int, int, const double* const*, const double*, double* const*, double*,
                                             int64_t, int64_t, int64_t, int, const DstTables<double>&, hipStream_t);

template <typename T, int L>
static hipError_t go_dxt(int dir, const T* in, T* out, int64_t N, int64_t M, const DstTables<T>& tb,
                         double* partials, int64_t* nparts, hipStream_t s) {
  constexpr int m = L / 2 - 1;
  if (M % m != 0) return hipErrorInvalidValue;
  const int64_t blocks = dstxt_blocks(M / m, N, dstxt_lines<T, L>());
  if (blocks < 1 || blocks > 2147483647LL) return hipErrorInvalidValue;
  if (nparts) *nparts = blocks;
  const size_t lds = dstxt_lds_bytes<T, L>();
  if (dir == 0)
    hipLaunchKernelGGL((k_dst_xt<T, L, 0>), dim3((unsigned)blocks), dim3(DSTXT_TPB), lds, s, in, out, N, M, tb,
                       partials);
  else
    hipLaunchKernelGGL((k_dst_xt<T, L, 1>), dim3((unsigned)blocks), dim3(DSTXT_TPB), lds, s, in, out, N, M, tb,
                       nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dst_xt(int L, int dir, const T* in, T* out, int64_t N, int64_t M, const DstTables<T>& tb,
                         double* partials, int64_t* nparts, hipStream_t s) {
  switch (L) {
#define BLTT_CASE(LL) \
  case LL: return go_dxt<T, LL>(dir, in, out, N, M, tb, partials, nparts, s);
    BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64) BLTT_CASE(128) BLTT_CASE(256)
    BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_dst_xt<double>(int, int, const double*, double*, int64_t, int64_t,
                                          const DstTables<double>&, double*, int64_t*, hipStream_t);

template <typename T, int L>
static hipError_t go_dx(int kind, const T* in, const T* v1, const T* v2, T* vout, const T* vdot, T* out,
                        int64_t nlines, const DstTables<T>& tb, const double* coef, double* partials,
                        const VupdStencil<T>& sten, hipStream_t s) {
  const int64_t blocks = fft_blocks<T, FK_DSTX>(L, nlines);
  const size_t lds = fft_lds_bytes<T, FK_DSTX>(L);
  const dim3 grid((unsigned)blocks), block(tpb_fft<T, FK_DSTX>());
  if (kind == KIND_DOT) {
    hipLaunchKernelGGL((k_dst_x<T, L, KIND_DOT, false, false>), grid, block, lds, s, in, v1, v2, vout, vdot, out,
                       nlines, tb, coef, partials, sten);
    return hipGetLastError();
  }
  const bool full = v1 || vout || sten.z;
  if (!full) {
    hipLaunchKernelGGL((k_dst_x<T, L, KIND_VUPD, false, false>), grid, block, lds, s, in, v1, v2, vout, vdot, out,
                       nlines, tb, coef, partials, sten);
    return hipGetLastError();
  }
  // the full Lanczos update needs v1 and vout; v2 may be absent (then coef[2] = 0);
  // without z there is no stencil term (the matvec carried the whole operator)
  if (!v1 || !vout) return hipErrorInvalidValue;
  if (!v2) v2 = v1;
  if (!sten.z) {
    hipLaunchKernelGGL((k_dst_x<T, L, KIND_VUPD, true, false, false>), grid, block, lds, s, in, v1, v2, vout, vdot,
                       out, nlines, tb, coef, partials, sten);
    return hipGetLastError();
  }
  if (sten.qtaps <= 1)
    hipLaunchKernelGGL((k_dst_x<T, L, KIND_VUPD, true, true>), grid, block, lds, s, in, v1, v2, vout, vdot, out,
                       nlines, tb, coef, partials, sten);
  else
    hipLaunchKernelGGL((k_dst_x<T, L, KIND_VUPD, true, false>), grid, block, lds, s, in, v1, v2, vout, vdot, out,
                       nlines, tb, coef, partials, sten);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t go_ds(T* x, int64_t nlines, int64_t S, const DstTables<T>& tb, hipStream_t s) {
  const int64_t blocks = fft_blocks<T, FK_DSTS>(L, nlines);
  const size_t lds = fft_lds_bytes<T, FK_DSTS>(L);
  // adjacent line pairs (S and nlines even) load and store as one 2-element access
  if (S % 2 == 0 && nlines % 2 == 0)
    hipLaunchKernelGGL((k_dst_strided<T, L, true>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_DSTS>()), lds, s, x,
                       nlines, S, tb);
  else
    hipLaunchKernelGGL((k_dst_strided<T, L, false>), dim3((unsigned)blocks), dim3(tpb_fft<T, FK_DSTS>()), lds, s, x,
                       nlines, S, tb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dst_x(int L, int kind, const T* in, const T* v1, const T* v2, T* vout, const T* vdot, T* out,
                        int64_t nlines, const DstTables<T>& tb, const double* coef, double* partials,
                        const VupdStencil<T>& sten, hipStream_t s) {
  switch (L) {
#define BLTT_CASE(LL) \
  case LL: return go_dx<T, LL>(kind, in, v1, v2, vout, vdot, out, nlines, tb, coef, partials, sten, s);
    BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64) BLTT_CASE(128) BLTT_CASE(256)
    BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dst_strided(int L, T* x, int64_t nlines, int64_t S, const DstTables<T>& tb, hipStream_t s) {
  switch (L) {
#define BLTT_CASE(LL) \
  case LL: return go_ds<T, LL>(x, nlines, S, tb, s);
    BLTT_CASE(4) BLTT_CASE(8) BLTT_CASE(16) BLTT_CASE(32) BLTT_CASE(64) BLTT_CASE(128) BLTT_CASE(256)
    BLTT_CASE(512) BLTT_CASE(1024) BLTT_CASE(2048)
#undef BLTT_CASE
  }
  return hipErrorInvalidValue;
}

#define BLTT_INST(T)                                                                                           \
  template hipError_t launch_dst_x<T>(int, int, const T*, const T*, const T*, T*, const T*, T*, int64_t,       \
                                      const DstTables<T>&, const double*, double*, const VupdStencil<T>&,      \
                                      hipStream_t);                                                            \
  template hipError_t launch_dst_strided<T>(int, T*, int64_t, int64_t, const DstTables<T>&, hipStream_t);
BLTT_INST(float)
BLTT_INST(double)
#undef BLTT_INST

template <typename T, int L>
static hipError_t attr_dst() {
  const int bx = (int)fft_lds_bytes<T, FK_DSTX>(L), bs = (int)fft_lds_bytes<T, FK_DSTS>(L);
  hipError_t e;
  const void* ks[5] = {reinterpret_cast<const void*>(&k_dst_x<T, L, KIND_VUPD, false, false>),
                       reinterpret_cast<const void*>(&k_dst_x<T, L, KIND_VUPD, true, true>),
                       reinterpret_cast<const void*>(&k_dst_x<T, L, KIND_VUPD, true, false>),
                       reinterpret_cast<const void*>(&k_dst_x<T, L, KIND_VUPD, true, false, false>),
                       reinterpret_cast<const void*>(&k_dst_x<T, L, KIND_DOT, false, false>)};
  for (const void* k : ks)
    if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bx)) != hipSuccess) return e;
  if constexpr (sizeof(T) == 8) {
    const int bt = (int)dstxt_lds_bytes<T, L>();
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_xt<T, L, 0>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bt)) != hipSuccess)
      return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_xt<T, L, 1>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bt)) != hipSuccess)
      return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_dst_xt<T, L, 0>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bt)) != hipSuccess)
      return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bt_dst_xt<T, L, 1>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bt)) != hipSuccess)
      return e;
  }
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_strided<T, L, false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bs)) != hipSuccess)
    return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dst_strided<T, L, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bs);
}

hipError_t configure_dst_kernels() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR(L)                                          \
  if ((e = attr_dst<float, L>()) != hipSuccess) return e;    \
  if ((e = attr_dst<double, L>()) != hipSuccess) return e;
  BLTT_ATTR(4) BLTT_ATTR(8) BLTT_ATTR(16) BLTT_ATTR(32) BLTT_ATTR(64) BLTT_ATTR(128) BLTT_ATTR(256)
  BLTT_ATTR(512) BLTT_ATTR(1024) BLTT_ATTR(2048)
#undef BLTT_ATTR
  return e;
}

}  // namespace bltt
