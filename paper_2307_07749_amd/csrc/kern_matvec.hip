// Symmetrised BLTT matvec q = Y A z: FFT form (dense p, line length 2N) and
// direct form (short p).
#include "launchers.hpp"

namespace bltt {

// R32: the residual is written as FP32 to up.r32 (FP64 sine-coordinate residual only)
template <typename T, int L, int MODE, int TERM, bool R32 = false>
__global__ __attribute__((amdgpu_waves_per_eu(2, max_waves_fft<T>()))) __launch_bounds__((tpb_fft<T, fk_mv<TERM == TERM_SPEC, L>()>()), waves_fft<T>()) void k_matvec_fft(T* z, T* __restrict__ out,
                                                             const T* __restrict__ fin, int64_t M,
                                                             MatvecTables<T> tb, IterUpd up,
                                                             double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NL = tpb_fft<T, fk_mv<TERM == TERM_SPEC, L>()>() / (L / fft_V(L));
  using F = LineFft<T, L, NL, TERM != TERM_SPEC, LAST_DEFAULT>;
  DevCtx ctx = make_ctx();
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<T>) * F::LDS_ELEMS);
  // the sine-coordinate forms work on the mode-major layout
  matvec_fft_body<T, L, MODE, TERM, TERM == TERM_SPEC, R32>(ctx, reinterpret_cast<cx<T>*>(smem), red, z, out, fin,
                                                            M, tb, up, partials);
}

template <typename T, int MODE>
__global__ __launch_bounds__(TPB_EW) void k_matvec_short(const T* __restrict__ z, T* __restrict__ out,
                                                         const T* __restrict__ fin, int64_t M, ShortTables<T> tb,
                                                         double* __restrict__ partials) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  matvec_short_body<T, MODE>(ctx, red, z, out, fin, M, tb, partials);
}

// (mode, term) combinations in use: Y A z with the stencil (step entry point,
// variable-coefficient MINRES), Y (p * z) alone (physical-space MINRES), the
// residual without the stencil (its spatial term follows on x-lines) or with
// it (variable coefficient), and the FP64 sine-coordinate forms (FP32 uses
// the N-point kernel of kern_cs.hip).
#define BLTT_MV_VARIANTS(X) X(MV_DOT, TERM_STENCIL) X(MV_DOT, TERM_NONE) X(MV_RESID, TERM_NONE) \
  X(MV_DOT, TERM_SPEC) X(MV_RESID, TERM_SPEC) X(MV_RESID, TERM_STENCIL)

template <typename T, int L>
static hipError_t go_mv(int mode, int term, T* z, T* out, const T* fin, int64_t M,
                        const MatvecTables<T>& tb, const IterUpd& up, double* partials, hipStream_t s) {
#define BLTT_GO(MO, TE)                                                                               \
  if (mode == MO && term == TE) {                                                                     \
    constexpr int FK = fk_mv<TE == TERM_SPEC, L>();                                                      \
    const unsigned blocks = (unsigned)fft_blocks<T, FK>(L, M);                                        \
    const unsigned tpb = (unsigned)tpb_fft<T, FK>();                                                  \
    const size_t lds = fft_lds_bytes<T, FK>(L);                                                       \
    if constexpr (sizeof(T) == 8 && MO == MV_RESID && TE == TERM_SPEC) {                             \
      if (up.r32) {                                                                                   \
        hipLaunchKernelGGL((k_matvec_fft<T, L, MO, TE, true>), dim3(blocks), dim3(tpb), lds, s, z, out, fin, \
                           M, tb, up, partials);                                                      \
        return hipGetLastError();                                                                     \
      }                                                                                               \
    }                                                                                                 \
    if (up.r32) return hipErrorInvalidValue;                                                          \
    hipLaunchKernelGGL((k_matvec_fft<T, L, MO, TE>), dim3(blocks), dim3(tpb), lds, s, z, out, fin, M, tb, \
                       up, partials);                                                                 \
    return hipGetLastError();                                                                         \
  }
  BLTT_MV_VARIANTS(BLTT_GO)
#undef BLTT_GO
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_matvec_fft(int L, int mode, int term, T* z, T* out, const T* fin, int64_t M,
                             const MatvecTables<T>& tb, const IterUpd& up, double* partials, hipStream_t s) {
  if (up.k < 0 || up.k > ZB_MAX || (up.k > 0 && !(mode == MV_RESID && term == TERM_SPEC))) return hipErrorInvalidValue;
  switch (L) {
    case 4: return go_mv<T, 4>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 8: return go_mv<T, 8>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 16: return go_mv<T, 16>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 32: return go_mv<T, 32>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 64: return go_mv<T, 64>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 128: return go_mv<T, 128>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 256: return go_mv<T, 256>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 512: return go_mv<T, 512>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 1024: return go_mv<T, 1024>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 2048: return go_mv<T, 2048>(mode, term, z, out, fin, M, tb, up, partials, s);
    case 4096: return go_mv<T, 4096>(mode, term, z, out, fin, M, tb, up, partials, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int MODE>
__global__ __launch_bounds__(TPB_EW) void k_matvec_short_mm(const T* __restrict__ z, T* __restrict__ out,
                                                            const T* __restrict__ fin, int64_t M, ShortTables<T> tb,
                                                            int log2N, double* __restrict__ partials) {
  __shared__ double red[TPB_EW];
  DevCtx ctx = make_ctx();
  matvec_short_mm_body<T, MODE>(ctx, red, z, out, fin, M, tb, log2N, partials);
}

template <typename T>
hipError_t launch_matvec_short(int mode, const T* z, T* out, const T* fin, int64_t M, const ShortTables<T>& tb,
                               double* partials, int64_t* nparts, hipStream_t s) {
  if (tb.term == TERM_SPEC) {
    int log2N = 0;
    while ((1 << log2N) < tb.N) ++log2N;
    if ((1 << log2N) != tb.N) return hipErrorInvalidValue;
    const int64_t gx = ew_blocks((int64_t)tb.N * M);
    if (nparts) *nparts = gx;
    if (mode == MV_DOT)
      hipLaunchKernelGGL((k_matvec_short_mm<T, MV_DOT>), dim3((unsigned)gx), dim3(TPB_EW), 0, s, z, out, fin, M, tb,
                         log2N, partials);
    else
      hipLaunchKernelGGL((k_matvec_short_mm<T, MV_RESID>), dim3((unsigned)gx), dim3(TPB_EW), 0, s, z, out, fin, M,
                         tb, log2N, partials);
    return hipGetLastError();
  }
  const int64_t gx = (M + TPB_EW - 1) / TPB_EW;
  const int half = (tb.N + 1) / 2;
  const int64_t gy = (half + tb.chunk - 1) / tb.chunk;
  if (nparts) *nparts = gx * gy;
  if (mode == MV_DOT)
    hipLaunchKernelGGL((k_matvec_short<T, MV_DOT>), dim3((unsigned)gx, (unsigned)gy), dim3(TPB_EW), 0, s, z, out,
                       fin, M, tb, partials);
  else
    hipLaunchKernelGGL((k_matvec_short<T, MV_RESID>), dim3((unsigned)gx, (unsigned)gy), dim3(TPB_EW), 0, s, z,
                       out, fin, M, tb, partials);
  return hipGetLastError();
}

#define BLTT_INST(T)                                                                                          \
  template hipError_t launch_matvec_fft<T>(int, int, int, T*, T*, const T*, int64_t, const MatvecTables<T>&,  \
                                           const IterUpd&, double*, hipStream_t);                            \
  template hipError_t launch_matvec_short<T>(int, const T*, T*, const T*, int64_t, const ShortTables<T>&,     \
                                             double*, int64_t*, hipStream_t);
BLTT_INST(float)
BLTT_INST(double)
#undef BLTT_INST

template <typename T, int L>
static hipError_t attr_mv() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR1(MO, TE)                                                                           \
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_matvec_fft<T, L, MO, TE>),                \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                                \
                          (int)fft_lds_bytes<T, fk_mv<TE == TERM_SPEC, L>()>(L));                       \
  if (e != hipSuccess) return e;
  BLTT_MV_VARIANTS(BLTT_ATTR1)
#undef BLTT_ATTR1
  if constexpr (sizeof(T) == 8)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_matvec_fft<T, L, MV_RESID, TERM_SPEC, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fft_lds_bytes<T, fk_mv<true, L>()>(L));
  return e;
}

hipError_t configure_matvec_kernels() {
  hipError_t e = hipSuccess;
#define BLTT_ATTR(L)                                         \
  if ((e = attr_mv<float, L>()) != hipSuccess) return e;    \
  if ((e = attr_mv<double, L>()) != hipSuccess) return e;
  BLTT_ATTR(4) BLTT_ATTR(8) BLTT_ATTR(16) BLTT_ATTR(32) BLTT_ATTR(64) BLTT_ATTR(128)
  BLTT_ATTR(256) BLTT_ATTR(512) BLTT_ATTR(1024) BLTT_ATTR(2048) BLTT_ATTR(4096)
#undef BLTT_ATTR
  return e;
}

}  // namespace bltt
