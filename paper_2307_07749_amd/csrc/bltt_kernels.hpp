// Kernel bodies of the PMINRES hot path (Li, Lin, Hon, Wu, arXiv 2307.07749).
//
// Every body is a __host__ __device__ template taking a context `Ctx` that
// supplies the thread/block indices and the workgroup barrier, so the HIP
// launch wrappers and a CPU workgroup emulator run the same code.
//
// Vector layout: time-major, element (n, i) at n*M + i, i = x + m0*(y + m1*z).
//
// Hot-path steps per MINRES iteration (one pass = one kernel):
//   matvec      q = Y A z   (Section 2 eq. (4); Section 5.1: Toeplitz product
//               along time by FFT, spatial stencil of the blocks, time
//               reversal) + the partial sums of <q, z>
//   dst_x_vupd  vhat = cq q + cv v_j + cvp v_{j-1} (Lanczos three-term step)
//               fused with the sine transform along x (Step 1 of Section 5.1)
//   dst_strided sine transform along y (and z) of every time slice
//   time_prec   per sine mode, the two alpha-circulant half-solves of Section
//               5.1: D^{-1} F Lambda^{-1/2} F^* D^2 F conj(Lambda)^{-1/2} F^* D^{-1}
//   dst_strided inverse sine transform along (z and) y
//   dst_x_dot   inverse sine transform along x (Step 3) + partial sums of
//               <vhat, zhat>
//   wx_update   MINRES direction and iterate update
// The orthonormal DST-I is symmetric and its own inverse, so forward and
// inverse sine passes are the same kernel.
#pragma once

#include "fft_engine.hpp"

namespace bltt {

// Workgroup size of each line-FFT kernel class.  NL = TPB / G lines of length
// L (G = L/16 threads per line) share a workgroup.
// FK_SPEC: the sine-basis time-line kernels (mode-major lines, one wavefront
// per line pair): smaller workgroups schedule independently of each other.
// FK_MVS: the 2N-point matvec on mode-major lines (FP64 sine basis, 2N <= 2048):
// one line (two waves) per workgroup, so each exchange barrier waits on two
// waves only.
enum FftKernel { FK_TIME = 0, FK_MV = 1, FK_DSTS = 2, FK_DSTX = 3, FK_SPEC = 4, FK_MVS = 5 };
template <bool MM, int L>
constexpr int fk_mv() { return MM && L <= 2048 ? FK_MVS : FK_MV; }
template <typename T, int FK>
constexpr int tpb_fft() {
  return FK == FK_SPEC ? 256 : (sizeof(T) == 4 ? 512 : (FK == FK_MVS ? 128 : 256));
}
template <typename T, int FK>
constexpr int lines_per_block(int L) {
  return tpb_fft<T, FK>() / (L / (L < 16 ? L : 16));
}
// The FP64 sine transforms (strided lines, and x-lines fused with the layout
// change) exchange real and imaginary parts in turn (LineFft SPLIT): half the
// LDS per workgroup, so three waves per SIMD fit where two did.
template <typename T>
constexpr bool dst_split() { return sizeof(T) == 8; }
// dynamic LDS: NL padded lines (half as many bytes for a split exchange) + one
// double per thread for reductions
template <typename T, int FK>
constexpr size_t fft_lds_bytes(int L) {
  const size_t slots = (size_t)lines_per_block<T, FK>(L) * (size_t)fft_padded(L);
  const bool split = FK == FK_DSTS && dst_split<T>();
  return (split ? (slots + 1) / 2 : slots) * sizeof(cx<T>) + (size_t)tpb_fft<T, FK>() * sizeof(double);
}
// workgroups of a launch over `units` spatial points or lines, rounded up to a
// multiple of 8 for the XCD-aware tile order
template <typename T, int FK>
inline int64_t fft_blocks(int L, int64_t units) {
  const int64_t per = 2 * (int64_t)lines_per_block<T, FK>(L);
  const int64_t nb = (units + per - 1) / per;
  return (nb + 7) / 8 * 8;
}
// tiles of 2*NL sine modes of the sine-basis kernels
template <typename T, int FK>
BLTT_HD int64_t fft_tiles(int L, int64_t units) {
  const int64_t per = 2 * (int64_t)lines_per_block<T, FK>(L);
  return (units + per - 1) / per;
}

// minimum waves per SIMD requested from the compiler for the FFT kernels
// (1: no constraint beyond the workgroup size)
// launch sizes of the 2N-point matvec (mm: mode-major lines), for host code
template <typename T>
inline int64_t mv_blocks(bool mm, int L, int64_t units) {
  return mm && L <= 2048 ? fft_blocks<T, FK_MVS>(L, units) : fft_blocks<T, FK_MV>(L, units);
}
template <typename T>
inline int64_t mv_tiles(bool mm, int L, int64_t units) {
  return mm && L <= 2048 ? fft_tiles<T, FK_MVS>(L, units) : fft_tiles<T, FK_MV>(L, units);
}
template <typename T>
constexpr int waves_fft() { return 1; }
// LDS (about 74 KB per workgroup) admits two workgroups per CU, i.e. at most 4
// waves per SIMD (FP32, 512 threads) or 2 (FP64, 256 threads); telling the
// compiler so lets its scheduler keep more loads in flight instead of
// minimising registers for an occupancy that can never be reached.
template <typename T>
constexpr int max_waves_fft() { return sizeof(T) == 4 ? 4 : 2; }
// The FP32 time pass is bound by instruction issue: two waves per SIMD (at
// most 256 VGPRs) let one wave's LDS and memory waits overlap the other's ALU
// work.
template <typename T>
constexpr int min_waves_upd() { return sizeof(T) == 4 ? 2 : 1; }
constexpr int TPB_EW = 256;  // elementwise / streaming kernels
constexpr int ZB_MAX = 32;   // stored Z vectors of one FP32 sweep, at most

// ---------------------------------------------------------------------------
// XCD-aware tile order.  Workgroups are dealt round-robin to the 8 XCDs
// (workgroup b runs on XCD b mod 8), each with its own L2.  Mapping b to tile
// (b mod 8) * (nb/8) + b/8 gives every XCD a contiguous run of tiles, so
// neighbouring tiles (which share 128-byte lines at their edges and stencil
// rows) run at the same time on the same L2.  nb must be a multiple of 8;
// tiles past the end are empty (every load and store is masked).
// ---------------------------------------------------------------------------
BLTT_HD int64_t xcd_tile(int bid, int nb) { return (int64_t)(bid & 7) * (nb >> 3) + (bid >> 3); }

// The two sine modes that share complex line t of the sine-basis kernels
// (mode-major vectors, modes numbered x fastest in rows of mx = m_0, which is
// odd).  Pairing 2j with 2j+1 throughout would put the last mode of every
// other row, the highest x frequency and the smallest in a solve, in one line
// with the first of the next row, the lowest and the largest; FP32 transforms
// of that line leave the small mode with the large one's rounding, amplified
// by their ratio (about 4 (m_0 + 1)^2 / pi^2).  Instead each row pairs its
// modes 2j, 2j+1 within the row, and the last modes of rows r and r+1 (r even)
// pair with each other: both carry the highest x frequency, so their scales
// stay within a small factor.  There are ceil(M/2) lines either way; ib = M
// (no partner) for a lone last mode, and ia >= M past the last line.  With
// mx = 1 this is the plain 2j, 2j+1 pairing.
BLTT_HD void mode_pair(int64_t t, int64_t M, int mx, int64_t& ia, int64_t& ib) {
  const uint32_t pr = (uint32_t)(mx - 1) >> 1;
  const uint32_t rows = (uint32_t)M / (uint32_t)mx;
  const uint32_t within = rows * pr;
  const uint32_t tt = (uint32_t)t;
  if (tt < within) {
    const uint32_t r = tt / pr, j = tt - r * pr;
    ia = (int64_t)r * mx + 2 * (int64_t)j;
    ib = ia + 1;
  } else {
    const int64_t r = 2 * (int64_t)(tt - within);
    ia = r * mx + mx - 1;
    ib = r + 1 < (int64_t)rows ? ia + mx : M;
  }
}

// ---------------------------------------------------------------------------
// workgroup sum of one double per thread, result valid in thread 0
// ---------------------------------------------------------------------------
template <int TPB, class Ctx>
BLTT_HD double block_sum(Ctx& ctx, double* red, double v) {
  const int tid = ctx.tid;
  ctx.sync();
  red[tid] = v;
  ctx.sync();
#pragma unroll
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    ctx.sync();
  }
  return red[0];
}

// ---------------------------------------------------------------------------
// spatial stencil L_h = -Delta_h, zero Dirichlet (Section 5), or, with face
// coefficients, L_{a,h} = -Delta_{a,h}, the central-difference form of
// -div(a grad) (Section 5.2):
//   (L_{a,h} v)_i = sum_d [a_{d,hi}(i) (v_i - v_{i+e_d}) + a_{d,lo}(i) (v_i - v_{i-e_d})] / h_d^2,
// v = 0 outside the grid.  face[d] holds a at the faces along d: an array with
// the grid's extents except m_d + 1 along d (lexicographic, x fastest); entry
// j along d lies between points j-1 and j, so point c has its low face at
// j = c_d and its high face at j = c_d + 1.  a = 1 gives L_h.
// ---------------------------------------------------------------------------
struct Grid {
  int dim;
  int m[3];
  double inv_h2[3];
  const double* face[3];  // nullptr: constant coefficient 1
};

// low/high face coefficients of point coords c along dimension d
BLTT_HD void face_pair(const Grid& gr, const int* c, int d, double& lo, double& hi) {
  if (!gr.face[d]) {
    lo = hi = 1.0;
    return;
  }
  int64_t idx = 0, stride = 1, sd = 1;
  for (int e = 0; e < gr.dim; ++e) {
    if (e == d) sd = stride;
    idx += (int64_t)c[e] * stride;
    stride *= gr.m[e] + (e == d ? 1 : 0);
  }
  lo = gr.face[d][idx];
  hi = gr.face[d][idx + sd];
}

template <typename T>
BLTT_HD T lap_at(const T* __restrict__ z, int64_t base, int64_t i, const Grid& gr) {
  // base = n*M, i = spatial index
  const T zc = z[base + i];
  int c[3] = {0, 0, 0};
  int64_t rest = i;
  for (int d = 0; d < gr.dim; ++d) {
    c[d] = (int)(rest % gr.m[d]);
    rest /= gr.m[d];
  }
  T acc = T(0);
  int64_t stride = 1;
  for (int d = 0; d < gr.dim; ++d) {
    const int md = gr.m[d];
    double alo, ahi;
    face_pair(gr, c, d, alo, ahi);
    T s = T(alo + ahi) * zc;
    if (c[d] > 0) s -= T(alo) * z[base + i - stride];
    if (c[d] < md - 1) s -= T(ahi) * z[base + i + stride];
    acc += T(gr.inv_h2[d]) * s;
    stride *= md;
  }
  return acc;
}

// Neighbour offsets and face coefficients of one spatial point, computed once
// per thread (the point is fixed; only the time row changes).
struct Stencil {
  int64_t off[6];  // +-stride per dimension, 0 when the neighbour is the boundary
  float has[6];    // 1 inside, 0 on the boundary
  double w[6];     // face coefficient (low, high) per dimension
  int nd;
};

BLTT_HD Stencil make_stencil(int64_t i, const Grid& gr) {
  Stencil st;
  int c[3] = {0, 0, 0};
  int64_t rest = i, stride = 1;
  st.nd = gr.dim;
  for (int d = 0; d < gr.dim; ++d) {
    c[d] = (int)(rest % gr.m[d]);
    rest /= gr.m[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < gr.dim) {
      const int md = gr.m[d];
      const int coord = c[d];
      st.off[2 * d] = coord > 0 ? -stride : 0;
      st.has[2 * d] = coord > 0 ? 1.f : 0.f;
      st.off[2 * d + 1] = coord < md - 1 ? stride : 0;
      st.has[2 * d + 1] = coord < md - 1 ? 1.f : 0.f;
      face_pair(gr, c, d, st.w[2 * d], st.w[2 * d + 1]);
      stride *= md;
    } else {
      st.off[2 * d] = st.off[2 * d + 1] = 0;
      st.has[2 * d] = st.has[2 * d + 1] = 0.f;
      st.w[2 * d] = st.w[2 * d + 1] = 0.0;
    }
  }
  return st;
}

// (L_{a,h} z)_i on the row starting at zrow (zrow points at element (n, i))
template <typename T>
BLTT_HD T lap_row(const T* __restrict__ zrow, const Stencil& st, const Grid& gr) {
  const T zc = zrow[0];
  T acc = T(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < st.nd) {
      const T wl = T(st.w[2 * d]), wh = T(st.w[2 * d + 1]);
      T s = (wl + wh) * zc;
      if (st.has[2 * d] != 0.f) s -= wl * zrow[st.off[2 * d]];
      if (st.has[2 * d + 1] != 0.f) s -= wh * zrow[st.off[2 * d + 1]];
      acc += T(gr.inv_h2[d]) * s;
    }
  }
  return acc;
}

// ---------------------------------------------------------------------------
// matvec, FFT form: (A z)_n = sum_{k<=n} p_k z_{n-k} + sum_{k<qtaps} q_k L_h z_{n-k}.
// The causal Toeplitz product along time is the first N samples of the cyclic
// convolution of length L = 2N of z padded with N zeros: ifft(fft(p) fft(z)).
// Two spatial points are packed as the real and imaginary part of one complex
// line (every operation is complex-linear with a real kernel).  The time
// reversal Y is applied on the store; <Y A z, z> needs z at the mirrored time,
// which comes from LDS.  The spatial term of the blocks is
//   TERM_NONE     absent: only Y (p * z) is formed (and its dot with z); inside
//                 the physical-space MINRES the spatial term is added by the
//                 x-line pass and its dot product by the preceding time pass;
//   TERM_STENCIL  the finite-difference stencil L_h on physical-space lines;
//   TERM_SPEC     sine coordinates (Remark 1): L_h is diag(mu), so line i gets
//                 mu_i sum_k q_k z[n-k], with z[n-k] read from LDS.
// ---------------------------------------------------------------------------
template <typename T>
struct MatvecTables {
  const cx<T>* tw;    // length 2N: exp(-2 pi i k/(2N))
  const cx<T>* phat;  // length 2N: fft(p padded to 2N)/(2N)
  const T* mu;        // TERM_SPEC: Laplacian eigenvalue of each sine mode (length M)
  T q[4];
  int qtaps;
  Grid grid;
  int mx = 1;         // mode-major lines: modes per x-row (mode_pair)
};

enum { MV_DOT = 0, MV_RESID = 1 };
enum { TERM_NONE = 0, TERM_STENCIL = 1, TERM_SPEC = 2 };

// Iterate update fused into the FP64 residual of the refinement loop:
// u <- (u_zero ? 0 : u) + sum_{i<k} (*s) y[i] Z_i (Z_i the stored FP32 vectors
// of the sweep, added in order in FP64), written back to u, and the residual
// formed from the new u.
struct IterUpd {
  const float* z[ZB_MAX];
  int k;             // 0: no update
  const double* y;
  const double* s;
  int u_zero;        // u not read (first sweep: the iterate starts at zero)
  // non-null: the residual goes to r32 as FP32, times r32_scale, instead of
  // to `out` (the next sweep's right-hand side, read once in FP32); its norm
  // is still summed in FP64 before the rounding
  float* r32 = nullptr;
  double r32_scale = 1.0;
};

// Layout (MM): false = time-major vectors (element (i, n) at n*M + i, the ABI
// layout), lines interleaved across the workgroup so that a row of 2*NL
// consecutive points is one coalesced access; true = mode-major (element at
// i*N + n, the sine-basis working layout), each line contiguous in memory and
// owned by consecutive threads, and for N <= 512 by one wavefront.
// Batched use: the stored vectors of system s start at up.z[i] + zoff, and
// k >= 0 / y / sptr replace up.k / up.y / up.s (the pointer table stays in the
// kernel arguments instead of a per-thread copy).
template <typename T, int L, int MODE, int TERM, bool MM, bool R32 = false, class Ctx>
BLTT_HD double matvec_fft_tile(Ctx& ctx, cx<T>* lds, int64_t tile, T* z, T* __restrict__ out,
                               const T* __restrict__ fin, int64_t M, const MatvecTables<T>& tb, const IterUpd& up,
                               int64_t zoff = 0, int k = -1, const double* y = nullptr,
                               const double* sptr = nullptr, float* r32o = nullptr, double r32so = 1.0) {
  static_assert(!(MM && TERM == TERM_STENCIL), "the stencil needs the time-major layout");
  constexpr int TPB = tpb_fft<T, fk_mv<MM, L>()>();
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0);
  constexpr int N = L / 2, VH = V / 2;  // slots t < VH hold times g + t*s0 < N
  using F = LineFft<T, L, NL, !MM, LAST_DEFAULT>;
  const int tid = ctx.tid, c = MM ? tid / G : tid % NL, g = MM ? tid % G : tid / NL;
  int64_t ia = tile * (2 * NL) + 2 * c, ib = ia + 1;
  if constexpr (MM) mode_pair(tile * NL + c, M, tb.mx, ia, ib);
  const bool va = ia < M, vb = ib < M;
  const T* za = z + ia;
  const T* zb = z + ib;

  const int64_t iac = va ? ia : M - 1, ibc = vb ? ib : M - 1;
  // time stride and line bases (clamped for loads, exact for stores)
  const int64_t ts = MM ? 1 : M;
  const int64_t la = MM ? iac * N : iac, lb = MM ? ibc * N : ibc;
  const int64_t sa = MM ? ia * N : ia, sb = MM ? ib * N : ib;
  const int uk = k >= 0 ? k : up.k;
  const double* uy = y ? y : up.y;
  const bool upd = MODE == MV_RESID && uk > 0;
  const double us = upd ? *(sptr ? sptr : up.s) : 0.0;
  // FP32 residual output (R32): the batched caller passes its system's
  // buffer and scale here instead of in up
  float* const r32p = r32o ? r32o : up.r32;
  const double r32s = r32o ? r32so : up.r32_scale;
  cx<T> v[V], zin[VH];
  T ra[VH], rb[VH];
#pragma unroll
  for (int t = 0; t < VH; ++t) {
    const int64_t off = (int64_t)(g + t * s0) * ts;
    ra[t] = T(0);
    rb[t] = T(0);
    if (!(MODE == MV_RESID && up.u_zero)) {
      ra[t] = z[la + off];
      rb[t] = z[lb + off];
    }
  }
  if (upd) {
    // refinement update of the iterate, written back before its use; the
    // loop over the stored vectors is outside the one over times, so each
    // vector's loads are all in flight together
    double da[VH], db[VH];
#pragma unroll
    for (int t = 0; t < VH; ++t) {
      da[t] = (double)ra[t];
      db[t] = (double)rb[t];
    }
    // ZG vectors per group: their loads are issued together, so a sweep of k
    // vectors costs about k/ZG memory round trips instead of k
    constexpr int ZG = 4;
    for (int i0 = 0; i0 < uk; i0 += ZG) {
      float xa[ZG][VH], xb[ZG][VH];
#pragma unroll
      for (int j = 0; j < ZG; ++j) {
        if (i0 + j < uk) {
          const float* zi = up.z[i0 + j] + zoff;
#pragma unroll
          for (int t = 0; t < VH; ++t) {
            const int64_t off = (int64_t)(g + t * s0) * ts;
            xa[j][t] = zi[la + off];
            xb[j][t] = zi[lb + off];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < ZG; ++j) {
        if (i0 + j < uk) {
          const double yi = us * uy[i0 + j];
#pragma unroll
          for (int t = 0; t < VH; ++t) {
            da[t] += yi * (double)xa[j][t];
            db[t] += yi * (double)xb[j][t];
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < VH; ++t) {
      const int64_t off = (int64_t)(g + t * s0) * ts;
      ra[t] = T(da[t]);
      rb[t] = T(db[t]);
      if (va) z[sa + off] = ra[t];
      if (vb) z[sb + off] = rb[t];
    }
  }
#pragma unroll
  for (int t = 0; t < VH; ++t) {
    zin[t] = mkc<T>(va ? ra[t] : T(0), vb ? rb[t] : T(0));
    v[t] = zin[t];
  }
#pragma unroll
  for (int t = VH; t < V; ++t) v[t] = mkc<T>(T(0), T(0));
  F::forward(ctx, v, lds, c, g, tb.tw);
#pragma unroll
  for (int w = 0; w < V / F::RL; ++w)
#pragma unroll
    for (int u = 0; u < F::RL; ++u) v[w * F::RL + u] = v[w * F::RL + u] * tb.phat[F::freq(g, w, u)];
  F::inverse(ctx, v, lds, c, g, tb.tw);

  // z at the mirrored time N-1-n, for <Y A z, z> (and z[n-k] for TERM_SPEC)
  F::xsync(ctx);
#pragma unroll
  for (int t = 0; t < VH; ++t) lds[F::idx(c, g + t * s0)] = zin[t];
  F::xsync(ctx);
  // the right-hand side: all loads in flight together (clamped line bases, so
  // unconditional), after the barrier so that they are not hoisted into the
  // transforms; inside the guarded epilogue each would wait for the stores
  // before it
  T fa[MODE == MV_RESID ? VH : 1], fb[MODE == MV_RESID ? VH : 1];
  if constexpr (MODE == MV_RESID) {
#pragma unroll
    for (int t = 0; t < VH; ++t) {
      const int64_t off = (int64_t)(g + t * s0) * ts;
      fa[t] = fin[la + off];
      fb[t] = fin[lb + off];
    }
  }

  Stencil sta{}, stb{};
  if constexpr (TERM == TERM_STENCIL) {
    sta = make_stencil(va ? ia : 0, tb.grid);
    stb = make_stencil(vb ? ib : 0, tb.grid);
  }
  T mua = T(0), mub = T(0);
  if (TERM == TERM_SPEC) {
    mua = tb.mu[iac];
    mub = tb.mu[ibc];
  }
  T* oa = out + sa;
  T* ob = out + sb;
  double part = 0.0;
#pragma unroll
  for (int t = 0; t < VH; ++t) {
    const int n = g + t * s0;
    T ya = v[t].re, yb = v[t].im;
    if (TERM == TERM_STENCIL) {
      for (int k = 0; k < tb.qtaps && k <= n; ++k) {
        const int64_t off = (int64_t)(n - k) * M;
        if (va) ya += tb.q[k] * lap_row(za + off, sta, tb.grid);
        if (vb) yb += tb.q[k] * lap_row(zb + off, stb, tb.grid);
      }
    }
    if (TERM == TERM_SPEC) {
      // taps beyond qtaps have q_k = 0; times before 0 read slot 0 with weight 0
      T sa = tb.q[0] * zin[t].re, sb = tb.q[0] * zin[t].im;
      if (tb.qtaps > 1) {
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          const int nk = n - k;
          const T w = nk >= 0 ? tb.q[k] : T(0);
          const cx<T> zk = lds[F::idx(c, nk >= 0 ? nk : 0)];
          sa += w * zk.re;
          sb += w * zk.im;
        }
      }
      ya += mua * sa;
      yb += mub * sb;
    }
    const int64_t offr = (int64_t)(N - 1 - n) * ts;
    if (MODE == MV_DOT) {
      const cx<T> zr = lds[F::idx(c, N - 1 - n)];
      if (va) {
        oa[offr] = ya;
        part += (double)ya * (double)zr.re;
      }
      if (vb) {
        ob[offr] = yb;
        part += (double)yb * (double)zr.im;
      }
    } else {
      const int64_t off = (int64_t)n * ts;
      (void)off;
      if (va) {
        const T r = fa[MODE == MV_RESID ? t : 0] - ya;
        if constexpr (R32) r32p[sa + offr] = (float)(r * r32s);
        else oa[offr] = r;
        part += (double)r * (double)r;
      }
      if (vb) {
        const T r = fb[MODE == MV_RESID ? t : 0] - yb;
        if constexpr (R32) r32p[sb + offr] = (float)(r * r32s);
        else ob[offr] = r;
        part += (double)r * (double)r;
      }
    }
  }
  // a following tile of the same workgroup must not overwrite z in LDS early
  F::xsync(ctx);
  return part;
}

template <typename T, int L, int MODE, int TERM, bool MM, bool R32 = false, class Ctx>
BLTT_HD void matvec_fft_body(Ctx& ctx, cx<T>* lds, double* red, T* z, T* __restrict__ out,
                             const T* __restrict__ fin, int64_t M, const MatvecTables<T>& tb, const IterUpd& up,
                             double* __restrict__ partials) {
  const double part = matvec_fft_tile<T, L, MODE, TERM, MM, R32>(ctx, lds, xcd_tile(ctx.bid, ctx.nbx), z, out, fin, M,
                                                              tb, up);
  const double s = block_sum<tpb_fft<T, fk_mv<MM, L>()>()>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = s;
}

// ---------------------------------------------------------------------------
// matvec in sine coordinates, mode-major, with N-point transforms: the causal
// Toeplitz product is T = (C + S)/2, C the circulant and S the skew-circulant
// with first column p (S = D^{-1} C' D, C' circulant of D p, D = diag(e^{i pi
// n/N}): the zero-padded 2N-point product split into its even and odd
// frequencies).  Each line stays in the N-point layout of the time pass (one
// wavefront per line pair for N <= 1024).  Line i gets, as in the 2N form,
// Y (p * z + mu_i (q * z)) and the partial sums of <., z> (MV_DOT) or of the
// squared residual Y (fin - ...) (MV_RESID).
// ---------------------------------------------------------------------------
template <typename T>
struct MatvecCSTables {
  const cx<T>* tw;     // length N
  const cx<T>* chat;   // fft(p)/(2N)
  const cx<T>* shat;   // fft(D p)/(2N)
  const cx<T>* omega;  // e^{i pi n/N}
  const T* mu;
  T q[4];
  int qtaps;
  int mx = 1;          // modes per x-row (mode_pair)
};

// Index of the spectrum entry register slot (w, u) of lane g multiplies: the
// frequency itself, or, for tables staged in LDS (STAGED), the slot's position
// in register order, (w RL + u) G + g, so consecutive lanes read consecutive
// entries (by frequency they would hit a few banks).
template <class F, bool STAGED>
BLTT_HD int spec_index(int g, int w, int u) {
  return STAGED ? (w * F::RL + u) * F::G + g : F::freq(g, w, u);
}

// The N-point matvec's tables staged in LDS per workgroup, in two steps so
// that the tile can put its own line loads between them: load() issues every
// global load (clamped indices, so unconditional) into registers; store()
// writes them to LDS (stage twiddles as build_twl lays them out, spectra in
// register order: entry (w RL + u) G + g holds frequency freq(g, w, u)), with
// no barrier (the tile takes one).
template <typename T, int L, int TPB, int PLAN = 0>
struct CsStage {
  using F = LineFft<T, L, TPB / (L / fft_V(L)), false, LAST_DEFAULT, true, PLAN>;
  static constexpr int PER = (L + TPB - 1) / TPB;
  cx<T> tv[F::template twl_per<TPB>()];
  cx<T> ch[PER], sh[PER], om[PER];
  cx<T>* tabs;

  template <class Ctx>
  BLTT_HD void load(Ctx& ctx, const MatvecCSTables<T>& tb) {
    F::template twl_load<TPB>(ctx, tb.tw, tv);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = ctx.tid + r * TPB, ii = i < L ? i : L - 1;
      const int g = ii % F::G, j = ii / F::G;
      const int k = F::freq(g, j / F::RL, j % F::RL);
      ch[r] = tb.chat[k];
      sh[r] = tb.shat[k];
      om[r] = tb.omega[ii];
    }
  }
  template <class Ctx>
  BLTT_HD void store(Ctx& ctx) {
    F::template twl_store<TPB>(ctx, tabs, tv);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = ctx.tid + r * TPB;
      if (i < L) {
        tabs[L + i] = ch[r];
        tabs[2 * L + i] = sh[r];
        tabs[3 * L + i] = om[r];
      }
    }
  }
  // the tables as the tile reads them
  BLTT_HD MatvecCSTables<T> tables(const MatvecCSTables<T>& tb) const {
    MatvecCSTables<T> t = tb;
    t.tw = tabs;
    t.chat = tabs + L;
    t.shat = tabs + 2 * L;
    t.omega = tabs + 3 * L;
    return t;
  }
};

// TPB: workgroup size (2*TPB/G modes per tile); the batched kernels choose it per shape.
// TWL: the tables are the LDS copies of CsStage (stage twiddles, spectra in
// register order), whose registers `stage` holds: the tile stores them and
// synchronises once its line loads are issued (a null `stage`: the tables are
// in LDS already, stored by an earlier tile of the workgroup).
template <typename T, int L, int MODE, int TPB = tpb_fft<T, FK_SPEC>(), bool TWL = false, int PLAN = 0, class Ctx,
          class Stage = CsStage<T, L, TPB, PLAN>>
BLTT_HD double matvec_cs_tile(Ctx& ctx, cx<T>* lds, int64_t tile, T* z, T* __restrict__ out,
                              const T* __restrict__ fin, int64_t M, const MatvecCSTables<T>& tb, const IterUpd& up,
                              Stage* stage = nullptr) {
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0);
  constexpr int N = L;
  using F = LineFft<T, L, NL, false, LAST_DEFAULT, TWL, PLAN>;
  const int tid = ctx.tid, c = tid / G;
  int g = tid % G;
#if defined(__HIP_DEVICE_COMPILE__)
  // g opaque to the compiler, so that a tile loop around this function does
  // not keep g-dependent table reads live across tiles at the cost of occupancy
  asm volatile("" : "+v"(g));
  g &= G - 1;
#endif
  int64_t ia, ib;
  mode_pair(tile * NL + c, M, tb.mx, ia, ib);
  const bool va = ia < M, vb = ib < M;
  const int64_t iac = va ? ia : M - 1, ibc = vb ? ib : M - 1;
  const int64_t la = iac * N, lb = ibc * N;
  // per-lane pointers at time g (the reversed output at N-1-g): time offsets
  // t*s0 are then compile-time constants (memory-instruction immediates);
  // stores go through the clamped bases, equal to the exact ones wherever the
  // store's guard holds
  const int64_t gr = N - 1 - g;
  const bool upd = MODE == MV_RESID && up.k > 0;
  const double us = upd ? *up.s : 0.0;
  T mua = tb.mu[iac], mub = tb.mu[ibc];
  cx<T> zin[V], v[V], acc[V];
  T ra[V], rb[V];
#pragma unroll
  for (int t = 0; t < V; ++t) {
    ra[t] = T(0);
    rb[t] = T(0);
    if (!(MODE == MV_RESID && up.u_zero)) {
      ra[t] = (z + la + g)[t * s0];
      rb[t] = (z + lb + g)[t * s0];
    }
  }
  // the staged tables (CsStage) are stored and become visible here, with the
  // line's loads already in flight
  if constexpr (TWL) {
    if (stage) {
      stage->store(ctx);
      ctx.sync();
    }
  }
  if (upd) {
    // stored-vector loop outside the time loop: one vector's loads in flight together
    double da[V], db[V];
#pragma unroll
    for (int t = 0; t < V; ++t) {
      da[t] = (double)ra[t];
      db[t] = (double)rb[t];
    }
    for (int i = 0; i < up.k; ++i) {
      const double yi = us * up.y[i];
      const float* zi = up.z[i];
      float xa[V], xb[V];
#pragma unroll
      for (int t = 0; t < V; ++t) {
        xa[t] = (zi + la + g)[t * s0];
        xb[t] = (zi + lb + g)[t * s0];
      }
#pragma unroll
      for (int t = 0; t < V; ++t) {
        da[t] += yi * (double)xa[t];
        db[t] += yi * (double)xb[t];
      }
    }
#pragma unroll
    for (int t = 0; t < V; ++t) {
      const int n = g + t * s0;
      ra[t] = T(da[t]);
      rb[t] = T(db[t]);
      if (va) (z + la + g)[t * s0] = ra[t];
      if (vb) (z + lb + g)[t * s0] = rb[t];
    }
  }
#pragma unroll
  for (int t = 0; t < V; ++t) {
    // a line past M holds the clamped line M-1: its products stay in their
    // own half of the packed line (C, S and the q taps are real) and all its
    // stores and dot terms are guarded
    zin[t] = mkc<T>(ra[t], rb[t]);
    v[t] = zin[t];
  }
#if defined(__HIP_DEVICE_COMPILE__)
  // mu in registers with the line, before the transforms: loaded late, its
  // first use would sit inside each guarded store of the epilogue and make
  // every store wait for the one before it (the load counter is merged
  // pessimistically where the guards join)
  asm volatile("" : "+v"(mua), "+v"(mub));
#endif
  // circulant part
  F::forward(ctx, v, lds, c, g, tb.tw);
#pragma unroll
  for (int w = 0; w < V / F::RL; ++w)
#pragma unroll
    for (int u = 0; u < F::RL; ++u) v[w * F::RL + u] = v[w * F::RL + u] * tb.chat[spec_index<F, TWL>(g, w, u)];
  F::inverse(ctx, v, lds, c, g, tb.tw);
#pragma unroll
  for (int t = 0; t < V; ++t) {
    acc[t] = v[t];
    v[t] = zin[t] * tb.omega[g + t * s0];
  }
  // skew-circulant part
  F::forward(ctx, v, lds, c, g, tb.tw);
#pragma unroll
  for (int w = 0; w < V / F::RL; ++w)
#pragma unroll
    for (int u = 0; u < F::RL; ++u) v[w * F::RL + u] = v[w * F::RL + u] * tb.shat[spec_index<F, TWL>(g, w, u)];
  F::inverse(ctx, v, lds, c, g, tb.tw);
#pragma unroll
  for (int t = 0; t < V; ++t) acc[t] = acc[t] + v[t] * conjg(tb.omega[g + t * s0]);

  // z in LDS: the mirrored time N-1-n for the dot, z[n-k] for the mu term
  F::xsync(ctx);
#pragma unroll
  for (int t = 0; t < V; ++t) lds[F::idx(c, g + t * s0)] = zin[t];
  F::xsync(ctx);
  double part = 0.0;
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int n = g + t * s0;
    T sqa = tb.q[0] * zin[t].re, sqb = tb.q[0] * zin[t].im;
    if (tb.qtaps > 1) {
      // taps beyond qtaps have q_k = 0; times before 0 read slot 0 with weight 0
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        const int nk = n - k;
        const T w = nk >= 0 ? tb.q[k] : T(0);
        const cx<T> zk = lds[F::idx(c, nk >= 0 ? nk : 0)];
        sqa += w * zk.re;
        sqb += w * zk.im;
      }
    }
    const T ya = acc[t].re + mua * sqa, yb = acc[t].im + mub * sqb;
    T* ora = out + la + gr;
    T* orb = out + lb + gr;
    if (MODE == MV_DOT) {
      const cx<T> zr = lds[F::idx(c, N - 1 - n)];
      if (va) {
        ora[-(t * s0)] = ya;
        part += (double)ya * (double)zr.re;
      }
      if (vb) {
        orb[-(t * s0)] = yb;
        part += (double)yb * (double)zr.im;
      }
    } else {
      if (va) {
        const T r = (fin + la + g)[t * s0] - ya;
        ora[-(t * s0)] = r;
        part += (double)r * (double)r;
      }
      if (vb) {
        const T r = (fin + lb + g)[t * s0] - yb;
        orb[-(t * s0)] = r;
        part += (double)r * (double)r;
      }
    }
  }
  // the next tile's first exchange must not overwrite z before every lane has read it
  F::xsync(ctx);
  return part;
}

// LDS staging of the four N-entry tables of the N-point matvec (when they fit
// beside the exchange lines, two workgroups per CU): the stage twiddles in the
// LineFft TWL layout, the two spectra and e^{i pi n/N}.
template <typename T, int L>
constexpr size_t cs_lds_base() { return fft_lds_bytes<T, FK_SPEC>(L); }
template <typename T, int L>
constexpr bool cs_stage() { return cs_lds_base<T, L>() + 4 * (size_t)L * sizeof(cx<T>) <= 80 * 1024; }
template <typename T, int L>
constexpr size_t cs_lds_bytes() { return cs_lds_base<T, L>() + (cs_stage<T, L>() ? 4 * (size_t)L * sizeof(cx<T>) : 0); }

// One tile per workgroup (a loop over tiles lets the compiler keep the
// loop-invariant twiddle and spectrum loads live across tiles, which costs
// half the occupancy here); one partial sum per workgroup.  `tabs`: LDS for
// the staged tables when cs_stage holds.  Workgroup b takes tiles b, b + nbx,
// ...: one tile each when the grid covers every tile, or persistently, with
// the tables staged once by the first tile.
template <typename T, int L, int MODE, int PLAN = 0, class Ctx>
BLTT_HD void matvec_cs_body(Ctx& ctx, cx<T>* lds, double* red, cx<T>* tabs, T* z, T* __restrict__ out,
                            const T* __restrict__ fin, int64_t M, const MatvecCSTables<T>& tb, const IterUpd& up,
                            double* __restrict__ partials) {
  constexpr int TPB = tpb_fft<T, FK_SPEC>();
  const int64_t ntiles = fft_tiles<T, FK_SPEC>(L, M);
  double part = 0.0;
  if constexpr (cs_stage<T, L>()) {
    using Stage = CsStage<T, L, TPB, PLAN>;
    Stage st;
    st.tabs = tabs;
    st.load(ctx, tb);
    const MatvecCSTables<T> lt = st.tables(tb);
    int64_t tile = ctx.bid;
    if (tile < ntiles)
      part = matvec_cs_tile<T, L, MODE, TPB, true, PLAN>(ctx, lds, tile, z, out, fin, M, lt, up, &st);
    for (tile += ctx.nbx; tile < ntiles; tile += ctx.nbx)
      part += matvec_cs_tile<T, L, MODE, TPB, true, PLAN>(ctx, lds, tile, z, out, fin, M, lt, up,
                                                          static_cast<Stage*>(nullptr));
  } else {
    for (int64_t tile = ctx.bid; tile < ntiles; tile += ctx.nbx)
      part += matvec_cs_tile<T, L, MODE, TPB, false, PLAN>(ctx, lds, tile, z, out, fin, M, tb, up);
  }
  const double sum = block_sum<TPB>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

// matvec, direct form for short p (ptaps <= 8): one thread per spatial point
// and a chunk of time steps together with their mirrors N-1-n, so the dot
// product <Y A z, z> needs no second pass over z.
template <typename T>
struct ShortTables {
  T p[8];
  int ptaps;
  T q[4];
  int qtaps;
  Grid grid;
  int N;
  int chunk;    // time steps per thread (from the first half)
  int term;     // TERM_NONE / TERM_STENCIL / TERM_SPEC, as for the FFT form
  const T* mu;  // TERM_SPEC: Laplacian eigenvalue of each sine mode
};

template <typename T, int MODE, class Ctx>
BLTT_HD void matvec_short_body(Ctx& ctx, double* red, const T* __restrict__ z, T* __restrict__ out,
                               const T* __restrict__ fin, int64_t M, const ShortTables<T>& tb,
                               double* __restrict__ partials) {
  const int tid = ctx.tid;
  const int64_t i = (int64_t)ctx.bid * TPB_EW + tid;
  const int N = tb.N;
  const int half = (N + 1) / 2;
  const int n0 = ctx.bid_y * tb.chunk;
  double part = 0.0;
  if (i < M) {
    for (int nn = n0; nn < n0 + tb.chunk && nn < half; ++nn) {
      for (int side = 0; side < 2; ++side) {
        const int n = side == 0 ? nn : N - 1 - nn;
        if (side == 1 && n == nn) break;  // odd N: middle step once
        T y = T(0);
        for (int k = 0; k < tb.ptaps && k <= n; ++k) y += tb.p[k] * z[(int64_t)(n - k) * M + i];
        if (tb.term == TERM_STENCIL)
          for (int k = 0; k < tb.qtaps && k <= n; ++k) y += tb.q[k] * lap_at(z, (int64_t)(n - k) * M, i, tb.grid);
        if (tb.term == TERM_SPEC) {
          T s = T(0);
          for (int k = 0; k < tb.qtaps && k <= n; ++k) s += tb.q[k] * z[(int64_t)(n - k) * M + i];
          y += tb.mu[i] * s;
        }
        const int64_t nr = (int64_t)(N - 1 - n);
        if (MODE == MV_DOT) {
          out[nr * M + i] = y;
          part += (double)y * (double)z[nr * M + i];
        } else {
          const T r = fin[(int64_t)n * M + i] - y;
          out[nr * M + i] = r;
          part += (double)r * (double)r;
        }
      }
    }
  }
  const double s = block_sum<TPB_EW>(ctx, red, part);
  if (tid == 0) partials[(int64_t)ctx.bid_y * ctx.nbx + ctx.bid] = s;
}

// Direct form in the mode-major sine-basis layout (element (i, n) at i*N + n):
// one thread per output element, consecutive threads along time, so every
// access is coalesced and the few neighbours k <= 8 back are cache hits.
// out[i*N + N-1-n] = (p * z_i)[n] + mu_i (q * z_i)[n] (MV_DOT, with the partial
// sums of <out, z>) or Y (fin - ...) (MV_RESID, partial sums of ||out||^2).
template <typename T, int MODE, class Ctx>
BLTT_HD void matvec_short_mm_body(Ctx& ctx, double* red, const T* __restrict__ z, T* __restrict__ out,
                                  const T* __restrict__ fin, int64_t M, const ShortTables<T>& tb, int log2N,
                                  double* __restrict__ partials) {
  const int N = tb.N;
  const int64_t n_total = (int64_t)N * M;
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  double part = 0.0;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) {
    const int64_t i = e >> log2N;
    const int n = (int)(e & (N - 1));
    const T* zl = z + (i << log2N);
    T y = T(0), sq = T(0);
    for (int k = 0; k < tb.ptaps && k <= n; ++k) y += tb.p[k] * zl[n - k];
    for (int k = 0; k < tb.qtaps && k <= n; ++k) sq += tb.q[k] * zl[n - k];
    y += tb.mu[i] * sq;
    const int64_t er = (i << log2N) + (N - 1 - n);
    if (MODE == MV_DOT) {
      out[er] = y;
      part += (double)y * (double)zl[N - 1 - n];
    } else {
      const T r = fin[e] - y;
      out[er] = r;
      part += (double)r * (double)r;
    }
  }
  const double sum = block_sum<TPB_EW>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

// ---------------------------------------------------------------------------
// sine transforms.  DST-I of length m = L/2 - 1 through one complex FFT of
// length L = 2(m+1) shared by two lines a, b: with e the odd extension
// (e_0 = e_{m+1} = 0, e_p = x_{p-1}, e_{L-p} = -x_{p-1}), fft(e_a + i e_b)_k =
// -2i S_a(k) + 2 S_b(k), S(k) = sum_j x_j sin(pi j k/(m+1)).  The orthonormal
// transform is y_{k-1} = sqrt(2/(m+1)) S(k).
// ---------------------------------------------------------------------------
template <typename T>
struct DstTables {
  const cx<T>* tw;  // length L
  int m;            // line length
  T nrm;            // 1/sqrt(L) = sqrt(2/(m+1))/2
};

// Spatial part of the matvec, added where x-lines are streamed: the Lanczos
// update of line (n, r) needs (Y L_h (q * z))[n, r, x] = sum_k q_k
// (L_h z)[N-1-n-k, r, x]; the neighbours along y and z are adjacent x-lines.
// Lines are indexed l = n R + r with R = M / m0 lines per time slice.
template <typename T>
struct VupdStencil {
  const T* z;  // z_j (nullptr: no stencil term)
  T q[4];
  int qtaps;
  Grid grid;
  int N;
  int64_t R;
};

// Per-line data of the stencil term for one x-line, computed once per thread.
// Neighbour rows outside the grid are replaced by the centre row with weight 0
// so that every load is unconditional (no branches around memory accesses).
template <typename T>
struct LineStencil {
  const T* row[4];   // centre row at reversed time N-1-n-k, k < 4 (clamped)
  T wk[4];           // q_k, or 0 when the tap falls before t = 0 or k >= qtaps
  int64_t dy_m, dy_p, dz_m, dz_p;  // element offsets of the y/z neighbours (0 when outside)
  T wy_m, wy_p, wz_m, wz_p;
};

template <typename T>
BLTT_HD LineStencil<T> line_stencil(const VupdStencil<T>& st, int64_t line) {
  LineStencil<T> ls;
  const int m0 = st.grid.m[0];
  const int64_t n = line / st.R, r = line - n * st.R;
  const int yc = st.grid.dim > 1 ? (int)(r % st.grid.m[1]) : 0;
  const int zc = st.grid.dim > 2 ? (int)(r / st.grid.m[1]) : 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t nt = (int64_t)st.N - 1 - n - k;
    const bool ok = nt >= 0 && k < st.qtaps;
    ls.row[k] = st.z + ((ok ? nt : 0) * st.R + r) * m0;
    ls.wk[k] = ok ? st.q[k] : T(0);
  }
  const bool ym = st.grid.dim > 1 && yc > 0, yp = st.grid.dim > 1 && yc < st.grid.m[1] - 1;
  const bool zm = st.grid.dim > 2 && zc > 0, zp = st.grid.dim > 2 && zc < st.grid.m[2] - 1;
  const int64_t pl = (int64_t)m0 * st.grid.m[1];
  ls.dy_m = ym ? -m0 : 0;
  ls.dy_p = yp ? m0 : 0;
  ls.dz_m = zm ? -pl : 0;
  ls.dz_p = zp ? pl : 0;
  ls.wy_m = ym ? T(1) : T(0);
  ls.wy_p = yp ? T(1) : T(0);
  ls.wz_m = zm ? T(1) : T(0);
  ls.wz_p = zp ? T(1) : T(0);
  return ls;
}

// sum_k q_k (L_h z)[N-1-n-k, r, x] for one element of an x-line.  Dimensions
// beyond the grid's have zero weight and zero offset, so the same straight-line
// code (no branches between the loads) serves 1-D, 2-D and 3-D grids.
template <typename T, bool Q1>
BLTT_HD T line_stencil_at(const VupdStencil<T>& st, const LineStencil<T>& ls, int x) {
  const int m0 = st.grid.m[0];
  const T hx = T(st.grid.inv_h2[0]), hy = T(st.grid.inv_h2[1]), hz = T(st.grid.inv_h2[2]);
  const int xm = x > 0 ? x - 1 : x, xp = x < m0 - 1 ? x + 1 : x;
  const T wxm = x > 0 ? T(1) : T(0), wxp = x < m0 - 1 ? T(1) : T(0);
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < (Q1 ? 1 : 4); ++k) {
    const T* row = ls.row[k];
    const T c = row[x];
    const T s = hx * (T(2) * c - wxm * row[xm] - wxp * row[xp]) +
                hy * (T(2) * c - ls.wy_m * row[x + ls.dy_m] - ls.wy_p * row[x + ls.dy_p]) +
                hz * (T(2) * c - ls.wz_m * row[x + ls.dz_m] - ls.wz_p * row[x + ls.dz_p]);
    acc += ls.wk[k] * s;
  }
  return acc;
}

// The odd extension holds every value twice (e_p and e_{L-p} = -e_p).  Only
// the positions 1..m are loaded from memory; the mirrored half is filled from
// LDS after one barrier.  The FFT that follows synchronises before it first
// writes LDS, so the mirror reads cannot race with it.
template <class F, typename T, int L, class Ctx>
BLTT_HD void odd_mirror(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g) {
  constexpr int V = fft_V(L), s0 = fft_sigma(L, 0), VH = V / 2;
  // slots t < V/2 hold positions p = g + t*s0 < L/2 (loaded), slots t >= V/2
  // the positions p >= L/2, whose values are -e_{L-p} (e_{L/2} = 0)
  if constexpr (F::SPLIT_X) {
    // real parts, then imaginary parts, through the T buffer
    T* ls = reinterpret_cast<T*>(lds);
#pragma unroll
    for (int t = 0; t < VH; ++t) ls[F::idx(c, g + t * s0)] = v[t].re;
    ctx.sync();
    T re[VH];
#pragma unroll
    for (int t = VH; t < V; ++t) {
      const int p = g + t * s0;
      re[t - VH] = ls[F::idx(c, p == L / 2 ? 0 : L - p)];
    }
    ctx.sync();
#pragma unroll
    for (int t = 0; t < VH; ++t) ls[F::idx(c, g + t * s0)] = v[t].im;
    ctx.sync();
#pragma unroll
    for (int t = VH; t < V; ++t) {
      const int p = g + t * s0;
      const T im = ls[F::idx(c, p == L / 2 ? 0 : L - p)];
      v[t] = p == L / 2 ? mkc<T>(T(0), T(0)) : mkc<T>(-re[t - VH], -im);
    }
  } else {
#pragma unroll
    for (int t = 0; t < VH; ++t) lds[F::idx(c, g + t * s0)] = v[t];
    ctx.sync();
#pragma unroll
    for (int t = VH; t < V; ++t) {
      const int p = g + t * s0;
      const cx<T> w = lds[F::idx(c, p == L / 2 ? 0 : L - p)];
      v[t] = p == L / 2 ? mkc<T>(T(0), T(0)) : mkc<T>(-w.re, -w.im);
    }
  }
}

// Lines along x (contiguous).  KIND_VUPD: input is the Lanczos update
// cq*(Q + Y L_h (q*z)) + cv*V1 + cvp*V2 (optionally written to vout) ->
// out = U_x(input); the stencil term is skipped when sten.z is null.
// KIND_DOT: out = U_x(in) and partial sums of <vdot, out>.
// `out` may alias `in` (each workgroup owns whole lines and reads them before
// its first barrier); vout never aliases in, v1 or v2.
enum { KIND_VUPD = 0, KIND_DOT = 1 };

// VUPD variants: FULL = the Lanczos vectors are present (v2 may equal v1 with
// cvp = 0); STEN = the stencil term is added (the constant-coefficient split
// matvec); Q1 = q has a single tap.
template <typename T, int L, int KIND, bool FULL, bool Q1, bool STEN = FULL, class Ctx>
BLTT_HD void dst_x_body(Ctx& ctx, cx<T>* lds, double* red, const T* in,
                        const T* __restrict__ v1, const T* __restrict__ v2, T* __restrict__ vout,
                        const T* __restrict__ vdot, T* out, int64_t nlines,
                        const DstTables<T>& tb, const double* __restrict__ coef,
                        double* __restrict__ partials, const VupdStencil<T>& sten) {
  constexpr int TPB = tpb_fft<T, FK_DSTX>();
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0), VH = V / 2;
  using F = LineFft<T, L, NL, false, LAST_LINEAR>;
  const int m = L / 2 - 1;
  const int tid = ctx.tid, c = tid / G, g = tid % G;
  const int64_t la = (int64_t)ctx.bid * (2 * NL) + 2 * c, lb = la + 1;
  const bool va = la < nlines, vb = lb < nlines;
  // clamped line indices: every load below is in bounds and unconditional
  const int64_t lac = va ? la : nlines - 1, lbc = vb ? lb : nlines - 1;
  const T ma = va ? T(1) : T(0), mb = vb ? T(1) : T(0);
  T cq = T(1), cv = T(0), cvp = T(0);
  if (KIND == KIND_VUPD) {
    cq = T(coef[0]);
    cv = T(coef[1]);
    cvp = T(coef[2]);
  }
  LineStencil<T> lsa, lsb;
  if (KIND == KIND_VUPD && STEN) {
    lsa = line_stencil(sten, lac);
    lsb = line_stencil(sten, lbc);
  }
  cx<T> v[V];
  // positions p = g + t*s0 < L/2 for t < V/2: element x = p - 1 (p = 0 is the zero of the extension)
#pragma unroll
  for (int t = 0; t < VH; ++t) {
    const int p = g + t * s0;
    const int x = p > 0 ? p - 1 : 0;
    const T wp = p > 0 ? T(1) : T(0);
    const int64_t ea = lac * m + x, eb = lbc * m + x;
    T a = in[ea], b = in[eb];
    if (KIND == KIND_VUPD && STEN) {
      a += line_stencil_at<T, Q1>(sten, lsa, x);
      b += line_stencil_at<T, Q1>(sten, lsb, x);
    }
    a *= cq;
    b *= cq;
    if (KIND == KIND_VUPD && FULL) {
      a += cv * v1[ea] + cvp * v2[ea];
      b += cv * v1[eb] + cvp * v2[eb];
    }
    a *= wp * ma;
    b *= wp * mb;
    v[t] = mkc<T>(a, b);
  }
  if (KIND == KIND_VUPD && FULL) {
    // the updated Lanczos vector (vout never aliases in, v1, v2); stores come
    // after all loads so the loads above can all be in flight together
#pragma unroll
    for (int t = 0; t < VH; ++t) {
      const int p = g + t * s0;
      if (p > 0) {
        if (va) vout[la * m + p - 1] = v[t].re;
        if (vb) vout[lb * m + p - 1] = v[t].im;
      }
    }
  }
  odd_mirror<F, T, L>(ctx, v, lds, c, g);
  F::forward(ctx, v, lds, c, g, tb.tw);
  double part = 0.0;
#pragma unroll
  for (int w = 0; w < V / F::RL; ++w) {
#pragma unroll
    for (int u = 0; u < F::RL; ++u) {
      const int k = F::freq(g, w, u);
      if (k >= 1 && k <= m) {
        const cx<T> zk = v[w * F::RL + u];
        const T ya = -zk.im * tb.nrm, yb = zk.re * tb.nrm;
        if (va) {
          out[la * m + k - 1] = ya;
          if (KIND == KIND_DOT) part += (double)ya * (double)vdot[la * m + k - 1];
        }
        if (vb) {
          out[lb * m + k - 1] = yb;
          if (KIND == KIND_DOT) part += (double)yb * (double)vdot[lb * m + k - 1];
        }
      }
    }
  }
  if (KIND == KIND_DOT) {
    const double s = block_sum<TPB>(ctx, red, part);
    if (tid == 0) partials[ctx.bid] = s;
  }
}

// Lines along a strided dimension: line l has elements at
// (l / S) * S * m + (l % S) + j * S, j < m.  In place.
// PAIRED (S and nlines even): the two lines of a thread's pair, la even and
// la + 1, are adjacent in memory and share one 2-element access.
template <typename T>
struct alignas(2 * sizeof(T)) Pair2 {
  T a, b;
};
template <typename T, int L, bool PAIRED, class Ctx>
BLTT_HD void dst_strided_body(Ctx& ctx, cx<T>* lds, T* __restrict__ x, int64_t nlines, int64_t S,
                              const DstTables<T>& tb) {
  constexpr int TPB = tpb_fft<T, FK_DSTS>();
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0);
  using F = LineFft<T, L, NL, true, LAST_DEFAULT, false, 0, dst_split<T>()>;
  const int m = L / 2 - 1;
  const int tid = ctx.tid, c = tid % NL, g = tid / NL;
  const int64_t la = xcd_tile(ctx.bid, ctx.nbx) * (2 * NL) + 2 * c, lb = la + 1;
  const bool va = la < nlines, vb = lb < nlines;
  // PAIRED: va implies vb, and a missing pair reads the last pair (in bounds)
  const int64_t lac = va ? la : (PAIRED ? nlines - 2 : nlines - 1), lbc = vb ? lb : nlines - 1;
  const int64_t basea = (lac / S) * S * m + (lac % S);
  const int64_t baseb = PAIRED ? basea + 1 : (lbc / S) * S * m + (lbc % S);
  const T ma = va ? T(1) : T(0), mb = vb ? T(1) : T(0);
  constexpr int VH = V / 2;
  // every stage's twiddle bases in flight with the line's loads, so no stage
  // waits for its table after an exchange barrier
  cx<T> pre[F::PF_LEN > 0 ? F::PF_LEN : 1];
  F::template pf_load<0>(pre, tb.tw, g);
  cx<T> v[V];
#pragma unroll
  for (int t = 0; t < VH; ++t) {
    const int p = g + t * s0;
    const int64_t xi = p > 0 ? p - 1 : 0;
    const T w = p > 0 ? T(1) : T(0);
    if constexpr (PAIRED) {
      const Pair2<T> ab = *reinterpret_cast<const Pair2<T>*>(x + basea + xi * S);
      v[t] = mkc<T>(ab.a * (w * ma), ab.b * (w * mb));
    } else {
      v[t] = mkc<T>(x[basea + xi * S] * (w * ma), x[baseb + xi * S] * (w * mb));
    }
  }
  odd_mirror<F, T, L>(ctx, v, lds, c, g);
  F::forward_pf(ctx, v, lds, c, g, pre);
  // all reads of this workgroup's lines happened before the barriers inside forward()
#pragma unroll
  for (int w = 0; w < V / F::RL; ++w) {
#pragma unroll
    for (int u = 0; u < F::RL; ++u) {
      const int k = F::freq(g, w, u);
      if (k >= 1 && k <= m) {
        const cx<T> zk = v[w * F::RL + u];
        if constexpr (PAIRED) {
          Pair2<T> ab;
          ab.a = -zk.im * tb.nrm;
          ab.b = zk.re * tb.nrm;
          if (va) *reinterpret_cast<Pair2<T>*>(x + basea + (int64_t)(k - 1) * S) = ab;
        } else {
          if (va) x[basea + (int64_t)(k - 1) * S] = -zk.im * tb.nrm;
          if (vb) x[baseb + (int64_t)(k - 1) * S] = zk.re * tb.nrm;
        }
      }
    }
  }
}

// Sine transform along x fused with the move between the time-major layout
// (element (n, i) at n*M + i) and the mode-major one (i*N + n).  The x-line of
// row r (r < M/m, i = r*m + x) at time n is one line; a workgroup takes 2*NL
// consecutive times of one row, so the mode-major side is read or written in
// runs of 2*NL elements and the time-major side in whole x-lines.  The
// mode-major side goes through LDS (the exchange buffer, before or after the
// transform).
// DIR 0: time-major `in` -> mode-major `out`, and one partial sum of ||in||^2
//        per workgroup (= ||out||^2, U being orthogonal; partials may be null).
// DIR 1: mode-major `in` -> time-major `out`.
constexpr int DSTXT_TPB = 256;
template <typename T, int L>
constexpr int dstxt_lines() { return 2 * (DSTXT_TPB / (L / fft_V(L))); }
// workgroups of a launch: rows x time blocks, rounded up to a multiple of 8
BLTT_HD int64_t dstxt_blocks(int64_t rows, int64_t N, int W2) {
  const int64_t nb = rows * ((N + W2 - 1) / W2);
  return (nb + 7) / 8 * 8;
}
template <typename T, int L, int DIR, class Ctx>
BLTT_HD void dst_xt_body(Ctx& ctx, cx<T>* lds, double* red, const T* __restrict__ in, T* __restrict__ out,
                         int64_t N, int64_t M, const DstTables<T>& tb, double* __restrict__ partials) {
  constexpr int TPB = DSTXT_TPB;
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0), VH = V / 2, W2 = 2 * NL;
  // linear last stage both ways: lane g holds frequencies g + G w + u K, so
  // DIR 1's global stores coalesce and DIR 0's stage writes hit consecutive
  // banks (the default deal puts consecutive lanes 16 entries apart)
  using F = LineFft<T, L, NL, false, LAST_LINEAR, false, 0, dst_split<T>()>;
  static_assert((size_t)W2 * (L / 2 - 1) * sizeof(T) <= (size_t)F::LDS_ELEMS * sizeof(cx<T>),
                "the staging rows fit in the exchange buffer");
  static_assert(G <= TPB, "one line per at most one workgroup");
  const int m = L / 2 - 1;
  const int64_t rows = M / m, nblk = (N + W2 - 1) / W2;
  const int64_t tile = xcd_tile(ctx.bid, ctx.nbx);
  const bool live = tile < rows * nblk;
  const int64_t r = live ? tile / nblk : 0, n0 = live ? (tile % nblk) * W2 : N;
  const int tid = ctx.tid, c = tid / G, g = tid % G;
  const int64_t na = n0 + 2 * c, nb = na + 1;
  const bool va = na < N, vb = nb < N;
  T* stage = reinterpret_cast<T*>(lds);  // W2 x m values, line-major
  // DIR 1: every stage's twiddles in flight with the line's loads (faster
  // for DIR 1 as measured, slower for DIR 0)
  constexpr bool PF = DIR == 1;
  cx<T> pre[PF && F::PF_LEN > 0 ? F::PF_LEN : 1];
  if constexpr (PF) F::template pf_load<0>(pre, tb.tw, g);
  cx<T> v[V];
  double part = 0.0;
  if (DIR == 0) {
    const int64_t nac = va ? na : 0, nbc = vb ? nb : 0;
    const T* pa = in + nac * M + r * m;
    const T* pb = in + nbc * M + r * m;
    const T ma = va ? T(1) : T(0), mb = vb ? T(1) : T(0);
#pragma unroll
    for (int t = 0; t < VH; ++t) {
      const int p = g + t * s0;
      const int x = p > 0 ? p - 1 : 0;
      const T wp = p > 0 ? T(1) : T(0);
      const T a = pa[x] * (wp * ma), b = pb[x] * (wp * mb);
      part += (double)a * (double)a + (double)b * (double)b;
      v[t] = mkc<T>(a, b);
    }
  } else {
    // runs of W2 consecutive times per x, into LDS line-major; all loads are
    // issued before the first LDS store
    constexpr int IT = (W2 * m + TPB - 1) / TPB;
    T val[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + it * TPB;
      const int x = e / W2, j = e % W2;
      const int64_t n = n0 + j;
      val[it] = (e < W2 * m && n < N) ? in[(r * m + x) * N + n] : T(0);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + it * TPB;
      if (e < W2 * m) stage[(e % W2) * m + e / W2] = val[it];
    }
    ctx.sync();
#pragma unroll
    for (int t = 0; t < VH; ++t) {
      const int p = g + t * s0;
      const int x = p > 0 ? p - 1 : 0;
      const T wp = p > 0 ? T(1) : T(0);
      v[t] = mkc<T>(stage[(2 * c) * m + x] * wp, stage[(2 * c + 1) * m + x] * wp);
    }
    // the mirror below writes the exchange buffer the stage lives in
    ctx.sync();
  }
  odd_mirror<F, T, L>(ctx, v, lds, c, g);
  if constexpr (PF)
    F::forward_pf(ctx, v, lds, c, g, pre);
  else
    F::forward(ctx, v, lds, c, g, tb.tw);
  if (DIR == 0) {
    ctx.sync();
#pragma unroll
    for (int w = 0; w < V / F::RL; ++w) {
#pragma unroll
      for (int u = 0; u < F::RL; ++u) {
        const int k = F::freq(g, w, u);
        if (k >= 1 && k <= m) {
          const cx<T> zk = v[w * F::RL + u];
          stage[(2 * c) * m + k - 1] = -zk.im * tb.nrm;
          stage[(2 * c + 1) * m + k - 1] = zk.re * tb.nrm;
        }
      }
    }
    ctx.sync();
    if (live) {
      constexpr int IT = (W2 * m + TPB - 1) / TPB;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = tid + it * TPB;
        const int k = e / W2, j = e % W2;
        const int64_t n = n0 + j;
        if (e < W2 * m && n < N) out[(r * m + k) * N + n] = stage[j * m + k];
      }
    }
    if (partials) {
      const double sum = block_sum<TPB>(ctx, red, part);
      if (tid == 0) partials[ctx.bid] = sum;
    }
  } else {
    T* oa = out + na * M + r * m;
    T* ob = out + nb * M + r * m;
#pragma unroll
    for (int w = 0; w < V / F::RL; ++w) {
#pragma unroll
      for (int u = 0; u < F::RL; ++u) {
        const int k = F::freq(g, w, u);
        if (k >= 1 && k <= m) {
          const cx<T> zk = v[w * F::RL + u];
          if (live && va) oa[k - 1] = -zk.im * tb.nrm;
          if (live && vb) ob[k - 1] = zk.re * tb.nrm;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// time pass of the preconditioner, per sine mode i (Section 5.1 Step 2, both
// halves):  t <- alpha^{-n/N} t;  t <- F conj(Lambda_i)^{-1/2} F^* t;
// t <- alpha^{2n/N} t;  t <- F Lambda_i^{-1/2} F^* t;  t <- alpha^{-n/N} t.
// lambda_{i,k} = sigma_k + mu_i rho_k (eq. (9) for blocks p_k I + q_k L_h),
// square roots on the principal branch (Definition 2), computed on the fly.
// Two modes a, b share one complex line; their spectra are separated with
// A_k = (Z_k + conj Z_{N-k})/2, B_k = (Z_k - conj Z_{N-k})/(2i).
// ---------------------------------------------------------------------------
template <typename T>
struct TimeTables {
  const cx<T>* tw;     // length N
  const T* dinv;       // alpha^{-n/N}
  const T* d2;         // alpha^{2n/N}
  const cx<T>* sigma;  // fft(alpha^{j/N} p_j)
  const cx<T>* rho;    // fft(alpha^{j/N} q_j)
  const T* mu;         // length M, Laplacian eigenvalue of each sine mode
  T log2_alpha_over_N; // log2(alpha)/N for the FP32 scalings
  T q[4];              // leading taps of q
  int qtaps;
  double* aux;         // per-workgroup sum_i mu_i sum_n (q * t_i)[N-1-n] t_i[n] (or null)
  int mx = 1;          // mode-major lines: modes per x-row (mode_pair)
};

// 1 / (N s), s the principal square root of lambda (Re lambda > 0, Definition 2):
// with r = |lambda|, s = sqrt((r + Re l)/2) + i Im l / (2 sqrt((r + Re l)/2))
// and 1/s = conj(s)/r.  FP32 uses the hardware reciprocal square root.
BLTT_HD cx<float> inv_sqrt_scaled(cx<float> lam, float invN) {
  const float r2 = lam.re * lam.re + lam.im * lam.im;
#if defined(__HIP_DEVICE_COMPILE__)
  const float rinv = __builtin_amdgcn_rsqf(r2);
#else
  const float rinv = 1.0f / sqrtf(r2);
#endif
  const float r = r2 * rinv;
  const float t = (r + lam.re) * 0.5f;
#if defined(__HIP_DEVICE_COMPILE__)
  const float w = __builtin_amdgcn_rsqf(t);
#else
  const float w = 1.0f / sqrtf(t);
#endif
  const float sr = t * w, si = 0.5f * lam.im * w;
  const float f = invN * rinv;
  return mkc<float>(sr * f, -si * f);
}
BLTT_HD cx<double> inv_sqrt_scaled(cx<double> lam, double invN) {
  const double r = sqrt(lam.re * lam.re + lam.im * lam.im);
  const double sr = sqrt((r + lam.re) * 0.5);
  const double si = lam.im / (2.0 * sr);
  const double f = invN / r;
  return mkc<double>(sr * f, -si * f);
}

// alpha^{e n / N}: FP32 evaluates exp2 on the fly, FP64 reads the table.
BLTT_HD float alpha_pow_n(const TimeTables<float>& tb, const float* tab, float e, int n) {
  (void)tab;
  return exp2f(e * tb.log2_alpha_over_N * (float)n);
}
BLTT_HD double alpha_pow_n(const TimeTables<double>& tb, const double* tab, double e, int n) {
  (void)tb;
  (void)e;
  return tab[n];
}

// Multiplies v[t] (time n = g + t*s0) by alpha^{e n/N}.  FP32: two exp2 per
// thread and a product chain over t (relative error below 2e-6 for V = 16);
// FP64: the table.  With DOT, also returns sum_t re(v_t before) re(v_t after)
// (the real line's share of the dot), and the imaginary line's in *dot_im.
template <typename T, int V, int s0, bool DOT = false>
BLTT_HD T scale_alpha(cx<T>* v, const TimeTables<T>& tb, const T* tab, T e, int g, T* dot_im = nullptr) {
  T acc0 = T(0), acc1 = T(0);
  T d = T(0), st = T(0);
  if constexpr (sizeof(T) == 4) {
    d = alpha_pow_n(tb, tab, e, g);
    st = alpha_pow_n(tb, tab, e, s0);
  }
#pragma unroll
  for (int t = 0; t < V; ++t) {
    if constexpr (sizeof(T) != 4) d = alpha_pow_n(tb, tab, e, g + t * s0);
    const cx<T> w = v[t] * d;
    if (DOT) {
      acc0 += v[t].re * w.re;
      acc1 += v[t].im * w.im;
    }
    v[t] = w;
    if constexpr (sizeof(T) == 4) d *= st;
  }
  if (DOT) *dot_im = acc1;
  return acc0;
}

// The two-for-one spectral step.  A packed line holds mode a in its real part
// and mode b in its imaginary part; with A_k = (Z_k + conj Z_{L-k})/2 and
// B_k = (Z_k - conj Z_{L-k})/(2i) and per-mode multipliers g_a, g_b at k, the
// new values are Z_k <- Z_k hp + conj(Z_{L-k}) hm with hp = (g_a + g_b)/2,
// hm = (g_a - g_b)/2; the multipliers of L - k are the conjugates of those of
// k.  The multipliers are 1/(N s), s the principal square root of lambda; the
// first half-solve uses their conjugates.  The first half computes them and
// keeps (hp, hm) in `gm`, the second reuses them.
template <typename T>
struct SpecMul {
  cx<T> p, m;
};

template <typename T>
BLTT_HD SpecMul<T> spectral_mul(int k, T mua, T mub, const TimeTables<T>& tb, T halfInvN) {
  const cx<T> sg = tb.sigma[k];
  const cx<T> rh = tb.rho[k];
  const cx<T> ga = inv_sqrt_scaled(sg + rh * mua, halfInvN);
  const cx<T> gb = inv_sqrt_scaled(sg + rh * mub, halfInvN);
  SpecMul<T> r;
  r.p = ga + gb;
  r.m = ga - gb;
  return r;
}

// frequencies k (Z1) and L - k (Z2)
template <typename T, int HALF>
BLTT_HD void spectral_apply(cx<T>& Z1, cx<T>& Z2, const SpecMul<T>& g) {
  const cx<T> hp = HALF == 0 ? conjg(g.p) : g.p, hm = HALF == 0 ? conjg(g.m) : g.m;
  const cx<T> n1 = Z1 * hp + conjg(Z2) * hm;
  const cx<T> n2 = Z2 * conjg(hp) + conjg(Z1) * conjg(hm);
  Z1 = n1;
  Z2 = n2;
}

// a frequency equal to its own mirror (k = 0 or L/2)
template <typename T, int HALF>
BLTT_HD void spectral_self(cx<T>& Z, const SpecMul<T>& g) {
  const cx<T> hp = HALF == 0 ? conjg(g.p) : g.p, hm = HALF == 0 ? conjg(g.m) : g.m;
  Z = Z * hp + conjg(Z) * hm;
}

// multiplier slots one thread keeps between the halves
template <int L, class F>
constexpr int spec_slots() {
  return F::S == 1 ? L / 2 + 1 : (F::V / F::RL / 2) * F::RL + 1;
}

// After the forward transform a thread holds, per pair p of its last-stage
// butterflies, s0[u] at frequency q + u K and s1[RL-1-u] at L - (q + u K)
// (q = g PP + p), except on the one lane with q = 0, whose butterflies hold
// k = u K and k = K/2 + u K: there the mirrors sit at s0[RL-u] and
// s1[RL-1-u], and k = 0, L/2 are their own mirrors.  That lane's values are
// re-dealt with selects into the common pattern (the two self frequencies
// sharing the last slot), so every lane runs the same instructions.
// select between two values (a conditional expression on two class lvalues
// would select their addresses and keep the operands in memory)
template <typename T>
BLTT_HD cx<T> csel(bool c, cx<T> a, cx<T> b) {
  return mkc<T>(c ? a.re : b.re, c ? a.im : b.im);
}

template <typename T, int L, class F, int HALF>
BLTT_HD void time_spectral(cx<T>* v, int g, T mua, T mub, const TimeTables<T>& tb, T invN, SpecMul<T>* gm) {
  constexpr int RL = F::RL, NB = F::V / RL, K = F::K;
  const T hinv = T(0.5) * invN;
  if constexpr (F::S == 1) {
    if (HALF == 0)
      for (int u = 0; u <= L / 2; ++u) gm[u] = spectral_mul(u, mua, mub, tb, hinv);
    spectral_self<T, HALF>(v[0], gm[0]);
#pragma unroll
    for (int u = 1; u < L / 2; ++u) spectral_apply<T, HALF>(v[u], v[L - u], gm[u]);
    if constexpr (L >= 2) spectral_self<T, HALF>(v[L / 2], gm[L / 2]);
  } else {
    constexpr int PP = NB / 2;
#pragma unroll
    for (int p = 0; p < PP; ++p) {
      const int q = g * PP + p;
      cx<T>* s0 = v + (2 * p) * RL;
      cx<T>* s1 = v + (2 * p + 1) * RL;
      SpecMul<T>* m = gm + p * RL;
      if (p != 0) {
        // q >= 1 on every lane
#pragma unroll
        for (int u = 0; u < RL; ++u) {
          if (HALF == 0) m[u] = spectral_mul(q + u * K, mua, mub, tb, hinv);
          spectral_apply<T, HALF>(s0[u], s1[RL - 1 - u], m[u]);
        }
        continue;
      }
      const bool q0 = q == 0;
      cx<T> X[RL], Y[RL];
#pragma unroll
      for (int u = 0; u < RL; ++u) {
        Y[u] = s1[u];
        if (u < RL / 2) {
          X[u] = csel(q0, s1[u], s0[u]);
        } else if (u < RL - 1) {
          X[u] = csel(q0, s0[u - RL / 2 + 1], s0[u]);
          Y[RL - 1 - u] = csel(q0, s0[3 * RL / 2 - 1 - u], s1[RL - 1 - u]);
        } else {
          X[u] = csel(q0, s0[0], s0[u]);
        }
      }
      Y[0] = csel(q0, s0[RL / 2], s1[0]);
      if (HALF == 0) {
#pragma unroll
        for (int u = 0; u < RL; ++u) {
          const int kq0 = u < RL / 2 ? K / 2 + u * K : (u < RL - 1 ? (u - RL / 2 + 1) * K : 0);
          m[u] = spectral_mul(q0 ? kq0 : q + u * K, mua, mub, tb, hinv);
        }
        gm[PP * RL] = spectral_mul(L / 2, mua, mub, tb, hinv);
      }
#pragma unroll
      for (int u = 0; u < RL - 1; ++u) spectral_apply<T, HALF>(X[u], Y[RL - 1 - u], m[u]);
      {
        cx<T> x = X[RL - 1], y = Y[0], xs = x, ys = y;
        spectral_apply<T, HALF>(x, y, m[RL - 1]);
        spectral_self<T, HALF>(xs, m[RL - 1]);
        spectral_self<T, HALF>(ys, gm[PP * RL]);
        X[RL - 1] = csel(q0, xs, x);
        Y[0] = csel(q0, ys, y);
      }
      // deal back
#pragma unroll
      for (int u = 0; u < RL; ++u) {
        cx<T> a0;  // s0[u] on the q = 0 lane
        if (u == 0)
          a0 = X[RL - 1];
        else if (u < RL / 2)
          a0 = X[u + RL / 2 - 1];
        else if (u == RL / 2)
          a0 = Y[0];
        else
          a0 = Y[u - RL / 2];
        s0[u] = csel(q0, a0, X[u]);
        s1[u] = u < RL / 2 ? csel(q0, X[u], Y[u]) : Y[u];
      }
    }
  }
}

template <typename T, int L, class Ctx>
BLTT_HD void time_prec_body(Ctx& ctx, cx<T>* lds, double* red, T* __restrict__ x, int64_t M,
                            const TimeTables<T>& tb) {
  constexpr int TPB = tpb_fft<T, FK_TIME>();
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0);
  using F = LineFft<T, L, NL, true, LAST_PAIRED>;
  const T invN = T(1) / T(L);
  const int tid = ctx.tid, c = tid % NL, g = tid / NL;
  const int64_t ia = xcd_tile(ctx.bid, ctx.nbx) * (2 * NL) + 2 * c, ib = ia + 1;
  const bool va = ia < M, vb = ib < M;
  const int64_t iac = va ? ia : M - 1, ibc = vb ? ib : M - 1;
  const T mua = tb.mu[iac], mub = tb.mu[ibc];
  const T wa = va ? T(1) : T(0), wb = vb ? T(1) : T(0);
  T* xa = x + ia;
  T* xb = x + ib;

  cx<T> v[V];
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int n = g + t * s0;
    const T d = alpha_pow_n(tb, tb.dinv, T(-1), n);
    const int64_t off = (int64_t)n * M;
    v[t] = mkc<T>(x[iac + off] * (d * wa), x[ibc + off] * (d * wb));
  }
  SpecMul<T> gm[spec_slots<L, F>()];
  F::forward(ctx, v, lds, c, g, tb.tw);
  time_spectral<T, L, F, 0>(v, g, mua, mub, tb, invN, gm);
  F::inverse(ctx, v, lds, c, g, tb.tw);
  scale_alpha<T, V, s0>(v, tb, tb.d2, T(2), g);
  F::forward(ctx, v, lds, c, g, tb.tw);
  time_spectral<T, L, F, 1>(v, g, mua, mub, tb, invN, gm);
  F::inverse(ctx, v, lds, c, g, tb.tw);
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int n = g + t * s0;
    const T d = alpha_pow_n(tb, tb.dinv, T(-1), n);
    v[t] = v[t] * d;
    const int64_t off = (int64_t)n * M;
    if (va) xa[off] = v[t].re;
    if (vb) xb[off] = v[t].im;
  }
  if (tb.aux) {
    // The output t = U z in sine coordinates, where L_h = diag(mu): the
    // spatial part of the next matvec's <Y A z, z> is
    // sum_i mu_i sum_n sum_k q_k t_i[N-1-n-k] t_i[n].
    ctx.sync();
#pragma unroll
    for (int t = 0; t < V; ++t) lds[F::idx(c, g + t * s0)] = v[t];
    ctx.sync();
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < V; ++t) {
      const int n = g + t * s0;
      double sa = 0.0, sb = 0.0;
      for (int k = 0; k < tb.qtaps; ++k) {
        const int nr = L - 1 - n - k;
        if (nr < 0) break;
        const cx<T> w = lds[F::idx(c, nr)];
        sa += (double)tb.q[k] * (double)w.re;
        sb += (double)tb.q[k] * (double)w.im;
      }
      if (va) part += (double)mua * sa * (double)v[t].re;
      if (vb) part += (double)mub * sb * (double)v[t].im;
    }
    const double sum = block_sum<TPB>(ctx, red, part);
    if (tid == 0) tb.aux[ctx.bid] = sum;
  }
}

// ---------------------------------------------------------------------------
// Lanczos update fused with the time pass, for MINRES run in sine coordinates.
// When every block is p_k I + q_k L_h, the orthonormal sine transform U
// diagonalises L_h (Remark 1) and commutes with Y, so MINRES on
// (I x U) Y A (I x U) with P^{-1} carried along is MINRES on Y A in another
// orthonormal basis: the same scalars, and iterates that differ by the change
// of basis.  In that basis P^{-1} is the time pass alone (Section 5.1 Step 2).
// Per pair of modes a, b (one complex line):
//   vhat = cq Q + cv V1 + cvp V2   (FULL; cq Q alone otherwise), stored to Vout
//                                  when Vout is non-null;
//   zhat = P^{-1} vhat             stored to Zout;
//   partial sums of <vhat, zhat>   one per workgroup.
// Q may be FP64 for an FP32 pass (the refinement right-hand side, scaled by cq
// in FP64 before rounding), and the start may read it time-reversed (Y Q).  Since P^{-1} = C^{-1/2} (C^{-1/2})^* with C^{-1/2}
// real (Section 3), <vhat, P^{-1} vhat> = ||(C^{-1/2})^* vhat||^2: the dot is
// taken on the intermediate after the first half-solve, so vhat need not be
// kept or read again.
// ---------------------------------------------------------------------------
// PREC false: no preconditioner (zhat = vhat), the MINRES-I comparator
template <typename T, int L, typename TQ, bool FULL, bool MM, int TPB = tpb_fft<T, FK_SPEC>(), bool PREC = true,
          bool TWL = false, int PLAN = 0, class Ctx>
BLTT_HD double time_upd_tile(Ctx& ctx, cx<T>* lds, int64_t tile, const TQ* __restrict__ Q,
                             const T* __restrict__ V1, const T* __restrict__ V2, T* __restrict__ Vout,
                             T* __restrict__ Zout, int64_t M, const TimeTables<T>& tb,
                             const double* __restrict__ coef, bool qrev = false) {
  constexpr int V = fft_V(L), G = L / V, NL = TPB / G, s0 = fft_sigma(L, 0);
  using F = LineFft<T, L, NL, !MM, LAST_PAIRED, TWL, PLAN>;
  const T invN = T(1) / T(L);
  const int tid = ctx.tid, c = MM ? tid / G : tid % NL;
  int g = MM ? tid % G : tid / NL;
#if defined(__HIP_DEVICE_COMPILE__)
  // g is opaque to the compiler here, so that a tile loop around this function
  // does not keep g-dependent table loads (twiddles, spectra) live across
  // tiles at the cost of occupancy
  asm volatile("" : "+v"(g));
  // g < G again for the compiler: LDS positions g + t*s0 then split into a
  // per-lane base and compile-time offsets (the ds instructions' immediates)
  g &= G - 1;
#endif
  int64_t ia = tile * (2 * NL) + 2 * c, ib = ia + 1;
  if constexpr (MM) mode_pair(tile * NL + c, M, tb.mx, ia, ib);
  const bool va = ia < M, vb = ib < M;
  const int64_t iac = va ? ia : M - 1, ibc = vb ? ib : M - 1;
  // element (i, n): time-major n*M + i, or mode-major i*N + n (N = L)
  const int64_t ts = MM ? 1 : M;
  const int64_t la = MM ? iac * L : iac, lb = MM ? ibc * L : ibc;
  // per-lane pointers at time g (Q reversed: L-1-g); the time offset t*s0*ts
  // is then a compile-time constant in the mode-major layout (the memory
  // instructions' immediates).  Stores go through the clamped line bases,
  // equal to the exact ones wherever the store's guard holds.
  const bool rq = !FULL && qrev;
  const int64_t gq = (int64_t)(rq ? L - 1 - g : g) * ts, gv = (int64_t)g * ts;
  const TQ* qa = Q + la + gq;
  const TQ* qb = Q + lb + gq;
  const T mua = tb.mu[iac], mub = tb.mu[ibc];
  const double cq = coef[0];
  T cv = T(0), cvp = T(0);
  if (FULL) {
    cv = T(coef[1]);
    cvp = T(coef[2]);
  }

  // every load of the tile first, one wait after them all: the empty asm
  // statements keep the loads above the "memory" barrier and the arithmetic
  // on them below it (left alone, the scheduler may trade the batch for
  // registers and wait after every few loads, once per memory round trip)
  TQ xqa[V], xqb[V];
  T x1a[FULL ? V : 1], x1b[FULL ? V : 1], x2a[FULL ? V : 1], x2b[FULL ? V : 1];
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int64_t off = (int64_t)(t * s0) * ts;
    // qrev (start only): Q read with its time lines reversed, i.e. Y Q
    const int64_t offq = rq ? -off : off;
    xqa[t] = qa[offq];
    xqb[t] = qb[offq];
    if constexpr (FULL) {
      x1a[t] = V1[la + gv + off];
      x1b[t] = V1[lb + gv + off];
      x2a[t] = V2[la + gv + off];
      x2b[t] = V2[lb + gv + off];
    }
  }
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" ::: "memory");
#pragma unroll
  for (int t = 0; t < V; ++t) {
    asm volatile("" : "+v"(xqa[t]), "+v"(xqb[t]));
    if constexpr (FULL) asm volatile("" : "+v"(x1a[t]), "+v"(x1b[t]), "+v"(x2a[t]), "+v"(x2b[t]));
  }
#endif
  cx<T> v[V];
#pragma unroll
  for (int t = 0; t < V; ++t) {
    T a, b;
    if constexpr (sizeof(TQ) > sizeof(T)) {
      a = T((double)xqa[t] * cq);
      b = T((double)xqb[t] * cq);
    } else {
      a = T(cq) * xqa[t];
      b = T(cq) * xqb[t];
    }
    if constexpr (FULL) {
      a += cv * x1a[t] + cvp * x2a[t];
      b += cv * x1b[t] + cvp * x2b[t];
    }
    // a line past M reads the clamped line M-1: finite values whose
    // transforms stay in their own half of the packed line; its stores are
    // guarded and its share of the dot is masked
    v[t] = mkc<T>(a, b);
  }
  if (Vout) {
    T* oa = Vout + la + gv;
    T* ob = Vout + lb + gv;
#pragma unroll
    for (int t = 0; t < V; ++t) {
      const int64_t off = (int64_t)(t * s0) * ts;
      if (va) oa[off] = v[t].re;
      if (vb) ob[off] = v[t].im;
    }
  }
  double part = 0.0;
  if constexpr (PREC) {
    SpecMul<T> gm[spec_slots<L, F>()];
    scale_alpha<T, V, s0>(v, tb, tb.dinv, T(-1), g);
    F::forward(ctx, v, lds, c, g, tb.tw);
    time_spectral<T, L, F, 0>(v, g, mua, mub, tb, invN, gm);
    F::inverse(ctx, v, lds, c, g, tb.tw);
    // v = D^{-1} (C^{-1/2})^* vhat here, so with w = (C^{-1/2})^* vhat,
    // ||w||^2 = sum_t <v, D^2 v>, taken while scaling by the middle D^2
    T dot_b;
    const T dot_a = scale_alpha<T, V, s0, true>(v, tb, tb.d2, T(2), g, &dot_b);
    part = (va ? (double)dot_a : 0.0) + (vb ? (double)dot_b : 0.0);
    F::forward(ctx, v, lds, c, g, tb.tw);
    time_spectral<T, L, F, 1>(v, g, mua, mub, tb, invN, gm);
    F::inverse(ctx, v, lds, c, g, tb.tw);
    scale_alpha<T, V, s0>(v, tb, tb.dinv, T(-1), g);
  }
  T* za = Zout + la + gv;
  T* zb = Zout + lb + gv;
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int64_t off = (int64_t)(t * s0) * ts;
    if (va) za[off] = v[t].re;
    if (vb) zb[off] = v[t].im;
    if constexpr (!PREC)
      part += (va ? (double)v[t].re * (double)v[t].re : 0.0) + (vb ? (double)v[t].im * (double)v[t].im : 0.0);
  }
  return part;
}

// The persistent FP32 time pass takes its stage twiddles from an LDS table
// (tb.tw then points to it; built once per workgroup).
template <typename T>
constexpr bool upd_twl() { return sizeof(T) == 4; }
// The spectra sigma_k, rho_k of eq. (9) go to LDS beside the twiddles where
// that still leaves two workgroups per CU: every tile reads 2 (V/2 + 1)
// entries of each, which from global memory are dependent L2 round trips
// inside the transform pipeline.
template <typename T, int L>
constexpr bool upd_spec_lds() {
  return upd_twl<T>() && fft_lds_bytes<T, FK_SPEC>(L) + 3 * (size_t)L * sizeof(cx<T>) <= 80 * 1024;
}
template <typename T, int L>
constexpr size_t upd_twl_bytes() {
  return upd_twl<T>() ? (size_t)(upd_spec_lds<T, L>() ? 3 : 1) * L * sizeof(cx<T>) : 0;
}

// FP32 runs persistently (workgroup b takes tiles b, b + nbx, ...); FP64,
// whose registers allow one wavefront per SIMD, one tile per workgroup.  One
// partial sum of <vhat, zhat> per workgroup.
template <typename T>
constexpr bool upd_persistent() { return sizeof(T) == 4; }

template <typename T, int L, typename TQ, bool FULL, bool MM, bool PREC = true, int PLAN = 0, class Ctx>
BLTT_HD void time_upd_body(Ctx& ctx, cx<T>* lds, double* red, const TQ* __restrict__ Q,
                           const T* __restrict__ V1, const T* __restrict__ V2, T* __restrict__ Vout,
                           T* __restrict__ Zout, int64_t M, const TimeTables<T>& tb,
                           const double* __restrict__ coef, double* __restrict__ partials, bool qrev = false) {
  constexpr int TPB = tpb_fft<T, FK_SPEC>();
  const int64_t ntiles = fft_tiles<T, FK_SPEC>(L, M);
  TimeTables<T> tl = tb;
  if constexpr (upd_twl<T>() && PREC) {
    // the stage twiddles in LDS, after the exchange lines and the reduction slots
    using F = LineFft<T, L, TPB / (L / fft_V(L)), !MM, LAST_PAIRED, true, PLAN>;
    cx<T>* twl = reinterpret_cast<cx<T>*>(red + TPB);
    F::template build_twl<TPB>(ctx, twl, tb.tw);
    if constexpr (upd_spec_lds<T, L>()) {
      cx<T>* sgl = twl + L;
      cx<T>* rhl = sgl + L;
      for (int i = ctx.tid; i < L; i += TPB) {
        sgl[i] = tb.sigma[i];
        rhl[i] = tb.rho[i];
      }
      tl.sigma = sgl;
      tl.rho = rhl;
    }
    ctx.sync();
    tl.tw = twl;
  }
  double part = 0.0;
  if constexpr (upd_persistent<T>()) {
    for (int64_t tile = ctx.bid; tile < ntiles; tile += ctx.nbx)
      part += time_upd_tile<T, L, TQ, FULL, MM, TPB, PREC, upd_twl<T>() && PREC, PLAN>(ctx, lds, tile, Q, V1, V2,
                                                                                       Vout, Zout, M, tl, coef, qrev);
  } else {
    part = time_upd_tile<T, L, TQ, FULL, MM, TPB, PREC, upd_twl<T>() && PREC, PLAN>(ctx, lds, ctx.bid, Q, V1, V2,
                                                                                     Vout, Zout, M, tl, coef, qrev);
  }
  const double sum = block_sum<tpb_fft<T, FK_SPEC>()>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

// ---------------------------------------------------------------------------
// streaming kernels
// ---------------------------------------------------------------------------

// Spatial part of the residual r = Y (f - A u): one workgroup per x-line l of
// r (threads along x), r[l, x] -= sum_k q_k (L_h u)[N-1-n-k, rr, x], plus the
// partial sums of ||r||^2.  The neighbours along y and z are the adjacent
// x-lines, read by neighbouring workgroups at the same time.
template <typename T, bool Q1, class Ctx>
BLTT_HD void resid_stencil_body(Ctx& ctx, double* red, T* __restrict__ r, const VupdStencil<T>& st,
                                double* __restrict__ partials) {
  const int64_t line = (int64_t)ctx.bid_y * ctx.nbx + ctx.bid;
  const int m0 = st.grid.m[0];
  const LineStencil<T> ls = line_stencil(st, line);
  double part = 0.0;
  for (int x = ctx.tid; x < m0; x += TPB_EW) {
    const int64_t e = line * m0 + x;
    const T v = r[e] - line_stencil_at<T, Q1>(st, ls, x);
    r[e] = v;
    part += (double)v * (double)v;
  }
  const double sum = block_sum<TPB_EW>(ctx, red, part);
  if (ctx.tid == 0) partials[line] = sum;
}

// b = Y f (time reversal, Section 2) and partial sums of ||b||^2
template <typename TO, class Ctx>
BLTT_HD void rhs_body(Ctx& ctx, double* red, const double* __restrict__ f, TO* __restrict__ b, int64_t N,
                      int64_t M, double scale, double* __restrict__ partials) {
  const int64_t n_total = N * M;
  double part = 0.0;
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) {
    const int64_t n = e / M, i = e - n * M;
    const double val = f[(N - 1 - n) * M + i] * scale;
    b[e] = (TO)val;
    part += val * val;
  }
  const double s = block_sum<TPB_EW>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = s;
}

// out = in^T for an R x C row-major matrix (out is C x R), through a 64 x 64
// LDS tile (padded rows); REV also reverses the order of the R index in out.
// Moves per-system vectors of the batched solves between the time-major ABI
// layout (R = N, C = M) and the mode-major sine-basis layout (R = M, C = N).
constexpr int TR_TILE = 64;
template <typename T, bool REV, class Ctx>
BLTT_HD void transpose_body(Ctx& ctx, T* tile, const T* __restrict__ in, T* __restrict__ out, int64_t R,
                            int64_t C) {
  constexpr int P = TR_TILE + 1, ROWS = TPB_EW / TR_TILE;
  const int64_t tiles_c = (C + TR_TILE - 1) / TR_TILE;
  const int64_t c0 = ((int64_t)ctx.bid % tiles_c) * TR_TILE, r0 = ((int64_t)ctx.bid / tiles_c) * TR_TILE;
  const int tx = ctx.tid % TR_TILE, ty = ctx.tid / TR_TILE;
#pragma unroll
  for (int k = 0; k < TR_TILE; k += ROWS) {
    const int64_t r = r0 + ty + k, c = c0 + tx;
    if (r < R && c < C) tile[(ty + k) * P + tx] = in[r * C + c];
  }
  ctx.sync();
#pragma unroll
  for (int k = 0; k < TR_TILE; k += ROWS) {
    const int64_t c = c0 + ty + k, r = r0 + tx;
    if (r < R && c < C) out[c * R + (REV ? R - 1 - r : r)] = tile[tx * P + ty + k];
  }
}

// W_new = cz Z + ca Wa + cb Wb  (stored over Wa);  X += cx W_new
template <typename T, typename TX, class Ctx>
BLTT_HD void wx_body(Ctx& ctx, const T* __restrict__ Z, T* __restrict__ Wa, const T* __restrict__ Wb,
                     TX* __restrict__ X, int64_t n_total, const double* __restrict__ coef) {
  const T cz = T(coef[0]), ca = T(coef[1]), cb = T(coef[2]);
  const TX cxv = TX(coef[3]);
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) {
    const T w = cz * Z[e] + ca * Wa[e] + cb * Wb[e];
    Wa[e] = w;
    X[e] += cxv * TX(w);
  }
}

template <typename T, class Ctx>
BLTT_HD void fill_body(Ctx& ctx, T* __restrict__ x, int64_t n_total, T val) {
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) x[e] = val;
}

// u += s * sum_{i<k} y[i] Z_i: the iterate of a sweep kept as a combination
// of its stored Z vectors, added to the FP64 solution (s = *sptr)
template <typename T>
struct ZList {
  const T* z[ZB_MAX];
  int k;
};

template <typename T, class Ctx>
BLTT_HD void combine_body(Ctx& ctx, double* __restrict__ u, const ZList<T>& zl, const double* __restrict__ y,
                          const double* __restrict__ sptr, int64_t n_total) {
  const double s = *sptr;
  double c[ZB_MAX];
#pragma unroll
  for (int i = 0; i < ZB_MAX; ++i) c[i] = i < zl.k ? s * y[i] : 0.0;
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) {
    double acc = u[e];
    for (int i = 0; i < zl.k; ++i) acc += c[i] * (double)zl.z[i][e];
    u[e] = acc;
  }
}

// y = (TO)(x * s)
template <typename TI, typename TO, class Ctx>
BLTT_HD void scale_cast_body(Ctx& ctx, const TI* __restrict__ x, TO* __restrict__ y, int64_t n_total,
                             const double* __restrict__ sptr, int invert) {
  double s = *sptr;
  if (invert) s = 1.0 / s;
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) y[e] = (TO)((double)x[e] * s);
}

// u += s d   (refinement update in FP64)
template <typename TD, class Ctx>
BLTT_HD void axpy64_body(Ctx& ctx, double* __restrict__ u, const TD* __restrict__ d, int64_t n_total,
                         const double* __restrict__ sptr) {
  const double s = *sptr;
  const int64_t stride = (int64_t)ctx.nbx * TPB_EW;
  for (int64_t e = (int64_t)ctx.bid * TPB_EW + ctx.tid; e < n_total; e += stride) u[e] += s * (double)d[e];
}

// ---------------------------------------------------------------------------
// MINRES scalar state (device resident, FP64)
// ---------------------------------------------------------------------------
struct SolverState {
  double beta;       // scale of the stored V_j, Z_j: v_j = V_j/beta, z_j = Z_j/beta
  double beta_prev;  // scale of V_{j-1}
  double blanc;      // Lanczos beta_j (0 for j = 1)
  double delta;
  double c, c_prev, s, s_prev;
  double eta, eta0;
  double coef_v[4];  // cq, cv, cvp, unused
  double coef_w[4];  // cz, ca, cb, cx
  double norm2;      // last reduced squared norm (rhs or residual)
  double rscale;     // ||r|| of the current refinement right-hand side
  double rinv;       // 1/||r|| (0 when r = 0)
  double dq;         // last reduced <q, z>
  double bsq;        // last reduced <vhat, zhat>
  int32_t iter;
  int32_t status;    // 0 running, 1 exact convergence (beta = 0), -3 NaN, -4 breakdown
  int32_t done;      // batched sweeps: this system's sweep has stopped
  int32_t seq;       // publications to the host mirror so far (k_scalar with a mirror)
};

// First stage of a long reduction: workgroup b sums partials
// [b*RED_CHUNK, (b+1)*RED_CHUNK) in a fixed order (deterministic), so the
// single-workgroup scalar kernel reads at most a few hundred values.
constexpr int RED_PER_THREAD = 16;
constexpr int RED_CHUNK = RED_PER_THREAD * TPB_EW;

template <class Ctx>
BLTT_HD void reduce_chunk_body(Ctx& ctx, double* red, const double* __restrict__ in, int64_t n,
                               double* __restrict__ out) {
  const int64_t base = (int64_t)ctx.bid * RED_CHUNK + ctx.tid;
  double v[RED_PER_THREAD];
#pragma unroll
  for (int k = 0; k < RED_PER_THREAD; ++k) {
    const int64_t e = base + (int64_t)k * TPB_EW;
    const double x = in[e < n ? e : n - 1];
    v[k] = e < n ? x : 0.0;
  }
#pragma unroll
  for (int w = RED_PER_THREAD / 2; w > 0; w >>= 1)
#pragma unroll
    for (int k = 0; k < w; ++k) v[k] += v[k + w];
  const double sum = block_sum<TPB_EW>(ctx, red, v[0]);
  if (ctx.tid == 0) out[ctx.bid] = sum;
}

template <class Ctx>
BLTT_HD double reduce_partials(Ctx& ctx, double* red, const double* __restrict__ partials, int64_t np) {
  double acc = 0.0;
  for (int64_t e = ctx.tid; e < np; e += TPB_EW) acc += partials[e];
  return block_sum<TPB_EW>(ctx, red, acc);
}

enum {
  SC_NORM = 0,   // norm2 = sum                              (rhs / residual norms)
  SC_START = 1,  // beta_1 = sqrt(<b, P^{-1} b>), state reset
  SC_DELTA = 2,  // delta_j = <q, z_j> (matvec part + stencil part), Lanczos coefficients
  SC_BETA = 3    // beta_{j+1}, Givens rotation, w/x coefficients, eta
};

// Iterate kept as a combination of the stored preconditioned Lanczos vectors:
// with Z_i the stored (unnormalised) z_{i+1}, w_j = sum_i om_j[i] Z_i follows
// the direction recurrence on coefficients, and x_j = x_0 + sum_i y[i] Z_i.
// om holds two coefficient vectors (w_{j-2}, w_{j-1}, alternating), each K long.
struct ZBasis {
  double* om;  // 2*K, or null when the direction vectors are kept explicitly
  double* y;   // K
  int K;
};

template <class Ctx>
BLTT_HD void scalar_body(Ctx& ctx, double* red, int phase, SolverState* __restrict__ st,
                         const double* __restrict__ partials, int64_t np, const double* __restrict__ aux,
                         int64_t naux, double* __restrict__ hist, ZBasis zb) {
  if (zb.om && phase == SC_START) {
    for (int i = ctx.tid; i < 2 * zb.K; i += TPB_EW) zb.om[i] = 0.0;
    for (int i = ctx.tid; i < zb.K; i += TPB_EW) zb.y[i] = 0.0;
  }
  double sum = reduce_partials(ctx, red, partials, np);
  if (aux) sum += reduce_partials(ctx, red, aux, naux);
  if (ctx.tid != 0) return;
  if (phase == SC_NORM) {
    st->norm2 = sum;
    st->rscale = sqrt(sum);
    st->rinv = sum > 0.0 ? 1.0 / st->rscale : 0.0;
    return;
  }
  if (phase == SC_START) {
    st->bsq = sum;
    st->iter = 0;
    st->status = 0;
    if (!(sum == sum) || sum > 1e300) {
      st->status = -3;
      return;
    }
    if (sum <= 0.0) {
      st->status = -4;
      return;
    }
    const double b1 = sqrt(sum);
    st->beta = b1;
    st->beta_prev = 1.0;
    st->blanc = 0.0;
    st->eta = b1;
    st->eta0 = b1;
    st->c = st->c_prev = 1.0;
    st->s = st->s_prev = 0.0;
    if (hist) hist[0] = 1.0;
    return;
  }
  if (phase == SC_DELTA) {
    st->dq = sum;
    const double b = st->beta;
    const double delta = sum / (b * b);
    st->delta = delta;
    st->coef_v[0] = 1.0 / b;
    st->coef_v[1] = -delta / b;
    st->coef_v[2] = st->iter == 0 ? 0.0 : -st->blanc / st->beta_prev;
    if (!(delta == delta)) st->status = -3;
    return;
  }
  // SC_BETA
  st->bsq = sum;
  if (!(sum == sum)) {
    st->status = -3;
    return;
  }
  if (sum < 0.0) {
    st->status = -4;
    return;
  }
  const double bn = sqrt(sum);
  const double delta = st->delta, bl = st->blanc;
  const double a0 = st->c * delta - st->c_prev * st->s * bl;
  const double a1 = sqrt(a0 * a0 + bn * bn);
  const double a2 = st->s * delta + st->c_prev * st->c * bl;
  const double a3 = st->s_prev * bl;
  const double cn = a0 / a1, sn = bn / a1;
  st->coef_w[0] = 1.0 / (a1 * st->beta);
  st->coef_w[1] = -a3 / a1;
  st->coef_w[2] = -a2 / a1;
  st->coef_w[3] = cn * st->eta;
  if (zb.om && st->iter < zb.K) {
    // w_j over Z_0..Z_{j-1} (j = iter + 1): overwrite the coefficients of w_{j-2}
    const int j0 = st->iter;
    double* oa = zb.om + (j0 & 1) * zb.K;
    const double* ob = zb.om + ((j0 + 1) & 1) * zb.K;
    for (int i = 0; i < j0; ++i) oa[i] = st->coef_w[1] * oa[i] + st->coef_w[2] * ob[i];
    oa[j0] = st->coef_w[0];
    for (int i = 0; i <= j0; ++i) zb.y[i] += st->coef_w[3] * oa[i];
  }
  st->eta = -sn * st->eta;
  st->c_prev = st->c;
  st->c = cn;
  st->s_prev = st->s;
  st->s = sn;
  st->beta_prev = st->beta;
  st->beta = bn;
  st->blanc = bn;
  st->iter += 1;
  if (hist) hist[st->iter] = fabs(st->eta) / st->eta0;
  if (bn == 0.0) st->status = 1;
}

}  // namespace bltt

namespace bltt {

// ---------------------------------------------------------------------------
// Batched scalar phase: workgroup s updates system s of a batch from its own
// range of partial sums (T per system).  Systems outside the outer loop
// (active[s] = 0) and, in the Lanczos phases, systems whose sweep has stopped
// are left alone.  After SC_BETA a sweep stops on |eta|/eta0 <= etol[s] (the
// system's own sweep tolerance; inner_tol when etol is null), on exact
// convergence, on error, or after cap iterations.
// ---------------------------------------------------------------------------
template <class Ctx>
BLTT_HD void batch_scalar_body(Ctx& ctx, double* red, int phase, SolverState* __restrict__ states,
                               const double* __restrict__ partials, int64_t T, double* __restrict__ hist,
                               int64_t hist_stride, double* __restrict__ zb, int K, double inner_tol, int cap,
                               const int* __restrict__ active, const double* __restrict__ etol = nullptr) {
  const int s = ctx.bid;
  if (!active[s]) return;
  SolverState* st = states + s;
  if ((phase == SC_DELTA || phase == SC_BETA) && st->done) return;
  ZBasis z;
  z.om = zb ? zb + (int64_t)s * 3 * K : nullptr;
  z.y = zb ? zb + (int64_t)s * 3 * K + 2 * K : nullptr;
  z.K = zb ? K : 0;
  scalar_body(ctx, red, phase, st, partials + (int64_t)s * T, T, (const double*)nullptr, 0,
              hist ? hist + (int64_t)s * hist_stride : nullptr, z);
  if (ctx.tid == 0) {
    if (phase == SC_START) st->done = st->status != 0 ? 1 : 0;
    const double tol_s = etol ? etol[s] : inner_tol;
    if (phase == SC_BETA && (st->status != 0 || fabs(st->eta) <= tol_s * st->eta0 || st->iter >= cap))
      st->done = 1;
  }
}

// ---------------------------------------------------------------------------
// batched sine-basis bodies: S systems of one shape, vectors back to back
// (system s at s*n), per-instance tables.  Workgroup g works on tile g % T of
// system g / T and writes one partial sum per tile, so each system's
// reductions stay separate; systems outside the outer loop (and, in the
// Lanczos phases, systems whose sweep has stopped) skip their tiles.
// ---------------------------------------------------------------------------
struct InstParams {
  float l2a;  // log2(alpha)/N
  int qtaps;
  float q32[4];
  double q64[4];
};
struct BatchTabs {
  const cx<float>* tw;     // N
  const cx<float>* sigma;  // I*N, fft(alpha^{j/N} p_j) per instance
  const cx<float>* rho;    // I*N
  const cx<float>* chat;   // I*N, circulant / skew-circulant spectra of p
  const cx<float>* shat;   // I*N
  const cx<float>* omega;  // N
  const float* mu32;       // M
  const cx<double>* tw2;   // 2N (FP64 residual)
  const cx<double>* phat;  // I*2N
  const double* mu64;      // M
  const InstParams* ip;    // I
  const int* sys_inst;     // S: instance of each system
};
struct BatchVec {
  int64_t n, M, T;        // elements per system, modes, tiles per system
  int S;
  int mx = 1;             // modes per x-row (mode_pair)
  // per system ||fhat||: a refinement residual pass writes r/||fhat|| in FP32
  // for the next sweep and scales the iterate update by ||fhat|| (null: the
  // residual goes out in FP64)
  const double* bscale = nullptr;
  const int* active;      // outer loop running (per system)
  const double* etol;     // sweep tolerance on |eta|/eta0 (per system)
  SolverState* states;    // per system
};
struct ZPool {
  float* z[ZB_MAX];       // stored Z vectors (class base pointers)
};

BLTT_HD bool bt_skip(const BatchVec& bv, int s, bool lanczos) {
  return !bv.active[s] || (lanczos && bv.states[s].done);
}

// time pass + Lanczos update (FULL) or start (cq = 1/||r|| of the system)
// LDS of the batched time-line kernels: NL exchange lines and one double per
// thread.  The batched time pass keeps its stage twiddles after them (as the
// single-system one does); the batched N-point matvec stages its system's
// tables (CsStage) there when everything fits in 80 KB (two workgroups per CU).
template <int L, int TPB>
constexpr size_t bt_lds_base() {
  return (size_t)(TPB / (L / fft_V(L))) * (size_t)fft_padded(L) * sizeof(cx<float>) + (size_t)TPB * sizeof(double);
}
template <int L, int TPB>
constexpr bool bt_cs_stage() { return bt_lds_base<L, TPB>() + 4 * (size_t)L * sizeof(cx<float>) <= 80 * 1024; }
template <int L, int TPB>
constexpr size_t bt_cs_lds() {
  return bt_lds_base<L, TPB>() + (bt_cs_stage<L, TPB>() ? 4 * (size_t)L * sizeof(cx<float>) : 0);
}

template <int L, int TPB>
constexpr size_t bt_upd_lds() { return bt_lds_base<L, TPB>() + (size_t)L * sizeof(cx<float>); }

template <int L, typename TQ, bool FULL, int TPB, int PLAN, class Ctx>
BLTT_HD void bt_upd_body(Ctx& ctx, unsigned char* smem, const TQ* __restrict__ Q, const float* __restrict__ V1,
                         const float* __restrict__ V2, float* __restrict__ Vout, float* __restrict__ Zout,
                         const BatchVec& bv, const BatchTabs& bt, double* __restrict__ partials) {
  constexpr int NL = TPB / (L / fft_V(L));
  using F = LineFft<float, L, NL, false, LAST_PAIRED>;
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<float>) * F::LDS_ELEMS);
  const int s = (int)(ctx.bid / bv.T);
  const int64_t tile = ctx.bid % bv.T;
  if (bt_skip(bv, s, FULL)) {
    if (ctx.tid == 0) partials[ctx.bid] = 0.0;
    return;
  }
  const int inst = bt.sys_inst[s];
  const InstParams& ip = bt.ip[inst];
  TimeTables<float> tb;
  tb.tw = bt.tw;
  tb.dinv = nullptr;
  tb.d2 = nullptr;
  tb.sigma = bt.sigma + (int64_t)inst * L;
  tb.rho = bt.rho + (int64_t)inst * L;
  tb.mu = bt.mu32;
  tb.log2_alpha_over_N = ip.l2a;
  for (int k = 0; k < 4; ++k) tb.q[k] = ip.q32[k];
  tb.qtaps = ip.qtaps;
  tb.aux = nullptr;
  tb.mx = bv.mx;
  // the stage twiddles in LDS (time pass with TWL), after the exchange lines
  // and the reduction slots
  {
    using FT = LineFft<float, L, NL, false, LAST_PAIRED, true, PLAN>;
    cx<float>* twl = reinterpret_cast<cx<float>*>(smem + bt_lds_base<L, TPB>());
    FT::template build_twl<TPB>(ctx, twl, bt.tw);
    ctx.sync();
    tb.tw = twl;
  }
  const int64_t o = (int64_t)s * bv.n;
  // a start from the FP32 residual r/||fhat|| runs on it as it is (the
  // iterate update carries ||fhat||); from FP64 it normalises by 1/||r||
  const double one[4] = {1.0, 0.0, 0.0, 0.0};
  const double* coef = FULL ? bv.states[s].coef_v : (sizeof(TQ) == 4 ? one : &bv.states[s].rinv);
  const double part = time_upd_tile<float, L, TQ, FULL, true, TPB, true, true, PLAN>(
      ctx, reinterpret_cast<cx<float>*>(smem), tile, Q + o, FULL ? V1 + o : nullptr, FULL ? V2 + o : nullptr,
      Vout ? Vout + o : nullptr, Zout + o, bv.M, tb, coef);
  const double sum = block_sum<TPB>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

// FP32 sine-coordinate matvec (N-point form): Q = Y T Z, partial sums of <Q, Z>
template <int L, int TPB, int PLAN, class Ctx>
BLTT_HD void bt_cs_body(Ctx& ctx, unsigned char* smem, const float* __restrict__ Z, float* __restrict__ Q,
                        const BatchVec& bv, const BatchTabs& bt, double* __restrict__ partials) {
  constexpr int NL = TPB / (L / fft_V(L));
  using F = LineFft<float, L, NL, false, LAST_DEFAULT>;
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<float>) * F::LDS_ELEMS);
  const int s = (int)(ctx.bid / bv.T);
  const int64_t tile = ctx.bid % bv.T;
  if (bt_skip(bv, s, true)) {
    if (ctx.tid == 0) partials[ctx.bid] = 0.0;
    return;
  }
  const int inst = bt.sys_inst[s];
  const InstParams& ip = bt.ip[inst];
  MatvecCSTables<float> tb;
  tb.tw = bt.tw;
  tb.chat = bt.chat + (int64_t)inst * L;
  tb.shat = bt.shat + (int64_t)inst * L;
  tb.omega = bt.omega;
  tb.mu = bt.mu32;
  for (int k = 0; k < 4; ++k) tb.q[k] = ip.q32[k];
  tb.qtaps = ip.qtaps;
  tb.mx = bv.mx;
  const int64_t o = (int64_t)s * bv.n;
  double part;
  if constexpr (bt_cs_stage<L, TPB>()) {
    CsStage<float, L, TPB, PLAN> st;
    st.tabs = reinterpret_cast<cx<float>*>(smem + bt_lds_base<L, TPB>());
    st.load(ctx, tb);
    part = matvec_cs_tile<float, L, MV_DOT, TPB, true, PLAN>(ctx, reinterpret_cast<cx<float>*>(smem), tile,
                                                       const_cast<float*>(Z) + o, Q + o, nullptr, bv.M,
                                                       st.tables(tb), IterUpd{}, &st);
  } else {
    part = matvec_cs_tile<float, L, MV_DOT, TPB, false, PLAN>(ctx, reinterpret_cast<cx<float>*>(smem), tile,
                                                              const_cast<float*>(Z) + o, Q + o, nullptr, bv.M, tb,
                                                              IterUpd{});
  }
  const double sum = block_sum<TPB>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

// FP64 refinement step per system: u_s <- u_s + rscale_s sum_i y_i Z_i (the
// sweep's stored vectors, pool.z[i] + s*n), R = Y(F - A u_s) (2N-point form),
// partial sums of ||R||^2.  T2 tiles per system.
// R32: the residual goes to r32 + s*n as FP32 r/||fhat_s|| (bv.bscale) for
// the next sweep, and the update is scaled by ||fhat_s||.
template <int L2, bool R32 = false, class Ctx>
BLTT_HD void bt_resid_body(Ctx& ctx, unsigned char* smem, double* const* __restrict__ u, double* __restrict__ R,
                           const double* __restrict__ Fh, const BatchVec& bv, const BatchTabs& bt,
                           const IterUpd& pool, const double* __restrict__ zb, int K, int64_t T2,
                           double* __restrict__ partials, float* __restrict__ r32 = nullptr) {
  constexpr int NL = tpb_fft<double, fk_mv<true, L2>()>() / (L2 / fft_V(L2));
  using F = LineFft<double, L2, NL, false, LAST_DEFAULT>;
  double* red = reinterpret_cast<double*>(smem + sizeof(cx<double>) * F::LDS_ELEMS);
  const int s = (int)(ctx.bid / T2);
  const int64_t tile = ctx.bid % T2;
  if (!bv.active[s]) {
    if (ctx.tid == 0) partials[ctx.bid] = 0.0;
    return;
  }
  const int inst = bt.sys_inst[s];
  const InstParams& ip = bt.ip[inst];
  MatvecTables<double> tb;
  tb.tw = bt.tw2;
  tb.phat = bt.phat + (int64_t)inst * L2;
  tb.mu = bt.mu64;
  for (int k = 0; k < 4; ++k) tb.q[k] = ip.q64[k];
  tb.qtaps = ip.qtaps;
  tb.mx = bv.mx;
  const int64_t o = (int64_t)s * bv.n;
  const int k = bv.states[s].iter < K ? bv.states[s].iter : K - 1;
  double part;
  if constexpr (R32) {
    part = matvec_fft_tile<double, L2, MV_RESID, TERM_SPEC, true, true>(
        ctx, reinterpret_cast<cx<double>*>(smem), tile, u[s], R + o, Fh + o, bv.M, tb, pool, o, k,
        zb + (int64_t)s * 3 * K + 2 * K, &bv.bscale[s], r32 + o, 1.0 / bv.bscale[s]);
  } else {
    part = matvec_fft_tile<double, L2, MV_RESID, TERM_SPEC, true>(
        ctx, reinterpret_cast<cx<double>*>(smem), tile, u[s], R + o, Fh + o, bv.M, tb, pool, o, k,
        zb + (int64_t)s * 3 * K + 2 * K, &bv.states[s].rscale);
  }
  const double sum = block_sum<tpb_fft<double, fk_mv<true, L2>()>()>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

// b = Y f per system (mode-major, each time line reversed) and per-system
// partial sums of ||b||^2 (BPS workgroups per system)
template <class Ctx>
BLTT_HD void bt_rhs_body(Ctx& ctx, double* red, const double* __restrict__ f, double* __restrict__ b, int log2N,
                         int64_t n, int64_t BPS, double* __restrict__ partials) {
  const int64_t s = ctx.bid / BPS, blk = ctx.bid % BPS;
  const int64_t N = (int64_t)1 << log2N;
  const double* fs = f + s * n;
  double* bs = b + s * n;
  double part = 0.0;
  for (int64_t e = blk * TPB_EW + ctx.tid; e < n; e += BPS * TPB_EW) {
    const int64_t i = e >> log2N, t = e & (N - 1);
    const double v = fs[(i << log2N) + (N - 1 - t)];
    bs[e] = v;
    part += v * v;
  }
  const double sum = block_sum<TPB_EW>(ctx, red, part);
  if (ctx.tid == 0) partials[ctx.bid] = sum;
}

}  // namespace bltt
