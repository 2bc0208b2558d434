// Register/LDS line FFT engine for gfx950 (CDNA4, 64-wide wavefronts).
//
// A workgroup holds NL complex "lines" of length L (a power of two, 2..4096).
// Each line is transformed by G = L/V threads that keep V = min(L,16) complex
// values in registers.  The transform is an in-place mixed-radix
// decimation-in-frequency FFT: stage s applies radix r_s butterflies of
// stride sigma_s, and consecutive stages exchange data through LDS.  The
// forward transform leaves frequency k = sum_s d_s rho_s at position
// sum_s d_s sigma_s (digit reversal), which is exactly the input order the
// mirrored decimation-in-time inverse consumes.  A forward/pointwise/inverse
// chain therefore needs no reordering, and the last forward stage, the
// pointwise multiply and the first inverse stage all stay in registers.
//
// Conventions: forward X[k] = sum_n x[n] exp(-2 pi i n k / L); the inverse
// returns L x (unnormalised).  Twiddles come from a table tw[k] =
// exp(-2 pi i k / L), k < L, computed on the host in double precision (or
// from a per-workgroup LDS copy of the entries each stage needs, TWL).
//
// Everything here is __host__ __device__ so the same code can be run by the
// CPU workgroup emulator used in the tests; `Ctx::sync()` is the workgroup
// barrier and `Ctx::wsync()` the wavefront-scope one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BLTT_HD __host__ __device__ __forceinline__

namespace bltt {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
BLTT_HD cx<T> mkc(T a, T b) {
  cx<T> r;
  r.re = a;
  r.im = b;
  return r;
}
template <typename T>
BLTT_HD cx<T> operator+(cx<T> a, cx<T> b) { return mkc<T>(a.re + b.re, a.im + b.im); }
template <typename T>
BLTT_HD cx<T> operator-(cx<T> a, cx<T> b) { return mkc<T>(a.re - b.re, a.im - b.im); }
template <typename T>
BLTT_HD cx<T> operator*(cx<T> a, cx<T> b) {
  return mkc<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
BLTT_HD cx<T> operator*(cx<T> a, T s) { return mkc<T>(a.re * s, a.im * s); }
template <typename T>
BLTT_HD cx<T> conjg(cx<T> a) { return mkc<T>(a.re, -a.im); }
// (SIGN * i) * a
template <int SIGN, typename T>
BLTT_HD cx<T> mul_si(cx<T> a) {
  return SIGN < 0 ? mkc<T>(a.im, -a.re) : mkc<T>(-a.im, a.re);
}

// ---------------------------------------------------------------------------
// plans: V values per thread, S stages, radix r(L, s)
// ---------------------------------------------------------------------------
constexpr int fft_V(int L) { return L < 16 ? L : 16; }
constexpr int fft_S(int L) { return L <= 16 ? 1 : (L <= 128 ? 2 : 3); }
constexpr int fft_r(int L, int s) {
  return L <= 16     ? L
         : L <= 128  ? (s == 0 ? 16 : L / 16)
         : L == 256  ? (s == 0 ? 16 : 4)
         : L == 512  ? (s == 0 ? 16 : (s == 1 ? 8 : 4))
         : L == 1024 ? (s == 0 ? 16 : 8)
         : L == 2048 ? (s == 2 ? 8 : 16)
                     : 16;  // 4096
}
// Radix plans.  Plan 0 is the table above; plan 1 splits the stages after the
// first radix-16 one the other way where that is possible with the same
// registers: 16*16*4 for L = 1024 and 16*4*8 for L = 512 (other lengths: plan 0).
// Which one runs faster is a property of the machine and the kernel around the
// transform, chosen at setup by timing both.
constexpr bool fft_plan_alt(int L) { return L == 512 || L == 1024; }
constexpr int fft_rp(int L, int s, int plan) {
  return plan == 1 && L == 1024  ? (s == 0 ? 16 : (s == 1 ? 16 : 4))
         : plan == 1 && L == 512 ? (s == 0 ? 16 : (s == 1 ? 4 : 8))
                                 : fft_r(L, s);
}
constexpr int fft_sigma_p(int L, int s, int plan) {
  int p = 1;
  for (int i = 0; i <= s; ++i) p *= fft_rp(L, i, plan);
  return L / p;
}
constexpr int fft_rho_p(int L, int s, int plan) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fft_rp(L, i, plan);
  return p;
}
constexpr int fft_sigma(int L, int s) {
  int p = 1;
  for (int i = 0; i <= s; ++i) p *= fft_r(L, i);
  return L / p;
}
constexpr int fft_rho(int L, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fft_r(L, i);
  return p;
}

// ---------------------------------------------------------------------------
// small DFTs in registers, natural order in and out:
//   y_u = sum_t a_t exp(SIGN 2 pi i t u / R)
// ---------------------------------------------------------------------------
template <int SIGN, typename T>
BLTT_HD void dft2(cx<T>* a) {
  cx<T> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}
template <int SIGN, typename T>
BLTT_HD void dft4(cx<T>* a) {
  cx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
  cx<T> t2 = a[1] + a[3], t3 = mul_si<SIGN>(a[1] - a[3]);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}
template <int SIGN, typename T>
BLTT_HD void dft8(cx<T>* a) {
  cx<T> e[4] = {a[0], a[2], a[4], a[6]};
  cx<T> o[4] = {a[1], a[3], a[5], a[7]};
  dft4<SIGN>(e);
  dft4<SIGN>(o);
  const T h = T(0.70710678118654752440);
  cx<T> t1 = o[1] * mkc<T>(h, SIGN * h);
  cx<T> t2 = mul_si<SIGN>(o[2]);
  cx<T> t3 = o[3] * mkc<T>(-h, SIGN * h);
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + t1;
  a[5] = e[1] - t1;
  a[2] = e[2] + t2;
  a[6] = e[2] - t2;
  a[3] = e[3] + t3;
  a[7] = e[3] - t3;
}
template <int SIGN, typename T>
BLTT_HD void dft16(cx<T>* a) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = a[2 * k];
    o[k] = a[2 * k + 1];
  }
  dft8<SIGN>(e);
  dft8<SIGN>(o);
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  const T h = T(0.70710678118654752440);
  const cx<T> w[8] = {mkc<T>(T(1), T(0)),     mkc<T>(c1, SIGN * s1), mkc<T>(h, SIGN * h),
                      mkc<T>(s1, SIGN * c1),  mkc<T>(T(0), T(SIGN)), mkc<T>(-s1, SIGN * c1),
                      mkc<T>(-h, SIGN * h),   mkc<T>(-c1, SIGN * s1)};
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    cx<T> t = (u == 0) ? o[0] : o[u] * w[u];
    a[u] = e[u] + t;
    a[u + 8] = e[u] - t;
  }
}
template <int R, int SIGN, typename T>
BLTT_HD void dft(cx<T>* a) {
  if constexpr (R == 2) dft2<SIGN>(a);
  else if constexpr (R == 4) dft4<SIGN>(a);
  else if constexpr (R == 8) dft8<SIGN>(a);
  else if constexpr (R == 16) dft16<SIGN>(a);
  else static_assert(R == 2, "unsupported radix");
}

// Twiddles w^u, 0 < u < R, of w = tw[e]: the powers w^(2^k) come from the
// table and the others are products of two or three of them (at most three
// roundings), so a radix-16 butterfly issues 4 table loads instead of 15.
constexpr int high_pow2(int u) {
  int h = 1;
  while (h * 2 <= u) h *= 2;
  return h;
}
// pw[U..R-1] from the powers of two below them (compile-time indices only, so
// pw stays in registers)
template <int R, int U, typename T>
BLTT_HD void twiddle_products(cx<T>* pw) {
  if constexpr (U < R) {
    constexpr int hi = high_pow2(U);
    if constexpr (hi != U) pw[U] = pw[hi] * pw[U - hi];
    twiddle_products<R, U + 1>(pw);
  }
}
template <int R, typename T>
BLTT_HD void twiddle_powers(cx<T>* pw, const cx<T>* tw, int e) {
#pragma unroll
  for (int u = 1; u < R; u <<= 1) pw[u] = tw[u * e];
  twiddle_products<R, 3>(pw);
}

// LDS padding of a line: one slot per 8 elements and one more per 128.  The
// exchanges read and write runs of consecutive positions, runs 8 apart, and
// (paired and linear last stages) positions 64 apart; one pad per 8 alone
// maps the latter to two banks per 16 lanes, the second pad spreads them.
BLTT_HD constexpr int fft_pad(int pos) { return pos + (pos >> 3) + (pos >> 7); }
BLTT_HD constexpr int fft_padded(int L) { return L + (L >> 3) + (L >> 7); }

// How the last stage's butterflies are dealt to the threads of a line.
enum LastMode {
  LAST_DEFAULT = 0,  // butterfly g + G*w (LDS friendly)
  LAST_LINEAR = 1,   // frequency base k_low = g + G*w (coalesced frequency stores)
  LAST_PAIRED = 2    // k_low and K - k_low in one thread (k <-> L-k pairs in registers)
};

// TWL: the stage twiddles come from a per-workgroup LDS table (built once with
// build_twl) instead of power products of the global table: for stage s, entry
// off_s + (u-1) sg_s + j holds w^(u j L/B_s) for butterfly j = beta mod sg_s,
// so consecutive lanes read consecutive entries.
// SPLIT: every exchange moves the real parts, then the imaginary parts,
// through an LDS buffer of T (half the bytes of one of cx<T>), so that more
// workgroups fit on a CU; `lds` then points to that T buffer.
template <typename T, int L, int NL, bool INTERLEAVED, int LAST, bool TWL = false, int PLAN = 0, bool SPLIT = false>
struct LineFft {
  static constexpr int V = fft_V(L);
  static constexpr int S = fft_S(L);
  static constexpr int G = L / V;             // threads per line
  static constexpr int RL = fft_rp(L, S - 1, PLAN);         // last radix
  static constexpr int K = L / RL;            // last-stage butterflies per line
  static constexpr int LP = fft_padded(L);    // padded line length
  // exchange buffer, in units of cx<T>
  static constexpr int LDS_ELEMS = SPLIT ? (NL * LP + 1) / 2 : NL * LP;
  static constexpr bool SPLIT_X = SPLIT;
  // Lines stored one after another (not interleaved) and at most one
  // wavefront per line: every exchange stays inside one wavefront, whose LDS
  // accesses execute in order, so a wavefront-scope barrier replaces the
  // workgroup barrier.
  static constexpr bool WAVE_LOCAL = !INTERLEAVED && G <= 64;

  template <class Ctx>
  BLTT_HD static void xsync(Ctx& ctx) {
    if constexpr (WAVE_LOCAL) ctx.wsync();
    else ctx.sync();
  }
  // LDS twiddle table: offset of stage s, and the total length (< L)
  static constexpr int twl_off(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i) o += (fft_rp(L, i, PLAN) - 1) * fft_sigma_p(L, i, PLAN);
    return o;
  }
  static constexpr int TWL_LEN = twl_off(S - 1) > 0 ? twl_off(S - 1) : 1;
  // fill the LDS table from the global one (all threads of the workgroup; the
  // caller synchronises before first use)
  template <int NT>
  static constexpr int twl_per() { return (TWL_LEN + NT - 1) / NT; }
  // split in a load phase and a store phase so that callers can put other
  // global loads between them (one memory round trip per workgroup)
  template <int NT, class Ctx>
  BLTT_HD static void twl_load(Ctx& ctx, const cx<T>* tw, cx<T>* val) {
#pragma unroll
    for (int k = 0; k < twl_per<NT>(); ++k) {
      const int i = ctx.tid + k * NT;
      val[k] = tw[twl_src(i < TWL_LEN ? i : TWL_LEN - 1)];
    }
  }
  template <int NT, class Ctx>
  BLTT_HD static void twl_store(Ctx& ctx, cx<T>* twl, const cx<T>* val) {
#pragma unroll
    for (int k = 0; k < twl_per<NT>(); ++k) {
      const int i = ctx.tid + k * NT;
      if (i < TWL_LEN) twl[i] = val[k];
    }
  }
  template <int NT, class Ctx>
  BLTT_HD static void build_twl(Ctx& ctx, cx<T>* twl, const cx<T>* tw) {
    cx<T> val[twl_per<NT>()];
    twl_load<NT>(ctx, tw, val);
    twl_store<NT>(ctx, twl, val);
  }
  // global-table index of LDS table entry i (stage s, entry off_s + (u-1) sg_s + j)
  BLTT_HD static constexpr int twl_src(int i) {
    int s = 0;
    while (s < S - 2 && i >= twl_off(s + 1)) ++s;
    const int sg = fft_sigma_p(L, s, PLAN), LB = L / (fft_rp(L, s, PLAN) * sg), e = i - twl_off(s);
    return (e / sg + 1) * (e % sg) * LB;
  }
  template <int s, int r>
  BLTT_HD static void stage_twiddles(cx<T>* pw, const cx<T>* tw, int b) {
    constexpr int sg = fft_sigma_p(L, s, PLAN), B = r * sg;
    if constexpr (TWL) {
      constexpr int o = twl_off(s);
      const int j = b % sg;
#pragma unroll
      for (int u = 1; u < r; ++u) pw[u] = tw[o + (u - 1) * sg + j];
    } else {
      twiddle_powers<r>(pw, tw, (b % sg) * (L / B));
    }
  }
  static_assert(S == 1 || fft_rp(L, 0, PLAN) == V, "first stage must use all registers");
  static_assert(LAST != LAST_PAIRED || S == 1 || V >= 2 * RL, "pairing needs two butterflies");

  BLTT_HD static int idx(int c, int pos) {
    const int pp = fft_pad(pos);
    return INTERLEAVED ? pp * NL + c : c * LP + pp;
  }

  template <int s>
  BLTT_HD static int pos(int b, int t) {
    constexpr int sg = fft_sigma_p(L, s, PLAN), r = fft_rp(L, s, PLAN);
    return (b / sg) * (r * sg) + (b % sg) + t * sg;
  }

  // frequency base of a last-stage butterfly, and its inverse
  BLTT_HD static int klow_of_blk(int b) {
    const int p = b * RL;
    int k = 0;
#pragma unroll
    for (int s = 0; s < S - 1; ++s) k += ((p / fft_sigma_p(L, s, PLAN)) % fft_rp(L, s, PLAN)) * fft_rho_p(L, s, PLAN);
    return k;
  }
  BLTT_HD static int blk_of_klow(int kl) {
    int b = 0;
#pragma unroll
    for (int s = 0; s < S - 1; ++s) b += ((kl / fft_rho_p(L, s, PLAN)) % fft_rp(L, s, PLAN)) * (fft_sigma_p(L, s, PLAN) / RL);
    return b;
  }

  BLTT_HD static int klow(int g, int w) {
    if constexpr (S == 1) {
      return 0;
    } else if constexpr (LAST == LAST_PAIRED) {
      constexpr int PP = V / (2 * RL);
      const int q = g * PP + (w >> 1);
      const bool first = (w & 1) == 0;
      if (q == 0) return first ? 0 : K / 2;
      return first ? q : K - q;
    } else if constexpr (LAST == LAST_LINEAR) {
      return g + G * w;
    } else {
      return klow_of_blk(g + G * w);
    }
  }

  template <int s>
  BLTT_HD static int beta(int g, int w) {
    if constexpr (s == S - 1 && S > 1 && LAST != LAST_DEFAULT) {
      return blk_of_klow(klow(g, w));
    } else {
      return g + G * w;
    }
  }

  // frequency held by register slot (w, u) after the forward transform
  BLTT_HD static int freq(int g, int w, int u) {
    if constexpr (S == 1) return u;
    else return klow(g, w) + u * K;
  }

  // ---- forward: v[w*r0+t] = x[pos<0>(beta<0>(g,w),t)]  ->  v[w*RL+u] = X[freq(g,w,u)]
  template <class Ctx>
  BLTT_HD static void forward(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g, const cx<T>* tw) {
    fwd_stage<0, false>(ctx, v, lds, c, g, tw, nullptr);
  }

  // Twiddle bases (table entries w^(u e), u = 1, 2, 4, ...) of every stage
  // loaded up front from the global table, so that no stage waits for its own
  // loads after an exchange barrier; costs the registers that hold them.
  template <int s>
  static constexpr int pf_per() {
    int n = 0;
    if (fft_sigma_p(L, s, PLAN) > 1)
      for (int u = 1; u < fft_rp(L, s, PLAN); u <<= 1) ++n;
    return n;
  }
  template <int s>
  static constexpr int pf_off() {
    int o = 0;
    if constexpr (s > 0) o = pf_off<s - 1>() + (V / fft_rp(L, s - 1, PLAN)) * pf_per<s - 1>();
    return o;
  }
  static constexpr int PF_LEN = pf_off<S - 1>() + (V / fft_rp(L, S - 1, PLAN)) * pf_per<S - 1>();
  template <int s>
  BLTT_HD static void pf_load(cx<T>* pre, const cx<T>* tw, int g) {
    if constexpr (s < S) {
      constexpr int r = fft_rp(L, s, PLAN), sg = fft_sigma_p(L, s, PLAN), NB = V / r, P = pf_per<s>();
      if constexpr (P > 0) {
#pragma unroll
        for (int w = 0; w < NB; ++w) {
          const int e = (beta<s>(g, w) % sg) * (L / (r * sg));
#pragma unroll
          for (int i = 0; i < P; ++i) pre[pf_off<s>() + w * P + i] = tw[(1 << i) * e];
        }
      }
      pf_load<s + 1>(pre, tw, g);
    }
  }
  // pre: PF_LEN entries filled by pf_load<0>, best issued before the caller's
  // own loads and exchanges
  template <class Ctx>
  BLTT_HD static void forward_pf(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g, const cx<T>* pre) {
    static_assert(!TWL, "the LDS twiddle table needs no prefetch");
    fwd_stage<0, true>(ctx, v, lds, c, g, nullptr, pre);
  }

  template <int s, bool PF, class Ctx>
  BLTT_HD static void fwd_stage(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g, const cx<T>* tw, const cx<T>* pre) {
    constexpr int r = fft_rp(L, s, PLAN), sg = fft_sigma_p(L, s, PLAN), NB = V / r;
    if constexpr (s > 0 && !SPLIT) {
#pragma unroll
      for (int w = 0; w < NB; ++w) {
        const int b = beta<s>(g, w);
#pragma unroll
        for (int t = 0; t < r; ++t) v[w * r + t] = lds[idx(c, pos<s>(b, t))];
      }
    }
#pragma unroll
    for (int w = 0; w < NB; ++w) {
      dft<r, -1>(v + w * r);
      if constexpr (sg > 1) {
        cx<T> pw[r];
        if constexpr (PF) {
#pragma unroll
          for (int i = 0; i < pf_per<s>(); ++i) pw[1 << i] = pre[pf_off<s>() + w * pf_per<s>() + i];
          twiddle_products<r, 3>(pw);
        } else {
          stage_twiddles<s, r>(pw, tw, beta<s>(g, w));
        }
#pragma unroll
        for (int u = 1; u < r; ++u) v[w * r + u] = v[w * r + u] * pw[u];
      }
    }
    if constexpr (s + 1 < S) {
      if constexpr (SPLIT) {
        split_exchange<s, s + 1>(ctx, v, lds, c, g);
      } else {
        xsync(ctx);
#pragma unroll
        for (int w = 0; w < NB; ++w) {
          const int b = beta<s>(g, w);
#pragma unroll
          for (int u = 0; u < r; ++u) lds[idx(c, pos<s>(b, u))] = v[w * r + u];
        }
        xsync(ctx);
      }
      fwd_stage<s + 1, PF>(ctx, v, lds, c, g, tw, pre);
    }
  }

  // SPLIT: the exchange from the slots of stage sw to those of stage sr, real
  // parts first (each part's writes, a barrier, its reads), then the
  // imaginary parts; a barrier between the two passes keeps the second
  // pass's writes behind every read of the first.
  template <int sw, int sr, class Ctx>
  BLTT_HD static void split_exchange(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g) {
    constexpr int rw = fft_rp(L, sw, PLAN), rr = fft_rp(L, sr, PLAN);
    T* ls = reinterpret_cast<T*>(lds);
    T re[V];
    xsync(ctx);
#pragma unroll
    for (int w = 0; w < V / rw; ++w)
#pragma unroll
      for (int u = 0; u < rw; ++u) ls[idx(c, pos<sw>(beta<sw>(g, w), u))] = v[w * rw + u].re;
    xsync(ctx);
#pragma unroll
    for (int w = 0; w < V / rr; ++w)
#pragma unroll
      for (int t = 0; t < rr; ++t) re[w * rr + t] = ls[idx(c, pos<sr>(beta<sr>(g, w), t))];
    xsync(ctx);
#pragma unroll
    for (int w = 0; w < V / rw; ++w)
#pragma unroll
      for (int u = 0; u < rw; ++u) ls[idx(c, pos<sw>(beta<sw>(g, w), u))] = v[w * rw + u].im;
    xsync(ctx);
#pragma unroll
    for (int w = 0; w < V / rr; ++w)
#pragma unroll
      for (int t = 0; t < rr; ++t) v[w * rr + t] = mkc<T>(re[w * rr + t], ls[idx(c, pos<sr>(beta<sr>(g, w), t))]);
  }

  // ---- inverse: v[w*RL+u] = X[freq(g,w,u)]  ->  v[w*r0+t] = L x[pos<0>(beta<0>(g,w),t)]
  template <class Ctx>
  BLTT_HD static void inverse(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g, const cx<T>* tw) {
    inv_stage<S - 1>(ctx, v, lds, c, g, tw);
  }

  template <int s, class Ctx>
  BLTT_HD static void inv_stage(Ctx& ctx, cx<T>* v, cx<T>* lds, int c, int g, const cx<T>* tw) {
    constexpr int r = fft_rp(L, s, PLAN), sg = fft_sigma_p(L, s, PLAN), NB = V / r;
    if constexpr (s < S - 1 && !SPLIT) {
#pragma unroll
      for (int w = 0; w < NB; ++w) {
        const int b = beta<s>(g, w);
#pragma unroll
        for (int u = 0; u < r; ++u) v[w * r + u] = lds[idx(c, pos<s>(b, u))];
      }
    }
#pragma unroll
    for (int w = 0; w < NB; ++w) {
      if constexpr (sg > 1) {
        cx<T> pw[r];
        stage_twiddles<s, r>(pw, tw, beta<s>(g, w));
#pragma unroll
        for (int u = 1; u < r; ++u) v[w * r + u] = v[w * r + u] * conjg(pw[u]);
      }
      dft<r, +1>(v + w * r);
    }
    if constexpr (s > 0) {
      if constexpr (SPLIT) {
        split_exchange<s, s - 1>(ctx, v, lds, c, g);
      } else {
        xsync(ctx);
#pragma unroll
        for (int w = 0; w < NB; ++w) {
          const int b = beta<s>(g, w);
#pragma unroll
          for (int t = 0; t < r; ++t) lds[idx(c, pos<s>(b, t))] = v[w * r + t];
        }
        xsync(ctx);
      }
      inv_stage<s - 1>(ctx, v, lds, c, g, tw);
    }
  }
};

}  // namespace bltt
