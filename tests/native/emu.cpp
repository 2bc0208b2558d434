// CPU workgroup emulator for the HIP kernel bodies (test infrastructure).
//
// Runs the __host__ __device__ kernel bodies of the GPU path on host threads:
// one host thread per GPU thread of a workgroup (from a pool that lives as
// long as the process), the workgroup barrier mapped to a host barrier and LDS
// to a host array.  The tests use it to check the
// kernels' index arithmetic and numerics on the CPU (with bounds-checked
// buffers) before anything runs on a GPU.  Built with hipcc as host code; never
// loaded by the solver.
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "bltt_kernels.hpp"
#include "host_tables.hpp"

using namespace bltt;

namespace {

struct Barrier {
  explicit Barrier(int n) : count(n) {}
  void wait() {
    std::unique_lock<std::mutex> lk(m);
    const int g = gen;
    if (++waiting == count) {
      waiting = 0;
      ++gen;
      cv.notify_all();
    } else {
      cv.wait(lk, [&] { return gen != g; });
    }
  }
  std::mutex m;
  std::condition_variable cv;
  int count;
  int waiting = 0;
  int gen = 0;
};

struct HostCtx {
  int tid, bid, bid_y, nbx;
  Barrier* bar;
  void sync() { bar->wait(); }
  // every thread of a workgroup runs the same sequence of barriers, so the
  // wavefront-scope barrier can be emulated by the workgroup one
  void wsync() { bar->wait(); }
};

// LDS with guard words: out-of-range accesses are detected at the end.
struct Lds {
  explicit Lds(size_t bytes) : buf(bytes + 2 * kGuard, 0xA5) {}
  unsigned char* base() { return buf.data() + kGuard; }
  bool intact() const {
    for (size_t i = 0; i < kGuard; ++i)
      if (buf[i] != 0xA5 || buf[buf.size() - 1 - i] != 0xA5) return false;
    return true;
  }
  static constexpr size_t kGuard = 256;
  std::vector<unsigned char> buf;
};

int g_error = 0;
int g_plan = 0;  // radix plan of the FP32 sine-basis transforms
int g_cs_blocks = 0;  // workgroups of the N-point matvec (0: one per tile)

// Worker threads for the emulated workgroups, created on first need and kept:
// run(n, job) runs job(t) on workers t = 0..n-1 at once (every one of them, as
// the workgroup barrier needs) and returns when all have finished.
class Pool {
 public:
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    go_.notify_all();
    for (auto& t : th_) t.join();
  }
  void run(int n, const std::function<void(int)>& job) {
    std::unique_lock<std::mutex> lk(m_);
    while ((int)th_.size() < n) {
      const int idx = (int)th_.size();
      th_.emplace_back([this, idx] { loop(idx); });
    }
    job_ = &job;
    active_ = n;
    pending_ = n;
    ++gen_;
    go_.notify_all();
    done_.wait(lk, [&] { return pending_ == 0; });
    job_ = nullptr;
  }

 private:
  void loop(int idx) {
    long seen = 0;
    std::unique_lock<std::mutex> lk(m_);
    for (;;) {
      go_.wait(lk, [&] { return stop_ || (gen_ != seen && idx < active_); });
      if (stop_) return;
      seen = gen_;
      const std::function<void(int)>* job = job_;
      lk.unlock();
      (*job)(idx);
      lk.lock();
      if (--pending_ == 0) done_.notify_all();
    }
  }
  std::mutex m_;
  std::condition_variable go_, done_;
  std::vector<std::thread> th_;
  const std::function<void(int)>* job_ = nullptr;
  long gen_ = 0;
  int active_ = 0, pending_ = 0;
  bool stop_ = false;
};
Pool g_pool;

void run_grid(int tpb, int gx, int gy, size_t lds_bytes,
              const std::function<void(HostCtx&, unsigned char*)>& body) {
  for (int by = 0; by < gy; ++by) {
    for (int bx = 0; bx < gx; ++bx) {
      Lds lds(lds_bytes);
      Barrier bar(tpb);
      g_pool.run(tpb, [&](int t) {
        HostCtx c{t, bx, by, gx, &bar};
        body(c, lds.base());
      });
      if (!lds.intact()) g_error = 1;
    }
  }
}

template <typename T>
std::vector<cx<T>> to_cx(const std::vector<host::cd>& v) {
  std::vector<cx<T>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = mkc<T>((T)v[i].real(), (T)v[i].imag());
  return o;
}
template <typename T>
std::vector<T> to_t(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

// ---- dispatch over the compile-time line length
// EMU_MAX_L (the sanitizer build): only line lengths up to it are compiled;
// longer ones set g_error = 2.
#ifndef EMU_MAX_L
#define EMU_MAX_L 4096
#endif
template <template <int> class F, int LL, typename... A>
void run_L(A&&... a) {
  if constexpr (LL <= EMU_MAX_L) F<LL>::run(a...);
  else g_error = 2;
}
template <template <int> class F, typename... A>
void with_L(int L, A&&... a) {
  switch (L) {
    case 2: run_L<F, 2>(a...); break;
    case 4: run_L<F, 4>(a...); break;
    case 8: run_L<F, 8>(a...); break;
    case 16: run_L<F, 16>(a...); break;
    case 32: run_L<F, 32>(a...); break;
    case 64: run_L<F, 64>(a...); break;
    case 128: run_L<F, 128>(a...); break;
    case 256: run_L<F, 256>(a...); break;
    case 512: run_L<F, 512>(a...); break;
    case 1024: run_L<F, 1024>(a...); break;
    case 2048: run_L<F, 2048>(a...); break;
    default: g_error = 2;
  }
}

// matvec line lengths are 2N (4..4096)
template <template <int> class F, typename... A>
void with_L2(int L, A&&... a) {
  if (L == 4096) run_L<F, 4096>(a...);
  else with_L<F>(L, a...);
}

template <typename T>
struct TimeRun {
  template <int L>
  struct R {
    static void run(T* x, int64_t M, const TimeTables<T>& tb) {
      constexpr int NL = lines_per_block<T, FK_TIME>(L);
      using Ft = LineFft<T, L, NL, true, LAST_PAIRED>;
      run_grid(tpb_fft<T, FK_TIME>(), (int)fft_blocks<T, FK_TIME>(L, M), 1, fft_lds_bytes<T, FK_TIME>(L),
               [&](HostCtx& c, unsigned char* lds) {
        double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Ft::LDS_ELEMS);
        time_prec_body<T, L>(c, reinterpret_cast<cx<T>*>(lds), red, x, M, tb);
      });
    }
  };
};

template <typename T>
struct DstXRun {
  template <int L>
  struct R {
    static void run(const T* in, T* out, int64_t nlines, const DstTables<T>& tb, const double* coef,
                    double* partials, const T* vdot, int kind, T* vout, const VupdStencil<T>& sten) {
      constexpr int NL = lines_per_block<T, FK_DSTX>(L);
      using Fx = LineFft<T, L, NL, false, LAST_LINEAR>;
      run_grid(tpb_fft<T, FK_DSTX>(), (int)fft_blocks<T, FK_DSTX>(L, nlines), 1, fft_lds_bytes<T, FK_DSTX>(L),
               [&](HostCtx& c, unsigned char* lds) {
        double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Fx::LDS_ELEMS);
        if (kind == KIND_VUPD && sten.z) {
          // full Lanczos variant: v1 = v2 = in with zero coefficients
          if (sten.qtaps <= 1)
            dst_x_body<T, L, KIND_VUPD, true, true>(c, reinterpret_cast<cx<T>*>(lds), red, in, in, in, vout,
                                                    nullptr, out, nlines, tb, coef, partials, sten);
          else
            dst_x_body<T, L, KIND_VUPD, true, false>(c, reinterpret_cast<cx<T>*>(lds), red, in, in, in, vout,
                                                     nullptr, out, nlines, tb, coef, partials, sten);
        } else if (kind == KIND_VUPD) {
          dst_x_body<T, L, KIND_VUPD, false, false>(c, reinterpret_cast<cx<T>*>(lds), red, in, nullptr, nullptr,
                                                    nullptr, nullptr, out, nlines, tb, coef, partials, sten);
        } else {
          dst_x_body<T, L, KIND_DOT, false, false>(c, reinterpret_cast<cx<T>*>(lds), red, in, nullptr, nullptr,
                                                   nullptr, vdot, out, nlines, tb, coef, partials, sten);
        }
      });
    }
  };
};

template <typename T>
struct DstSRun {
  template <int L>
  struct R {
    static void run(T* x, int64_t nlines, int64_t S, const DstTables<T>& tb) {
      run_grid(tpb_fft<T, FK_DSTS>(), (int)fft_blocks<T, FK_DSTS>(L, nlines), 1, fft_lds_bytes<T, FK_DSTS>(L),
               [&](HostCtx& c, unsigned char* lds) {
        if (S % 2 == 0 && nlines % 2 == 0)
          dst_strided_body<T, L, true>(c, reinterpret_cast<cx<T>*>(lds), x, nlines, S, tb);
        else
          dst_strided_body<T, L, false>(c, reinterpret_cast<cx<T>*>(lds), x, nlines, S, tb);
      });
    }
  };
};

template <typename T>
struct MvRun {
  template <int L>
  struct R {
    static void run(const T* z, T* out, int64_t M, const MatvecTables<T>& tb, double* partials, bool stencil) {
      constexpr int NL = lines_per_block<T, FK_MV>(L);
      using Fm = LineFft<T, L, NL, true, LAST_DEFAULT>;
      run_grid(tpb_fft<T, FK_MV>(), (int)fft_blocks<T, FK_MV>(L, M), 1, fft_lds_bytes<T, FK_MV>(L),
               [&](HostCtx& c, unsigned char* lds) {
        double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Fm::LDS_ELEMS);
        if (stencil)
          matvec_fft_body<T, L, MV_DOT, TERM_STENCIL, false>(c, reinterpret_cast<cx<T>*>(lds), red, const_cast<T*>(z),
                                                             out, nullptr, M, tb, IterUpd{}, partials);
        else
          matvec_fft_body<T, L, MV_DOT, TERM_NONE, false>(c, reinterpret_cast<cx<T>*>(lds), red, const_cast<T*>(z), out,
                                                          nullptr, M, tb, IterUpd{}, partials);
      });
    }
  };
};

struct Problem {
  int dim;
  int m[3];
  double h[3];
  int64_t N, M;
  double alpha;
  std::vector<double> p, q;
};

Problem make_problem(int dim, const int* m, const double* h, int64_t N, double alpha, const double* p,
                     const double* q) {
  Problem P;
  P.dim = dim;
  P.M = 1;
  for (int d = 0; d < 3; ++d) {
    P.m[d] = d < dim ? m[d] : 1;
    P.h[d] = d < dim ? h[d] : 1.0;
    if (d < dim) P.M *= m[d];
  }
  P.N = N;
  P.alpha = alpha;
  P.p.assign(p, p + N);
  P.q.assign(q, q + N);
  return P;
}

// face coefficients of a variable-coefficient operator (emu_set_faces; null: a = 1)
const double* g_faces[3] = {nullptr, nullptr, nullptr};

Grid grid_of(const Problem& P) {
  Grid g;
  g.dim = P.dim;
  for (int d = 0; d < 3; ++d) {
    g.m[d] = P.m[d];
    g.inv_h2[d] = d < P.dim ? 1.0 / (P.h[d] * P.h[d]) : 0.0;
    g.face[d] = d < P.dim ? g_faces[d] : nullptr;
  }
  return g;
}

template <typename T>
struct HostTables {
  std::vector<cx<T>> tw_time, tw_dst[3], sigma, rho, tw_mv, phat;
  std::vector<T> dinv, d2, mu;
  explicit HostTables(const Problem& P) {
    tw_time = to_cx<T>(host::twiddles((int)P.N));
    for (int d = 0; d < P.dim; ++d) tw_dst[d] = to_cx<T>(host::twiddles(2 * (P.m[d] + 1)));
    dinv = to_t<T>(host::alpha_pow(P.N, P.alpha, -1.0));
    d2 = to_t<T>(host::alpha_pow(P.N, P.alpha, 2.0));
    sigma = to_cx<T>(host::alpha_spectrum(P.p, P.alpha));
    rho = to_cx<T>(host::alpha_spectrum(P.q, P.alpha));
    mu = to_t<T>(host::lap_eigs(P.dim, P.m, P.h));
    tw_mv = to_cx<T>(host::twiddles((int)(2 * P.N)));
    phat = to_cx<T>(host::matvec_spectrum(P.p));
  }
  DstTables<T> dst(const Problem& P, int d) const {
    DstTables<T> tb;
    tb.tw = tw_dst[d].data();
    tb.m = P.m[d];
    tb.nrm = (T)(1.0 / std::sqrt(2.0 * (P.m[d] + 1)));
    return tb;
  }
};

template <typename T>
TimeTables<T> time_tables(const Problem& P, const HostTables<T>& ht) {
  int qtaps = 0;
  for (int64_t k = 0; k < P.N; ++k)
    if (P.q[(size_t)k] != 0.0) qtaps = (int)k + 1;
  TimeTables<T> tt;
  tt.tw = ht.tw_time.data();
  tt.dinv = ht.dinv.data();
  tt.d2 = ht.d2.data();
  tt.sigma = ht.sigma.data();
  tt.rho = ht.rho.data();
  tt.mu = ht.mu.data();
  tt.log2_alpha_over_N = (T)(std::log2(P.alpha) / (double)P.N);
  for (int k = 0; k < 4; ++k) tt.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
  tt.qtaps = qtaps;
  tt.mx = (int)P.m[0];
  tt.aux = nullptr;
  return tt;
}

template <typename T>
VupdStencil<T> vupd_stencil(const Problem& P, const T* z) {
  int qtaps = 0;
  for (int64_t k = 0; k < P.N; ++k)
    if (P.q[(size_t)k] != 0.0) qtaps = (int)k + 1;
  VupdStencil<T> st;
  st.z = z;
  for (int k = 0; k < 4; ++k) st.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
  st.qtaps = qtaps;
  st.grid = grid_of(P);
  st.N = (int)P.N;
  st.R = P.M / P.m[0];
  return st;
}

template <typename T>
void space_strided(const Problem& P, const HostTables<T>& ht, T* x, bool reverse) {
  const int64_t n = P.N * P.M;
  for (int k = 1; k < P.dim; ++k) {
    const int d = reverse ? P.dim - k : k;
    int64_t S = 1;
    for (int e = 0; e < d; ++e) S *= P.m[e];
    with_L<DstSRun<T>::template R>(2 * (P.m[d] + 1), x, n / P.m[d], S, ht.dst(P, d));
  }
}

// x-line transform fused with the layout move (FP64, the sine-basis in/out passes)
struct DstXtRun {
  template <int L>
  struct R {
    static void run(int dir, const double* in, double* out, int64_t N, int64_t M, const DstTables<double>& tb,
                    double* partials) {
      constexpr int NL = DSTXT_TPB / (L / fft_V(L));
      using Fx = LineFft<double, L, NL, false, LAST_LINEAR, false, 0, dst_split<double>()>;
      constexpr int m = L / 2 - 1;
      const int64_t blocks = dstxt_blocks(M / m, N, dstxt_lines<double, L>());
      run_grid(DSTXT_TPB, (int)blocks, 1, sizeof(cx<double>) * Fx::LDS_ELEMS + DSTXT_TPB * sizeof(double),
               [&](HostCtx& c, unsigned char* lds) {
                 double* red = reinterpret_cast<double*>(lds + sizeof(cx<double>) * Fx::LDS_ELEMS);
                 if (dir == 0)
                   dst_xt_body<double, L, 0>(c, reinterpret_cast<cx<double>*>(lds), red, in, out, N, M, tb, partials);
                 else
                   dst_xt_body<double, L, 1>(c, reinterpret_cast<cx<double>*>(lds), red, in, out, N, M, tb,
                                             nullptr);
               });
    }
  };
};

// strided transforms on a mode-major vector (stride N m_0 ... m_{d-1} along d)
void space_strided_mm(const Problem& P, const HostTables<double>& ht, double* x, bool reverse) {
  const int64_t n = P.N * P.M;
  for (int k = 1; k < P.dim; ++k) {
    const int d = reverse ? P.dim - k : k;
    int64_t S = P.N;
    for (int e = 0; e < d; ++e) S *= P.m[e];
    with_L<DstSRun<double>::template R>(2 * (P.m[d] + 1), x, n / P.m[d], S, ht.dst(P, d));
  }
}

// dir 0: y (mode-major) = (I x U) x with x time-major, returns the sum of the
// partial sums of ||x||^2; dir 1: y (time-major) = (I x U) x with x mode-major
double apply_sine_io(const Problem& P, const double* x, double* y, int dir) {
  HostTables<double> ht(P);
  const int64_t n = P.N * P.M;
  const int L = 2 * (P.m[0] + 1);
  std::vector<double> partials((size_t)(P.M / P.m[0]) * (size_t)P.N + 8, 0.0);
  if (dir == 0) {
    with_L<DstXtRun::template R>(L, 0, x, y, P.N, P.M, ht.dst(P, 0), partials.data());
    space_strided_mm(P, ht, y, false);
  } else {
    std::vector<double> t(x, x + n);
    space_strided_mm(P, ht, t.data(), true);
    with_L<DstXtRun::template R>(L, 1, (const double*)t.data(), y, P.N, P.M, ht.dst(P, 0), (double*)nullptr);
  }
  double s = 0.0;
  for (double v : partials) s += v;
  return s;
}

template <typename T>
void apply_space(const Problem& P, const T* x, T* y) {
  HostTables<T> ht(P);
  const int64_t n = P.N * P.M;
  const double one[4] = {1, 0, 0, 0};
  with_L<DstXRun<T>::template R>(2 * (P.m[0] + 1), x, y, n / P.m[0], ht.dst(P, 0), one, (double*)nullptr,
                                 (const T*)nullptr, (int)KIND_VUPD, (T*)nullptr, vupd_stencil<T>(P, nullptr));
  space_strided<T>(P, ht, y, false);
}

template <typename T>
void apply_time(const Problem& P, T* x) {
  HostTables<T> ht(P);
  TimeTables<T> tt = time_tables<T>(P, ht);
  with_L<TimeRun<T>::template R>((int)P.N, x, P.M, tt);
}

template <typename T>
void apply_precond(const Problem& P, const T* x, T* y) {
  HostTables<T> ht(P);
  const int64_t n = P.N * P.M;
  std::vector<T> tmp((size_t)n);
  const double one[4] = {1, 0, 0, 0};
  const int Lx = 2 * (P.m[0] + 1);
  with_L<DstXRun<T>::template R>(Lx, x, tmp.data(), n / P.m[0], ht.dst(P, 0), one, (double*)nullptr,
                                 (const T*)nullptr, (int)KIND_VUPD, (T*)nullptr, vupd_stencil<T>(P, nullptr));
  space_strided<T>(P, ht, tmp.data(), false);
  TimeTables<T> tt = time_tables<T>(P, ht);
  with_L<TimeRun<T>::template R>((int)P.N, tmp.data(), P.M, tt);
  space_strided<T>(P, ht, tmp.data(), true);
  std::vector<double> partials((size_t)fft_blocks<T, FK_DSTX>(Lx, n / P.m[0]) + 1);
  with_L<DstXRun<T>::template R>(Lx, tmp.data(), y, n / P.m[0], ht.dst(P, 0), one, partials.data(), x,
                                 (int)KIND_DOT, (T*)nullptr, vupd_stencil<T>(P, nullptr));
}

template <typename T>
double apply_sym(const Problem& P, const T* z, T* out, bool force_fft, bool stencil = true) {
  int ptaps = 0, qtaps = 0;
  for (int64_t k = 0; k < P.N; ++k) {
    if (P.p[(size_t)k] != 0.0) ptaps = (int)k + 1;
    if (P.q[(size_t)k] != 0.0) qtaps = (int)k + 1;
  }
  double dot = 0.0;
  if (ptaps <= 8 && !force_fft) {
    ShortTables<T> tb;
    for (int k = 0; k < 8; ++k) tb.p[k] = (T)(k < ptaps ? P.p[(size_t)k] : 0.0);
    tb.ptaps = ptaps;
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.grid = grid_of(P);
    tb.N = (int)P.N;
    tb.chunk = 8;
    tb.term = stencil ? TERM_STENCIL : TERM_NONE;
    tb.mu = nullptr;
    const int gx = (int)((P.M + TPB_EW - 1) / TPB_EW);
    const int gy = (int)(((P.N + 1) / 2 + tb.chunk - 1) / tb.chunk);
    std::vector<double> partials((size_t)gx * gy);
    run_grid(TPB_EW, gx, gy, TPB_EW * sizeof(double), [&](HostCtx& c, unsigned char* lds) {
      matvec_short_body<T, MV_DOT>(c, reinterpret_cast<double*>(lds), z, out, (const T*)nullptr, P.M, tb,
                                   partials.data());
    });
    for (double v : partials) dot += v;
  } else {
    HostTables<T> ht(P);
    MatvecTables<T> tb;
    tb.tw = ht.tw_mv.data();
    tb.phat = ht.phat.data();
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.mx = (int)P.m[0];
    tb.grid = grid_of(P);
    std::vector<double> partials((size_t)fft_blocks<T, FK_MV>((int)(2 * P.N), P.M));
    with_L2<MvRun<T>::template R>((int)(2 * P.N), z, out, P.M, tb, partials.data(), stencil);
    for (double v : partials) dot += v;
  }
  return dot;
}

// r = Y (f - A u) the way the solver forms it for dense p: time-line FFT pass
// without the stencil, then the x-line stencil pass; returns ||r||^2
template <typename T>
struct MvResRun {
  template <int L>
  struct R {
    static void run(const T* z, T* out, const T* fin, int64_t M, const MatvecTables<T>& tb, double* partials) {
      constexpr int NL = lines_per_block<T, FK_MV>(L);
      using Fm = LineFft<T, L, NL, true, LAST_DEFAULT>;
      run_grid(tpb_fft<T, FK_MV>(), (int)fft_blocks<T, FK_MV>(L, M), 1, fft_lds_bytes<T, FK_MV>(L),
               [&](HostCtx& c, unsigned char* lds) {
                 double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Fm::LDS_ELEMS);
                 matvec_fft_body<T, L, MV_RESID, TERM_NONE, false>(c, reinterpret_cast<cx<T>*>(lds), red,
                                                                   const_cast<T*>(z), out, fin, M, tb, IterUpd{},
                                                                   partials);
               });
    }
  };
};

// r = Y (f - A u) in one pass, stencil included (the variable-coefficient form)
template <typename T>
struct MvResFullRun {
  template <int L>
  struct R {
    static void run(const T* z, T* out, const T* fin, int64_t M, const MatvecTables<T>& tb, double* partials) {
      constexpr int NL = lines_per_block<T, FK_MV>(L);
      using Fm = LineFft<T, L, NL, true, LAST_DEFAULT>;
      run_grid(tpb_fft<T, FK_MV>(), (int)fft_blocks<T, FK_MV>(L, M), 1, fft_lds_bytes<T, FK_MV>(L),
               [&](HostCtx& c, unsigned char* lds) {
                 double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Fm::LDS_ELEMS);
                 matvec_fft_body<T, L, MV_RESID, TERM_STENCIL, false>(c, reinterpret_cast<cx<T>*>(lds), red,
                                                                      const_cast<T*>(z), out, fin, M, tb, IterUpd{},
                                                                      partials);
               });
    }
  };
};

template <typename T>
double apply_resid_full(const Problem& P, const T* u, const T* f, T* r, bool force_fft) {
  int ptaps = 0, qtaps = 0;
  for (int64_t k = 0; k < P.N; ++k) {
    if (P.p[(size_t)k] != 0.0) ptaps = (int)k + 1;
    if (P.q[(size_t)k] != 0.0) qtaps = (int)k + 1;
  }
  double s = 0.0;
  if (ptaps <= 8 && !force_fft) {
    ShortTables<T> tb;
    for (int k = 0; k < 8; ++k) tb.p[k] = (T)(k < ptaps ? P.p[(size_t)k] : 0.0);
    tb.ptaps = ptaps;
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.grid = grid_of(P);
    tb.N = (int)P.N;
    tb.chunk = 8;
    tb.term = TERM_STENCIL;
    tb.mu = nullptr;
    const int gx = (int)((P.M + TPB_EW - 1) / TPB_EW);
    const int gy = (int)(((P.N + 1) / 2 + tb.chunk - 1) / tb.chunk);
    std::vector<double> partials((size_t)gx * gy);
    run_grid(TPB_EW, gx, gy, TPB_EW * sizeof(double), [&](HostCtx& c, unsigned char* lds) {
      matvec_short_body<T, MV_RESID>(c, reinterpret_cast<double*>(lds), u, r, f, P.M, tb, partials.data());
    });
    for (double v : partials) s += v;
  } else {
    HostTables<T> ht(P);
    MatvecTables<T> tb;
    tb.tw = ht.tw_mv.data();
    tb.phat = ht.phat.data();
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.mx = (int)P.m[0];
    tb.grid = grid_of(P);
    std::vector<double> partials((size_t)fft_blocks<T, FK_MV>((int)(2 * P.N), P.M));
    with_L2<MvResFullRun<T>::template R>((int)(2 * P.N), u, r, f, P.M, tb, partials.data());
    for (double v : partials) s += v;
  }
  return s;
}

template <typename T>
double apply_resid(const Problem& P, const T* u, const T* f, T* r) {
  HostTables<T> ht(P);
  int qtaps = 0;
  for (int64_t k = 0; k < P.N; ++k)
    if (P.q[(size_t)k] != 0.0) qtaps = (int)k + 1;
  MatvecTables<T> tb;
  tb.tw = ht.tw_mv.data();
  tb.phat = ht.phat.data();
  for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
  tb.qtaps = qtaps;
  tb.mx = (int)P.m[0];
  tb.grid = grid_of(P);
  std::vector<double> partials((size_t)fft_blocks<T, FK_MV>((int)(2 * P.N), P.M));
  with_L2<MvResRun<T>::template R>((int)(2 * P.N), u, r, f, P.M, tb, partials.data());
  const int64_t nlines = P.N * P.M / P.m[0];
  std::vector<double> lp((size_t)nlines);
  const VupdStencil<T> st = vupd_stencil<T>(P, u);
  run_grid(TPB_EW, (int)nlines, 1, TPB_EW * sizeof(double), [&](HostCtx& c, unsigned char* lds) {
    if (st.qtaps <= 1)
      resid_stencil_body<T, true>(c, reinterpret_cast<double*>(lds), r, st, lp.data());
    else
      resid_stencil_body<T, false>(c, reinterpret_cast<double*>(lds), r, st, lp.data());
  });
  double s = 0.0;
  for (double v : lp) s += v;
  return s;
}

// q1 + Y L_h (q * z) through the x-line pass (coefficients 1, 0, 0)
template <typename T>
void apply_vupd_stencil(const Problem& P, const T* q1, const T* z, T* vout) {
  HostTables<T> ht(P);
  const int64_t n = P.N * P.M;
  std::vector<T> tmp((size_t)n);
  const double one[4] = {1, 0, 0, 0};
  with_L<DstXRun<T>::template R>(2 * (P.m[0] + 1), q1, tmp.data(), n / P.m[0], ht.dst(P, 0), one,
                                 (double*)nullptr, (const T*)nullptr, (int)KIND_VUPD, vout, vupd_stencil<T>(P, z));
}

// time pass in place, returning the summed spatial dot product of its output
template <typename T>
double apply_time_aux(const Problem& P, T* x) {
  HostTables<T> ht(P);
  TimeTables<T> tt = time_tables<T>(P, ht);
  std::vector<double> aux((size_t)fft_blocks<T, FK_TIME>((int)P.N, P.M), 0.0);
  tt.aux = aux.data();
  with_L<TimeRun<T>::template R>((int)P.N, x, P.M, tt);
  double s = 0.0;
  for (double v : aux) s += v;
  return s;
}

// Lanczos update + time pass (sine coordinates), returning the summed dot
template <typename T, typename TQ>
struct UpdRun {
  template <int L>
  struct R {
    static void run(const TQ* Q, const T* V1, const T* V2, T* Vout, T* Zout, int64_t M, const TimeTables<T>& tb,
                    const double* coef, double* partials, bool full, bool qrev) {
      constexpr int NL = lines_per_block<T, FK_SPEC>(L);
      using Ft = LineFft<T, L, NL, false, LAST_PAIRED>;
      // fewer workgroups than tiles: every workgroup walks several tiles
      const int64_t tiles = fft_tiles<T, FK_SPEC>(L, M);
      run_grid(tpb_fft<T, FK_SPEC>(), (int)(upd_persistent<T>() ? std::min<int64_t>(tiles, 3) : tiles), 1,
               fft_lds_bytes<T, FK_SPEC>(L) + upd_twl_bytes<T, L>(), [&](HostCtx& c, unsigned char* lds) {
                 double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Ft::LDS_ELEMS);
                 // radix plan 1 where it exists (FP32, L = 512, 1024), plan 0 otherwise
                 if constexpr (sizeof(T) == 4 && fft_plan_alt(L)) {
                   if (g_plan == 1) {
                     if (full)
                       time_upd_body<T, L, TQ, true, true, true, 1>(c, reinterpret_cast<cx<T>*>(lds), red, Q, V1, V2,
                                                                    Vout, Zout, M, tb, coef, partials);
                     else
                       time_upd_body<T, L, TQ, false, true, true, 1>(c, reinterpret_cast<cx<T>*>(lds), red, Q, V1, V2,
                                                                     Vout, Zout, M, tb, coef, partials, qrev);
                     return;
                   }
                 }
                 if (full)
                   time_upd_body<T, L, TQ, true, true>(c, reinterpret_cast<cx<T>*>(lds), red, Q, V1, V2, Vout, Zout, M,
                                                       tb, coef, partials);
                 else
                   time_upd_body<T, L, TQ, false, true>(c, reinterpret_cast<cx<T>*>(lds), red, Q, V1, V2, Vout, Zout,
                                                        M, tb, coef, partials, qrev);
               });
    }
  };
};

template <typename T, typename TQ>
double apply_time_upd(const Problem& P, const TQ* Q, const T* V1, const T* V2, T* Vout, T* Zout, const double* coef,
                      bool full, bool qrev = false) {
  HostTables<T> ht(P);
  TimeTables<T> tt = time_tables<T>(P, ht);
  std::vector<double> partials((size_t)fft_tiles<T, FK_SPEC>((int)P.N, P.M), 0.0);
  with_L<UpdRun<T, TQ>::template R>((int)P.N, Q, V1, V2, Vout, Zout, P.M, tt, coef, partials.data(), full, qrev);
  double s = 0.0;
  for (double v : partials) s += v;
  return s;
}

// sine-coordinate matvec (MV_DOT) or residual (MV_RESID), FFT or direct form
template <typename T, int MODE>
struct MvSpecRun {
  template <int L>
  struct R {
    static void run(T* z, T* out, const T* fin, int64_t M, const MatvecCSTables<T>& tb, const IterUpd& up,
                    double* partials) {
      constexpr int NL = lines_per_block<T, FK_SPEC>(L);
      using Fm = LineFft<T, L, NL, false, LAST_DEFAULT>;
      const int64_t tiles = fft_tiles<T, FK_SPEC>(L, M);
      const int blocks = (int)(g_cs_blocks > 0 ? std::min<int64_t>(tiles, g_cs_blocks) : tiles);
      run_grid(tpb_fft<T, FK_SPEC>(), blocks, 1,
               cs_lds_bytes<T, L>(), [&](HostCtx& c, unsigned char* lds) {
                 double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Fm::LDS_ELEMS);
                 cx<T>* tabs = reinterpret_cast<cx<T>*>(lds + cs_lds_base<T, L>());
                 if constexpr (sizeof(T) == 4 && fft_plan_alt(L)) {
                   if (g_plan == 1) {
                     matvec_cs_body<T, L, MODE, 1>(c, reinterpret_cast<cx<T>*>(lds), red, tabs, z, out, fin, M, tb,
                                                   up, partials);
                     return;
                   }
                 }
                 matvec_cs_body<T, L, MODE>(c, reinterpret_cast<cx<T>*>(lds), red, tabs, z, out, fin, M, tb, up,
                                            partials);
               });
    }
  };
};

// 2N-point form on mode-major vectors (the FP64 sine-coordinate kernels)
template <typename T, int MODE>
struct MvSpec2nRun {
  template <int L>
  struct R {
    static void run(T* z, T* out, const T* fin, int64_t M, const MatvecTables<T>& tb, const IterUpd& up,
                    double* partials) {
      constexpr int FK = fk_mv<true, L>();
      constexpr int NL = lines_per_block<T, FK>(L);
      using Fm = LineFft<T, L, NL, false, LAST_DEFAULT>;
      run_grid(tpb_fft<T, FK>(), (int)fft_blocks<T, FK>(L, M), 1, fft_lds_bytes<T, FK>(L),
               [&](HostCtx& c, unsigned char* lds) {
                 double* red = reinterpret_cast<double*>(lds + sizeof(cx<T>) * Fm::LDS_ELEMS);
                 if constexpr (sizeof(T) == 8 && MODE == MV_RESID) {
                   if (up.r32) {
                     matvec_fft_body<T, L, MODE, TERM_SPEC, true, true>(c, reinterpret_cast<cx<T>*>(lds), red, z,
                                                                        out, fin, M, tb, up, partials);
                     return;
                   }
                 }
                 matvec_fft_body<T, L, MODE, TERM_SPEC, true>(c, reinterpret_cast<cx<T>*>(lds), red, z, out, fin, M,
                                                              tb, up, partials);
               });
    }
  };
};

template <typename T, int MODE>
double apply_spec(const Problem& P, const T* z, T* out, const T* fin, bool force_fft, const IterUpd* upd = nullptr,
                  bool two_n = false) {
  int ptaps = 0, qtaps = 0;
  for (int64_t k = 0; k < P.N; ++k) {
    if (P.p[(size_t)k] != 0.0) ptaps = (int)k + 1;
    if (P.q[(size_t)k] != 0.0) qtaps = (int)k + 1;
  }
  HostTables<T> ht(P);
  double dot = 0.0;
  if (ptaps <= 8 && !force_fft) {
    ShortTables<T> tb;
    for (int k = 0; k < 8; ++k) tb.p[k] = (T)(k < ptaps ? P.p[(size_t)k] : 0.0);
    tb.ptaps = ptaps;
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.grid = grid_of(P);
    tb.N = (int)P.N;
    tb.chunk = 8;
    tb.term = TERM_SPEC;
    tb.mu = ht.mu.data();
    int log2N = 0;
    while ((1 << log2N) < P.N) ++log2N;
    // a grid smaller than the vector exercises the grid-stride loop
    const int gx = (int)std::min<int64_t>((P.N * P.M + TPB_EW - 1) / TPB_EW, 7);
    std::vector<double> partials((size_t)gx);
    run_grid(TPB_EW, gx, 1, TPB_EW * sizeof(double), [&](HostCtx& c, unsigned char* lds) {
      matvec_short_mm_body<T, MODE>(c, reinterpret_cast<double*>(lds), z, out, fin, P.M, tb, log2N, partials.data());
    });
    for (double v : partials) dot += v;
  } else if (two_n) {
    MatvecTables<T> tb;
    tb.tw = ht.tw_mv.data();
    tb.phat = ht.phat.data();
    tb.mu = ht.mu.data();
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.mx = (int)P.m[0];
    tb.grid = grid_of(P);
    IterUpd up{};
    if (upd) up = *upd;
    std::vector<double> partials((size_t)mv_blocks<T>(true, (int)(2 * P.N), P.M));
    with_L2<MvSpec2nRun<T, MODE>::template R>((int)(2 * P.N), const_cast<T*>(z), out, fin, P.M, tb, up,
                                             partials.data());
    for (double v : partials) dot += v;
  } else {
    const std::vector<cx<T>> chat = to_cx<T>(host::circulant_spectrum(P.p, false));
    const std::vector<cx<T>> shat = to_cx<T>(host::circulant_spectrum(P.p, true));
    const std::vector<cx<T>> omega = to_cx<T>(host::half_roots(P.N));
    MatvecCSTables<T> tb;
    tb.tw = ht.tw_time.data();
    tb.chat = chat.data();
    tb.shat = shat.data();
    tb.omega = omega.data();
    tb.mu = ht.mu.data();
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < qtaps ? P.q[(size_t)k] : 0.0);
    tb.qtaps = qtaps;
    tb.mx = (int)P.m[0];
    IterUpd up{};
    if (upd) up = *upd;
    std::vector<double> partials((size_t)fft_tiles<T, FK_SPEC>((int)P.N, P.M), 0.0);
    with_L<MvSpecRun<T, MODE>::template R>((int)P.N, const_cast<T*>(z), out, fin, P.M, tb, up, partials.data());
    for (double v : partials) dot += v;
  }
  return dot;
}

// scalar phase and direction/iterate update, as the solver sequences them
void apply_scalar(int phase, SolverState* st, const double* partials, int64_t np, double* hist, ZBasis zb) {
  run_grid(TPB_EW, 1, 1, TPB_EW * sizeof(double), [&](HostCtx& c, unsigned char* lds) {
    scalar_body(c, reinterpret_cast<double*>(lds), phase, st, partials, np, (const double*)nullptr, 0, hist, zb);
  });
}

template <typename T>
void apply_wx(const T* Z, T* Wa, const T* Wb, T* X, int64_t n, const double* coef) {
  const int nb = (int)std::min<int64_t>((n + TPB_EW - 1) / TPB_EW, 64);
  run_grid(TPB_EW, nb, 1, 0, [&](HostCtx& c, unsigned char*) { wx_body<T, T>(c, Z, Wa, Wb, X, n, coef); });
}

void apply_transpose(const double* in, double* out, int64_t R, int64_t C, bool rev) {
  const int64_t nb = ((C + TR_TILE - 1) / TR_TILE) * ((R + TR_TILE - 1) / TR_TILE);
  run_grid(TPB_EW, (int)nb, 1, sizeof(double) * TR_TILE * (TR_TILE + 1), [&](HostCtx& c, unsigned char* lds) {
    if (rev)
      transpose_body<double, true>(c, reinterpret_cast<double*>(lds), in, out, R, C);
    else
      transpose_body<double, false>(c, reinterpret_cast<double*>(lds), in, out, R, C);
  });
}

}  // namespace

extern "C" {

void emu_transpose_f64(const double* in, double* out, int64_t R, int64_t C, int rev) {
  apply_transpose(in, out, R, C, rev != 0);
}

int64_t emu_state_size(void) { return (int64_t)sizeof(SolverState); }
// byte offsets: coef_v, coef_w, eta, eta0, status, rinv, rscale, iter
void emu_state_offsets(int64_t* o) {
  o[0] = offsetof(SolverState, coef_v);
  o[1] = offsetof(SolverState, coef_w);
  o[2] = offsetof(SolverState, eta);
  o[3] = offsetof(SolverState, eta0);
  o[4] = offsetof(SolverState, status);
  o[5] = offsetof(SolverState, rinv);
  o[6] = offsetof(SolverState, rscale);
  o[7] = offsetof(SolverState, iter);
}
void emu_scalar(int phase, void* st, const double* partials, int64_t np, double* hist, double* om, double* y,
                int K) {
  ZBasis zb;
  zb.om = om;
  zb.y = y;
  zb.K = K;
  apply_scalar(phase, reinterpret_cast<SolverState*>(st), partials, np, hist, zb);
}
// u += s * sum_i y[i] Z_i, Z_i = zs + i*n (FP32)
void emu_combine_f32(double* u, const float* zs, int k, const double* y, double s, int64_t n) {
  ZList<float> zl;
  for (int i = 0; i < ZB_MAX; ++i) zl.z[i] = i < k ? zs + (int64_t)i * n : nullptr;
  zl.k = k;
  const int nb = (int)std::min<int64_t>((n + TPB_EW - 1) / TPB_EW, 9);
  run_grid(TPB_EW, nb, 1, 0, [&](HostCtx& c, unsigned char*) { combine_body<float>(c, u, zl, y, &s, n); });
}
void emu_wx_f64(const double* Z, double* Wa, const double* Wb, double* X, int64_t n, const double* coef) {
  apply_wx<double>(Z, Wa, Wb, X, n, coef);
}
void emu_wx_f32(const float* Z, float* Wa, const float* Wb, float* X, int64_t n, const double* coef) {
  apply_wx<float>(Z, Wa, Wb, X, n, coef);
}


// the kernels' assignment of sine modes to complex lines, for lines 0..count-1
void emu_mode_pairs(int64_t M, int mx, int64_t count, int64_t* ia, int64_t* ib) {
  for (int64_t t = 0; t < count; ++t) mode_pair(t, M, mx, ia[t], ib[t]);
}

int emu_error(void) { return g_error; }
// radix plan of the FP32 time pass and N-point matvec (0 or 1)
void emu_set_plan(int plan) { g_plan = plan; }
// workgroups of the N-point matvec (0: one per tile, else persistent)
void emu_set_cs_blocks(int blocks) { g_cs_blocks = blocks; }

#define EMU_ARGS int dim, const int *m, const double *h, int64_t N, double alpha, const double *p, const double *q
#define EMU_P make_problem(dim, m, h, N, alpha, p, q)

void emu_space_f64(EMU_ARGS, const double* x, double* y) { apply_space<double>(EMU_P, x, y); }
double emu_sine_io(EMU_ARGS, const double* x, double* y, int dir) { return apply_sine_io(EMU_P, x, y, dir); }
void emu_space_f32(EMU_ARGS, const float* x, float* y) { apply_space<float>(EMU_P, x, y); }
void emu_time_f64(EMU_ARGS, double* x) { apply_time<double>(EMU_P, x); }
void emu_time_f32(EMU_ARGS, float* x) { apply_time<float>(EMU_P, x); }
void emu_precond_f64(EMU_ARGS, const double* x, double* y) { apply_precond<double>(EMU_P, x, y); }
void emu_precond_f32(EMU_ARGS, const float* x, float* y) { apply_precond<float>(EMU_P, x, y); }
void emu_set_faces(const double* f0, const double* f1, const double* f2) {
  g_faces[0] = f0;
  g_faces[1] = f1;
  g_faces[2] = f2;
}
double emu_resid_full_f64(EMU_ARGS, const double* u, const double* f, double* r, int force_fft) {
  return apply_resid_full<double>(EMU_P, u, f, r, force_fft != 0);
}
double emu_sym_f64(EMU_ARGS, const double* x, double* y, int force_fft) {
  return apply_sym<double>(EMU_P, x, y, force_fft != 0);
}
double emu_sym_f32(EMU_ARGS, const float* x, float* y, int force_fft) {
  return apply_sym<float>(EMU_P, x, y, force_fft != 0);
}
double emu_sym_nostencil_f64(EMU_ARGS, const double* x, double* y, int force_fft) {
  return apply_sym<double>(EMU_P, x, y, force_fft != 0, false);
}
double emu_sym_nostencil_f32(EMU_ARGS, const float* x, float* y, int force_fft) {
  return apply_sym<float>(EMU_P, x, y, force_fft != 0, false);
}
void emu_vupd_stencil_f64(EMU_ARGS, const double* q1, const double* z, double* v) {
  apply_vupd_stencil<double>(EMU_P, q1, z, v);
}
void emu_vupd_stencil_f32(EMU_ARGS, const float* q1, const float* z, float* v) {
  apply_vupd_stencil<float>(EMU_P, q1, z, v);
}
double emu_time_aux_f64(EMU_ARGS, double* x) { return apply_time_aux<double>(EMU_P, x); }
double emu_resid_f64(EMU_ARGS, const double* u, const double* f, double* r) {
  return apply_resid<double>(EMU_P, u, f, r);
}
double emu_time_aux_f32(EMU_ARGS, float* x) { return apply_time_aux<float>(EMU_P, x); }
double emu_time_upd_f64(EMU_ARGS, const double* Q, const double* V1, const double* V2, double* Vout, double* Zout,
                        const double* coef, int full) {
  return apply_time_upd<double, double>(EMU_P, Q, V1, V2, Vout, Zout, coef, full == 1, full == 2);
}
double emu_time_upd_f32(EMU_ARGS, const float* Q, const float* V1, const float* V2, float* Vout, float* Zout,
                        const double* coef, int full) {
  return apply_time_upd<float, float>(EMU_P, Q, V1, V2, Vout, Zout, coef, full == 1, full == 2);
}
double emu_time_upd_mixed(EMU_ARGS, const double* Q, float* Vout, float* Zout, const double* coef, int qrev) {
  return apply_time_upd<float, double>(EMU_P, Q, (const float*)nullptr, (const float*)nullptr, Vout, Zout, coef,
                                       false, qrev != 0);
}
// form: 0 direct (short p), 1 N-point circulant + skew-circulant, 2 zero-padded 2N-point
double emu_sym_spec_f64(EMU_ARGS, const double* z, double* out, int form) {
  return apply_spec<double, MV_DOT>(EMU_P, z, out, (const double*)nullptr, form != 0, nullptr, form == 2);
}
double emu_sym_spec_f32(EMU_ARGS, const float* z, float* out, int form) {
  return apply_spec<float, MV_DOT>(EMU_P, z, out, (const float*)nullptr, form != 0, nullptr, form == 2);
}
double emu_resid_spec_f64(EMU_ARGS, const double* u, const double* f, double* r, int form) {
  return apply_spec<double, MV_RESID>(EMU_P, u, r, f, form != 0, nullptr, form == 2);
}
// u <- (u_zero ? 0 : u) + s sum_i y[i] Z_i (Z_i = zs + i*n, FP32), then r = Y(f - A u): the
// refinement step of the mixed path in one pass (FFT form)
double emu_resid_upd_f64(EMU_ARGS, double* u, const double* f, double* r, const float* zs, int k, const double* y,
                         double s, int u_zero, int two_n) {
  const Problem P = EMU_P;
  IterUpd up{};
  for (int i = 0; i < ZB_MAX; ++i) up.z[i] = i < k ? zs + (int64_t)i * P.N * P.M : nullptr;
  up.k = k;
  up.y = y;
  up.s = &s;
  up.u_zero = u_zero;
  return apply_spec<double, MV_RESID>(P, u, r, f, true, &up, two_n != 0);
}
// as emu_resid_upd_f64 in the 2N-point form, with the residual written as FP32
// to r32, times r32_scale (r is not written)
double emu_resid_upd_r32_f64(EMU_ARGS, double* u, const double* f, float* r32, double r32_scale, const float* zs,
                             int k, const double* y, double s, int u_zero) {
  const Problem P = EMU_P;
  IterUpd up{};
  for (int i = 0; i < ZB_MAX; ++i) up.z[i] = i < k ? zs + (int64_t)i * P.N * P.M : nullptr;
  up.k = k;
  up.y = y;
  up.s = &s;
  up.u_zero = u_zero;
  up.r32 = r32;
  up.r32_scale = r32_scale;
  std::vector<double> unused((size_t)(P.N * P.M), 0.0);
  return apply_spec<double, MV_RESID>(P, u, unused.data(), f, true, &up, true);
}

}  // extern "C"
