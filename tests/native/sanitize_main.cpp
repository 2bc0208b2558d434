// Main program of the sanitizer build of the kernel-body emulator (emu.cpp): runs
// every emulated kernel family once per problem on exactly sized host arrays,
// so that AddressSanitizer flags any access outside them and
// UndefinedBehaviorSanitizer any undefined arithmetic (shifts, overflow,
// misaligned loads) in the index code the GPU kernels share.  The numbers are
// not checked here (the emulator tests do that); a clean exit is the result.
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
#define EMU_ARGS int dim, const int *m, const double *h, int64_t N, double alpha, const double *p, const double *q
void emu_space_f64(EMU_ARGS, const double* x, double* y);
void emu_space_f32(EMU_ARGS, const float* x, float* y);
double emu_sine_io(EMU_ARGS, const double* x, double* y, int dir);
void emu_time_f64(EMU_ARGS, double* x);
void emu_time_f32(EMU_ARGS, float* x);
void emu_precond_f64(EMU_ARGS, const double* x, double* y);
void emu_precond_f32(EMU_ARGS, const float* x, float* y);
double emu_sym_f64(EMU_ARGS, const double* x, double* y, int force_fft);
double emu_sym_f32(EMU_ARGS, const float* x, float* y, int force_fft);
double emu_time_upd_f64(EMU_ARGS, const double* Q, const double* V1, const double* V2, double* Vout, double* Zout,
                        const double* coef, int full);
double emu_time_upd_f32(EMU_ARGS, const float* Q, const float* V1, const float* V2, float* Vout, float* Zout,
                        const double* coef, int full);
double emu_time_upd_mixed(EMU_ARGS, const double* Q, float* Vout, float* Zout, const double* coef, int qrev);
double emu_sym_spec_f64(EMU_ARGS, const double* z, double* out, int form);
double emu_sym_spec_f32(EMU_ARGS, const float* z, float* out, int form);
double emu_resid_spec_f64(EMU_ARGS, const double* u, const double* f, double* r, int form);
double emu_resid_upd_f64(EMU_ARGS, double* u, const double* f, double* r, const float* zs, int k, const double* y,
                         double s, int u_zero, int two_n);
void emu_wx_f64(const double* Z, double* Wa, const double* Wb, double* X, int64_t n, const double* coef);
void emu_wx_f32(const float* Z, float* Wa, const float* Wb, float* X, int64_t n, const double* coef);
void emu_combine_f32(double* u, const float* zs, int k, const double* y, double s, int64_t n);
void emu_transpose_f64(const double* in, double* out, int64_t R, int64_t C, int rev);
int emu_error(void);
}

namespace {

struct Case {
  int dim;
  int m[3];
  int64_t N;
  bool dense;  // dense p (fractional-like) or two taps (heat-like)
};

double value(int64_t i) { return std::sin(0.37 * (double)i + 0.11) + 0.25 * std::cos(1.3 * (double)i); }

template <typename T>
std::vector<T> filled(int64_t n, int64_t seed) {
  std::vector<T> v((size_t)n);
  for (int64_t i = 0; i < n; ++i) v[(size_t)i] = (T)value(i + 7919 * seed);
  return v;
}

int run(const Case& c) {
  int64_t M = 1;
  double h[3];
  for (int d = 0; d < 3; ++d) {
    h[d] = 1.0 / (c.m[d] + 1);
    if (d < c.dim) M *= c.m[d];
  }
  const int64_t N = c.N, n = N * M;
  std::vector<double> p((size_t)N, 0.0), q((size_t)N, 0.0);
  p[0] = 2.0 * N;
  if (c.dense) {
    for (int64_t k = 1; k < N; ++k) p[(size_t)k] = -1.5 * N / (double)((k + 1) * (k + 1));
  } else if (N > 1) {
    p[1] = -1.0 * N;
  }
  q[0] = 1.0;
  if (N > 1 && !c.dense) q[1] = 0.5;
  const double alpha = 0.05;
#define A c.dim, c.m, h, N, alpha, p.data(), q.data()
  std::vector<double> x = filled<double>(n, 1), y((size_t)n), z = filled<double>(n, 2), w = filled<double>(n, 3);
  std::vector<float> xf = filled<float>(n, 4), yf((size_t)n), zf = filled<float>(n, 5), wf = filled<float>(n, 6);
  std::vector<double> vout((size_t)n), zout((size_t)n);
  std::vector<float> voutf((size_t)n), zoutf((size_t)n);
  const double coef[4] = {0.7, -0.2, 0.1, 0.0};
  emu_space_f64(A, x.data(), y.data());
  emu_space_f32(A, xf.data(), yf.data());
  emu_sine_io(A, x.data(), y.data(), 0);
  emu_sine_io(A, y.data(), x.data(), 1);
  emu_time_f64(A, y.data());
  emu_time_f32(A, yf.data());
  emu_precond_f64(A, x.data(), y.data());
  emu_precond_f32(A, xf.data(), yf.data());
  for (int fft = 0; fft < 2; ++fft) {
    emu_sym_f64(A, x.data(), y.data(), fft);
    emu_sym_f32(A, xf.data(), yf.data(), fft);
  }
  for (int full = 0; full < 3; ++full) {
    emu_time_upd_f64(A, x.data(), z.data(), w.data(), vout.data(), zout.data(), coef, full);
    emu_time_upd_f32(A, xf.data(), zf.data(), wf.data(), voutf.data(), zoutf.data(), coef, full);
  }
  emu_time_upd_mixed(A, x.data(), voutf.data(), zoutf.data(), coef, 0);
  emu_time_upd_mixed(A, x.data(), voutf.data(), zoutf.data(), coef, 1);
  for (int form = c.dense ? 1 : 0; form < 3; ++form) {
    emu_sym_spec_f64(A, x.data(), y.data(), form);
    emu_sym_spec_f32(A, xf.data(), yf.data(), form);
    emu_resid_spec_f64(A, x.data(), z.data(), y.data(), form);
  }
  {
    const int k = 3;
    std::vector<float> zs = filled<float>(k * n, 8);
    const double yk[3] = {0.5, -0.25, 0.125};
    std::vector<double> u = x;
    emu_resid_upd_f64(A, u.data(), z.data(), y.data(), zs.data(), k, yk, 1.5, 0, 0);
    emu_resid_upd_f64(A, u.data(), z.data(), y.data(), zs.data(), k, yk, 1.5, 1, 1);
    emu_combine_f32(u.data(), zs.data(), k, yk, 0.5, n);
  }
  {
    std::vector<double> wa = filled<double>(n, 9), xx = filled<double>(n, 10);
    std::vector<float> waf = filled<float>(n, 11), xxf = filled<float>(n, 12);
    emu_wx_f64(z.data(), wa.data(), w.data(), xx.data(), n, coef);
    emu_wx_f32(zf.data(), waf.data(), wf.data(), xxf.data(), n, coef);
  }
  emu_transpose_f64(x.data(), y.data(), N, M, 0);
  emu_transpose_f64(y.data(), x.data(), M, N, 1);
#undef A
  return emu_error();
}

}  // namespace

int main() {
  // line lengths up to 64 (the build's EMU_MAX_L): N <= 32 (2N-point matvec)
  // and 2(m + 1) <= 64: one- and two-stage transforms, ragged mode pairs
  const Case cases[] = {
      {2, {7, 3, 1}, 32, true},   // dense p, 21 modes (a ragged pair), N = 32
      {3, {1, 3, 7}, 4, false},   // 3D, two-tap p and q, a one-point dimension
      {1, {15, 1, 1}, 2, false},  // the shortest time line
  };
  int bad = 0;
  for (const Case& c : cases) {
    const auto t0 = std::chrono::steady_clock::now();
    const int e = run(c);
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::printf("dim=%d m=(%d,%d,%d) N=%lld dense=%d: emulator error %d (%.1f s)\n", c.dim, c.m[0], c.m[1], c.m[2],
                (long long)c.N, (int)c.dense, e, s);
    bad |= e;
  }
  std::printf(bad ? "FAILED\n" : "ok\n");
  return bad ? 1 : 0;
}
