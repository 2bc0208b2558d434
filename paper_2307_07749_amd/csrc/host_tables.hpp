// Host-side (FP64) construction of the tables the kernels read.
//
//  * twiddles exp(-2 pi i k / L), k < L, with exact angle reduction;
//  * D_alpha = diag(alpha^{j/N}) powers used by the time pass (eq. (8));
//  * sigma_k = sum_j alpha^{j/N} p_j exp(-2 pi i j k/N) and rho_k likewise
//    from q, so that lambda_i^{(k,alpha)} = sigma_k + mu_i rho_k (eq. (9) for
//    blocks p_k I + q_k L_h, whose eigenvalues are p_k + q_k mu_i);
//  * matvec spectrum fft(p zero-padded to 2N)/(2N);
//  * mu_i, the eigenvalue of L_h for each sine mode (Remark 1):
//    sum_d 4 h_d^-2 sin^2(pi k_d / (2(m_d+1))), k_d = 1..m_d.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

namespace bltt {
namespace host {

using cd = std::complex<double>;

// exp(-2 pi i k / L) for k in [0, L), angle reduced mod L and evaluated in
// long double so every entry is within an ulp or two of the exact root.
inline cd unit_root(int64_t k, int64_t L) {
  k %= L;
  if (k < 0) k += L;
  const long double two_pi = 6.283185307179586476925286766559L;
  const long double a = two_pi * (long double)k / (long double)L;
  return cd((double)std::cos(a), -(double)std::sin(a));
}

inline std::vector<cd> twiddles(int L) {
  std::vector<cd> t((size_t)L);
  for (int k = 0; k < L; ++k) t[(size_t)k] = unit_root(k, L);
  // clean exact values
  for (int k = 0; k < L; ++k) {
    if ((4 * k) % L == 0) {
      const int q = (4 * k) / L;
      t[(size_t)k] = q == 0 ? cd(1, 0) : q == 1 ? cd(0, -1) : q == 2 ? cd(-1, 0) : cd(0, 1);
    }
  }
  return t;
}

// sum_j c_j w_j exp(-2 pi i j k / N), k < N  (direct DFT, exact twiddle table)
inline std::vector<cd> dft(const std::vector<cd>& c) {
  const int64_t N = (int64_t)c.size();
  std::vector<cd> tw((size_t)N);
  for (int64_t k = 0; k < N; ++k) tw[(size_t)k] = unit_root(k, N);
  std::vector<cd> out((size_t)N);
  for (int64_t k = 0; k < N; ++k) {
    cd acc(0, 0);
    for (int64_t j = 0; j < N; ++j) acc += c[(size_t)j] * tw[(size_t)((j * k) % N)];
    out[(size_t)k] = acc;
  }
  return out;
}

inline std::vector<double> alpha_pow(int64_t N, double alpha, double expo) {
  std::vector<double> d((size_t)N);
  const double la = std::log(alpha);
  for (int64_t n = 0; n < N; ++n) d[(size_t)n] = std::exp(expo * la * (double)n / (double)N);
  return d;
}

inline std::vector<cd> alpha_spectrum(const std::vector<double>& c, double alpha) {
  const int64_t N = (int64_t)c.size();
  const std::vector<double> d = alpha_pow(N, alpha, 1.0);
  std::vector<cd> s((size_t)N);
  for (int64_t j = 0; j < N; ++j) s[(size_t)j] = cd(c[(size_t)j] * d[(size_t)j], 0.0);
  return dft(s);
}

// fft of p zero-padded to length 2N, divided by 2N (the unnormalised inverse
// FFT of the kernels then returns the causal convolution directly)
inline std::vector<cd> matvec_spectrum(const std::vector<double>& p) {
  const int64_t N = (int64_t)p.size();
  std::vector<cd> s((size_t)(2 * N), cd(0, 0));
  for (int64_t j = 0; j < N; ++j) s[(size_t)j] = cd(p[(size_t)j], 0.0);
  std::vector<cd> out = dft(s);
  for (auto& v : out) v /= (double)(2 * N);
  return out;
}

// Causal Toeplitz product as circulant + skew-circulant (both N x N, first
// column p): T = (C + S)/2 with C = F^{-1} diag(fft(p)) F and
// S = D^{-1} F^{-1} diag(fft(D p)) F D, D = diag(e^{i pi n/N}).  Returns
// fft(p)/(2N) and fft(D p)/(2N) (the kernels' inverse FFT is unnormalised).
inline std::vector<cd> circulant_spectrum(const std::vector<double>& p, bool skew) {
  const int64_t N = (int64_t)p.size();
  std::vector<cd> s((size_t)N);
  for (int64_t j = 0; j < N; ++j)
    s[(size_t)j] = skew ? std::conj(unit_root(j, 2 * N)) * p[(size_t)j] : cd(p[(size_t)j], 0.0);
  std::vector<cd> out = dft(s);
  for (auto& v : out) v /= (double)(2 * N);
  return out;
}

// e^{i pi n / N}, n < N
inline std::vector<cd> half_roots(int64_t N) {
  std::vector<cd> r((size_t)N);
  for (int64_t n = 0; n < N; ++n) r[(size_t)n] = std::conj(unit_root(n, 2 * N));
  return r;
}

inline std::vector<double> lap_eigs_1d(int m, double h) {
  std::vector<double> mu((size_t)m);
  const long double pi = 3.141592653589793238462643383279L;
  for (int k = 1; k <= m; ++k) {
    const long double s = std::sin(pi * (long double)k / (2.0L * (long double)(m + 1)));
    mu[(size_t)(k - 1)] = (double)(4.0L / ((long double)h * (long double)h) * s * s);
  }
  return mu;
}

inline std::vector<double> lap_eigs(int dim, const int* m, const double* h) {
  int64_t M = 1;
  for (int d = 0; d < dim; ++d) M *= m[d];
  std::vector<double> mu((size_t)M, 0.0);
  int64_t stride = 1;
  for (int d = 0; d < dim; ++d) {
    const std::vector<double> e = lap_eigs_1d(m[d], h[d]);
    for (int64_t i = 0; i < M; ++i) mu[(size_t)i] += e[(size_t)((i / stride) % m[d])];
    stride *= m[d];
  }
  return mu;
}

// Assumption 1(ii) margin min_i (l_i^(0) - sum_{k>=1} |l_i^(k)|), l_i^(k) = p_k + q_k mu_i.
// The function of mu is concave, so its minimum over [mu_min, mu_max] is at an end.
inline double assumption_margin(const std::vector<double>& p, const std::vector<double>& q, double mu_min,
                                double mu_max) {
  auto c0 = [&](double mu) {
    double v = p[0] + q[0] * mu;
    for (size_t k = 1; k < p.size(); ++k) v -= std::fabs(p[k] + q[k] * mu);
    return v;
  };
  return std::min(c0(mu_min), c0(mu_max));
}

}  // namespace host
}  // namespace bltt
