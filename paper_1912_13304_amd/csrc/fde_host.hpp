// Host-side helpers shared by the library's translation units: error
// reporting, float64 setup arithmetic (Grunwald weights, symbol samples, a
// radix-2 FFT for circulant eigenvalues) and small integer utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fde.h"

namespace fde {

inline thread_local std::string g_err;

inline fde_status fail(fde_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::fde::fail(FDE_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                            \
  } while (0)

#define TRY(expr)                   \
  do {                              \
    fde_status s_ = (expr);         \
    if (s_ != FDE_OK) return s_;    \
  } while (0)

inline int ilog2(long v) {
  int l = 0;
  while ((1L << l) < v) ++l;
  return l;
}

inline bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

// In-place radix-2 FFT, exponent sign -1, float64 (host setup only).
inline void host_fft(std::vector<std::complex<double>>& a) {
  const size_t L = a.size();
  for (size_t i = 1, j = 0; i < L; ++i) {
    size_t bit = L >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= L; len <<= 1) {
    const size_t half = len >> 1;
    std::vector<std::complex<double>> w(half);
    for (size_t k = 0; k < half; ++k) {
      const double ang = -2.0 * M_PI * (double)k / (double)len;
      w[k] = std::complex<double>(std::cos(ang), std::sin(ang));
    }
    for (size_t i = 0; i < L; i += len)
      for (size_t k = 0; k < half; ++k) {
        const std::complex<double> u = a[i + k], v = a[i + k + half] * w[k];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

// Grunwald weights g_0..g_K (eq. grunwald1) or the second-order weights w_k
// (Section 1.3), by the ratio g_k/g_{k-1} = (k - 1 - alpha)/k.
inline std::vector<double> weights(double alpha, int K, int kind) {
  std::vector<double> g(K + 2);
  g[0] = 1.0;
  for (int k = 1; k <= K + 1; ++k) g[k] = g[k - 1] * ((double)(k - 1) - alpha) / (double)k;
  if (kind == FDE_W_SHIFTED) return g;
  std::vector<double> w(K + 2);
  w[0] = 0.5 * alpha * g[0];
  for (int k = 1; k <= K + 1; ++k) w[k] = 0.5 * alpha * g[k] + 0.5 * (2.0 - alpha) * g[k - 1];
  return w;
}

// Symbol F_a(theta) = f(theta) + f(-theta) with f = g_a (first order,
// Section 2.1: g_a(t) = -e^{-it}(1 - e^{it})^a) or w_a (second order,
// w_a(t) = -((2 - a(1 - e^{-it}))/2)(1 - e^{it})^a); principal branch.
inline double symbol(double a, double t, int kind) {
  auto f = [&](double th) {
    const std::complex<double> I(0.0, 1.0);
    const std::complex<double> base = std::pow(1.0 - std::exp(I * th), a);
    if (kind == FDE_W_SHIFTED) return -std::exp(-I * th) * base;
    return -((2.0 - a * (1.0 - std::exp(-I * th))) / 2.0) * base;
  };
  return (f(t) + f(-t)).real();
}

}  // namespace fde
