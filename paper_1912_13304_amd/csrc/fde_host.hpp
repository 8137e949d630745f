// Host-side helpers shared by the library's translation units: error
// reporting, float64 setup arithmetic (Grunwald weights, symbol samples, a
// radix-2 FFT for circulant eigenvalues) and small integer utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <utility>
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

// Device memory cache.  A plan's buffers go back to a per-device list keyed
// by their exact size when the plan is destroyed (after the device has been
// synchronised), and the next plan of the same shape takes them instead of
// calling hipMalloc; hipMalloc and hipFree each cost about a millisecond at
// these sizes, which a time-stepping job that builds one plan per run would
// pay every run.  At most CACHE_MAX bytes are held; fde_release_cache frees
// them.  Blocks are handed out uninitialised, as hipMalloc's are.
struct MemCache {
  static constexpr size_t CACHE_MAX = size_t(16) << 30;
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> blocks;
  size_t held = 0;
};

inline MemCache& memcache() {
  static MemCache* c = new MemCache();   // never destroyed: no hipFree after the runtime is gone
  return *c;
}

inline hipError_t cache_malloc(void** p, size_t bytes, int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  *dev_out = dev;
  {
    MemCache& c = memcache();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.blocks.find({dev, bytes});
    if (it != c.blocks.end() && !it->second.empty()) {
      *p = it->second.back();
      it->second.pop_back();
      c.held -= bytes;
      return hipSuccess;
    }
  }
  return hipMalloc(p, bytes);
}

// The device that owns p must have no pending work on it.
inline void cache_free(void* p, size_t bytes, int dev) {
  MemCache& c = memcache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    if (c.held + bytes <= MemCache::CACHE_MAX) {
      c.blocks[{dev, bytes}].push_back(p);
      c.held += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

inline void cache_release() {
  MemCache& c = memcache();
  std::lock_guard<std::mutex> g(c.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : c.blocks) {
    (void)hipSetDevice(kv.first.first);
    for (void* q : kv.second) (void)hipFree(q);
  }
  (void)hipSetDevice(cur);
  c.blocks.clear();
  c.held = 0;
}

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

// Partitioned factorisation of a tridiagonal matrix (sub[i] = A[i][i-1],
// diag[i], sup[i] = A[i][i+1]) for the P_tri solve: rows split into p chunks
// [cs[k], cs[k+1]) of at least two rows; the last row r of chunk k is the
// interface unknown X_k, rows cs[k]..r-1 its interior.  Per row: the interior
// Thomas pivots (ai = sub with the chunk's first entry zeroed, cp, den) and
// the interior responses sv, sw to the couplings sub[cs[k]] X_{k-1} and
// sup[r-1] X_k; per chunk: ar = sub[r], cr = sup[r] (0 for the last chunk) and
// the tridiagonal system (ra, rb, rc) in the X_k left after the interiors are
// eliminated.  A strictly diagonally dominant A needs no pivoting.
struct TriFactors {
  long n = 0;
  int p = 0;
  std::vector<int> cs;
  std::vector<double> ai, cp, den, sv, sw;
  std::vector<double> ar, cr, ra, rb, rc;
};

inline TriFactors tri_factor(const std::vector<double>& sub, const std::vector<double>& diag,
                             const std::vector<double>& sup, int pmax) {
  TriFactors F;
  const long n = (long)diag.size();
  F.n = n;
  F.p = (int)std::max(1L, std::min((long)pmax, n / 2));
  const int p = F.p;
  F.cs.resize(p + 1);
  for (int k = 0; k <= p; ++k) F.cs[k] = (int)(((long)k * n) / p);
  F.ai.assign(n, 0.0);
  F.cp.assign(n, 0.0);
  F.den.assign(n, 0.0);
  F.sv.assign(n, 0.0);
  F.sw.assign(n, 0.0);
  auto thomas = [&](long s, long r, std::vector<double>& x) {   // x: rhs of rows s..r-1, in place
    double d = 0.0;
    for (long i = s; i < r; ++i) {
      d = (x[i - s] - F.ai[i] * d) * F.den[i];
      x[i - s] = d;
    }
    double yn = 0.0;
    for (long i = r - 1; i >= s; --i) {
      yn = x[i - s] - F.cp[i] * yn;
      x[i - s] = yn;
    }
  };
  for (int k = 0; k < p; ++k) {
    const long s = F.cs[k], r = F.cs[k + 1] - 1;
    double prev = 0.0;
    for (long i = s; i < r; ++i) {
      const double a = i == s ? 0.0 : sub[i];
      const double c = i == r - 1 ? 0.0 : sup[i];
      const double dd = 1.0 / (diag[i] - a * prev);
      F.ai[i] = a;
      F.den[i] = dd;
      F.cp[i] = c * dd;
      prev = F.cp[i];
    }
    const long q = r - s;
    if (q >= 1) {
      std::vector<double> e(q, 0.0);
      e[0] = sub[s];
      thomas(s, r, e);
      for (long i = 0; i < q; ++i) F.sv[s + i] = e[i];
      std::fill(e.begin(), e.end(), 0.0);
      e[q - 1] = sup[r - 1];
      thomas(s, r, e);
      for (long i = 0; i < q; ++i) F.sw[s + i] = e[i];
    }
  }
  F.ar.assign(p, 0.0);
  F.cr.assign(p, 0.0);
  F.ra.assign(p, 0.0);
  F.rb.assign(p, 0.0);
  F.rc.assign(p, 0.0);
  for (int k = 0; k < p; ++k) {
    const long s = F.cs[k], r = F.cs[k + 1] - 1, q = r - s;
    F.ar[k] = sub[r];
    F.cr[k] = k + 1 < p ? sup[r] : 0.0;
    const double aL = q >= 1 ? F.sv[r - 1] : -1.0, bL = q >= 1 ? F.sw[r - 1] : 0.0;
    double aR = 0.0, bR = 0.0;
    if (k + 1 < p) {
      const long s2 = F.cs[k + 1], q2 = F.cs[k + 2] - 1 - s2;
      aR = q2 >= 1 ? F.sv[s2] : 0.0;
      bR = q2 >= 1 ? F.sw[s2] : -1.0;
    }
    F.ra[k] = -F.ar[k] * aL;
    F.rb[k] = diag[r] - F.ar[k] * bL - F.cr[k] * aR;
    F.rc[k] = -F.cr[k] * bR;
  }
  return F;
}

// Tridiagonal part of the 1D M = nu I + D+ T + D- T^T (T = -[g_{i-j+1}]):
// M[i][i] = nu - (d+_i + d-_i) g_1, M[i][i-1] = -d+_i g_2 - d-_i g_0,
// M[i][i+1] = -d+_i g_0 - d-_i g_2 (P_tri of Table 2).
inline void tri_part(const std::vector<double>& g, double nu, const double* dp, const double* dm, long n,
                     std::vector<double>& sub, std::vector<double>& diag, std::vector<double>& sup) {
  sub.assign(n, 0.0);
  diag.assign(n, 0.0);
  sup.assign(n, 0.0);
  for (long i = 0; i < n; ++i) {
    diag[i] = nu - (dp[i] + dm[i]) * g[1];
    if (i > 0) sub[i] = -dp[i] * g[2] - dm[i] * g[0];
    if (i + 1 < n) sup[i] = -dp[i] * g[0] - dm[i] * g[2];
  }
}

}  // namespace fde
