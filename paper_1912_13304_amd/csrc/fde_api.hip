// C ABI of libfde (include/fde.h): plan assembly, the operator and
// preconditioner entry points and the Krylov drivers.
//
// Host work is limited to O(n) float64 setup (Grunwald weights, circulant
// eigenvalues of T by a host FFT, twiddles, symbol samples) and to enqueueing
// kernels.  The Krylov state lives on the device (fde_krylov.hpp); the host
// reads it back once per GMRES cycle, and polls a mapped host flag written by
// the device one step behind the launch front so that it stops enqueueing
// after convergence without stalling the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fde.h"
#include "fde_bigline.hpp"
#include "fde_dense.hpp"
#include "fde_fgmres1.hpp"
#include "fde_host.hpp"
#include "fde_krylov.hpp"
#include "fde_lines.hpp"
#include "fde_pcg.hpp"
#include "fde_tri.hpp"

using namespace fde;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
extern "C" const char* fde_last_error(void) { return fde::g_err.c_str(); }

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
constexpr int DENSE_NMAX = 1023;      // largest n per direction of the dense 2D form
constexpr int CHIRP_NMAX = 1 << 21;   // largest 1D n whose n + 1 need not be a power of two
constexpr int FOURSTEP_MIN = 4096;    // smallest four-step FFT length (both factors >= 64)

// FFT lengths of a 1D line on the four-step path: the Toeplitz embedding's
// (a power of two >= n + 1, = n + 1 when that is one) and, for the chirp-z
// DST, the convolution's (a power of two >= 2n - 1); both at least FOURSTEP_MIN.
static long toep_len(long n) { return std::max<long>(FOURSTEP_MIN, 1L << ilog2(n + 1)); }
static long chirp_len(long n) { return std::max<long>(FOURSTEP_MIN, 1L << ilog2(std::max(2 * n - 1, 1L))); }

struct Dir {
  int n = 0, P = 0, logP = 0, nlines = 0, B = 1, logB = 0;
  long ls = 0, es = 0;
  bool cols = false;   // lines are columns of a row-major array (line_kernel<.., COLS = true, ..>)
};

template <typename T>
struct Consts {
  cx<T> *W2p1 = nullptr, *W2p2 = nullptr;                        // four-step factor twiddles (big lines)
  cx<T>* cw = nullptr;                                           // big-line complex work, 6 max(P, Q)
  // chirp-z DST of a 1D line whose n + 1 is not a power of two: four-step
  // factor twiddles and exp(-i pi m/Q) of the length-Q FFTs, chirp c_j
  // (j <= n) and the chirp filter's spectrum (Q entries)
  cx<T> *Ws1 = nullptr, *Ws2 = nullptr, *Wsb = nullptr, *chirp = nullptr, *bhat = nullptr;
  T *dp = nullptr, *dm = nullptr, *ep = nullptr, *em = nullptr;  // coefficients
  T *ept = nullptr, *emt = nullptr;                              // e+- transposed (n1 x n2)
  T* dinv = nullptr;                                             // D^{-1} (null: no D factor)
  T *fx = nullptr, *fy = nullptr, *fzero = nullptr;              // symbol samples
  cx<T> *W2x = nullptr, *W2y = nullptr, *lamx = nullptr, *lamy = nullptr;
  T *stabx = nullptr, *staby = nullptr, *gx = nullptr, *gy = nullptr;  // dense 2D: sine tables, weights
};

struct fde_plan_s {
  fde_params p;
  int dim = 1, n1 = 0, n2 = 1;
  long N = 0;
  long ld = 0;   // leading dimension of the Krylov bases: N rounded up to 64 (aligned slots)
  double hx = 0, hy = 0, hxa = 0, nu = 0, kappa = 0, shift = 0;
  bool has_dinv = false;
  int dside = FDE_D_LEFT;
  TriDev<double> tri64;   // P_tri factors and work (FDE_P_TRI)
  TriDev<float> tri32;
  Dir rows, trows;   // lines along x (rows of the (n2, n1) array); along y (rows of its transpose)
  Dir ycols;         // lines along y read in place (columns of the (n2, n1) array)
  bool use_cols = false;   // y-direction passes on ycols (no transposes)
  bool big = false;  // 1D line longer than one workgroup: four-step FFT over kernels
  bool dense = false;  // 2D: line operators as dense MFMA products (fde_dense.hpp)
  int P1 = 0, P2 = 0, log1 = 0, log2 = 0;   // four-step factors of the Toeplitz FFT length rows.P
  bool blue = false;  // 1D, n + 1 not a power of two: rows.P >= n + 1 pads the Toeplitz embedding and
                      // the DST takes the chirp-z form with FFTs of length sQ
  long sQ = 0;
  int sQ1 = 0, sQ2 = 0, slog1 = 0, slog2 = 0;
  Consts<double> c64;
  Consts<float> c32;
  int m = 30, kin = 0;
  double *V = nullptr, *Z = nullptr, *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
  float *Vf = nullptr, *t1f = nullptr, *t2f = nullptr, *t3f = nullptr, *uf = nullptr, *zf = nullptr;
  template <typename T> T* tmp(int i);
  double* part = nullptr;
  // Gram-Schmidt partials left for the next update pass to sum (no finalize
  // launch in between; grids of at most HANDOFF_MAXG workgroups), or null
  const double* pend_part = nullptr;
  int pend_G = 0;
  // Toeplitz extraction of a long 1D line left to the first Gram-Schmidt
  // pass (CG_XDOT): set by big_toep while defer_x is on (the outer step's
  // operator, whose result w that pass reads next)
  bool defer_x = false, xpend = false;
  XArgs xpa;
  double* xout = nullptr;
  double* stats_buf = nullptr;   // 3 + 3*256 doubles for the setup statistics
  KState *ks = nullptr, *ksi = nullptr;
  double* hstat = nullptr;      // mapped pinned host memory
  double* hstat_dev = nullptr;  // its device address
  KState* hks = nullptr;        // pinned host copy of the state header
  hipEvent_t ev[4] = {};
  // timing probe
  int probe = FDE_PROBE_OFF;
  long long pseen = 0;              // launches of the probed class since fde_probe
  static constexpr int PSTRIDE = 32; // every PSTRIDE-th launch is bracketed
  std::vector<hipEvent_t> pev;      // event pool, pairs (start, stop)
  size_t pused = 0;                 // pairs recorded since the last read
  double pbytes = 0.0;
  struct Alloc {
    void* p;
    size_t bytes;
    int dev;
  };
  std::vector<Alloc> allocs;   // device buffers, returned to the memory cache on destroy
  size_t bytes = 0;
};

template <> double* fde_plan_s::tmp<double>(int i) { return i == 1 ? t1 : i == 2 ? t2 : t3; }
template <> float* fde_plan_s::tmp<float>(int i) { return i == 1 ? t1f : i == 2 ? t2f : t3f; }

// Lines per workgroup for a transform of size P: B*P/8 threads per
// workgroup.  One line per workgroup (at least one wavefront) lets several
// workgroups share a CU, so that the load, transform and store phases of
// different lines overlap.
static void choose_tile(Dir& d) {
  const int B = d.cols ? cols_per_tile(d.P) : rows_per_tile(d.P);
  d.B = B;
  d.logB = ilog2(B);
}

void fde_default_params_impl(fde_params* p) {
  std::memset(p, 0, sizeof *p);
  p->dim = 1;
  p->n[0] = 1023;
  p->n[1] = 1;
  p->alpha[0] = 1.5;
  p->alpha[1] = 1.5;
  p->lo[0] = p->lo[1] = 0.0;
  p->hi[0] = p->hi[1] = 2.0;
  p->dt = 2.0 / 1024.0;
  p->weights = FDE_W_SHIFTED;
  p->time = FDE_T_EULER;
  p->prec = FDE_P_TAU;
  p->dside = FDE_D_LEFT;
  p->shift = NAN;
  p->solver = FDE_S_GMRES;
  p->restart = 30;
  p->maxit = 10000;
  p->tol = 1e-8;
  p->precision = FDE_FP64;
  p->inner_steps = 16;
}

extern "C" void fde_default_params(fde_params* p) {
  if (p) fde_default_params_impl(p);
}

static fde_status validate(const fde_params* p) {
  if (!p) return fail(FDE_EINVAL, "params is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(FDE_EINVAL, "dim must be 1 or 2 (got %d)", p->dim);
  for (int i = 0; i < p->dim; ++i) {
    if (p->n[i] < 1) return fail(FDE_EINVAL, "n[%d] must be >= 1 (got %d)", i, p->n[i]);
    if (!(p->alpha[i] > 1.0 && p->alpha[i] < 2.0))
      return fail(FDE_EINVAL, "alpha[%d] must lie in (1,2) (got %g)", i, p->alpha[i]);
    if (!(p->hi[i] > p->lo[i]) || !std::isfinite(p->hi[i]) || !std::isfinite(p->lo[i]))
      return fail(FDE_EINVAL, "domain [%g, %g] is empty", p->lo[i], p->hi[i]);
    const long lim = p->dim == 1 ? (1L << 22) : 4096;
    const bool dense_ok = p->dim == 2 && p->n[0] <= DENSE_NMAX && p->n[1] <= DENSE_NMAX;
    const bool chirp_ok = p->dim == 1 && p->n[0] <= CHIRP_NMAX;
    if ((!is_pow2((long)p->n[i] + 1) && !dense_ok && !chirp_ok) || p->n[i] + 1 > lim)
      return fail(FDE_EUNSUPPORTED,
                  "n[%d] + 1 = %d must be a power of two <= %ld (1D lines with n <= %d and 2D grids with both "
                  "n <= %d take any n)", i, p->n[i] + 1, lim, CHIRP_NMAX, DENSE_NMAX);
  }
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(FDE_EINVAL, "dt must be > 0 (got %g)", p->dt);
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(FDE_EINVAL, "tol must be > 0 (got %g)", p->tol);
  if (p->weights != FDE_W_SHIFTED && p->weights != FDE_W_WEIGHTED) return fail(FDE_EINVAL, "bad weights");
  if (p->time != FDE_T_EULER && p->time != FDE_T_CN) return fail(FDE_EINVAL, "bad time scheme");
  if (p->prec < FDE_P_NONE || p->prec > FDE_P_TRI) return fail(FDE_EINVAL, "bad preconditioner");
  if (p->prec == FDE_P_TILDE && p->dim != 1) return fail(FDE_EINVAL, "P_tilde is defined in 1D only");
  if (p->prec == FDE_P_TRI && p->dim != 1) return fail(FDE_EINVAL, "P_tri is defined in 1D only");
  if (p->dside != FDE_D_LEFT && p->dside != FDE_D_RIGHT) return fail(FDE_EINVAL, "bad dside");
  if (p->solver != FDE_S_GMRES && p->solver != FDE_S_PCG) return fail(FDE_EINVAL, "bad solver");
  if (p->restart < 1 || p->restart > 32) return fail(FDE_EINVAL, "restart must be in 1..32");
  if (p->maxit < 1) return fail(FDE_EINVAL, "maxit must be >= 1");
  if (p->precision != FDE_FP64 && p->precision != FDE_MIXED) return fail(FDE_EINVAL, "bad precision");
  if (p->precision == FDE_MIXED && (p->inner_steps < 0 || p->inner_steps > 32))
    return fail(FDE_EINVAL, "inner_steps must be in 0..32");
  if (p->precision == FDE_MIXED && p->solver != FDE_S_GMRES)
    return fail(FDE_EINVAL, "the mixed form wraps an FGMRES outer loop");
  if (!std::isnan(p->shift) && !std::isfinite(p->shift)) return fail(FDE_EINVAL, "shift must be finite or NaN");
  return FDE_OK;
}

// 2D plans whose n_1 + 1 or n_2 + 1 is not a power of two run their line
// operators as dense products (both n <= DENSE_NMAX); FDE_DENSE_LINES=1 in
// the environment selects that form for every 2D plan within the limit (to
// compare the two forms).
static bool use_dense(const fde_params* p) {
  if (p->dim != 2 || p->n[0] > DENSE_NMAX || p->n[1] > DENSE_NMAX) return false;
  if (!is_pow2((long)p->n[0] + 1) || !is_pow2((long)p->n[1] + 1)) return true;
  const char* e = std::getenv("FDE_DENSE_LINES");
  return e && e[0] == '1';
}

// Device bytes of a plan (buffers only; the kernels need no other memory).
static size_t plan_bytes_impl(const fde_params* p) {
  const long n1 = p->n[0], n2 = p->dim == 2 ? p->n[1] : 1;
  const long N = n1 * n2;
  const long m = p->restart;
  size_t b = 0;
  const int ncoef = p->dim == 2 ? 4 : 2;
  b += (size_t)N * (ncoef + 1) * (8 + 4);       // coefficients and D^{-1}, both precisions
  if (p->dim == 2 && n2 + 1 > 2048) b += (size_t)N * 2 * (8 + 4);   // e+- transposed (y passes on the transpose)
  b += (size_t)(n1 + n2 + 1) * (8 + 4);         // symbol samples
  b += (size_t)4 * (2 * (n1 + 1) + 2 * (n2 + 1)) * (16 + 8);  // twiddles and eigenvalues
  if (p->solver == FDE_S_PCG) b += (size_t)N * 8 * 6;
  else b += (size_t)((N + 63) / 64 * 64) * 8 * (2 * m + 1) + (size_t)N * 8 * 3;
  if (p->precision == FDE_MIXED) b += (size_t)((N + 63) / 64 * 64) * 4 * (p->inner_steps + 1) + (size_t)N * 4 * 6;
  b += (size_t)RED_MAXG * (KMAX + 1) * 8 + 2 * sizeof(KState);
  if (p->dim == 1 && !is_pow2(n1 + 1)) {
    const size_t L = (size_t)std::max(toep_len(n1), chirp_len(n1));
    b += L * (6 * 16 + (p->precision == FDE_MIXED ? 6 * 8 : 0) + 8 * 24) + (size_t)(n1 + 1 + chirp_len(n1)) * 24;
  } else if (p->dim == 1 && n1 + 1 > 4096) {
    b += (size_t)(n1 + 1) * (6 * 16 + (p->precision == FDE_MIXED ? 6 * 8 : 0) + 8 * 24);
  }
  if (p->prec == FDE_P_TRI) b += (size_t)N * 6 * (8 + 4) + (size_t)TRI_PMAX * (7 * (8 + 4) + 4) + 4;
  return b;
}

extern "C" size_t fde_plan_bytes(const fde_params* p) {
  if (validate(p) != FDE_OK) return 0;
  return plan_bytes_impl(p);
}

template <typename T>
static fde_status dalloc(fde_plan pl, T** ptr, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  int dev = 0;
  hipError_t e = cache_malloc(&q, bytes, &dev);
  if (e != hipSuccess) return fail(FDE_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  pl->allocs.push_back({q, bytes, dev});
  pl->bytes += bytes;
  *ptr = static_cast<T*>(q);
  return FDE_OK;
}

template <typename T>
static fde_status upload(fde_plan pl, T** dst, const std::vector<double>& src) {
  TRY(dalloc(pl, dst, src.size()));
  std::vector<T> tmp(src.begin(), src.end());
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return FDE_OK;
}

template <typename T>
static fde_status upload_cx(fde_plan pl, cx<T>** dst, const std::vector<std::complex<double>>& src) {
  TRY(dalloc(pl, dst, src.size()));
  std::vector<cx<T>> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) {
    tmp[i].x = (T)src[i].real();
    tmp[i].y = (T)src[i].imag();
  }
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(cx<T>), hipMemcpyHostToDevice));
  return FDE_OK;
}

// Twiddles W2[m] = exp(-i pi m/P), m < 2P, and circulant eigenvalues of the
// 2P x 2P circulant whose leading n x n block is T (or S): first column
// (-g_1, ..., -g_n, 0, ..., 0, -g_0).
static void direction_host(double alpha, int n, int kind, std::vector<std::complex<double>>& W2,
                           std::vector<std::complex<double>>& lam, long Pt = 0) {
  const long P = Pt ? Pt : n + 1;   // FFT length; the circulant of length 2P embeds T when P >= n + 1
  W2.assign(2 * P, 0.0);
  lam.assign(2 * P, 0.0);
  for (int m = 0; m < 2 * P; ++m) {
    // angle pi m/P, reduced by symmetry to keep the argument small
    const double t = (double)m / (double)P;  // exact
    W2[m] = std::complex<double>(std::cos(M_PI * t), -std::sin(M_PI * t));
  }
  // exact values at multiples of pi/2
  for (long m = 0; m < 2 * P; m += std::max(1L, P / 2)) {
    const int q = (int)((2L * m) / P) & 3;
    if ((2L * m) % P == 0) W2[m] = q == 0 ? 1.0 : q == 1 ? std::complex<double>(0, -1) : q == 2 ? -1.0 : std::complex<double>(0, 1);
  }
  std::vector<double> g = weights(alpha, n, kind);
  for (int k = 0; k < n; ++k) lam[k] = -g[k + 1];
  lam[2 * P - 1] = -g[0];
  host_fft(lam);
  lam.resize(P + 1);
}

static fde_status direction_tables(fde_plan pl, double alpha, int n, cx<double>** W2d, cx<float>** W2f,
                                   cx<double>** lamd, cx<float>** lamf, long Pt = 0) {
  std::vector<std::complex<double>> W2, lam;
  direction_host(alpha, n, pl->p.weights, W2, lam, Pt);
  TRY(upload_cx(pl, W2d, W2));
  TRY(upload_cx(pl, W2f, W2));
  TRY(upload_cx(pl, lamd, lam));
  TRY(upload_cx(pl, lamf, lam));
  return FDE_OK;
}

static void destroy_impl(fde_plan pl) {
  if (!pl) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  const int dev = pl->allocs.empty() ? cur : pl->allocs[0].dev;
  if (dev != cur) (void)hipSetDevice(dev);
  (void)hipDeviceSynchronize();   // no pending work may touch buffers handed to the cache
  for (auto& e : pl->pev) (void)hipEventDestroy(e);
  for (const auto& a : pl->allocs) cache_free(a.p, a.bytes, a.dev);   // the device is synchronised above
  if (pl->hstat) (void)hipHostFree(pl->hstat);
  if (pl->hks) (void)hipHostFree(pl->hks);
  for (auto& e : pl->ev)
    if (e) (void)hipEventDestroy(e);
  if (dev != cur) (void)hipSetDevice(cur);
  delete pl;
}

extern "C" void fde_destroy(fde_plan pl) { destroy_impl(pl); }

extern "C" void fde_release_cache(void) {
  (void)hipDeviceSynchronize();
  cache_release();
}

static fde_status coef_stats(fde_plan pl, const double* a, double* st3, hipStream_t st) {
  double* d = pl->stats_buf;
  const int G = 256;
  hipLaunchKernelGGL(stats_part_kernel, dim3(G), dim3(RED_THREADS), 0, st, a, pl->N, d + 3);
  hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(64), 0, st, d + 3, G, d);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(st3, d, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return FDE_OK;
}

// P_tri: tridiagonal part of M (Table 2), factored on the host in float64.
template <typename T>
static fde_status tri_upload(fde_plan pl, const TriFactors& F, const int* dcs, TriDev<T>& t) {
  t.p = F.p;
  t.cs = dcs;
  T *ai, *cp, *den, *sv, *sw, *ar, *cr, *ra, *rb, *rc;
  TRY(upload(pl, &ai, F.ai));
  TRY(upload(pl, &cp, F.cp));
  TRY(upload(pl, &den, F.den));
  TRY(upload(pl, &sv, F.sv));
  TRY(upload(pl, &sw, F.sw));
  TRY(upload(pl, &ar, F.ar));
  TRY(upload(pl, &cr, F.cr));
  TRY(upload(pl, &ra, F.ra));
  TRY(upload(pl, &rb, F.rb));
  TRY(upload(pl, &rc, F.rc));
  t.ai = ai;
  t.cp = cp;
  t.den = den;
  t.sv = sv;
  t.sw = sw;
  t.ar = ar;
  t.cr = cr;
  t.ra = ra;
  t.rb = rb;
  t.rc = rc;
  TRY(dalloc(pl, &t.y, (size_t)F.n));
  TRY(dalloc(pl, &t.part, (size_t)F.p));
  TRY(dalloc(pl, &t.X, (size_t)F.p));
  return FDE_OK;
}

static fde_status tri_setup(fde_plan pl, const double* dp, const double* dm) {
  const long n = pl->n1;
  std::vector<double> hp(n), hm(n);
  HIPCHK(hipMemcpy(hp.data(), dp, n * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(hm.data(), dm, n * sizeof(double), hipMemcpyDeviceToHost));
  const std::vector<double> g = weights(pl->p.alpha[0], (int)std::max(n, 2L), pl->p.weights);
  std::vector<double> sub, diag, sup;
  tri_part(g, pl->nu, hp.data(), hm.data(), n, sub, diag, sup);
  for (long i = 0; i < n; ++i)
    if (!(std::fabs(diag[i]) > std::fabs(sub[i]) + std::fabs(sup[i])))
      return fail(FDE_EINVAL, "P_tri: the tridiagonal part of M is not strictly diagonally dominant at row %ld", i);
  const TriFactors F = tri_factor(sub, diag, sup, TRI_PMAX);
  int* dcs = nullptr;
  TRY(dalloc(pl, &dcs, F.cs.size()));
  HIPCHK(hipMemcpy(dcs, F.cs.data(), F.cs.size() * sizeof(int), hipMemcpyHostToDevice));
  TRY(tri_upload<double>(pl, F, dcs, pl->tri64));
  TRY(tri_upload<float>(pl, F, dcs, pl->tri32));
  return FDE_OK;
}

static fde_status assemble_impl(const fde_params* p, const double* dp, const double* dm, const double* ep,
                                const double* em, hipStream_t st, fde_plan pl) {
  pl->p = *p;
  pl->dim = p->dim;
  pl->n1 = p->n[0];
  pl->n2 = p->dim == 2 ? p->n[1] : 1;
  pl->N = (long)pl->n1 * pl->n2;
  pl->ld = (pl->N + 63) / 64 * 64;
  pl->hx = (p->hi[0] - p->lo[0]) / (pl->n1 + 1);
  pl->hxa = std::pow(pl->hx, p->alpha[0]);
  pl->nu = (p->time == FDE_T_EULER ? 1.0 : 2.0) * pl->hxa / p->dt;
  if (p->dim == 2) {
    pl->hy = (p->hi[1] - p->lo[1]) / (pl->n2 + 1);
    pl->kappa = pl->hxa / std::pow(pl->hy, p->alpha[1]);
  }
  pl->dside = p->dside;
  pl->m = p->restart;
  pl->kin = p->precision == FDE_MIXED ? p->inner_steps : 0;
  const long N = pl->N;

  // geometry
  pl->rows.n = pl->n1;
  pl->rows.P = pl->n1 + 1;
  pl->rows.logP = ilog2(pl->rows.P);
  pl->rows.nlines = pl->n2;
  pl->rows.ls = pl->n1;
  pl->rows.es = 1;
  choose_tile(pl->rows);
  if (p->dim == 2) {
    pl->trows.n = pl->n2;
    pl->trows.P = pl->n2 + 1;
    pl->trows.logP = ilog2(pl->trows.P);
    pl->trows.nlines = pl->n1;
    pl->trows.ls = pl->n2;
    pl->trows.es = 1;
    choose_tile(pl->trows);
    pl->ycols = pl->trows;
    pl->ycols.ls = 1;
    pl->ycols.es = pl->n1;
    pl->ycols.cols = true;
    choose_tile(pl->ycols);
    // with one column per tile every global access would be a lone element:
    // such sizes keep the transposes
    pl->use_cols = pl->ycols.B >= 2;
    pl->dense = use_dense(p);
    if (pl->dense) pl->use_cols = true;   // no transposed coefficient copies
  }

  // coefficients: validate and copy
  TRY(dalloc(pl, &pl->stats_buf, 3 + 3 * 256));
  const double* src[4] = {dp, dm, ep, em};
  const int ncoef = p->dim == 2 ? 4 : 2;
  double stats[4][3];
  for (int i = 0; i < ncoef; ++i) {
    if (!src[i]) return fail(FDE_EINVAL, "coefficient array %d is NULL", i);
    TRY(coef_stats(pl, src[i], stats[i], st));
    if (stats[i][2] != 0.0) return fail(FDE_EINVAL, "coefficient array %d has a non-finite value", i);
    if (stats[i][0] < 0.0) return fail(FDE_EINVAL, "coefficient array %d has a negative value", i);
  }
  double* d64[4] = {nullptr, nullptr, nullptr, nullptr};
  float* d32[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < ncoef; ++i) {
    TRY(dalloc(pl, &d64[i], N));
    TRY(dalloc(pl, &d32[i], N));
    HIPCHK(hipMemcpyAsync(d64[i], src[i], N * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(256), dim3(256), 0, st, src[i], d32[i], N);
    HIPCHK(hipGetLastError());
  }
  pl->c64.dp = d64[0];
  pl->c64.dm = d64[1];
  pl->c64.ep = d64[2];
  pl->c64.em = d64[3];
  if (p->dim == 2 && !pl->use_cols) {   // e+- transposed for the y passes that run on the transpose
    TRY(dalloc(pl, &pl->c64.ept, N));
    TRY(dalloc(pl, &pl->c64.emt, N));
    TRY(dalloc(pl, &pl->c32.ept, N));
    TRY(dalloc(pl, &pl->c32.emt, N));
    const dim3 tg((pl->n1 + 31) / 32, (pl->n2 + 31) / 32);
    hipLaunchKernelGGL((transpose_kernel<double, false>), tg, dim3(256), 0, st, d64[2], pl->c64.ept, pl->n2, pl->n1,
                       (const double*)nullptr, (const int*)nullptr, (const int*)nullptr);
    hipLaunchKernelGGL((transpose_kernel<double, false>), tg, dim3(256), 0, st, d64[3], pl->c64.emt, pl->n2, pl->n1,
                       (const double*)nullptr, (const int*)nullptr, (const int*)nullptr);
    hipLaunchKernelGGL((transpose_kernel<float, false>), tg, dim3(256), 0, st, d32[2], pl->c32.ept, pl->n2, pl->n1,
                       (const float*)nullptr, (const int*)nullptr, (const int*)nullptr);
    hipLaunchKernelGGL((transpose_kernel<float, false>), tg, dim3(256), 0, st, d32[3], pl->c32.emt, pl->n2, pl->n1,
                       (const float*)nullptr, (const int*)nullptr, (const int*)nullptr);
    HIPCHK(hipGetLastError());
  }
  pl->c32.dp = d32[0];
  pl->c32.dm = d32[1];
  pl->c32.ep = d32[2];
  pl->c32.em = d32[3];

  // constancy (Section 3.1, Case I): all coefficients one constant c
  bool constant = true;
  double cval = stats[0][0];
  for (int i = 0; i < ncoef; ++i)
    if (stats[i][0] != cval || stats[i][1] != cval) constant = false;

  // D^{-1}
  pl->has_dinv = (p->prec == FDE_P_TAU);
  if (pl->has_dinv) {
    TRY(dalloc(pl, &pl->c64.dinv, N));
    TRY(dalloc(pl, &pl->c32.dinv, N));
    if (p->dim == 2)
      hipLaunchKernelGGL((dinv_kernel<true>), dim3(256), dim3(256), 0, st, d64[0], d64[1], d64[2], d64[3],
                         pl->c64.dinv, pl->c32.dinv, N);
    else
      hipLaunchKernelGGL((dinv_kernel<false>), dim3(256), dim3(256), 0, st, d64[0], d64[1], d64[2], d64[3],
                         pl->c64.dinv, pl->c32.dinv, N);
    HIPCHK(hipGetLastError());
    double ds[3];
    TRY(coef_stats(pl, pl->c64.dinv, ds, st));
    if (ds[2] != 0.0 || !(ds[0] > 0.0))
      return fail(FDE_EINVAL, "D = mean of the coefficients has a zero (d+ and d- share a zero)");
  }

  // symbol samples at theta_j = j pi/(n+1)
  const int n1 = pl->n1, n2 = pl->n2;
  std::vector<double> Fa(n1), Fb(p->dim == 2 ? n2 : 1, 0.0);
  for (int i = 0; i < n1; ++i) Fa[i] = symbol(p->alpha[0], M_PI * (i + 1) / (double)(n1 + 1), p->weights);
  if (p->dim == 2)
    for (int j = 0; j < n2; ++j) Fb[j] = symbol(p->alpha[1], M_PI * (j + 1) / (double)(n2 + 1), p->weights);
  std::vector<double> fx(n1), fy(p->dim == 2 ? n2 : 1, 0.0), fz(1, 0.0);
  double shift = 0.0;
  if (p->prec == FDE_P_TAU) {
    shift = std::isnan(p->shift) ? (constant ? pl->nu / cval : 0.0) : p->shift;
    for (int i = 0; i < n1; ++i) fx[i] = Fa[i];
    if (p->dim == 2)
      for (int j = 0; j < n2; ++j) fy[j] = pl->kappa * Fb[j] + shift;
    else
      for (int i = 0; i < n1; ++i) fx[i] += shift;
  } else if (p->prec == FDE_P_TAU_HAT) {
    // constant d+- = d, e+- = e required
    const double d = stats[0][0];
    if (!(stats[0][0] == stats[0][1] && stats[1][0] == d && stats[1][1] == d))
      return fail(FDE_EINVAL, "P_hat needs constant, equal d+ and d-");
    double e = 0.0;
    if (p->dim == 2) {
      e = stats[2][0];
      if (!(stats[2][0] == stats[2][1] && stats[3][0] == e && stats[3][1] == e))
        return fail(FDE_EINVAL, "P_hat needs constant, equal e+ and e-");
    }
    for (int i = 0; i < n1; ++i) fx[i] = d * Fa[i];
    if (p->dim == 2)
      for (int j = 0; j < n2; ++j) fy[j] = pl->kappa * e * Fb[j] + pl->nu;
    else
      for (int i = 0; i < n1; ++i) fx[i] += pl->nu;
    if (!(d > 0.0) || (p->dim == 2 && !(e > 0.0))) return fail(FDE_EINVAL, "P_hat needs positive coefficients");
  } else if (p->prec == FDE_P_TILDE) {
    std::vector<double> hp(N), hm(N);
    HIPCHK(hipMemcpy(hp.data(), dp, N * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hm.data(), dm, N * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < n1; ++i) {
      fx[i] = 0.5 * (hp[i] + hm[i]) * Fa[i];
      if (!(fx[i] > 0.0)) return fail(FDE_EINVAL, "P_tilde: D_j p(theta_j) must be positive");
    }
  }
  pl->shift = shift;
  if (p->prec == FDE_P_TRI) TRY(tri_setup(pl, dp, dm));
  TRY(upload(pl, &pl->c64.fx, fx));
  TRY(upload(pl, &pl->c32.fx, fx));
  TRY(upload(pl, &pl->c64.fy, fy));
  TRY(upload(pl, &pl->c32.fy, fy));
  TRY(upload(pl, &pl->c64.fzero, fz));
  TRY(upload(pl, &pl->c32.fzero, fz));
  if (p->dim == 1 && (pl->n1 + 1 > 4096 || !is_pow2(pl->n1 + 1))) {
    // the four-step path: Toeplitz FFT length rows.P (n + 1, or a padded
    // power of two for the chirp-z form)
    pl->big = true;
    pl->blue = !is_pow2(pl->n1 + 1);
    pl->rows.P = (int)toep_len(pl->n1);
    pl->rows.logP = ilog2(pl->rows.P);
  }
  if (pl->dense) {
    // sine tables sqrt(2/P) sin(pi m/P), m < 2P, and the weights g_0..g_n, per direction
    auto dense_tables = [&](double alpha, int n, double** s64, float** s32, double** g64, float** g32) -> fde_status {
      const int P = n + 1;
      std::vector<double> st(2 * P);
      const double c = std::sqrt(2.0 / (double)P);
      for (int m = 0; m < 2 * P; ++m) st[m] = c * std::sin(M_PI * (double)m / (double)P);
      st[0] = st[P] = 0.0;
      const std::vector<double> g = weights(alpha, n, p->weights);
      TRY(upload(pl, s64, st));
      TRY(upload(pl, s32, st));
      TRY(upload(pl, g64, g));
      TRY(upload(pl, g32, g));
      return FDE_OK;
    };
    TRY(dense_tables(p->alpha[0], n1, &pl->c64.stabx, &pl->c32.stabx, &pl->c64.gx, &pl->c32.gx));
    TRY(dense_tables(p->alpha[1], n2, &pl->c64.staby, &pl->c32.staby, &pl->c64.gy, &pl->c32.gy));
  } else {
    TRY(direction_tables(pl, p->alpha[0], n1, &pl->c64.W2x, &pl->c32.W2x, &pl->c64.lamx, &pl->c32.lamx,
                         pl->rows.P));
  }
  if (pl->big) {
    const int L = pl->rows.logP;
    pl->log1 = (L + 1) / 2;
    pl->log2 = L / 2;
    pl->P1 = 1 << pl->log1;
    pl->P2 = 1 << pl->log2;
    auto sub = [&](int Ps, cx<double>** d, cx<float>** f) -> fde_status {
      std::vector<std::complex<double>> W(2 * Ps);
      for (int m = 0; m < 2 * Ps; ++m)
        W[m] = std::complex<double>(std::cos(M_PI * m / (double)Ps), -std::sin(M_PI * m / (double)Ps));
      TRY(upload_cx(pl, d, W));
      TRY(upload_cx(pl, f, W));
      return FDE_OK;
    };
    TRY(sub(pl->P1, &pl->c64.W2p1, &pl->c32.W2p1));
    TRY(sub(pl->P2, &pl->c64.W2p2, &pl->c32.W2p2));
    long work = pl->rows.P;
    if (pl->blue) {
      // chirp-z DST: FFT length sQ >= 2n - 1, its four-step factors, the chirp
      // c_j = exp(i pi j^2/(2P)) (j <= n, P = n + 1; j^2 reduced mod 4P) and the
      // spectrum of the filter conj(c_m), |m| < n, times sqrt(2/P)/sQ
      pl->sQ = chirp_len(n1);
      const int LQ = ilog2(pl->sQ);
      pl->slog1 = (LQ + 1) / 2;
      pl->slog2 = LQ / 2;
      pl->sQ1 = 1 << pl->slog1;
      pl->sQ2 = 1 << pl->slog2;
      TRY(sub(pl->sQ1, &pl->c64.Ws1, &pl->c32.Ws1));
      TRY(sub(pl->sQ2, &pl->c64.Ws2, &pl->c32.Ws2));
      TRY(sub((int)pl->sQ, &pl->c64.Wsb, &pl->c32.Wsb));
      const long P = n1 + 1;
      auto ph = [&](long j, double sgn) {
        const long r = (j * j) % (4 * P);
        const double t = M_PI * (double)r / (2.0 * (double)P);
        return std::complex<double>(std::cos(t), sgn * std::sin(t));
      };
      std::vector<std::complex<double>> chirp(n1 + 1), bhat(pl->sQ, 0.0);
      for (long j = 0; j <= n1; ++j) chirp[j] = ph(j, 1.0);
      for (long r = 0; r < n1; ++r) {
        bhat[r] = ph(r, -1.0);
        if (r) bhat[pl->sQ - r] = bhat[r];
      }
      host_fft(bhat);
      const double sc = std::sqrt(2.0 / (double)P) / (double)pl->sQ;
      for (auto& v : bhat) v *= sc;
      TRY(upload_cx(pl, &pl->c64.chirp, chirp));
      TRY(upload_cx(pl, &pl->c32.chirp, chirp));
      TRY(upload_cx(pl, &pl->c64.bhat, bhat));
      TRY(upload_cx(pl, &pl->c32.bhat, bhat));
      work = std::max(work, pl->sQ);
    }
    TRY(dalloc(pl, &pl->c64.cw, 6 * (size_t)work));
    if (p->precision == FDE_MIXED) TRY(dalloc(pl, &pl->c32.cw, 6 * (size_t)work));
  }
  if (p->dim == 2 && !pl->dense)
    TRY(direction_tables(pl, p->alpha[1], n2, &pl->c64.W2y, &pl->c32.W2y, &pl->c64.lamy, &pl->c32.lamy));

  // workspace
  const int m = pl->m;
  const long nvec = p->solver == FDE_S_PCG ? 3 : (m + 1);
  TRY(dalloc(pl, &pl->V, (size_t)nvec * pl->ld));
  TRY(dalloc(pl, &pl->Z, (size_t)(p->solver == FDE_S_PCG ? 2 : m) * pl->ld));
  TRY(dalloc(pl, &pl->t1, N));
  TRY(dalloc(pl, &pl->t2, N));
  TRY(dalloc(pl, &pl->t3, N));
  if (p->precision == FDE_MIXED) {
    TRY(dalloc(pl, &pl->Vf, (size_t)(pl->kin + 1) * pl->ld));
    TRY(dalloc(pl, &pl->t1f, N));
    TRY(dalloc(pl, &pl->t2f, N));
    TRY(dalloc(pl, &pl->t3f, N));
    TRY(dalloc(pl, &pl->uf, N));
    TRY(dalloc(pl, &pl->zf, N));
  }
  TRY(dalloc(pl, &pl->part, (size_t)RED_MAXG * (KMAX + 1)));
  TRY(dalloc(pl, &pl->ks, 1));
  TRY(dalloc(pl, &pl->ksi, 1));
  HIPCHK(hipMemsetAsync(pl->ks, 0, sizeof(KState), st));
  HIPCHK(hipMemsetAsync(pl->ksi, 0, sizeof(KState), st));
  void* hs = nullptr;
  HIPCHK(hipHostMalloc(&hs, 4 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
  pl->hstat = static_cast<double*>(hs);
  std::memset(pl->hstat, 0, 4 * sizeof(double));
  void* hd = nullptr;
  HIPCHK(hipHostGetDevicePointer(&hd, hs, 0));
  pl->hstat_dev = static_cast<double*>(hd);
  void* hk = nullptr;
  HIPCHK(hipHostMalloc(&hk, sizeof(KState), hipHostMallocDefault));
  pl->hks = static_cast<KState*>(hk);
  for (auto& e : pl->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipStreamSynchronize(st));
  return FDE_OK;
}

extern "C" fde_status fde_assemble(const fde_params* p, const double* dplus, const double* dminus,
                                   const double* eplus, const double* eminus, void* stream, fde_plan* out) {
  if (!out) return fail(FDE_EINVAL, "out is NULL");
  *out = nullptr;
  TRY(validate(p));
  fde_plan pl = new (std::nothrow) fde_plan_s();
  if (!pl) return fail(FDE_ENOMEM, "host allocation failed");
  fde_status s = assemble_impl(p, dplus, dminus, eplus, eminus, (hipStream_t)stream, pl);
  if (s != FDE_OK) {
    std::string keep = g_err;
    destroy_impl(pl);
    g_err = keep;
    return s;
  }
  *out = pl;
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Timing probe
// ---------------------------------------------------------------------------
struct ProbeScope {
  fde_plan pl;
  hipStream_t st;
  bool on;
  // cls: the launch's class; cls2: a second class it also belongs to (or 0)
  ProbeScope(fde_plan p, int cls, hipStream_t s, double bytes, int cls2 = 0)
      : pl(p), st(s), on(p && cls != 0 && (p->probe == cls || (cls2 != 0 && p->probe == cls2))) {
    if (!on) return;
    on = (pl->pseen++ % fde_plan_s::PSTRIDE) == 0;   // sample: keeps the event overhead small
    if (!on) return;
    if (pl->pev.size() < 2 * (pl->pused + 1)) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
          on = false;
          return;
        }
        pl->pev.push_back(e);
      }
    }
    (void)hipEventRecord(pl->pev[2 * pl->pused], st);
    pl->pbytes += bytes;
  }
  ~ProbeScope() {
    if (!on) return;
    (void)hipEventRecord(pl->pev[2 * pl->pused + 1], st);
    ++pl->pused;
  }
};

extern "C" fde_status fde_probe(fde_plan pl, int cls) {
  if (!pl) return fail(FDE_EINVAL, "NULL plan");
  if (cls < FDE_PROBE_OFF || cls >= 128 || (cls > FDE_PROBE_CGS32 && cls < FDE_PROBE_LINE64_VARIANT))
    return fail(FDE_EINVAL, "bad probe class %d", cls);
  pl->probe = cls;
  pl->pseen = 0;
  return FDE_OK;
}

extern "C" fde_status fde_probe_read(fde_plan pl, double* ms, long long* launches, double* bytes) {
  if (!pl) return fail(FDE_EINVAL, "NULL plan");
  double tot = 0.0;
  if (pl->pused) HIPCHK(hipEventSynchronize(pl->pev[2 * pl->pused - 1]));
  for (size_t i = 0; i < pl->pused; ++i) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, pl->pev[2 * i], pl->pev[2 * i + 1]));
    tot += t;
  }
  if (ms) *ms = tot;
  if (launches) *launches = (long long)pl->pused;
  if (bytes) *bytes = pl->pbytes;
  pl->pused = 0;
  pl->pbytes = 0.0;
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
static thread_local fde_plan g_probe_plan = nullptr;   // plan whose launches are being issued

struct ProbePlanScope {
  explicit ProbePlanScope(fde_plan pl) { g_probe_plan = pl; }
  ~ProbePlanScope() { g_probe_plan = nullptr; }
};

template <typename T, bool COLS, int FL, int LOGP>
static void launch_line_k(const LineArgs<T>& a, int grid, int nth, size_t lds, hipStream_t st) {
  // function-local static: initialised once, thread-safe (server workers launch concurrently)
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&line_kernel<T, COLS, FL, LOGP>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)attr;
  hipLaunchKernelGGL((line_kernel<T, COLS, FL, LOGP>), dim3(grid), dim3(nth), lds, st, a);
}

// COLS = true: d is a column direction (d.cols); only the y-direction
// programs are instantiated in that form.
// The direction's sizes and strides into the line program's arguments.
template <typename T>
static void fill_line_args(const Dir& d, LineArgs<T>& a) {
  a.n = d.n;
  a.P = d.P;
  a.logP = d.logP;
  a.nlines = d.nlines;
  a.B = d.B;
  a.logB = d.logB;
  a.LS = d.cols ? cols_line_stride(d.P) : line_stride(d.P);
  a.ls = d.ls;
  a.es = d.es;
  a.ntiles = (d.nlines + d.B - 1) / d.B;
}

template <typename T, int FL, bool COLS = false>
static void launch_line(const Dir& d, LineArgs<T> a, hipStream_t st) {
  fill_line_args(d, a);
  const int nth = std::max(1, d.B * d.P / 8);
  const size_t lds = ((size_t)d.B * a.LS + 2 * d.B + (size_t)d.P) * sizeof(cx<T>);
  const int grid = 8 * ((a.ntiles + 7) / 8);
  // algorithmic bytes: every vector operand read or written once
  const int nvec = (a.in != nullptr) + (a.pre != nullptr) + (a.post != nullptr) + (a.zout != nullptr) +
                   ((FL & LF_TOEP) ? 2 : 0) + ((FL & LF_EXTBASE) ? 1 : 0) + 1;
  const double bytes = (double)nvec * (double)d.n * (double)d.nlines * sizeof(T);
  ProbeScope ps(g_probe_plan, sizeof(T) == 8 ? FDE_PROBE_LINE64 : FDE_PROBE_LINE32, st, bytes,
                (sizeof(T) == 8 ? FDE_PROBE_LINE64_VARIANT : FDE_PROBE_LINE32_VARIANT) + FL);
  if constexpr (COLS) {
    switch (d.logP) {   // cols_per_tile(P) >= 2: P <= 2048
      case 3: launch_line_k<T, true, FL, 3>(a, grid, nth, lds, st); break;
      case 4: launch_line_k<T, true, FL, 4>(a, grid, nth, lds, st); break;
      case 5: launch_line_k<T, true, FL, 5>(a, grid, nth, lds, st); break;
      case 6: launch_line_k<T, true, FL, 6>(a, grid, nth, lds, st); break;
      case 7: launch_line_k<T, true, FL, 7>(a, grid, nth, lds, st); break;
      case 8: launch_line_k<T, true, FL, 8>(a, grid, nth, lds, st); break;
      case 9: launch_line_k<T, true, FL, 9>(a, grid, nth, lds, st); break;
      case 10: launch_line_k<T, true, FL, 10>(a, grid, nth, lds, st); break;
      case 11: launch_line_k<T, true, FL, 11>(a, grid, nth, lds, st); break;
      default: launch_line_k<T, true, FL, 0>(a, grid, nth, lds, st); break;
    }
  } else {
    switch (d.logP) {
      case 3: launch_line_k<T, false, FL, 3>(a, grid, nth, lds, st); break;
      case 4: launch_line_k<T, false, FL, 4>(a, grid, nth, lds, st); break;
      case 5: launch_line_k<T, false, FL, 5>(a, grid, nth, lds, st); break;
      case 6: launch_line_k<T, false, FL, 6>(a, grid, nth, lds, st); break;
      case 7: launch_line_k<T, false, FL, 7>(a, grid, nth, lds, st); break;
      case 8: launch_line_k<T, false, FL, 8>(a, grid, nth, lds, st); break;
      case 9: launch_line_k<T, false, FL, 9>(a, grid, nth, lds, st); break;
      case 10: launch_line_k<T, false, FL, 10>(a, grid, nth, lds, st); break;
      case 11: launch_line_k<T, false, FL, 11>(a, grid, nth, lds, st); break;
      case 12: launch_line_k<T, false, FL, 12>(a, grid, nth, lds, st); break;
      default: launch_line_k<T, false, FL, 0>(a, grid, nth, lds, st); break;
    }
  }
}

static int ew_grid(long N) { return (int)std::max(1L, std::min<long>(2048, (N + 255) / 256)); }

template <typename T>
static const Consts<T>& consts(fde_plan pl);
template <>
const Consts<double>& consts<double>(fde_plan pl) { return pl->c64; }
template <>
const Consts<float>& consts<float>(fde_plan pl) { return pl->c32; }

// Toeplitz-type LineArgs.  ydir: lines along y, with e+- in the original
// layout (columns read in place) or transposed (rows of the transposed
// (n1, n2) array, for the sizes that keep the transposes).
template <typename T>
static LineArgs<T> toep_args(fde_plan pl, bool ydir, const int* skip, const int* skip2) {
  const Consts<T>& c = consts<T>(pl);
  LineArgs<T> a{};
  a.W2 = ydir ? c.W2y : c.W2x;
  a.lam = ydir ? c.lamy : c.lamx;
  a.cplus = ydir ? (pl->use_cols ? c.ep : c.ept) : c.dp;
  a.cminus = ydir ? (pl->use_cols ? c.em : c.emt) : c.dm;
  a.skip = skip;
  a.skip2 = skip2;
  return a;
}

// out (cols x rows) = in^T (+ addend)
template <typename T>
static void transpose(const T* in, T* out, int rows, int cols, const T* addend, hipStream_t st,
                      const int* skip, const int* skip2) {
  const dim3 g((cols + 31) / 32, (rows + 31) / 32);
  if (addend)
    hipLaunchKernelGGL((transpose_kernel<T, true>), g, dim3(256), 0, st, in, out, rows, cols, addend, skip, skip2);
  else
    hipLaunchKernelGGL((transpose_kernel<T, false>), g, dim3(256), 0, st, in, out, rows, cols, addend, skip, skip2);
}

// y-direction part added to an x-direction part: y = xpart + tscale * kappa *
// (E+ (T_y (x) I) + E- (T_y^T (x) I)) x, on the columns of x in place, or on
// its transpose.
template <typename T>
static void add_y_part(fde_plan pl, const T* x, const T* xpart, T* y, T tscale, hipStream_t st, const int* skip,
                       const int* skip2) {
  if (pl->use_cols) {
    LineArgs<T> q = toep_args<T>(pl, true, skip, skip2);
    q.in = x;
    q.base = xpart;
    q.bscale = xpart ? T(1) : T(0);
    q.tscale = tscale * (T)pl->kappa;
    q.out = y;
    if (xpart) launch_line<T, LF_TOEP | LF_EXTBASE, true>(pl->ycols, q, st);
    else launch_line<T, LF_TOEP, true>(pl->ycols, q, st);
    return;
  }
  T* xt = pl->tmp<T>(1);
  T* yt = pl->tmp<T>(2);
  transpose<T>(x, xt, pl->n2, pl->n1, nullptr, st, skip, skip2);
  LineArgs<T> q = toep_args<T>(pl, true, skip, skip2);
  q.in = xt;
  q.bscale = T(0);
  q.tscale = tscale * (T)pl->kappa;
  q.out = yt;
  launch_line<T, LF_TOEP>(pl->trows, q, st);
  transpose<T>(yt, y, pl->n1, pl->n2, xpart, st, skip, skip2);
}

// ---------------------------------------------------------------------------
// Big 1D lines (P > 4096)
// ---------------------------------------------------------------------------
template <typename T, int LOG, bool CIN, bool COUT, class LD>
static void fourstep_k(LD in, cx<T>* out, long P, int npl, int batch, long ils, long ies, long ols, long oes,
                       const cx<T>* Wsub, const cx<T>* Wbig, int apply, hipStream_t st, const int* skip,
                       const int* skip2) {
  constexpr int L = 1 << LOG;
  constexpr int B = fourstep_lines(L);
  constexpr int EPT = fourstep_ept(L);
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&fourstep_kernel<T, LOG, CIN, COUT, LD>), hipFuncAttributeMaxDynamicSharedMemorySize,
      160 * 1024);
  (void)attr;
  const size_t lds = ((size_t)B * line_stride(L) + (size_t)B * L) * sizeof(cx<T>);
  const long lines = (long)batch * npl;   // B divides npl (both powers of two, npl >= 64 >= B)
  hipLaunchKernelGGL((fourstep_kernel<T, LOG, CIN, COUT, LD>), dim3((unsigned)(lines / B)), dim3(B * L / EPT), lds, st, in,
                     out, P, npl, ils, ies, ols, oes, Wsub, Wbig, apply, skip, skip2);
}

// Column pass (lines = the P2 columns of the P1 x P2 view, length P1, in
// place layout, twiddled) or row pass (lines = the P1 rows, length P2,
// written in natural order).
template <typename T, bool COLPASS, class LD>
static void fourstep(int lg, LD in, cx<T>* out, long P, int P1, int P2, int batch, const cx<T>* Wsub,
                     const cx<T>* Wbig, hipStream_t st, const int* skip, const int* skip2) {
#define FDE_FOURSTEP_CASE(LG)                                                                                   \
  case LG:                                                                                                     \
    if constexpr (COLPASS)                                                                                     \
      fourstep_k<T, LG, true, true>(in, out, P, P2, batch, 1, P2, 1, P2, Wsub, Wbig, 1, st, skip, skip2);     \
    else                                                                                                       \
      fourstep_k<T, LG, false, true>(in, out, P, P1, batch, P2, 1, 1, P1, Wsub, Wbig, 0, st, skip, skip2);    \
    break;
  switch (lg) {
    FDE_FOURSTEP_CASE(6)
    FDE_FOURSTEP_CASE(7)
    FDE_FOURSTEP_CASE(8)
    FDE_FOURSTEP_CASE(9)
    FDE_FOURSTEP_CASE(10)
    FDE_FOURSTEP_CASE(11)
    default: break;   // P = n + 1 <= 2^22: both factors have 6..11 bits
  }
#undef FDE_FOURSTEP_CASE
}

// P-point FFT of the `batch` arrays the loader produces, into `out`
// (natural order); `tmp` (batch P entries) is scratch.  The column pass has
// finished reading the loader's sources before the row pass writes `out`, so
// `out` may be one of them.
template <typename T, class LD>
static void big_fft(fde_plan pl, LD ld, cx<T>* out, cx<T>* tmp, int batch, hipStream_t st, const int* skip,
                    const int* skip2, bool chirp = false) {
  const Consts<T>& c = consts<T>(pl);
  if (chirp) {   // the chirp-z DST's length-sQ FFT
    const long Q = pl->sQ;
    fourstep<T, true>(pl->slog1, ld, tmp, Q, pl->sQ1, pl->sQ2, batch, c.Ws1, c.Wsb, st, skip, skip2);
    fourstep<T, false>(pl->slog2, LdArray<T>{tmp, Q}, out, Q, pl->sQ1, pl->sQ2, batch, c.Ws2, c.Wsb, st, skip,
                       skip2);
    return;
  }
  const long P = pl->rows.P;
  fourstep<T, true>(pl->log1, ld, tmp, P, pl->P1, pl->P2, batch, c.W2p1, c.W2x, st, skip, skip2);   // columns
  fourstep<T, false>(pl->log2, LdArray<T>{tmp, P}, out, P, pl->P1, pl->P2, batch, c.W2p2, c.W2x, st, skip,
                     skip2);                                                                          // rows
}

static int ew_grid(long N);

// z = S F^{-1} S (pre .* sc v) .* post   (1D big line); z2: optional second copy
template <typename T, typename TI = T>
static void big_tau(fde_plan pl, const TI* v, const double* sc, const T* pre, const T* post, T* z, T* z2,
                    hipStream_t st, const int* skip, const int* skip2, bool raw = false) {
  const Consts<T>& c = consts<T>(pl);
  const int P = pl->rows.P, n = pl->n1;
  if (pl->blue) {   // chirp-z DST, divide by F, chirp-z DST
    const long Q = pl->sQ;
    cx<T>* a0 = c.cw;
    cx<T>* a1 = c.cw + Q;
    big_fft<T>(pl, LdChirpIn<T, TI>{v, pre, sc, c.chirp, n}, a0, a1, 1, st, skip, skip2, true);
    big_fft<T>(pl, LdChirpMul<T>{a0, c.bhat}, a0, a1, 1, st, skip, skip2, true);
    big_fft<T>(pl, LdChirpMid<T>{a0, c.chirp, c.fx, n}, a0, a1, 1, st, skip, skip2, true);
    big_fft<T>(pl, LdChirpMul<T>{a0, c.bhat}, a0, a1, 1, st, skip, skip2, true);
    if (raw) return;   // the caller unpacks from a0 (LdChirpPackToep)
    hipLaunchKernelGGL((unpack_chirp_kernel<T>), dim3(ew_grid(n)), dim3(256), 0, st, a0, c.chirp, post, z, z2, n,
                       skip, skip2);
    return;
  }
  cx<T>* c0 = c.cw;
  cx<T>* c1 = c.cw + P;
  const int g = ew_grid(P);
  big_fft<T>(pl, LdPackDst<T, TI>{v, pre, sc, P}, c0, c1, 1, st, skip, skip2);
  big_fft<T>(pl, LdFRepack<T>{c0, c.W2x, c.fx, P}, c0, c1, 1, st, skip, skip2);
  if (raw) return;   // the caller unpacks from c0 (LdDstPackToep)
  hipLaunchKernelGGL((unpack_dst_kernel<T>), dim3(g), dim3(256), 0, st, c0, c.W2x, post, z, z2, n, P, skip, skip2);
}

// out = bscale * base + tscale * (D+ T x + D- T^T x)   (1D big line); the
// loader supplies the packed x (LdPackToep, or LdDstPackToep straight from
// the preconditioner's last FFT).  With defer_x (float64) the extraction is
// left to the first Gram-Schmidt pass of the outer step.
template <typename T, class LD>
static void big_toep_ld(fde_plan pl, LD ld, const T* base, T bscale, T tscale, T* out, hipStream_t st,
                        const int* skip, const int* skip2) {
  const Consts<T>& c = consts<T>(pl);
  const int P = pl->rows.P, n = pl->n1;
  cx<T>* c0 = c.cw;
  cx<T>* c1 = c.cw + P;
  cx<T>* c2 = c.cw + 2 * P;
  cx<T>* c3 = c.cw + 4 * P;
  const int g = ew_grid(P);
  big_fft<T>(pl, ld, c0, c1, 1, st, skip, skip2);
  big_fft<T>(pl, LdPairToep<T>{c0, c.lamx, c.W2x, P}, c3, c2, 2, st, skip, skip2);
  if constexpr (sizeof(T) == 8) {
    if (pl->defer_x) {
      pl->xpa = XArgs{reinterpret_cast<const double*>(c3), reinterpret_cast<const double*>(c3 + P), c.dp, c.dm,
                      base, bscale, tscale, P};
      pl->xout = out;
      pl->xpend = true;
      return;
    }
  }
  hipLaunchKernelGGL((extract_toep_kernel<T>), dim3(g), dim3(256), 0, st, c3, c3 + P, c.dp, c.dm, base, bscale, tscale,
                     out, n, P, skip, skip2);
}

template <typename T>
static void big_toep(fde_plan pl, const T* x, const T* base, T bscale, T tscale, T* out, hipStream_t st,
                     const int* skip, const int* skip2) {
  big_toep_ld<T>(pl, LdPackToep<T>{x, pl->n1}, base, bscale, tscale, out, st, skip, skip2);
}

// z = P^{-1}(sc * v) (stored when z != null; the DST-side factors D^{-1} as
// dside says) and w = M z: the fused operator step of the solvers.  With
// prec NONE, z = sc * v.
template <typename T>
static const TriDev<T>& tri_dev(fde_plan pl);
template <>
const TriDev<double>& tri_dev<double>(fde_plan pl) { return pl->tri64; }
template <>
const TriDev<float>& tri_dev<float>(fde_plan pl) { return pl->tri32; }

// z = P_tri^{-1}(sc v): chunk sweeps, reduced system, back substitution.
template <typename T>
static void tri_apply(fde_plan pl, const T* v, const double* sc, T* z, hipStream_t st, const int* skip,
                      const int* skip2) {
  const TriDev<T>& t = tri_dev<T>(pl);
  hipLaunchKernelGGL((tri_chunk_kernel<T, T>), dim3((t.p + 255) / 256), dim3(256), 0, st, v, sc, t, skip, skip2);
  hipLaunchKernelGGL((tri_reduce_kernel<T>), dim3(1), dim3(TRI_PMAX), 0, st, t, skip, skip2);
  hipLaunchKernelGGL((tri_back_kernel<T, T>), dim3(ew_grid(pl->N)), dim3(256), 0, st, t, pl->N, z, skip, skip2);
}

// 2D: out = (S (x) I) F^{-1} (S (x) I) applied along y to t (the middle of
// P^{-1}: DST along y, division by F_N, DST along y), in place on the
// columns, or on the transpose (t is overwritten then).
template <typename T>
static void y_dst_f_dst(fde_plan pl, T* t, T* out, hipStream_t st, const int* skip, const int* skip2) {
  const Consts<T>& c = consts<T>(pl);
  LineArgs<T> b{};
  b.fline = c.fx;
  b.felem = c.fy;
  b.W2 = c.W2y;
  b.skip = skip;
  b.skip2 = skip2;
  if (pl->use_cols) {
    b.in = t;
    b.out = out;
    launch_line<T, LF_DST1 | LF_FDST2, true>(pl->ycols, b, st);
    return;
  }
  transpose<T>(t, out, pl->n2, pl->n1, nullptr, st, skip, skip2);
  b.in = out;
  b.out = t;
  launch_line<T, LF_DST1 | LF_FDST2>(pl->trows, b, st);
  transpose<T>(t, out, pl->n1, pl->n2, nullptr, st, skip, skip2);
}

template <typename T>
static void matvec_only(fde_plan pl, const T* x, T* y, T bscale, T tscale, hipStream_t st, const int* skip,
                        const int* skip2 = nullptr);

// ---------------------------------------------------------------------------
// Dense 2D form (fde_dense.hpp)
// ---------------------------------------------------------------------------
template <typename T, int MODE>
static void dense_launch(fde_plan pl, DenseArgs<T> a, hipStream_t st, const int* skip, const int* skip2) {
  a.n1 = pl->n1;
  a.n2 = pl->n2;
  a.skip = skip;
  a.skip2 = skip2;
  const dim3 grid((pl->n1 + 31) / 32, (pl->n2 + 31) / 32);
  constexpr bool TOEP = MODE == DM_ROW_TOEP || MODE == DM_COL_TOEP;
  const double bytes = (double)pl->N * sizeof(T) *
                       ((a.pre != nullptr) + (a.post != nullptr) + (TOEP ? 3 + (a.base != nullptr) : 0) + 2);
  ProbeScope ps(g_probe_plan, sizeof(T) == 8 ? FDE_PROBE_LINE64 : FDE_PROBE_LINE32, st, bytes);
  hipLaunchKernelGGL((dense_kernel<T, MODE>), grid, dim3(256), 0, st, a);
}

// z = P^{-1}(sc * v): rows DST (D^{-1} first for D tau), columns DST, / F,
// columns DST, rows DST (D^{-1} after for tau D).
template <typename T>
static void dense_tau(fde_plan pl, const T* v, const double* sc, const T* pre, const T* post, T* z, hipStream_t st,
                      const int* skip, const int* skip2) {
  const Consts<T>& c = consts<T>(pl);
  T* t1 = pl->tmp<T>(1);
  T* t2 = pl->tmp<T>(2);
  DenseArgs<T> a{};
  a.in = v;
  a.sc = sc;
  a.pre = pre;
  a.stab = c.stabx;
  a.out = t1;
  dense_launch<T, DM_ROW_DST>(pl, a, st, skip, skip2);
  DenseArgs<T> b{};
  b.in = t1;
  b.stab = c.staby;
  b.fx = c.fx;
  b.fy = c.fy;
  b.out = t2;
  dense_launch<T, DM_COL_DST>(pl, b, st, skip, skip2);
  b.in = t2;
  b.fx = b.fy = nullptr;
  b.out = t1;
  dense_launch<T, DM_COL_DST>(pl, b, st, skip, skip2);
  DenseArgs<T> r{};
  r.in = t1;
  r.stab = c.stabx;
  r.post = post;
  r.out = z;
  dense_launch<T, DM_ROW_DST>(pl, r, st, skip, skip2);
}

// y = bscale x + tscale (A_x x + kappa A_y x)
template <typename T>
static void dense_toep(fde_plan pl, const T* x, T* y, T bscale, T tscale, hipStream_t st, const int* skip,
                       const int* skip2) {
  const Consts<T>& c = consts<T>(pl);
  T* t3 = pl->tmp<T>(3);
  DenseArgs<T> a{};
  a.in = x;
  a.g = c.gx;
  a.cp = c.dp;
  a.cm = c.dm;
  a.bscale = bscale;
  a.tscale = tscale;
  a.out = t3;
  dense_launch<T, DM_ROW_TOEP>(pl, a, st, skip, skip2);
  DenseArgs<T> b{};
  b.in = x;
  b.g = c.gy;
  b.cp = c.ep;
  b.cm = c.em;
  b.base = t3;
  b.bscale = T(1);
  b.tscale = tscale * (T)pl->kappa;
  b.out = y;
  dense_launch<T, DM_COL_TOEP>(pl, b, st, skip, skip2);
}

template <typename T>
static void tau_matvec(fde_plan pl, const T* v, const double* sc, T* z, T* w, hipStream_t st, const int* skip,
                       const int* skip2) {
  if (pl->dense) {   // 2D callers always pass z
    const Consts<T>& c = consts<T>(pl);
    if (pl->p.prec == FDE_P_NONE)
      hipLaunchKernelGGL((scale_cast_kernel<T, T>), dim3(ew_grid(pl->N)), dim3(256), 0, st, v, z, pl->N, sc, skip,
                         skip2);
    else
      dense_tau<T>(pl, v, sc, (pl->has_dinv && pl->dside == FDE_D_LEFT) ? c.dinv : nullptr,
                   (pl->has_dinv && pl->dside == FDE_D_RIGHT) ? c.dinv : nullptr, z, st, skip, skip2);
    dense_toep<T>(pl, z, w, (T)pl->nu, T(1), st, skip, skip2);
    return;
  }
  if (pl->p.prec == FDE_P_TRI) {
    tri_apply<T>(pl, v, sc, z, st, skip, skip2);
    matvec_only<T>(pl, z, w, (T)pl->nu, T(1), st, skip, skip2);
    return;
  }
  const Consts<T>& c = consts<T>(pl);
  const bool tau = pl->p.prec != FDE_P_NONE;
  const T* pre = (pl->has_dinv && pl->dside == FDE_D_LEFT) ? c.dinv : nullptr;
  const T* post = (pl->has_dinv && pl->dside == FDE_D_RIGHT) ? c.dinv : nullptr;
  if (pl->dim == 1 && pl->big) {
    T* zz = z ? z : pl->tmp<T>(1);
    if (tau) {
      // the second DST's unpacking is the Toeplitz product's packing loader
      // (the DST's output occupies c.cw below the Toeplitz FFT's scratch,
      // which starts at c.cw + P, P > n)
      big_tau<T>(pl, v, sc, pre, post, zz, nullptr, st, skip, skip2, true);
      if (pl->blue)
        big_toep_ld<T>(pl, LdChirpPackToep<T>{c.cw, c.chirp, post, zz, pl->n1}, zz, (T)pl->nu, T(1), w, st, skip,
                       skip2);
      else
        big_toep_ld<T>(pl, LdDstPackToep<T>{c.cw, c.W2x, post, zz, pl->n1, pl->rows.P}, zz, (T)pl->nu, T(1), w, st,
                       skip, skip2);
      return;
    }
    hipLaunchKernelGGL((scale_cast_kernel<T, T>), dim3(ew_grid(pl->N)), dim3(256), 0, st, v, zz, pl->N, sc, skip,
                       skip2);
    big_toep<T>(pl, zz, zz, (T)pl->nu, T(1), w, st, skip, skip2);
    return;
  }
  if (pl->dim == 1) {
    LineArgs<T> a = toep_args<T>(pl, false, skip, skip2);
    a.in = v;
    a.sc = sc;
    a.pre = pre;
    a.post = post;
    a.fline = c.fzero;
    a.felem = c.fx;
    a.zout = z;
    a.bscale = (T)pl->nu;
    a.tscale = T(1);
    a.out = w;
    if (tau) {
      if (z) launch_line<T, LF_DST1 | LF_FDST2 | LF_STOREZ | LF_TOEP>(pl->rows, a, st);
      else launch_line<T, LF_DST1 | LF_FDST2 | LF_TOEP>(pl->rows, a, st);
    } else {
      if (z) launch_line<T, LF_STOREZ | LF_TOEP>(pl->rows, a, st);
      else launch_line<T, LF_TOEP>(pl->rows, a, st);
    }
    return;
  }
  T* t1 = pl->tmp<T>(1);
  T* t2 = pl->tmp<T>(2);
  T* t3 = pl->tmp<T>(3);
  T* zz = z;   // 2D callers always pass z: the y-direction pass reads it
  if (tau) {
    // rows: DST along x (D^{-1} first for the D tau order)
    LineArgs<T> a{};
    a.in = v;
    a.sc = sc;
    a.pre = pre;
    a.W2 = c.W2x;
    a.out = t1;
    a.skip = skip;
    a.skip2 = skip2;
    launch_line<T, LF_DST1>(pl->rows, a, st);
    // along y: DST, divide by F, DST
    y_dst_f_dst<T>(pl, t1, t2, st, skip, skip2);
    // rows: DST along x (D^{-1} after for tau D), store z, x-direction Toeplitz
    LineArgs<T> r = toep_args<T>(pl, false, skip, skip2);
    r.in = t2;
    r.post = post;
    r.zout = zz;
    r.bscale = (T)pl->nu;
    r.tscale = T(1);
    r.out = t3;
    launch_line<T, LF_DST1 | LF_STOREZ | LF_TOEP>(pl->rows, r, st);
  } else {
    LineArgs<T> r = toep_args<T>(pl, false, skip, skip2);
    r.in = v;
    r.sc = sc;
    r.zout = zz;
    r.bscale = (T)pl->nu;
    r.tscale = T(1);
    r.out = t3;
    launch_line<T, LF_STOREZ | LF_TOEP>(pl->rows, r, st);
  }
  add_y_part<T>(pl, zz, t3, w, T(1), st, skip, skip2);
}

// z = P^{-1}(sc * v)
template <typename T>
static void tau_only(fde_plan pl, const T* v, const double* sc, T* z, hipStream_t st, const int* skip,
                     const int* skip2 = nullptr) {
  const Consts<T>& c = consts<T>(pl);
  const T* pre = (pl->has_dinv && pl->dside == FDE_D_LEFT) ? c.dinv : nullptr;
  const T* post = (pl->has_dinv && pl->dside == FDE_D_RIGHT) ? c.dinv : nullptr;
  if (pl->p.prec == FDE_P_NONE) {
    hipLaunchKernelGGL((scale_cast_kernel<T, T>), dim3(ew_grid(pl->N)), dim3(256), 0, st, v, z, pl->N, sc,
                       skip, skip2);
    return;
  }
  if (pl->p.prec == FDE_P_TRI) {
    tri_apply<T>(pl, v, sc, z, st, skip, skip2);
    return;
  }
  if (pl->dim == 1 && pl->big) {
    big_tau<T>(pl, v, sc, pre, post, z, nullptr, st, skip, skip2);
    return;
  }
  if (pl->dense) {
    dense_tau<T>(pl, v, sc, pre, post, z, st, skip, skip2);
    return;
  }
  if (pl->dim == 1) {
    LineArgs<T> a{};
    a.in = v;
    a.sc = sc;
    a.pre = pre;
    a.post = post;
    a.fline = c.fzero;
    a.felem = c.fx;
    a.W2 = c.W2x;
    a.out = z;
    a.skip = skip;
    a.skip2 = skip2;
    launch_line<T, LF_DST1 | LF_FDST2>(pl->rows, a, st);
    return;
  }
  T* t1 = pl->tmp<T>(1);
  T* t2 = pl->tmp<T>(2);
  LineArgs<T> a{};
  a.in = v;
  a.sc = sc;
  a.pre = pre;
  a.W2 = c.W2x;
  a.out = t1;
  a.skip = skip;
  a.skip2 = skip2;
  launch_line<T, LF_DST1>(pl->rows, a, st);
  y_dst_f_dst<T>(pl, t1, t2, st, skip, skip2);
  LineArgs<T> r{};
  r.in = t2;
  r.post = post;
  r.W2 = c.W2x;
  r.out = z;
  r.skip = skip;
  r.skip2 = skip2;
  launch_line<T, LF_DST1>(pl->rows, r, st);
}

// y = bscale*x + tscale*(A_x x + kappa A_y x)   (bscale = nu, tscale = 1: y = M x)
template <typename T>
static void matvec_only(fde_plan pl, const T* x, T* y, T bscale, T tscale, hipStream_t st, const int* skip,
                        const int* skip2) {
  if (pl->dim == 1 && pl->big) {
    big_toep<T>(pl, x, x, bscale, tscale, y, st, skip, skip2);
    return;
  }
  if (pl->dense) {
    dense_toep<T>(pl, x, y, bscale, tscale, st, skip, skip2);
    return;
  }
  LineArgs<T> a = toep_args<T>(pl, false, skip, skip2);
  a.in = x;
  a.bscale = bscale;
  a.tscale = tscale;
  if (pl->dim == 1) {
    a.out = y;
    launch_line<T, LF_TOEP>(pl->rows, a, st);
    return;
  }
  T* t3 = pl->tmp<T>(3);
  a.out = t3;
  launch_line<T, LF_TOEP>(pl->rows, a, st);
  add_y_part<T>(pl, x, t3, y, tscale, st, skip, skip2);
}

extern "C" fde_status fde_matvec(fde_plan pl, const double* x, double* y, void* stream) {
  if (!pl || !x || !y) return fail(FDE_EINVAL, "NULL argument");
  ProbePlanScope pps(pl);
  matvec_only<double>(pl, x, y, pl->nu, 1.0, (hipStream_t)stream, nullptr);
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

extern "C" fde_status fde_tau_apply(fde_plan pl, const double* v, double* z, void* stream) {
  if (!pl || !v || !z) return fail(FDE_EINVAL, "NULL argument");
  ProbePlanScope pps(pl);
  tau_only<double>(pl, v, nullptr, z, (hipStream_t)stream, nullptr);
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

// The same operators in float32 arithmetic (those of the mixed form's inner
// solves): the float64 input rounded to float32, the float32 result widened.
static fde_status op_f32(fde_plan pl, const double* in, double* out, hipStream_t st, bool tau) {
  if (!pl || !in || !out) return fail(FDE_EINVAL, "NULL argument");
  if (pl->p.precision != FDE_MIXED) return fail(FDE_EINVAL, "float32 operators need a plan assembled with FDE_MIXED");
  ProbePlanScope pps(pl);
  const long N = pl->N;
  hipLaunchKernelGGL((scale_cast_kernel<double, float>), dim3(ew_grid(N)), dim3(256), 0, st, in, pl->uf, N,
                     (const double*)nullptr, (const int*)nullptr, (const int*)nullptr);
  if (tau) tau_only<float>(pl, pl->uf, nullptr, pl->zf, st, nullptr);
  else matvec_only<float>(pl, pl->uf, pl->zf, (float)pl->nu, 1.0f, st, nullptr);
  hipLaunchKernelGGL((scale_cast_kernel<float, double>), dim3(ew_grid(N)), dim3(256), 0, st, pl->zf, out, N,
                     (const double*)nullptr, (const int*)nullptr, (const int*)nullptr);
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

extern "C" fde_status fde_matvec_f32(fde_plan pl, const double* x, double* y, void* stream) {
  return op_f32(pl, x, y, (hipStream_t)stream, false);
}

extern "C" fde_status fde_tau_apply_f32(fde_plan pl, const double* v, double* z, void* stream) {
  return op_f32(pl, v, z, (hipStream_t)stream, true);
}

extern "C" fde_status fde_rhs(fde_plan pl, const double* u, const double* f, double* b, void* stream) {
  if (!pl || !u || !b) return fail(FDE_EINVAL, "NULL argument");
  ProbePlanScope pps(pl);
  hipStream_t st = (hipStream_t)stream;
  const long N = pl->N;
  if (pl->p.time == FDE_T_EULER) {
    hipLaunchKernelGGL(axpby_kernel, dim3(ew_grid(N)), dim3(256), 0, st, pl->nu, u, pl->hxa, f, b, N);
  } else {
    matvec_only<double>(pl, u, b, pl->nu, -1.0, st, nullptr);
    if (f) hipLaunchKernelGGL(axpby_kernel, dim3(ew_grid(N)), dim3(256), 0, st, 1.0, b, 2.0 * pl->hxa, f, b, N);
  }
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Solvers
// ---------------------------------------------------------------------------
__global__ void ks_init_kernel(KState* ks, int maxit, int m, double tol) {
  if (threadIdx.x != 0) return;
  ks->kdone = 0;
  ks->done = 0;
  ks->conv = 0;
  ks->iters = 0;
  ks->maxit = maxit;
  ks->m = m;
  ks->nonfinite = 0;
  ks->breakdown = 0;
  ks->bnorm = 0;
  ks->tolabs = tol;   // multiplied by ||b|| once it is known
  ks->beta = ks->est = ks->hn = 0;
  ks->rz = ks->pq = ks->alpha = ks->betacg = 0;
  for (int i = 0; i <= KMAX; ++i) ks->scale[i] = 0.0;
}

__global__ void ks_settol_kernel(KState* ks) {
  if (threadIdx.x == 0) ks->tolabs = ks->tolabs * ks->bnorm;
}

static int red_grid(long N, long per) {
  return (int)std::max(1L, std::min<long>(RED_MAXG, (N + per - 1) / per));
}

static void finalize(fde_plan pl, int G, int nq, KState* ks, int fkind, int emode, int col, double* hstat,
                     hipStream_t st, const int* skip, const int* skip2, const double* part = nullptr) {
  if (G <= 1) return;
  hipLaunchKernelGGL(finalize_kernel, dim3(fkind == FK_H ? nq : 1), dim3(RED_THREADS), 0, st,
                     part ? part : pl->part, G, nq, ks, fkind, emode, col, hstat, skip, skip2);
}

// A Gram-Schmidt pass with a grid of at most HANDOFF_MAXG workgroups leaves
// its k coefficient partials to the update pass that follows it, whose
// workgroups each sum them (k * G <= 32 * HANDOFF_MAXG values from L2) in
// place of a finalize launch; the passes alternate between two regions of
// the partials buffer so that a pass never overwrites what it reads.
constexpr int HANDOFF_MAXG = 8 * HANDOFF_PER_THREAD;
constexpr size_t PART_B = (size_t)HANDOFF_MAXG * 32;   // offset of the second region

// ||a - b||^2 with an epilogue; out = a - b when out != null.
template <typename T>
static void norm_red(fde_plan pl, const T* a, const T* b, T* out, KState* ks, int emode, hipStream_t st,
                     const int* skip = nullptr, const int* skip2 = nullptr) {
  const int G = red_grid(pl->N, (long)RED_THREADS * 8);
  hipLaunchKernelGGL((norm_kernel<T>), dim3(G), dim3(RED_THREADS), 0, st, a, b, out, pl->N, pl->part, ks, emode,
                     skip, skip2);
  finalize(pl, G, 1, ks, FK_NORM, emode, 0, nullptr, st, skip, skip2);
}

template <typename T, int KC, int EPI, int MODE>
static void cgs_launch(fde_plan pl, const T* V, int k, T* w, KState* ks, int emode, int col, double* hstat,
                       hipStream_t st, const int* skip, const int* skip2) {
  const long N = pl->N;
  // float32 kernels take element pairs: the same grid as float64 covers them in one pass
  const int G = red_grid(N, (long)RED_THREADS * EPI * 2);
  constexpr bool DOT = MODE == CG_DOT || MODE == CG_XDOT;
  const int cls = sizeof(T) == 8 ? (DOT ? FDE_PROBE_MDOT64 : FDE_PROBE_MAXPY64)
                                 : (DOT ? FDE_PROBE_MDOT32 : FDE_PROBE_MAXPY32);
  // (the extraction pass also reads the two FFT lines, base and d+-, and writes w)
  const double bytes = (double)(k + (DOT ? 1 : 2) + (MODE == CG_XDOT ? 7 : 0)) * N * sizeof(T);
  // partials of the previous pass (update passes only), and where this pass writes its own
  const double* pin = !DOT ? pl->pend_part : nullptr;
  const int gin = pin ? pl->pend_G : 0;
  pl->pend_part = nullptr;
  double* pout = pin == pl->part ? pl->part + PART_B : pl->part;
  {
    ProbeScope ps(pl, cls, st, bytes, sizeof(T) == 8 ? FDE_PROBE_CGS64 : FDE_PROBE_CGS32);
    hipLaunchKernelGGL((cgs_kernel<T, KC, EPI, MODE>), dim3(G), dim3(RED_THREADS), 0, st, V, pl->ld, k, w, w, N, emode,
                       col, pout, ks, hstat, pin, gin, MODE == CG_XDOT ? pl->xpa : XArgs{}, skip, skip2);
  }
  if (MODE == CG_AXPY_NORM) {
    finalize(pl, G, 1, ks, FK_NORM, emode, col, hstat, st, skip, skip2, pout);
  } else if (G > 1 && G <= HANDOFF_MAXG) {
    pl->pend_part = pout;   // summed by the next update pass
    pl->pend_G = G;
  } else {
    finalize(pl, G, k, ks, FK_H, MODE == CG_AXPY_DOT ? EP_H2 : emode, col, hstat, st, skip, skip2, pout);
  }
}

template <typename T, int MODE>
static void cgs_pass_k(fde_plan pl, const T* V, int k, T* w, KState* ks, int emode, int col, double* hstat,
                       hipStream_t st, const int* skip, const int* skip2) {
  // (twice the elements per thread for float32 was measured slower: fewer workgroups)
  constexpr int X = 1;
  if (k <= 8) cgs_launch<T, 8, 4 * X, MODE>(pl, V, k, w, ks, emode, col, hstat, st, skip, skip2);
  else if (k <= 16) cgs_launch<T, 16, 2 * X, MODE>(pl, V, k, w, ks, emode, col, hstat, st, skip, skip2);
  else cgs_launch<T, 32, 1 * X, MODE>(pl, V, k, w, ks, emode, col, hstat, st, skip, skip2);
}

template <typename T, int MODE>
static void cgs_pass(fde_plan pl, const T* V, int k, T* w, KState* ks, int emode, int col, double* hstat,
                     hipStream_t st, const int* skip, const int* skip2) {
  if constexpr (MODE == CG_DOT && sizeof(T) == 8) {
    if (pl->xpend) {   // w still to be extracted from the Toeplitz product's FFT lines
      pl->xpend = false;
      if (pl->xout == w) {
        cgs_pass_k<double, CG_XDOT>(pl, V, k, w, ks, emode, col, hstat, st, skip, skip2);
        return;
      }
      const XArgs& a = pl->xpa;
      hipLaunchKernelGGL((extract_toep_kernel<double>), dim3(ew_grid(pl->rows.P)), dim3(256), 0, st,
                         reinterpret_cast<const cx<double>*>(a.r1), reinterpret_cast<const cx<double>*>(a.r2), a.cp,
                         a.cm, a.base, a.bscale, a.tscale, pl->xout, pl->n1, a.P, skip, skip2);
    }
  }
  cgs_pass_k<T, MODE>(pl, V, k, w, ks, emode, col, hstat, st, skip, skip2);
}

// One classical Gram-Schmidt pass (h = V^T w into h2, then w -= V h and
// ||w|| in one pass) and the Givens column j; h1 stays zero from the cycle
// start.
template <typename T>
static void cgs1_givens(fde_plan pl, const T* V, T* w, int j, KState* ks, double* hstat, hipStream_t st,
                        const int* skip, const int* skip2) {
  const int k = j + 1;
  cgs_pass<T, CG_DOT>(pl, V, k, w, ks, EP_H2, j, nullptr, st, skip, skip2);
  cgs_pass<T, CG_AXPY_NORM>(pl, V, k, w, ks, EP_GIVENS, j, hstat, st, skip, skip2);
}

// CGS2 of w (= basis slot j+1) against basis vectors 0..j, then the Givens
// column j: h1 = V^T w; w -= V h1 and h2 = V^T w in one pass; w -= V h2 and
// ||w|| in one pass.
template <typename T>
static void cgs2_givens(fde_plan pl, const T* V, T* w, int j, KState* ks, double* hstat, hipStream_t st,
                        const int* skip, const int* skip2) {
  const int k = j + 1;
  cgs_pass<T, CG_DOT>(pl, V, k, w, ks, EP_H1, j, nullptr, st, skip, skip2);
  cgs_pass<T, CG_AXPY_DOT>(pl, V, k, w, ks, EP_H2, j, nullptr, st, skip, skip2);
  cgs_pass<T, CG_AXPY_NORM>(pl, V, k, w, ks, EP_GIVENS, j, hstat, st, skip, skip2);
}

static fde_status read_header(fde_plan pl, KState* ks, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(pl->hks, ks, KSTATE_HEADER, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return FDE_OK;
}

// The float32 inner solve of one outer step of the mixed form: GMRES(kin)
// from x = 0 on the float32 copy of v_j (basis slot 0 of Vf), then
// zf = P^{-1} uf.  Every kernel skips when the outer cycle is over; the inner
// ones also when the inner cycle broke down.  The inner basis is
// orthogonalised with one classical Gram-Schmidt pass: the inner solve only
// shapes the flexible preconditioner, while the float64 outer cycle (CGS2)
// and its true-residual test decide the answer.
static void inner_solve(fde_plan pl, hipStream_t st) {
  const long N = pl->N, ld = pl->ld;
  const int* skip = &pl->ks->done;
  KState* ki = pl->ksi;
  const int* s2 = &ki->done;
  float* Vf = pl->Vf;
  norm_red<float>(pl, Vf, nullptr, nullptr, ki, EP_INNER0, st, skip, nullptr);
  for (int i = 0; i < pl->kin; ++i) {
    float* vi = Vf + (long)i * ld;
    float* wi = Vf + (long)(i + 1) * ld;
    tau_matvec<float>(pl, vi, &ki->scale[i], pl->zf, wi, st, s2, skip);
    cgs1_givens<float>(pl, Vf, wi, i, ki, nullptr, st, s2, skip);
  }
  hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(256), 0, st, ki, skip);
  hipLaunchKernelGGL((update_kernel<float, float>), dim3(ew_grid(N)), dim3(RED_THREADS), 0, st, Vf, ld,
                     (const float*)nullptr, pl->uf, N, ki, ki->scale, skip);
  tau_only<float>(pl, pl->uf, nullptr, pl->zf, st, skip);
}

// One outer Arnoldi step j: z_j = P^{-1} v_j (FP64, or the float32 inner
// solve), w = M z_j into basis slot j+1, CGS2, Givens.
static void outer_step(fde_plan pl, int j, hipStream_t st) {
  const long N = pl->N;
  KState* ks = pl->ks;
  const int* skip = &ks->done;
  const long ld = pl->ld;
  double* vj = pl->V + (long)j * ld;
  double* w = pl->V + (long)(j + 1) * ld;
  double* zj = pl->Z + (long)j * ld;
  pl->defer_x = pl->dim == 1 && pl->big;   // the CGS2 below starts with w
  if (pl->p.precision == FDE_FP64) {
    tau_matvec<double>(pl, vj, &ks->scale[j], zj, w, st, skip, nullptr);
  } else if (pl->kin == 0 && pl->dim == 1 && pl->big && pl->p.prec != FDE_P_NONE && pl->p.prec != FDE_P_TRI) {
    // long 1D line, float32 P^{-1} alone: its first loader scales and casts
    // v_j, and the Toeplitz product's loader casts its result (stored as z_j)
    const Consts<float>& c = pl->c32;
    const float* pre = (pl->has_dinv && pl->dside == FDE_D_LEFT) ? c.dinv : nullptr;
    const float* post = (pl->has_dinv && pl->dside == FDE_D_RIGHT) ? c.dinv : nullptr;
    big_tau<float, double>(pl, vj, &ks->scale[j], pre, post, nullptr, nullptr, st, skip, nullptr, true);
    if (pl->blue)
      big_toep_ld<double>(pl, LdChirpPackToep<double, float>{c.cw, c.chirp, post, zj, pl->n1}, zj, pl->nu, 1.0, w,
                          st, skip, nullptr);
    else
      big_toep_ld<double>(pl, LdDstPackToep<double, float>{c.cw, c.W2x, post, zj, pl->n1, pl->rows.P}, zj, pl->nu,
                          1.0, w, st, skip, nullptr);
  } else {
    if (pl->kin == 0) {
      hipLaunchKernelGGL((scale_cast_kernel<double, float>), dim3(ew_grid(N)), dim3(256), 0, st, vj, pl->uf, N,
                         &ks->scale[j], skip, nullptr);
      tau_only<float>(pl, pl->uf, nullptr, pl->zf, st, skip);
    } else {
      hipLaunchKernelGGL((scale_cast_kernel<double, float>), dim3(ew_grid(N)), dim3(256), 0, st, vj, pl->Vf, N,
                         &ks->scale[j], skip, nullptr);
      inner_solve(pl, st);
    }
    hipLaunchKernelGGL((scale_cast_kernel<float, double>), dim3(ew_grid(N)), dim3(256), 0, st, pl->zf, zj, N,
                       nullptr, skip, nullptr);
    matvec_only<double>(pl, zj, w, pl->nu, 1.0, st, skip);
  }
  pl->defer_x = false;
  cgs2_givens<double>(pl, pl->V, w, j, ks, pl->hstat_dev, st, skip, nullptr);
}

// r = b - M x into basis slot 0 and its norm (cycle start / true residual).
static void residual(fde_plan pl, const double* b, const double* x, hipStream_t st) {
  double* tmp = pl->V + pl->ld;   // slot 1 is free between cycles
  matvec_only<double>(pl, x, tmp, pl->nu, 1.0, st, nullptr);
  norm_red<double>(pl, b, tmp, pl->V, pl->ks, EP_RESID, st);
}

// ---------------------------------------------------------------------------
// Residual-history trace.  With FDE_TRACE set to "1" (standard error) or to a
// file name (appended to), every solve writes one line per iteration with the
// solver's residual estimate and one per true-residual check, both relative
// to ||b||:
//   fde_trace solve=<k> solver=<gmres|pcg> kind=<est|true> iter=<i> relres=<v>
// The FGMRES estimates after the iterations of a cycle are rebuilt from the
// cycle's starting residual and the sines of its Givens rotations,
// beta |s_0| ... |s_j|, in the order the device formed them, so they equal
// the device's values.  The one-workgroup PCG solve reports its final
// estimate and true residual only.  Tracing adds host reads per cycle (PCG:
// per iteration) and is meant for inspection, not for timing.
// ---------------------------------------------------------------------------
struct Trace {
  FILE* f = nullptr;
  bool own = false;
  long id = 0;
  const char* solver = "";
  Trace(const char* solver_name) : solver(solver_name) {
    static std::mutex mu;
    static long next = 0;
    const char* e = std::getenv("FDE_TRACE");
    if (!e || !*e || std::strcmp(e, "0") == 0) return;
    if (std::strcmp(e, "1") == 0) {
      f = stderr;
    } else {
      f = std::fopen(e, "a");
      own = f != nullptr;
    }
    std::lock_guard<std::mutex> g(mu);
    id = next++;
  }
  ~Trace() {
    if (own) std::fclose(f);
  }
  bool on() const { return f != nullptr; }
  void line(const char* kind, int iter, double relres) const {
    if (f) std::fprintf(f, "fde_trace solve=%ld solver=%s kind=%s iter=%d relres=%.17g\n", id, solver, kind, iter, relres);
  }
};

// Estimates after the iterations iters0+1 .. iters of the cycle that just
// ended (its Givens sines are still in the state), then its true residual.
static fde_status trace_cycle(fde_plan pl, const Trace& tr, double beta0, int iters0, hipStream_t st) {
  const KState h = *pl->hks;
  const int k = h.iters - iters0;
  if (k > 0) {
    std::vector<double> sn(k);
    HIPCHK(hipMemcpyAsync(sn.data(), pl->ks->sn, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double g = beta0;
    for (int j = 0; j < k; ++j) {
      g = -sn[j] * g;
      tr.line("est", iters0 + j + 1, std::fabs(g) / h.bnorm);
    }
  }
  tr.line("true", h.iters, h.beta / h.bnorm);
  return FDE_OK;
}

static bool trace_requested() {
  const char* e = std::getenv("FDE_TRACE");
  return e && *e && std::strcmp(e, "0") != 0;
}

// The whole FGMRES solve in one workgroup (fde_fgmres1.hpp): float64 1D
// plans with n + 1 <= 1024 and a line-program preconditioner (measured
// against the multi-kernel path: 1.6x faster at n = 255, 1.3x at 511 and
// 1023, even at 2047, slower at 4095, where one CU's Gram-Schmidt passes
// over the basis cost more than the launches they replace).  A traced solve
// takes the multi-kernel path, which reports every iteration.
static bool gmres_one_workgroup(fde_plan pl) {
  return pl->dim == 1 && !pl->big && pl->p.prec != FDE_P_NONE && pl->p.prec != FDE_P_TRI &&
         pl->p.precision == FDE_FP64 && pl->rows.logP >= 3 && pl->rows.logP <= 10 && pl->m <= FG1_KMAX &&
         !trace_requested();
}

template <int LOGP>
static fde_status fgmres1d_launch(fde_plan pl, const LineArgs<double>& ta, const LineArgs<double>& ma,
                                  const double* b, double* x, hipStream_t st) {
  const Dir& d = pl->rows;
  const size_t lds = ((size_t)d.B * line_stride(d.P) + 2 * d.B + (size_t)d.P) * sizeof(cx<double>);
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&fgmres1d_kernel<LOGP>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  HIPCHK(attr);
  hipLaunchKernelGGL((fgmres1d_kernel<LOGP>), dim3(1), dim3(pcg_threads(LOGP)), lds, st, ta, ma, b, x, pl->V, pl->Z,
                     pl->ld, (int)pl->N, pl->m, pl->p.tol, pl->p.maxit, pl->ks);
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

static fde_status solve_gmres_one_workgroup(fde_plan pl, const double* b, double* x, fde_info* info,
                                            hipStream_t st) {
  const Consts<double>& c = consts<double>(pl);
  LineArgs<double> ta{};   // z = P^{-1}(s v), as tau_only (in, sc, out set per step)
  ta.pre = (pl->has_dinv && pl->dside == FDE_D_LEFT) ? c.dinv : nullptr;
  ta.post = (pl->has_dinv && pl->dside == FDE_D_RIGHT) ? c.dinv : nullptr;
  ta.fline = c.fzero;
  ta.felem = c.fx;
  ta.W2 = c.W2x;
  fill_line_args(pl->rows, ta);
  LineArgs<double> ma = toep_args<double>(pl, false, nullptr, nullptr);   // nu v + T-part v
  ma.bscale = pl->nu;
  ma.tscale = 1.0;
  fill_line_args(pl->rows, ma);
  switch (pl->rows.logP) {
    case 3: TRY(fgmres1d_launch<3>(pl, ta, ma, b, x, st)); break;
    case 4: TRY(fgmres1d_launch<4>(pl, ta, ma, b, x, st)); break;
    case 5: TRY(fgmres1d_launch<5>(pl, ta, ma, b, x, st)); break;
    case 6: TRY(fgmres1d_launch<6>(pl, ta, ma, b, x, st)); break;
    case 7: TRY(fgmres1d_launch<7>(pl, ta, ma, b, x, st)); break;
    case 8: TRY(fgmres1d_launch<8>(pl, ta, ma, b, x, st)); break;
    case 9: TRY(fgmres1d_launch<9>(pl, ta, ma, b, x, st)); break;
    default: TRY(fgmres1d_launch<10>(pl, ta, ma, b, x, st)); break;   // gmres_one_workgroup: logP <= 10
  }
  TRY(read_header(pl, pl->ks, st));
  const KState h = *pl->hks;
  if (!std::isfinite(h.bnorm)) return fail(FDE_ENONFINITE, "the right-hand side has a non-finite value");
  if (h.bnorm == 0.0) {
    if (info) *info = fde_info{0, 0, 0, 1, 0.0, 0.0, 0.0};
    return FDE_OK;
  }
  if (info) {
    info->iters = h.iters;
    info->inner_iters = 0;
    info->restarts = h.restarts;
    info->converged = h.conv;
    info->relres_true = h.beta / h.bnorm;
    info->relres_est = h.est / h.bnorm;
  }
  if (h.nonfinite) return fail(FDE_ENONFINITE, "a residual became non-finite");
  if (!h.conv) return fail(FDE_ENOTCONV, "tolerance not reached in %d iterations", h.iters);
  return FDE_OK;
}

static fde_status solve_gmres(fde_plan pl, const double* b, double* x, fde_info* info, hipStream_t st) {
  if (gmres_one_workgroup(pl)) return solve_gmres_one_workgroup(pl, b, x, info, st);
  const long N = pl->N;
  KState* ks = pl->ks;
  pl->pend_part = nullptr;
  hipLaunchKernelGGL(ks_init_kernel, dim3(1), dim3(1), 0, st, ks, pl->p.maxit, pl->m, pl->p.tol);
  hipLaunchKernelGGL(ks_init_kernel, dim3(1), dim3(1), 0, st, pl->ksi, 1 << 30, std::max(1, pl->kin), 0.0);
  norm_red<double>(pl, b, nullptr, nullptr, ks, EP_BNORM, st);
  hipLaunchKernelGGL(ks_settol_kernel, dim3(1), dim3(1), 0, st, ks);
  residual(pl, b, x, st);
  HIPCHK(hipGetLastError());
  TRY(read_header(pl, ks, st));
  if (!std::isfinite(pl->hks->bnorm)) return fail(FDE_ENONFINITE, "the right-hand side has a non-finite value");
  if (pl->hks->bnorm == 0.0) {
    hipLaunchKernelGGL(axpby_kernel, dim3(ew_grid(N)), dim3(256), 0, st, 0.0, b, 0.0, (const double*)nullptr, x, N);
    HIPCHK(hipStreamSynchronize(st));
    if (info) *info = fde_info{0, 0, 0, 1, 0.0, 0.0, 0.0};
    return FDE_OK;
  }
  Trace tr("gmres");
  tr.line("true", 0, pl->hks->beta / pl->hks->bnorm);
  int restarts = 0;
  while (!pl->hks->conv && !pl->hks->nonfinite && pl->hks->iters < pl->p.maxit) {
    const double beta0 = pl->hks->beta;
    const int iters0 = pl->hks->iters;
    pl->hstat[0] = 0.0;
    for (int j = 0; j < pl->m; ++j) {
      if (j >= 2) {
        HIPCHK(hipEventSynchronize(pl->ev[(j - 2) & 3]));
        if (*(volatile double*)&pl->hstat[0] != 0.0) break;
      }
      outer_step(pl, j, st);
      HIPCHK(hipEventRecord(pl->ev[j & 3], st));
    }
    hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(256), 0, st, ks, (const int*)nullptr);
    hipLaunchKernelGGL((update_kernel<double, double>), dim3(ew_grid(N)), dim3(RED_THREADS), 0, st, pl->Z, pl->ld, x, x,
                       N, ks, (const double*)nullptr, (const int*)nullptr);
    residual(pl, b, x, st);
    HIPCHK(hipGetLastError());
    TRY(read_header(pl, ks, st));
    if (tr.on()) TRY(trace_cycle(pl, tr, beta0, iters0, st));
    if (!pl->hks->conv) ++restarts;
  }
  const KState h = *pl->hks;
  if (info) {
    info->iters = h.iters;
    info->restarts = restarts;
    info->converged = h.conv;
    info->relres_true = h.beta / h.bnorm;
    info->relres_est = h.est / h.bnorm;
    info->inner_iters = 0;
    if (pl->p.precision == FDE_MIXED) {
      TRY(read_header(pl, pl->ksi, st));
      info->inner_iters = pl->hks->iters;
    }
  }
  if (h.nonfinite) return fail(FDE_ENONFINITE, "a residual became non-finite");
  if (!h.conv) return fail(FDE_ENOTCONV, "tolerance not reached in %d iterations", h.iters);
  return FDE_OK;
}

template <typename T>
static void dot_red(fde_plan pl, const T* a, const T* b, KState* ks, int emode, hipStream_t st, const int* skip) {
  const int G = red_grid(pl->N, (long)RED_THREADS * 8);
  hipLaunchKernelGGL((dot_kernel<T>), dim3(G), dim3(RED_THREADS), 0, st, a, b, pl->N, pl->part, ks, emode, skip);
  finalize(pl, G, 1, ks, FK_DOT, emode, 0, nullptr, st, skip, nullptr);
}

// The whole PCG solve in a single workgroup (fde_pcg.hpp): 1D plans whose
// line fits one workgroup, with a line-program preconditioner.
static bool pcg_one_workgroup(fde_plan pl) {
  return pl->dim == 1 && !pl->big && pl->p.prec != FDE_P_NONE && pl->p.prec != FDE_P_TRI && pl->rows.logP >= 3 &&
         pl->rows.logP <= 12;
}

struct PcgArgs {
  LineArgs<double> ta, ma;
  const double* b;
  double *x, *r, *p, *q, *z;
};

template <int LOGP>
static fde_status pcg1d_launch(fde_plan pl, const PcgArgs& g, hipStream_t st) {
  const Dir& d = pl->rows;
  const size_t lds = ((size_t)d.B * line_stride(d.P) + 2 * d.B + (size_t)d.P) * sizeof(cx<double>);
  // the kernel also holds a few hundred bytes of static LDS, so the dynamic
  // size asked for is the launch's own (one value per LOGP), not the CU's 160 KB
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&pcg1d_kernel<LOGP>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  HIPCHK(attr);
  hipLaunchKernelGGL((pcg1d_kernel<LOGP>), dim3(1), dim3(pcg_threads(LOGP)), lds, st, g.ta, g.ma, g.b, g.x, g.r,
                     g.p, g.q, g.z, (int)pl->N, pl->p.tol, pl->p.maxit, pl->ks);
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

static fde_status solve_pcg_one_workgroup(fde_plan pl, const double* b, double* x, fde_info* info,
                                          hipStream_t st) {
  const Consts<double>& c = consts<double>(pl);
  PcgArgs g{};
  g.b = b;
  g.x = x;
  g.r = pl->V;
  g.p = pl->V + pl->ld;
  g.q = pl->V + 2 * pl->ld;
  g.z = pl->Z;
  g.ta.in = g.r;   // z = P^{-1} r, as tau_only
  g.ta.pre = (pl->has_dinv && pl->dside == FDE_D_LEFT) ? c.dinv : nullptr;
  g.ta.post = (pl->has_dinv && pl->dside == FDE_D_RIGHT) ? c.dinv : nullptr;
  g.ta.fline = c.fzero;
  g.ta.felem = c.fx;
  g.ta.W2 = c.W2x;
  g.ta.out = g.z;
  fill_line_args(pl->rows, g.ta);
  g.ma = toep_args<double>(pl, false, nullptr, nullptr);   // q = M p, as matvec_only
  g.ma.in = g.p;
  g.ma.bscale = pl->nu;
  g.ma.tscale = 1.0;
  g.ma.out = g.q;
  fill_line_args(pl->rows, g.ma);
  switch (pl->rows.logP) {
    case 3: TRY(pcg1d_launch<3>(pl, g, st)); break;
    case 4: TRY(pcg1d_launch<4>(pl, g, st)); break;
    case 5: TRY(pcg1d_launch<5>(pl, g, st)); break;
    case 6: TRY(pcg1d_launch<6>(pl, g, st)); break;
    case 7: TRY(pcg1d_launch<7>(pl, g, st)); break;
    case 8: TRY(pcg1d_launch<8>(pl, g, st)); break;
    case 9: TRY(pcg1d_launch<9>(pl, g, st)); break;
    case 10: TRY(pcg1d_launch<10>(pl, g, st)); break;
    case 11: TRY(pcg1d_launch<11>(pl, g, st)); break;
    default: TRY(pcg1d_launch<12>(pl, g, st)); break;   // pcg_one_workgroup: logP <= 12
  }
  TRY(read_header(pl, pl->ks, st));
  const KState h = *pl->hks;
  if (!std::isfinite(h.bnorm)) return fail(FDE_ENONFINITE, "the right-hand side has a non-finite value");
  if (h.bnorm == 0.0) {
    if (info) *info = fde_info{0, 0, 0, 1, 0.0, 0.0, 0.0};
    return FDE_OK;
  }
  {
    Trace tr("pcg");
    tr.line("est", h.iters, h.est / h.bnorm);
    tr.line("true", h.iters, h.beta / h.bnorm);
  }
  if (info) {
    info->iters = h.iters;
    info->inner_iters = 0;
    info->restarts = h.restarts;
    info->converged = h.conv;
    info->relres_true = h.beta / h.bnorm;
    info->relres_est = h.est / h.bnorm;
  }
  if (h.nonfinite) return fail(FDE_ENONFINITE, "a residual became non-finite");
  if (!h.conv) return fail(FDE_ENOTCONV, "tolerance not reached in %d iterations", h.iters);
  return FDE_OK;
}

static fde_status solve_pcg(fde_plan pl, const double* b, double* x, fde_info* info, hipStream_t st) {
  if (pcg_one_workgroup(pl)) return solve_pcg_one_workgroup(pl, b, x, info, st);
  const long N = pl->N;
  KState* ks = pl->ks;
  const int* skip = &ks->done;
  double* r = pl->V;
  double* p = pl->V + pl->ld;
  double* q = pl->V + 2 * pl->ld;
  double* z = pl->Z;
  hipLaunchKernelGGL(ks_init_kernel, dim3(1), dim3(1), 0, st, ks, pl->p.maxit, 1, pl->p.tol);
  norm_red<double>(pl, b, nullptr, nullptr, ks, EP_BNORM, st);
  hipLaunchKernelGGL(ks_settol_kernel, dim3(1), dim3(1), 0, st, ks);
  matvec_only<double>(pl, x, q, pl->nu, 1.0, st, nullptr);
  norm_red<double>(pl, b, q, r, ks, EP_RESID, st);
  HIPCHK(hipGetLastError());
  TRY(read_header(pl, ks, st));
  if (!std::isfinite(pl->hks->bnorm)) return fail(FDE_ENONFINITE, "the right-hand side has a non-finite value");
  if (pl->hks->bnorm == 0.0) {
    hipLaunchKernelGGL(axpby_kernel, dim3(ew_grid(N)), dim3(256), 0, st, 0.0, b, 0.0, (const double*)nullptr, x, N);
    HIPCHK(hipStreamSynchronize(st));
    if (info) *info = fde_info{0, 0, 0, 1, 0.0, 0.0, 0.0};
    return FDE_OK;
  }
  const int G = red_grid(N, (long)RED_THREADS * 8);
  Trace tr("pcg");
  tr.line("true", 0, pl->hks->beta / pl->hks->bnorm);
  int restarts = 0;
  while (!pl->hks->conv && !pl->hks->nonfinite && pl->hks->iters < pl->p.maxit) {
    // (re)start: z = P^{-1} r, rz = r.z, p = z
    tau_only<double>(pl, r, nullptr, z, st, skip);
    dot_red<double>(pl, r, z, ks, EP_CG_RZ, st, skip);
    hipLaunchKernelGGL((scale_cast_kernel<double, double>), dim3(ew_grid(N)), dim3(256), 0, st, z, p, N,
                       (const double*)nullptr, skip, (const int*)nullptr);
    pl->hstat[0] = 0.0;
    for (int it = 0; it < pl->p.maxit; ++it) {
      if (it >= 2) {
        HIPCHK(hipEventSynchronize(pl->ev[(it - 2) & 3]));
        if (*(volatile double*)&pl->hstat[0] != 0.0) break;
      }
      matvec_only<double>(pl, p, q, pl->nu, 1.0, st, skip);
      dot_red<double>(pl, p, q, ks, EP_CG_PQ, st, skip);
      hipLaunchKernelGGL(cg_update_kernel, dim3(G), dim3(RED_THREADS), 0, st, x, r, p, q, N, pl->part, ks,
                         pl->hstat_dev, skip);
      finalize(pl, G, 1, ks, FK_NORM, EP_CG_R, 0, pl->hstat_dev, st, skip, nullptr);
      tau_only<double>(pl, r, nullptr, z, st, skip);
      dot_red<double>(pl, r, z, ks, EP_CG_RZ, st, skip);
      hipLaunchKernelGGL(cg_direction_kernel, dim3(ew_grid(N)), dim3(256), 0, st, p, z, N, ks, skip);
      HIPCHK(hipEventRecord(pl->ev[it & 3], st));
      if (tr.on()) {
        const int before = pl->hks->iters;
        TRY(read_header(pl, ks, st));
        if (pl->hks->iters == before) break;   // the iteration was skipped: the solve had stopped
        tr.line("est", pl->hks->iters, pl->hks->est / pl->hks->bnorm);
        if (pl->hks->done) break;
      }
    }
    // true residual
    matvec_only<double>(pl, x, q, pl->nu, 1.0, st, nullptr);
    norm_red<double>(pl, b, q, r, ks, EP_RESID, st);
    HIPCHK(hipGetLastError());
    TRY(read_header(pl, ks, st));
    tr.line("true", pl->hks->iters, pl->hks->beta / pl->hks->bnorm);
    if (!pl->hks->conv) ++restarts;
  }
  const KState h = *pl->hks;
  if (info) {
    info->iters = h.iters;
    info->inner_iters = 0;
    info->restarts = restarts;
    info->converged = h.conv;
    info->relres_true = h.beta / h.bnorm;
    info->relres_est = h.est / h.bnorm;
  }
  if (h.nonfinite) return fail(FDE_ENONFINITE, "a residual became non-finite");
  if (!h.conv) return fail(FDE_ENOTCONV, "tolerance not reached in %d iterations", h.iters);
  return FDE_OK;
}

extern "C" fde_status fde_solve(fde_plan pl, const double* b, double* x, fde_info* info, void* stream) {
  if (!pl || !b || !x) return fail(FDE_EINVAL, "NULL argument");
  ProbePlanScope pps(pl);
  auto t0 = std::chrono::steady_clock::now();
  fde_status s = pl->p.solver == FDE_S_PCG ? solve_pcg(pl, b, x, info, (hipStream_t)stream)
                                           : solve_gmres(pl, b, x, info, (hipStream_t)stream);
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

// ---------------------------------------------------------------------------
// Allocation-free one-shot 1D PCG solve (fde_pcg1d_solve_noalloc)
//
// The same set-up arithmetic and the same one-workgroup PCG kernel as
// fde_assemble + fde_solve for a 1D PCG plan whose line fits one workgroup,
// with every device table and work vector in one static device array instead
// of plan buffers.  The coefficient arrays are read where the caller keeps
// them.  Nothing in the array needs to start at zero: every entry is written
// before it is read in the same call.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)512 << 10;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];   // device address of `scratch`, per device

// Device address of `scratch` on the current device, looked up once per device
// (each device holds its own copy at its own address).
static fde_status scratch_address(unsigned char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(FDE_EUNSUPPORTED, "device %d: the allocation-free entry point handles devices 0..%d", dev,
                NOALLOC_MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FDE_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return FDE_OK;
}

struct NoallocLayout {
  size_t stats, dinv, dinvf, fx, fzero, W2, lam, vec, ks, total;
};

static NoallocLayout noalloc_layout(int n, long ld) {
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t P = (size_t)n + 1;
  NoallocLayout L{};
  size_t o = 0;
  L.stats = o;  o = up(o + (3 + 3 * 256) * sizeof(double));
  L.dinv = o;   o = up(o + (size_t)n * sizeof(double));
  L.dinvf = o;  o = up(o + (size_t)n * sizeof(float));
  L.fx = o;     o = up(o + (size_t)n * sizeof(double));
  L.fzero = o;  o = up(o + sizeof(double));
  L.W2 = o;     o = up(o + 2 * P * sizeof(cx<double>));
  L.lam = o;    o = up(o + (P + 1) * sizeof(cx<double>));
  L.vec = o;    o = up(o + 4 * (size_t)ld * sizeof(double));   // r, p, q, z
  L.ks = o;     o = up(o + sizeof(KState));
  L.total = o;
  return L;
}

extern "C" fde_status fde_pcg1d_solve_noalloc(const fde_params* p, const double* dplus, const double* dminus,
                                              const double* b, double* x, fde_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!dplus || !dminus || !b || !x) return fail(FDE_EINVAL, "NULL argument");
  TRY(validate(p));
  if (p->dim != 1 || p->solver != FDE_S_PCG || p->precision != FDE_FP64)
    return fail(FDE_EUNSUPPORTED, "the allocation-free solve is the 1D float64 PCG (dim = 1, FDE_S_PCG, FDE_FP64)");
  if (p->prec != FDE_P_TAU && p->prec != FDE_P_TAU_HAT && p->prec != FDE_P_TILDE)
    return fail(FDE_EUNSUPPORTED, "the allocation-free solve takes FDE_P_TAU, FDE_P_TAU_HAT or FDE_P_TILDE");
  const int n = p->n[0];
  if (n + 1 < 8 || n + 1 > 4096)
    return fail(FDE_EUNSUPPORTED, "the allocation-free solve needs 8 <= n + 1 <= 4096 (got n = %d)", n);
  hipStream_t st = static_cast<hipStream_t>(stream);

  // host description of the plan (no device buffers of its own)
  fde_plan_s pl;
  pl.p = *p;
  pl.dim = 1;
  pl.n1 = n;
  pl.n2 = 1;
  pl.N = n;
  pl.ld = ((long)n + 63) / 64 * 64;
  pl.hx = (p->hi[0] - p->lo[0]) / (n + 1);
  pl.hxa = std::pow(pl.hx, p->alpha[0]);
  pl.nu = (p->time == FDE_T_EULER ? 1.0 : 2.0) * pl.hxa / p->dt;
  pl.dside = p->dside;
  pl.m = p->restart;
  pl.rows.n = n;
  pl.rows.P = n + 1;
  pl.rows.logP = ilog2(pl.rows.P);
  pl.rows.nlines = 1;
  pl.rows.ls = n;
  pl.rows.es = 1;
  choose_tile(pl.rows);
  if (!pcg_one_workgroup(&pl)) return fail(FDE_EUNSUPPORTED, "this size does not run as one workgroup");
  const NoallocLayout L = noalloc_layout(n, pl.ld);
  if (L.total > NOALLOC_SCRATCH_BYTES)
    return fail(FDE_EUNSUPPORTED, "n = %d needs %zu bytes of scratch, more than the static %zu", n, L.total,
                NOALLOC_SCRATCH_BYTES);
  unsigned char* base = nullptr;
  TRY(scratch_address(&base));
  pl.stats_buf = reinterpret_cast<double*>(base + L.stats);

  // coefficients: validated where the caller keeps them, read there by the kernel
  double stats[2][3];
  const double* src[2] = {dplus, dminus};
  for (int i = 0; i < 2; ++i) {
    TRY(coef_stats(&pl, src[i], stats[i], st));
    if (stats[i][2] != 0.0) return fail(FDE_EINVAL, "coefficient array %d has a non-finite value", i);
    if (stats[i][0] < 0.0) return fail(FDE_EINVAL, "coefficient array %d has a negative value", i);
  }
  pl.c64.dp = const_cast<double*>(dplus);   // read only
  pl.c64.dm = const_cast<double*>(dminus);
  const bool constant = stats[0][0] == stats[0][1] && stats[1][0] == stats[0][0] && stats[1][1] == stats[0][0];
  const double cval = stats[0][0];
  pl.has_dinv = p->prec == FDE_P_TAU;
  if (pl.has_dinv) {
    pl.c64.dinv = reinterpret_cast<double*>(base + L.dinv);
    hipLaunchKernelGGL((dinv_kernel<false>), dim3(256), dim3(256), 0, st, dplus, dminus, (const double*)nullptr,
                       (const double*)nullptr, pl.c64.dinv, reinterpret_cast<float*>(base + L.dinvf), (long)n);
    HIPCHK(hipGetLastError());
    double ds[3];
    TRY(coef_stats(&pl, pl.c64.dinv, ds, st));
    if (ds[2] != 0.0 || !(ds[0] > 0.0))
      return fail(FDE_EINVAL, "D = mean of the coefficients has a zero (d+ and d- share a zero)");
  }
  // symbol samples (as fde_assemble)
  std::vector<double> fx(n), fz(1, 0.0);
  for (int i = 0; i < n; ++i) fx[i] = symbol(p->alpha[0], M_PI * (i + 1) / (double)(n + 1), p->weights);
  if (p->prec == FDE_P_TAU) {
    const double shift = std::isnan(p->shift) ? (constant ? pl.nu / cval : 0.0) : p->shift;
    for (int i = 0; i < n; ++i) fx[i] += shift;
  } else if (p->prec == FDE_P_TAU_HAT) {
    if (!constant || !(cval > 0.0)) return fail(FDE_EINVAL, "P_hat needs constant, equal, positive d+ and d-");
    for (int i = 0; i < n; ++i) fx[i] = cval * fx[i];
    for (int i = 0; i < n; ++i) fx[i] += pl.nu;
  } else {
    std::vector<double> hp(n), hm(n);
    HIPCHK(hipMemcpyAsync(hp.data(), dplus, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hm.data(), dminus, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
      fx[i] *= 0.5 * (hp[i] + hm[i]);
      if (!(fx[i] > 0.0)) return fail(FDE_EINVAL, "P_tilde: D_j p(theta_j) must be positive");
    }
  }
  std::vector<std::complex<double>> W2, lam;
  direction_host(p->alpha[0], n, p->weights, W2, lam);
  pl.c64.fx = reinterpret_cast<double*>(base + L.fx);
  pl.c64.fzero = reinterpret_cast<double*>(base + L.fzero);
  pl.c64.W2x = reinterpret_cast<cx<double>*>(base + L.W2);
  pl.c64.lamx = reinterpret_cast<cx<double>*>(base + L.lam);
  // std::complex<double> and cx<double> are both two adjacent doubles (real, imaginary)
  static_assert(sizeof(std::complex<double>) == sizeof(cx<double>), "complex layouts differ");
  HIPCHK(hipMemcpyAsync(pl.c64.fx, fx.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pl.c64.fzero, fz.data(), sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pl.c64.W2x, W2.data(), W2.size() * sizeof(cx<double>), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pl.c64.lamx, lam.data(), lam.size() * sizeof(cx<double>), hipMemcpyHostToDevice, st));
  pl.V = reinterpret_cast<double*>(base + L.vec);   // r, p, q
  pl.Z = pl.V + 3 * pl.ld;                          // z
  pl.ks = reinterpret_cast<KState*>(base + L.ks);
  KState hk{};
  pl.hks = &hk;   // the header is read back into host memory of this call
  const fde_status s = solve_pcg_one_workgroup(&pl, b, x, info, st);   // synchronises st
  pl.hks = nullptr;
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return s;
}
