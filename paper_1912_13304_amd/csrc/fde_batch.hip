// C ABI of the batched solver (fde_batch_* in include/fde.h): assembly of
// many independent 1D instances, the persistent solve launch, time stepping
// through a captured graph, and the launch-configuration autotuner.
//
// Assembly computes every table on the host in float64 (Grunwald weights,
// circulant eigenvalues, symbol samples, chirps and chirp-filter spectra) and
// uploads them, with each instance's Krylov workspace, into one device arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/fde.h"
#include "fde_batch.hpp"
#include "fde_host.hpp"

using namespace fde;
using namespace fde::bat;

namespace {

// Queue reset before a launch (a kernel, so that it can sit in a graph).
__global__ void batch_reset_kernel(unsigned* queue) {
  if (threadIdx.x == 0) queue[0] = 0u;
}

// Advances the step counter of a time-stepping run.
__global__ void batch_advance_kernel(int* step) {
  if (threadIdx.x == 0) step[0] += 1;
}


// Launch variants: 0 = 512 threads, radix 8; 1 = 512 threads, radix 4.
// Variants 2 and 3 (256 threads) are disabled: the 256-thread build took a
// GPU memory fault whose cause was not found (a CPU emulation of the same
// code with per-array bounds checking runs clean), so they are rejected.
constexpr int VARIANTS_ENABLED = 2;
constexpr long BATCH_NMAX = 65535;
constexpr size_t ALIGN = 256;

size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Geo {
  long n, Qt, Qs;
  int logQt, logQs;
  bool blue, staged;
};

Geo geometry(const fde_params& p) {
  Geo g{};
  g.n = p.n[0];
  g.logQt = ilog2(g.n);
  g.Qt = 1L << g.logQt;
  g.blue = !is_pow2(g.n + 1);
  g.logQs = g.blue ? ilog2(2 * g.n - 1) : ilog2(g.n + 1);
  g.Qs = 1L << g.logQs;
  g.staged = 2 * g.Qt > Cap<double>::value || g.Qs > Cap<double>::value;
  return g;
}

// Bytes of one instance's tables and workspace in the arena, sub-arrays aligned.
struct Layout {
  size_t tab64[7], tab32[7];   // dp dm dinv finv lam chirp bhat
  size_t tri64[11], tri32[11]; // P_tri: ai cp den sv sw (n), ar cr ra rb rc (p), work y (n)
  size_t tcs;                  // P_tri chunk starts (p + 1 ints)
  int tp;
  size_t V, Z, b, t, Vf, uf, zf, tf, fa, fb;
  size_t total;
};

Layout layout(const fde_params& p) {
  const Geo g = geometry(p);
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += up(std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t n = g.n;
  for (int k = 0; k < 2; ++k) {
    const size_t r = k == 0 ? 8 : 4;
    size_t* t = k == 0 ? L.tab64 : L.tab32;
    t[0] = take(n * r);
    t[1] = take(n * r);
    t[2] = take(n * r);
    t[3] = take(n * r);
    t[4] = take((g.Qt + 1) * 2 * r);
    t[5] = take(g.blue ? (n + 1) * 2 * r : 0);
    t[6] = take(g.blue ? g.Qs * 2 * r : 0);
  }
  const bool tri = p.prec == FDE_P_TRI;
  L.tp = tri ? (int)std::max(1L, std::min((long)TRI_CHUNKS, g.n / 2)) : 0;
  for (int k = 0; k < 2; ++k) {
    const size_t r = k == 0 ? 8 : 4;
    size_t* t = k == 0 ? L.tri64 : L.tri32;
    for (int a = 0; a < 11; ++a) t[a] = take(tri ? (a < 5 || a == 10 ? n : (size_t)L.tp) * r : 0);
  }
  L.tcs = take(tri ? (size_t)(L.tp + 1) * 4 : 0);
  const size_t m = p.restart;
  const bool mixed = p.precision == FDE_MIXED;
  const size_t kin = mixed ? p.inner_steps : 0;
  L.V = take((m + 1) * n * 8);
  L.Z = take(m * n * 8);
  L.b = take(n * 8);
  L.t = take(n * 8);
  L.Vf = take(mixed && kin > 0 ? (kin + 1) * n * 4 : 0);
  L.uf = take(mixed ? n * 4 : 0);
  L.zf = take(mixed ? n * 4 : 0);
  L.tf = take(mixed ? n * 4 : 0);
  L.fa = take(g.staged ? (size_t)std::max(2 * g.Qt, g.Qs) * 16 : 0);
  L.fb = take(g.staged ? (size_t)std::max(g.Qt, g.Qs) * 16 : 0);
  L.total = o;
  return L;
}

fde_status validate_one(const fde_params* p, int i) {
  if (p->dim != 1) return fail(FDE_EINVAL, "instance %d: batched solves are 1D (dim = %d)", i, p->dim);
  if (p->n[0] < 1) return fail(FDE_EINVAL, "instance %d: n must be >= 1 (got %d)", i, p->n[0]);
  if (p->n[0] > BATCH_NMAX)
    return fail(FDE_EUNSUPPORTED, "instance %d: n = %d exceeds %ld", i, p->n[0], BATCH_NMAX);
  if (!(p->alpha[0] > 1.0 && p->alpha[0] < 2.0))
    return fail(FDE_EINVAL, "instance %d: alpha must lie in (1,2) (got %g)", i, p->alpha[0]);
  if (!(p->hi[0] > p->lo[0]) || !std::isfinite(p->hi[0]) || !std::isfinite(p->lo[0]))
    return fail(FDE_EINVAL, "instance %d: empty domain", i);
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(FDE_EINVAL, "instance %d: dt must be > 0", i);
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(FDE_EINVAL, "instance %d: tol must be > 0", i);
  if (p->weights != FDE_W_SHIFTED && p->weights != FDE_W_WEIGHTED) return fail(FDE_EINVAL, "instance %d: bad weights", i);
  if (p->time != FDE_T_EULER && p->time != FDE_T_CN) return fail(FDE_EINVAL, "instance %d: bad time scheme", i);
  if (p->prec < FDE_P_NONE || p->prec > FDE_P_TRI) return fail(FDE_EINVAL, "instance %d: bad preconditioner", i);
  if (p->dside != FDE_D_LEFT && p->dside != FDE_D_RIGHT) return fail(FDE_EINVAL, "instance %d: bad dside", i);
  if (p->solver != FDE_S_GMRES)
    return fail(FDE_EUNSUPPORTED, "instance %d: batched solves use FGMRES (solver = FDE_S_GMRES)", i);
  if (p->restart < 1 || p->restart > MMAX) return fail(FDE_EINVAL, "instance %d: restart must be in 1..32", i);
  if (p->maxit < 1) return fail(FDE_EINVAL, "instance %d: maxit must be >= 1", i);
  if (p->precision != FDE_FP64 && p->precision != FDE_MIXED) return fail(FDE_EINVAL, "instance %d: bad precision", i);
  if (p->precision == FDE_MIXED && (p->inner_steps < 0 || p->inner_steps > MMAX))
    return fail(FDE_EINVAL, "instance %d: inner_steps must be in 0..32", i);
  if (!std::isnan(p->shift) && !std::isfinite(p->shift))
    return fail(FDE_EINVAL, "instance %d: shift must be finite or NaN", i);
  return FDE_OK;
}

fde_status validate_all(const fde_params* ps, int count) {
  if (!ps) return fail(FDE_EINVAL, "params is NULL");
  if (count < 1) return fail(FDE_EINVAL, "count must be >= 1 (got %d)", count);
  for (int i = 0; i < count; ++i) TRY(validate_one(&ps[i], i));
  return FDE_OK;
}

template <typename T>
void put(std::vector<unsigned char>& arena, size_t at, const std::vector<double>& v) {
  T* d = reinterpret_cast<T*>(arena.data() + at);
  for (size_t i = 0; i < v.size(); ++i) d[i] = (T)v[i];
}

template <typename T>
void put_cx(std::vector<unsigned char>& arena, size_t at, const std::vector<std::complex<double>>& v) {
  T* d = reinterpret_cast<T*>(arena.data() + at);
  for (size_t i = 0; i < v.size(); ++i) {
    d[2 * i] = (T)v[i].real();
    d[2 * i + 1] = (T)v[i].imag();
  }
}

}  // namespace

struct fde_batch_s {
  int count = 0;
  std::vector<fde_params> p;
  std::vector<long> off;
  long total = 0;
  int logTW = 0;
  Inst* dinst = nullptr;
  std::vector<int> hq;   // host copy of the queue order
  unsigned* queue = nullptr;
  int* step = nullptr;
  Info* info = nullptr;
  long info_cap = 0;
  cx<double>* tw64 = nullptr;
  cx<float>* tw32 = nullptr;
  double* tune_x = nullptr;
  std::vector<void*> allocs;
  size_t bytes = 0;
  fde_batch_cfg cfg{0, 0, 1, 0.0, 0};
  int cus = 256;
  int dev = 0;
  // captured graph of one time step
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* gx = nullptr;
  fde_batch_cfg gcfg{-1, -1, -1, 0.0, -1};
  std::vector<Info> hinfo;
  // instances taken out of the persistent launch (cfg.split of them, the
  // largest estimated work) and solved on the plan path by worker threads
  std::vector<double> cost;             // per-iteration work model of each instance
  std::vector<int> last_iters;          // iterations of each instance's last solve (0: not known)
  std::vector<const double*> hdp, hdm;  // the instance's coefficients in the arena
  std::vector<double*> hb;              // the instance's right-hand-side buffer in the arena
  std::vector<int> split_idx;           // current split set, largest estimated work first
  std::vector<fde_plan> plans;          // per instance, built when it is first split
  std::vector<hipStream_t> wstreams;    // worker streams
  int* order_q = nullptr;               // queue order of the launch (count entries, nq used)
  int nq = 0;
};

namespace {

template <typename T>
fde_status balloc(fde_batch bt, T** ptr, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(FDE_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  bt->allocs.push_back(q);
  bt->bytes += bytes;
  *ptr = static_cast<T*>(q);
  return FDE_OK;
}

void drop_graph(fde_batch bt) {
  if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->gexec = nullptr;
  bt->graph = nullptr;
  bt->gx = nullptr;
  bt->gcfg = fde_batch_cfg{-1, -1, -1, 0.0, -1};
}

void destroy_impl(fde_batch bt) {
  if (!bt) return;
  (void)hipDeviceSynchronize();
  drop_graph(bt);
  for (fde_plan pl : bt->plans)
    if (pl) fde_destroy(pl);
  for (hipStream_t w : bt->wstreams) (void)hipStreamDestroy(w);
  if (bt->cap) (void)hipStreamDestroy(bt->cap);
  for (void* q : bt->allocs) (void)hipFree(q);
  delete bt;
}

template <int NT, int RAD>
fde_status launch_v(const Args& a, int grid, hipStream_t st) {
  const size_t lds = sizeof(Shm<NT>);
  // function-local static: initialised once, thread-safe
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_kernel<NT, RAD>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  HIPCHK(attr);
  hipLaunchKernelGGL((batch_kernel<NT, RAD>), dim3(grid), dim3(NT), lds, st, a);
  HIPCHK(hipGetLastError());
  return FDE_OK;
}

// reset queue, persistent solve launch (and, for a time step, the step counter advance)
fde_status enqueue(fde_batch bt, const fde_batch_cfg& c, int mode, const double* b, double* x, const int* step,
                   hipStream_t st, int single = 0) {
  Args a{};
  a.inst = bt->dinst;
  a.count = bt->count;
  a.mode = mode;
  a.order = bt->order_q;
  a.nq = bt->nq;
  a.queue = bt->queue;
  a.tw64 = bt->tw64;
  a.tw32 = bt->tw32;
  a.logTW = bt->logTW;
  a.bin = b;
  a.x = x;
  a.info = bt->info;
  a.step = step;
  a.single = single;
  const int grid = std::max(1, std::min(c.grid > 0 ? c.grid : 2 * bt->cus, bt->count));
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, bt->queue);
  HIPCHK(hipGetLastError());
  switch (c.variant) {
    case 0: TRY((launch_v<512, 8>(a, grid, st))); break;
    case 1: TRY((launch_v<512, 4>(a, grid, st))); break;
    default: return fail(FDE_EUNSUPPORTED, "launch variant %d is disabled", c.variant);
  }
  if (step) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, st, bt->step);
    HIPCHK(hipGetLastError());
  }
  return FDE_OK;
}

fde_status ensure_info(fde_batch bt, long entries) {
  if (entries <= bt->info_cap) return FDE_OK;
  drop_graph(bt);   // the graph holds the old buffer
  Info* q = nullptr;
  TRY(balloc(bt, &q, (size_t)entries));
  bt->info = q;     // the old buffer stays allocated until destroy
  bt->info_cap = entries;
  return FDE_OK;
}

fde_status collect(fde_batch bt, long entries, fde_info* out, double seconds, hipStream_t st,
                   const std::vector<std::pair<long, Info>>* plan_info = nullptr) {
  bt->hinfo.resize(entries);
  HIPCHK(hipMemcpyAsync(bt->hinfo.data(), bt->info, entries * sizeof(Info), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (plan_info)
    for (const auto& e : *plan_info) bt->hinfo[e.first] = e.second;
  for (long e = 0; e < entries; ++e) bt->last_iters[e % bt->count] = bt->hinfo[e].iters;
  bool nonfinite = false, notconv = false;
  for (long e = 0; e < entries; ++e) {
    const Info& r = bt->hinfo[e];
    if (r.nonfinite) nonfinite = true;
    else if (!r.converged) notconv = true;
    if (out) {
      out[e].iters = r.iters;
      out[e].inner_iters = r.inner_iters;
      out[e].restarts = r.restarts;
      out[e].converged = r.converged;
      out[e].relres_true = r.relres_true;
      out[e].relres_est = r.relres_est;
      out[e].seconds = seconds;
    }
  }
  if (nonfinite) return fail(FDE_ENONFINITE, "a right-hand side or residual became non-finite");
  if (notconv) return fail(FDE_ENOTCONV, "some instances did not reach the tolerance");
  return FDE_OK;
}

constexpr int SPLIT_WORKERS = 4;   // worker threads (and streams) of the plan-path instances

// Estimated work of instance i: its per-iteration model times the iterations
// of its last solve (1 before any).
double est_work(const fde_batch bt, int i) {
  return (bt->last_iters[i] > 0 ? (double)bt->last_iters[i] : 1.0) * bt->cost[i];
}

// The split set of configuration c (its c.split instances of largest
// estimated work, largest first), their plans (built here, on the calling
// thread, before any launch of this call), the worker streams, and the queue
// order of the persistent launch without them (largest estimated work first
// with c.lpt, else as given), copied to the device on `st`.
fde_status prepare_queue(fde_batch bt, const fde_batch_cfg& c, hipStream_t st) {
  const int count = bt->count;
  const int k = std::max(0, std::min(c.split, count));
  std::vector<int> idx(count);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return est_work(bt, a) > est_work(bt, b); });
  bt->split_idx.assign(idx.begin(), idx.begin() + k);
  std::vector<char> split(count, 0);
  for (int i : bt->split_idx) split[i] = 1;
  bt->hq.clear();
  if (c.lpt) {
    for (int i : idx)
      if (!split[i]) bt->hq.push_back(i);
  } else {
    for (int i = 0; i < count; ++i)
      if (!split[i]) bt->hq.push_back(i);
  }
  bt->nq = (int)bt->hq.size();
  if (bt->nq) HIPCHK(hipMemcpyAsync(bt->order_q, bt->hq.data(), bt->nq * sizeof(int), hipMemcpyHostToDevice, st));
  for (int i : bt->split_idx)
    if (!bt->plans[i]) {
      const fde_params q = bt->p[i];
      TRY(fde_assemble(&q, bt->hdp[i], bt->hdm[i], nullptr, nullptr, st, &bt->plans[i]));
    }
  const int nw = std::min(k, SPLIT_WORKERS);
  while ((int)bt->wstreams.size() < nw) {
    hipStream_t w = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
    bt->wstreams.push_back(w);
  }
  HIPCHK(hipStreamSynchronize(st));   // the host copy of the order stays valid until here
  return FDE_OK;
}

// The split instances on the plan path, by SPLIT_WORKERS threads (the calling
// thread is one of them), each on its own stream, dealt largest work first:
// `steps` implicit steps from x (b = rhs(x), solve from x; step_mode) or one
// solve of b.  Their per-step results go to `res` as (info slot, Info).
fde_status run_split(fde_batch bt, const double* b, double* x, int steps, bool step_mode,
                     std::vector<std::pair<long, Info>>& res) {
  const int k = (int)bt->split_idx.size();
  if (!k) return FDE_OK;
  const int nw = std::min(k, (int)bt->wstreams.size());
  std::vector<fde_status> status(nw, FDE_OK);
  std::vector<std::string> errs(nw);
  std::vector<std::vector<std::pair<long, Info>>> out(nw);
  auto work = [&](int w) {
    if (hipSetDevice(bt->dev) != hipSuccess) {
      status[w] = FDE_EHIP;
      errs[w] = "hipSetDevice failed in a worker";
      return;
    }
    hipStream_t s = bt->wstreams[w];
    for (int j = w; j < k; j += nw) {
      const int i = bt->split_idx[j];
      fde_plan pl = bt->plans[i];
      const long off = bt->off[i];
      for (int t = 0; t < steps; ++t) {
        if (step_mode) {
          const fde_status r = fde_rhs(pl, x + off, nullptr, bt->hb[i], s);
          if (r != FDE_OK) {
            status[w] = r;
            errs[w] = fde_last_error();
            return;
          }
        }
        fde_info fi{};
        const fde_status r = fde_solve(pl, step_mode ? bt->hb[i] : b + off, x + off, &fi, s);
        if (r < 0 && r != FDE_ENONFINITE) {
          status[w] = r;
          errs[w] = fde_last_error();
          return;
        }
        Info in{fi.iters, fi.inner_iters, fi.restarts, fi.converged, r == FDE_ENONFINITE ? 1 : 0, 0,
                fi.relres_true, fi.relres_est};
        out[w].push_back({(long)t * bt->count + i, in});
      }
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < nw; ++w) th.emplace_back(work, w);
  work(0);
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w) {
    if (status[w] != FDE_OK) return fail(status[w], "plan-path instance: %s", errs[w].c_str());
    res.insert(res.end(), out[w].begin(), out[w].end());
  }
  return FDE_OK;
}

fde_status assemble_impl(const fde_params* ps, int count, const double* dp, const double* dm, hipStream_t st,
                         fde_batch bt) {
  bt->count = count;
  bt->p.assign(ps, ps + count);
  bt->off.resize(count + 1);
  bt->off[0] = 0;
  for (int i = 0; i < count; ++i) bt->off[i + 1] = bt->off[i] + ps[i].n[0];
  bt->total = bt->off[count];
  const long N = bt->total;
  if (!dp || !dm) return fail(FDE_EINVAL, "coefficient arrays must not be NULL");
  std::vector<double> hp(N), hm(N);
  HIPCHK(hipMemcpyAsync(hp.data(), dp, N * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hm.data(), dm, N * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  bt->cus = std::max(1, prop.multiProcessorCount);

  std::vector<Layout> lay(count);
  std::vector<size_t> base(count + 1, 0);
  int logTW = 1;
  for (int i = 0; i < count; ++i) {
    lay[i] = layout(ps[i]);
    base[i + 1] = base[i] + lay[i].total;
    const Geo g = geometry(ps[i]);
    logTW = std::max(logTW, std::max(g.logQt, g.logQs) + 1);
  }
  bt->logTW = logTW;
  // tables are written into a host image of the arena (workspace left zero)
  unsigned char* arena = nullptr;
  TRY(balloc(bt, &arena, base[count]));
  HIPCHK(hipMemsetAsync(arena, 0, base[count], st));
  std::vector<Inst> hinst(count);
  bt->hdp.assign(count, nullptr);
  bt->hdm.assign(count, nullptr);
  bt->hb.assign(count, nullptr);
  bt->plans.assign(count, nullptr);
  bt->last_iters.assign(count, 0);
  bt->dev = dev;
  std::vector<unsigned char> img;
  for (int i = 0; i < count; ++i) {
    const fde_params& p = ps[i];
    const Layout& L = lay[i];
    const Geo g = geometry(p);
    const long n = g.n;
    const double* ip = hp.data() + bt->off[i];
    const double* im = hm.data() + bt->off[i];
    double mn = ip[0], mx = ip[0];
    for (long k = 0; k < n; ++k) {
      if (!std::isfinite(ip[k]) || !std::isfinite(im[k]))
        return fail(FDE_EINVAL, "instance %d: a coefficient is not finite", i);
      if (ip[k] < 0.0 || im[k] < 0.0) return fail(FDE_EINVAL, "instance %d: a coefficient is negative", i);
      mn = std::min(mn, std::min(ip[k], im[k]));
      mx = std::max(mx, std::max(ip[k], im[k]));
    }
    const bool constant = mn == mx;
    const double h = (p.hi[0] - p.lo[0]) / (double)(n + 1);
    const double hxa = std::pow(h, p.alpha[0]);
    const double nu = (p.time == FDE_T_EULER ? 1.0 : 2.0) * hxa / p.dt;

    std::vector<double> dinv(n, 0.0), finv(n), Fa(n);
    for (long k = 0; k < n; ++k) Fa[k] = symbol(p.alpha[0], M_PI * (double)(k + 1) / (double)(n + 1), p.weights);
    bool has_d = false;
    if (p.prec == FDE_P_TAU) {
      has_d = true;
      const double shift = std::isnan(p.shift) ? (constant ? nu / mn : 0.0) : p.shift;
      for (long k = 0; k < n; ++k) {
        const double D = 0.5 * (ip[k] + im[k]);
        if (!(D > 0.0)) return fail(FDE_EINVAL, "instance %d: D has a zero (d+ and d- share a zero)", i);
        dinv[k] = 1.0 / D;
        finv[k] = 1.0 / (Fa[k] + shift);
      }
    } else if (p.prec == FDE_P_TAU_HAT) {
      if (!constant || !(mn > 0.0)) return fail(FDE_EINVAL, "instance %d: P_hat needs constant, equal, positive d+ and d-", i);
      for (long k = 0; k < n; ++k) finv[k] = 1.0 / (mn * Fa[k] + nu);
    } else if (p.prec == FDE_P_TILDE) {
      for (long k = 0; k < n; ++k) {
        const double f = 0.5 * (ip[k] + im[k]) * Fa[k];
        if (!(f > 0.0)) return fail(FDE_EINVAL, "instance %d: P_tilde: D_j p(theta_j) must be positive", i);
        finv[k] = 1.0 / f;
      }
    } else {
      for (long k = 0; k < n; ++k) finv[k] = 1.0;
    }
    TriFactors TF;
    if (p.prec == FDE_P_TRI) {
      const std::vector<double> gw = weights(p.alpha[0], (int)std::max(n, 2L), p.weights);
      std::vector<double> sub, diag, sup;
      tri_part(gw, nu, ip, im, n, sub, diag, sup);
      for (long k = 0; k < n; ++k)
        if (!(std::fabs(diag[k]) > std::fabs(sub[k]) + std::fabs(sup[k])))
          return fail(FDE_EINVAL, "instance %d: P_tri: tridiagonal part not strictly diagonally dominant", i);
      TF = tri_factor(sub, diag, sup, L.tp);
    }
    // circulant of length 2 Qt embedding T: first column (-g_1..-g_n, 0.., -g_0)
    const long Lc = 2 * g.Qt;
    std::vector<double> w = weights(p.alpha[0], (int)n, p.weights);
    std::vector<std::complex<double>> lam(Lc, 0.0);
    for (long k = 0; k < n; ++k) lam[k] = -w[k + 1];
    lam[Lc - 1] += -w[0];
    host_fft(lam);
    lam.resize(g.Qt + 1);
    for (auto& v : lam) v /= (double)Lc;
    // chirp-z tables
    std::vector<std::complex<double>> chirp, bhat;
    if (g.blue) {
      const long P = n + 1;
      auto ph = [&](long j, double sgn) {
        const long r = (j * j) % (4 * P);
        const double t = M_PI * (double)r / (2.0 * (double)P);
        return std::complex<double>(std::cos(t), sgn * std::sin(t));
      };
      chirp.resize(n + 1);
      for (long j = 0; j <= n; ++j) chirp[j] = ph(j, 1.0);
      bhat.assign(g.Qs, 0.0);
      for (long r = 0; r < n; ++r) {
        bhat[r] = ph(r, -1.0);
        if (r) bhat[g.Qs - r] = bhat[r];
      }
      host_fft(bhat);
      const double s = std::sqrt(2.0 / (double)P) / (double)g.Qs;
      for (auto& v : bhat) v *= s;
    }
    // host image of this instance's tables
    img.assign(L.total, 0);
    std::vector<double> vdp(ip, ip + n), vdm(im, im + n);
    put<double>(img, L.tab64[0], vdp);
    put<double>(img, L.tab64[1], vdm);
    put<double>(img, L.tab64[2], dinv);
    put<double>(img, L.tab64[3], finv);
    put_cx<double>(img, L.tab64[4], lam);
    put<float>(img, L.tab32[0], vdp);
    put<float>(img, L.tab32[1], vdm);
    put<float>(img, L.tab32[2], dinv);
    put<float>(img, L.tab32[3], finv);
    put_cx<float>(img, L.tab32[4], lam);
    if (g.blue) {
      put_cx<double>(img, L.tab64[5], chirp);
      put_cx<double>(img, L.tab64[6], bhat);
      put_cx<float>(img, L.tab32[5], chirp);
      put_cx<float>(img, L.tab32[6], bhat);
    }
    if (p.prec == FDE_P_TRI) {
      const std::vector<double>* arr[10] = {&TF.ai, &TF.cp, &TF.den, &TF.sv, &TF.sw,
                                            &TF.ar, &TF.cr, &TF.ra, &TF.rb, &TF.rc};
      for (int a = 0; a < 10; ++a) {
        put<double>(img, L.tri64[a], *arr[a]);
        put<float>(img, L.tri32[a], *arr[a]);
      }
      std::memcpy(img.data() + L.tcs, TF.cs.data(), TF.cs.size() * sizeof(int));
    }
    const size_t tab_end = L.V;   // tables precede the workspace
    HIPCHK(hipMemcpy(arena + base[i], img.data(), tab_end, hipMemcpyHostToDevice));
    unsigned char* a0 = arena + base[i];
    Inst& I = hinst[i];
    I.n = (int)n;
    I.logQt = g.logQt;
    I.logQs = g.logQs;
    I.blue = g.blue ? 1 : 0;
    I.prec = p.prec;
    I.dside = p.dside;
    I.time = p.time;
    I.precision = p.precision;
    I.kin = p.precision == FDE_MIXED ? p.inner_steps : 0;
    I.m = p.restart;
    I.maxit = p.maxit;
    I.tol = p.tol;
    I.nu = nu;
    I.off = bt->off[i];
    I.t64 = Tab<double>{reinterpret_cast<double*>(a0 + L.tab64[0]), reinterpret_cast<double*>(a0 + L.tab64[1]),
                        has_d ? reinterpret_cast<double*>(a0 + L.tab64[2]) : nullptr,
                        reinterpret_cast<double*>(a0 + L.tab64[3]), reinterpret_cast<cx<double>*>(a0 + L.tab64[4]),
                        g.blue ? reinterpret_cast<cx<double>*>(a0 + L.tab64[5]) : nullptr,
                        g.blue ? reinterpret_cast<cx<double>*>(a0 + L.tab64[6]) : nullptr};
    I.t32 = Tab<float>{reinterpret_cast<float*>(a0 + L.tab32[0]), reinterpret_cast<float*>(a0 + L.tab32[1]),
                       has_d ? reinterpret_cast<float*>(a0 + L.tab32[2]) : nullptr,
                       reinterpret_cast<float*>(a0 + L.tab32[3]), reinterpret_cast<cx<float>*>(a0 + L.tab32[4]),
                       g.blue ? reinterpret_cast<cx<float>*>(a0 + L.tab32[5]) : nullptr,
                       g.blue ? reinterpret_cast<cx<float>*>(a0 + L.tab32[6]) : nullptr};
    I.tp = p.prec == FDE_P_TRI ? TF.p : 0;
    I.tcs = p.prec == FDE_P_TRI ? reinterpret_cast<const int*>(a0 + L.tcs) : nullptr;
    {
      auto d64 = [&](int a) { return p.prec == FDE_P_TRI ? reinterpret_cast<double*>(a0 + L.tri64[a]) : nullptr; };
      auto d32 = [&](int a) { return p.prec == FDE_P_TRI ? reinterpret_cast<float*>(a0 + L.tri32[a]) : nullptr; };
      I.t64.ai = d64(0); I.t64.cp = d64(1); I.t64.den = d64(2); I.t64.sv = d64(3); I.t64.sw = d64(4);
      I.t64.ar = d64(5); I.t64.cr = d64(6); I.t64.ra = d64(7); I.t64.rb = d64(8); I.t64.rc = d64(9);
      I.t64.ty = d64(10);
      I.t32.ai = d32(0); I.t32.cp = d32(1); I.t32.den = d32(2); I.t32.sv = d32(3); I.t32.sw = d32(4);
      I.t32.ar = d32(5); I.t32.cr = d32(6); I.t32.ra = d32(7); I.t32.rb = d32(8); I.t32.rc = d32(9);
      I.t32.ty = d32(10);
    }
    bt->hdp[i] = I.t64.dp;
    bt->hdm[i] = I.t64.dm;
    bt->hb[i] = reinterpret_cast<double*>(a0 + L.b);
    I.V = reinterpret_cast<double*>(a0 + L.V);
    I.Z = reinterpret_cast<double*>(a0 + L.Z);
    I.b = reinterpret_cast<double*>(a0 + L.b);
    I.t = reinterpret_cast<double*>(a0 + L.t);
    I.Vf = reinterpret_cast<float*>(a0 + L.Vf);
    I.uf = reinterpret_cast<float*>(a0 + L.uf);
    I.zf = reinterpret_cast<float*>(a0 + L.zf);
    I.tf = reinterpret_cast<float*>(a0 + L.tf);
    I.fa = g.staged ? reinterpret_cast<cx<double>*>(a0 + L.fa) : nullptr;
    I.fb = g.staged ? reinterpret_cast<cx<double>*>(a0 + L.fb) : nullptr;
  }
  TRY(balloc(bt, &bt->dinst, count));
  HIPCHK(hipMemcpy(bt->dinst, hinst.data(), count * sizeof(Inst), hipMemcpyHostToDevice));

  // twiddles exp(-2 pi i m/TW)
  const long TW = 1L << logTW;
  std::vector<std::complex<double>> tw(TW);
  for (long m = 0; m < TW; ++m) {
    const double t = 2.0 * M_PI * (double)m / (double)TW;
    tw[m] = std::complex<double>(std::cos(t), -std::sin(t));
  }
  for (long q = 0; q < 4; ++q) {   // exact quarter turns
    const long m = q * (TW / 4);
    if (TW >= 4) tw[m] = q == 0 ? 1.0 : q == 1 ? std::complex<double>(0, -1) : q == 2 ? -1.0 : std::complex<double>(0, 1);
  }
  {
    std::vector<unsigned char> t64(TW * 16), t32(TW * 8);
    put_cx<double>(t64, 0, tw);
    put_cx<float>(t32, 0, tw);
    TRY(balloc(bt, &bt->tw64, TW));
    TRY(balloc(bt, &bt->tw32, TW));
    HIPCHK(hipMemcpy(bt->tw64, t64.data(), t64.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bt->tw32, t32.data(), t32.size(), hipMemcpyHostToDevice));
  }

  // per-iteration work model of each instance (the queue order's key, times
  // the iterations of its last solve once known)
  bt->cost.assign(count, 0.0);
  for (int i = 0; i < count; ++i) {
    const Geo g = geometry(ps[i]);
    bt->cost[i] = (double)g.n * (ps[i].restart + 8.0) + (double)g.Qs * g.logQs * (g.blue ? 4.0 : 2.0) +
                  3.0 * (double)g.Qt * g.logQt;
  }
  TRY(balloc(bt, &bt->order_q, count));
  TRY(balloc(bt, &bt->queue, 1));
  TRY(balloc(bt, &bt->step, 1));
  TRY(ensure_info(bt, count));
  bt->cfg = fde_batch_cfg{0, 2 * bt->cus, 1, 0.0, 0};
  HIPCHK(hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking));
  TRY(prepare_queue(bt, bt->cfg, st));
  HIPCHK(hipStreamSynchronize(st));
  return FDE_OK;
}

}  // namespace

extern "C" size_t fde_batch_layout(const fde_params* params, int count, long long* offsets) {
  if (validate_all(params, count) != FDE_OK) return 0;
  long long o = 0;
  for (int i = 0; i < count; ++i) {
    if (offsets) offsets[i] = o;
    o += params[i].n[0];
  }
  if (offsets) offsets[count] = o;
  return (size_t)o;
}

extern "C" size_t fde_batch_bytes(const fde_params* params, int count) {
  if (validate_all(params, count) != FDE_OK) return 0;
  size_t b = 0;
  int logTW = 1;
  for (int i = 0; i < count; ++i) {
    b += layout(params[i]).total;
    const Geo g = geometry(params[i]);
    logTW = std::max(logTW, std::max(g.logQt, g.logQs) + 1);
  }
  b += (size_t)count * (sizeof(Inst) + 2 * sizeof(int) + sizeof(Info)) + (24UL << logTW) + 64;
  return b;
}

extern "C" fde_status fde_batch_assemble(const fde_params* params, int count, const double* dplus,
                                         const double* dminus, void* stream, fde_batch* out) {
  if (!out) return fail(FDE_EINVAL, "out is NULL");
  *out = nullptr;
  TRY(validate_all(params, count));
  fde_batch bt = new (std::nothrow) fde_batch_s();
  if (!bt) return fail(FDE_ENOMEM, "host allocation failed");
  const fde_status s = assemble_impl(params, count, dplus, dminus, static_cast<hipStream_t>(stream), bt);
  if (s != FDE_OK) {
    const std::string keep = g_err;
    destroy_impl(bt);
    g_err = keep;
    return s;
  }
  *out = bt;
  return FDE_OK;
}

extern "C" fde_status fde_batch_solve(fde_batch bt, const double* b, double* x, fde_info* info, void* stream) {
  if (!bt || !b || !x) return fail(FDE_EINVAL, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  TRY(prepare_queue(bt, bt->cfg, st));
  TRY(enqueue(bt, bt->cfg, MODE_SOLVE, b, x, nullptr, st));
  std::vector<std::pair<long, Info>> pinfo;
  const fde_status ws = run_split(bt, b, x, 1, false, pinfo);   // concurrently with the launch
  HIPCHK(hipStreamSynchronize(st));
  TRY(ws);
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return collect(bt, bt->count, info, sec, st, &pinfo);
}

// Batched operators: every instance's operator applied with its own plan
// (built on first use, as for the instances split off the persistent launch),
// one launch sequence per instance on `stream`.  The persistent kernel's own
// operator modes stay disabled: their first GPU run (an earlier build) took a
// memory fault whose cause was not found.
static fde_status batch_apply(fde_batch bt, int mode, int precision, const double* in, double* out, void* stream) {
  if (!bt || !in || !out) return fail(FDE_EINVAL, "NULL argument");
  if (precision != FDE_FP64 && precision != FDE_MIXED) return fail(FDE_EINVAL, "bad precision");
  if (precision == FDE_MIXED)
    for (int i = 0; i < bt->count; ++i)
      if (bt->p[i].precision != FDE_MIXED)
        return fail(FDE_EINVAL, "float32 operators need a batch assembled with FDE_MIXED (instance %d)", i);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int i = 0; i < bt->count; ++i) {
    if (!bt->plans[i]) {
      const fde_params q = bt->p[i];
      TRY(fde_assemble(&q, bt->hdp[i], bt->hdm[i], nullptr, nullptr, st, &bt->plans[i]));
    }
    const long off = bt->off[i];
    fde_plan pl = bt->plans[i];
    fde_status r;
    if (mode == MODE_MATVEC)
      r = precision == FDE_FP64 ? fde_matvec(pl, in + off, out + off, st) : fde_matvec_f32(pl, in + off, out + off, st);
    else
      r = precision == FDE_FP64 ? fde_tau_apply(pl, in + off, out + off, st)
                                : fde_tau_apply_f32(pl, in + off, out + off, st);
    if (r != FDE_OK) return r;
  }
  return FDE_OK;
}

extern "C" fde_status fde_batch_matvec(fde_batch bt, int precision, const double* x, double* y, void* stream) {
  return batch_apply(bt, MODE_MATVEC, precision, x, y, stream);
}

extern "C" fde_status fde_batch_tau_apply(fde_batch bt, int precision, const double* v, double* z, void* stream) {
  return batch_apply(bt, MODE_TAU, precision, v, z, stream);
}

extern "C" fde_status fde_batch_run(fde_batch bt, double* u, int steps, int use_graph, fde_info* info,
                                    void* stream) {
  if (!bt || !u) return fail(FDE_EINVAL, "NULL argument");
  if (steps < 1) return fail(FDE_EINVAL, "steps must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  TRY(ensure_info(bt, (long)steps * bt->count));
  TRY(prepare_queue(bt, bt->cfg, st));
  HIPCHK(hipMemsetAsync(bt->step, 0, sizeof(int), st));
  const auto t0 = std::chrono::steady_clock::now();
  if (use_graph) {
    const fde_batch_cfg& c = bt->cfg;
    if (!bt->gexec || bt->gx != u || bt->gcfg.variant != c.variant || bt->gcfg.grid != c.grid ||
        bt->gcfg.lpt != c.lpt || bt->gcfg.split != c.split) {
      drop_graph(bt);
      HIPCHK(hipStreamBeginCapture(bt->cap, hipStreamCaptureModeThreadLocal));
      const fde_status s = enqueue(bt, c, MODE_STEP, nullptr, u, bt->step, bt->cap);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(bt->cap, &g);
      if (s != FDE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
      }
      HIPCHK(e);
      bt->graph = g;
      HIPCHK(hipGraphInstantiate(&bt->gexec, g, nullptr, nullptr, 0));
      bt->gx = u;
      bt->gcfg = c;
    }
    for (int s = 0; s < steps; ++s) HIPCHK(hipGraphLaunch(bt->gexec, st));
  } else {
    for (int s = 0; s < steps; ++s) TRY(enqueue(bt, bt->cfg, MODE_STEP, nullptr, u, bt->step, st));
  }
  std::vector<std::pair<long, Info>> pinfo;
  const fde_status ws = run_split(bt, nullptr, u, steps, true, pinfo);   // concurrently with the launches
  HIPCHK(hipStreamSynchronize(st));
  TRY(ws);
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return collect(bt, (long)steps * bt->count, info, sec, st, &pinfo);
}

// One time step of configuration c from u (copied to the tuning state), wall
// time in milliseconds (the persistent launch and the plan-path instances).
// With FDE_TRACE set (1: standard error, else a file name appended to), the
// tuner writes one line per timed trial:
//   fde_trace tune variant=<v> grid=<g> lpt=<l> split=<s> ms=<t>
static void trace_trial(const fde_batch_cfg& c, double ms) {
  const char* e = std::getenv("FDE_TRACE");
  if (!e || !*e || std::strcmp(e, "0") == 0) return;
  FILE* f = std::strcmp(e, "1") == 0 ? stderr : std::fopen(e, "a");
  if (!f) return;
  std::fprintf(f, "fde_trace tune variant=%d grid=%d lpt=%d split=%d ms=%.3f\n", c.variant, c.grid, c.lpt, c.split,
               ms);
  if (f != stderr) std::fclose(f);
}

static fde_status tune_trial(fde_batch bt, const fde_batch_cfg& c, const double* u, hipStream_t st, double* ms) {
  TRY(prepare_queue(bt, c, st));
  HIPCHK(hipMemcpyAsync(bt->tune_x, u, bt->total * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  const auto t0 = std::chrono::steady_clock::now();
  TRY(enqueue(bt, c, MODE_STEP, nullptr, bt->tune_x, nullptr, st));
  std::vector<std::pair<long, Info>> pinfo;
  const fde_status ws = run_split(bt, nullptr, bt->tune_x, 1, true, pinfo);
  HIPCHK(hipStreamSynchronize(st));
  TRY(ws);
  *ms = 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return FDE_OK;
}

extern "C" fde_status fde_batch_tune(fde_batch bt, const double* u, void* stream, fde_batch_cfg* chosen) {
  if (!bt || !u) return fail(FDE_EINVAL, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!bt->tune_x) TRY(balloc(bt, &bt->tune_x, (size_t)bt->total));
  fde_batch_cfg best{bt->cfg.variant, bt->cfg.grid, bt->cfg.lpt, 1e300, 0};
  // launch configurations, every instance in the persistent launch
  const std::vector<int> grids = {bt->cus, 2 * bt->cus};
  for (int v = 0; v < VARIANTS_ENABLED; ++v)
    for (int grid : grids)
      for (int lp = 1; lp >= 0; --lp) {
        const fde_batch_cfg c{v, grid, lp, 0.0, 0};
        double ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
          double t = 0.0;
          TRY(tune_trial(bt, c, u, st, &t));
          trace_trial(c, t);
          ms = std::min(ms, t);
        }
        if (ms < best.ms) best = fde_batch_cfg{v, grid, lp, ms, 0};
      }
  // the iterations of every instance (the trials' per-instance results) set the work estimates
  bt->hinfo.resize(bt->count);
  HIPCHK(hipMemcpyAsync(bt->hinfo.data(), bt->info, bt->count * sizeof(Info), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < bt->count; ++i) bt->last_iters[i] = bt->hinfo[i].iters;
  // then the instances of largest estimated work on the plan path
  for (int k : {4, 8, 16, 32, 64}) {
    if (k >= bt->count) break;
    fde_batch_cfg c = best;
    c.split = k;
    double ms = 1e300, t = 0.0;
    TRY(tune_trial(bt, c, u, st, &t));   // first run of new plans: not timed
    for (int rep = 0; rep < 2; ++rep) {
      TRY(tune_trial(bt, c, u, st, &t));
      trace_trial(c, t);
      ms = std::min(ms, t);
    }
    if (ms < best.ms) {
      best = c;
      best.ms = ms;
    }
  }
  bt->cfg = best;
  drop_graph(bt);
  if (chosen) *chosen = best;
  return FDE_OK;
}

extern "C" fde_status fde_batch_get_cfg(fde_batch bt, fde_batch_cfg* cfg) {
  if (!bt || !cfg) return fail(FDE_EINVAL, "NULL argument");
  *cfg = bt->cfg;
  return FDE_OK;
}

extern "C" fde_status fde_batch_set_cfg(fde_batch bt, const fde_batch_cfg* cfg) {
  if (!bt || !cfg) return fail(FDE_EINVAL, "NULL argument");
  if (cfg->variant < 0 || cfg->variant >= FDE_BATCH_VARIANTS)
    return fail(FDE_EINVAL, "variant must be in 0..%d", FDE_BATCH_VARIANTS - 1);
  if (cfg->variant >= VARIANTS_ENABLED) return fail(FDE_EUNSUPPORTED, "launch variant %d is disabled", cfg->variant);
  if (cfg->grid < 1) return fail(FDE_EINVAL, "grid must be >= 1");
  if (cfg->split < 0 || cfg->split > bt->count) return fail(FDE_EINVAL, "split must be in 0..%d", bt->count);
  bt->cfg = fde_batch_cfg{cfg->variant, cfg->grid, cfg->lpt ? 1 : 0, 0.0, cfg->split};
  drop_graph(bt);
  return FDE_OK;
}

extern "C" void fde_batch_destroy(fde_batch bt) { destroy_impl(bt); }
