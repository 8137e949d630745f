// Preconditioned conjugate gradients for a 1D plan whose line fits one
// workgroup (n + 1 <= 4096): the whole solve in a single workgroup, which a
// system with a few hundred to a few thousand unknowns otherwise spends in
// kernel launches and host round trips.  The steps are those of the
// multi-kernel driver (Section 3.1, Case I, for the preconditioner):
//   ||b||; tolerance tol ||b||; then until the true residual passes or the
//   iteration cap is met:
//     r = b - M x, beta = ||r|| (the true residual; a restart when PCG's own
//     estimate had passed but this one does not);
//     z = P^{-1} r, rz = r.z, p = z; then until done:
//       q = M p, alpha = rz / p.q, x += alpha p, r -= alpha q, est = ||r||,
//       stop when est <= tol ||b|| (or non-finite, or the iteration cap),
//       z = P^{-1} r, beta_cg = r.z / rz, p = z + beta_cg p.
// P^{-1} and M are the DST and Toeplitz line programs (line_body).  The
// scalars are computed identically by every thread from the workgroup sums;
// thread 0 records them in the Krylov state for the host at the end.
#pragma once

#include <hip/hip_runtime.h>

#include "fde_krylov.hpp"
#include "fde_lines.hpp"
#include "fde_reduce.hpp"

namespace fde {

// Elements per thread of the line programs: 4 up to P = 2048 (P/4 threads,
// at least 128: every SIMD of the CU takes a wave), 8 at P = 4096 (512
// threads).
__host__ __device__ constexpr int pcg_ept(int logP) { return logP <= 11 ? 4 : 8; }
__host__ __device__ constexpr int pcg_threads(int logP) {
  return rows_per_tile(1 << logP) * (1 << logP) / pcg_ept(logP);
}

// ta: z = P^{-1} r (in = r, out = z); ma: q = nu v + T-part v with out = q;
// its input is x for a true residual and p within the iteration.  The steps
// run as one loop with a single call site per line program (the Toeplitz
// product's input chosen per pass), so that only two copies of the programs'
// registers are live.  Launched with one workgroup of pcg_threads(LOGP)
// threads; the bound is that size.
template <int LOGP>
__global__ void __launch_bounds__(pcg_threads(LOGP))
pcg1d_kernel(LineArgs<double> ta, LineArgs<double> ma, const double* b, double* x, double* r, double* p, double* q,
             double* z, int n, double tol, int maxit, KState* ks) {
  __shared__ double red[16];
  __shared__ double tot[1];
  const int tid = threadIdx.x, nt = blockDim.x;
  // Each inlined line program's address arithmetic depends on its tile; a
  // tile index the compiler cannot see through keeps it from hoisting that
  // arithmetic out of the loop, which would not fit in registers.  The value
  // is always 0.
  auto tile0 = []() {
    int t = 0;
    asm volatile("" : "+s"(t));
    return t;
  };
  auto sum = [&](double v) -> double {
    double acc[1] = {v};
    block_multi_sum<1>(acc, red, tot);
    const double s = tot[0];
    __syncthreads();   // red and tot are reused by the next sum
    return s;
  };
  auto dot = [&](const double* u, const double* v) -> double {
    double acc = 0.0;
    for (int e = tid; e < n; e += nt) acc += u[e] * v[e];
    return sum(acc);
  };

  const double bnorm = sqrt(dot(b, b));
  const double tolabs = tol * bnorm;
  int iters = 0, restarts = 0, conv = 0, nonfinite = !isfinite(bnorm);
  double beta = 0.0, est = 0.0, rz = 0.0, pq = 0.0, alpha = 0.0, betacg = 0.0;
  if (!nonfinite && bnorm == 0.0) {
    for (int e = tid; e < n; e += nt) x[e] = 0.0;
    conv = 1;
  } else if (!nonfinite) {
    bool fresh = true;     // this pass's product is M x (a true residual); else M p
    bool started = false;  // a true residual was taken before
    bool first = true;     // the next direction is p = z (a (re)start)
    for (;;) {
      LineArgs<double> mv = ma;
      mv.in = fresh ? x : p;
      line_body<double, false, LF_TOEP, LOGP, pcg_ept(LOGP)>(mv, tile0());   // q = M x or q = M p
      __syncthreads();
      if (fresh) {
        double ss = 0.0;
        for (int e = tid; e < n; e += nt) {
          const double rv = b[e] - q[e];
          r[e] = rv;
          ss += rv * rv;
        }
        beta = sqrt(sum(ss));
        conv = beta <= tolabs;
        if (!isfinite(beta)) nonfinite = 1;
        if (started && !conv) ++restarts;
        started = true;
        if (conv || nonfinite || iters >= maxit) break;
        first = true;   // (re)start PCG from r
      } else {
        pq = dot(p, q);
        alpha = rz / pq;
        double rr = 0.0;
        for (int e = tid; e < n; e += nt) {
          x[e] += alpha * p[e];
          const double rv = r[e] - alpha * q[e];
          r[e] = rv;
          rr += rv * rv;
        }
        est = sqrt(sum(rr));
        ++iters;
        if (!isfinite(est)) nonfinite = 1;
        if (est <= tolabs || nonfinite || iters >= maxit) {   // uniform across the workgroup
          fresh = true;   // confirm with the true residual
          continue;
        }
      }
      line_body<double, false, LF_DST1 | LF_FDST2, LOGP, pcg_ept(LOGP)>(ta, tile0());   // z = P^{-1} r
      __syncthreads();
      const double rzn = dot(r, z);
      if (first) {
        betacg = 0.0;
        for (int e = tid; e < n; e += nt) p[e] = z[e];
      } else {
        betacg = rz != 0.0 ? rzn / rz : 0.0;
        for (int e = tid; e < n; e += nt) p[e] = z[e] + betacg * p[e];
      }
      rz = rzn;
      first = false;
      fresh = false;
      __syncthreads();
    }
  }
  if (tid == 0) {
    ks->kdone = 0;
    ks->done = 1;
    ks->conv = conv;
    ks->iters = iters;
    ks->maxit = maxit;
    ks->m = 1;
    ks->nonfinite = nonfinite;
    ks->breakdown = 0;
    ks->restarts = restarts;
    ks->bnorm = bnorm;
    ks->tolabs = tolabs;
    ks->beta = beta;
    ks->est = est;
    ks->hn = 0.0;
    ks->rz = rz;
    ks->pq = pq;
    ks->alpha = alpha;
    ks->betacg = betacg;
  }
}

}  // namespace fde
