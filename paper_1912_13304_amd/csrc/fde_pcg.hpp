// Preconditioned conjugate gradients for a 1D plan whose line fits one
// workgroup (n + 1 <= 4096): the whole iteration loop of one (re)start in a
// single workgroup, which a solve with a few hundred to a few thousand
// unknowns otherwise spends in kernel launches.  Each step is that of the
// multi-kernel driver (Section 3.1, Case I, for the preconditioner):
//   z = P^{-1} r, rz = r.z, p = z; then until done:
//   q = M p, alpha = rz / p.q, x += alpha p, r -= alpha q, est = ||r||,
//   stop when est <= tol ||b|| (or non-finite, or the iteration cap),
//   z = P^{-1} r, beta = r.z / rz, p = z + beta p.
// P^{-1} and M are the DST and Toeplitz line programs (line_body).  The
// scalars are computed identically by every thread from the workgroup sums;
// thread 0 records them in the Krylov state for the host.
#pragma once

#include <hip/hip_runtime.h>

#include "fde_krylov.hpp"
#include "fde_lines.hpp"
#include "fde_reduce.hpp"

namespace fde {

// ta: z = P^{-1} r (in = r, out = z); ma: q = nu p + T-part (in = p, out = q).
// Launched with one workgroup of the line program's size, P/8 threads (64
// below P = 512); the bound is that size so that the registers of the three
// inlined line programs fit without spilling.
template <int LOGP>
__global__ void __launch_bounds__((1 << LOGP) / 8 > 64 ? (1 << LOGP) / 8 : 64)
pcg1d_kernel(LineArgs<double> ta, LineArgs<double> ma, double* x, double* r, double* p, double* q, double* z,
             int n, KState* ks, double* hstat) {
  __shared__ double red[16];
  __shared__ double tot[1];
  const int tid = threadIdx.x, nt = blockDim.x;
  // set by earlier kernels; read before this kernel writes the state
  const double tolabs = ks->tolabs;
  const int maxit = ks->maxit;
  int iters = ks->iters;
  const double rz_prev = ks->rz;
  // Each inlined line program's address arithmetic depends on its tile; a
  // tile index the compiler cannot see through keeps it from hoisting three
  // copies of that arithmetic out of the loop, which would not fit in
  // registers.  The value is always 0.
  auto tile0 = []() {
    int t = 0;
    asm volatile("" : "+s"(t));
    return t;
  };
  auto dot = [&](const double* u, const double* v) -> double {
    double acc[1] = {0.0};
    for (int e = tid; e < n; e += nt) acc[0] += u[e] * v[e];
    block_multi_sum<1>(acc, red, tot);
    const double s = tot[0];
    __syncthreads();   // red and tot are reused by the next sum
    return s;
  };
  line_body<double, false, LF_DST1 | LF_FDST2, LOGP>(ta, tile0());   // z = P^{-1} r
  __syncthreads();
  double rz = dot(r, z);
  if (tid == 0) {
    ks->betacg = (rz_prev != 0.0 && iters > 0) ? rz / rz_prev : 0.0;
    ks->rz = rz;
  }
  for (int e = tid; e < n; e += nt) p[e] = z[e];
  __syncthreads();
  for (;;) {
    line_body<double, false, LF_TOEP, LOGP>(ma, tile0());   // q = M p
    __syncthreads();
    const double pq = dot(p, q);
    const double alpha = rz / pq;
    if (tid == 0) {
      ks->pq = pq;
      ks->alpha = alpha;
    }
    double ss[1] = {0.0};
    for (int e = tid; e < n; e += nt) {
      x[e] += alpha * p[e];
      const double rv = r[e] - alpha * q[e];
      r[e] = rv;
      ss[0] += rv * rv;
    }
    block_multi_sum<1>(ss, red, tot);
    const double est = sqrt(tot[0]);
    __syncthreads();
    iters += 1;
    const bool bad = !isfinite(est);
    const bool done = (est <= tolabs) || bad || iters >= maxit;
    if (tid == 0) {
      ks->est = est;
      ks->iters = iters;
      if (bad) ks->nonfinite = 1;
      ks->done = done;
      if (hstat) {
        hstat[0] = (double)done;
        hstat[1] = (double)iters;
      }
    }
    if (done) break;   // uniform: every thread holds the same est and iters
    line_body<double, false, LF_DST1 | LF_FDST2, LOGP>(ta, tile0());   // z = P^{-1} r
    __syncthreads();
    const double rzn = dot(r, z);
    const double beta = rz != 0.0 ? rzn / rz : 0.0;
    rz = rzn;
    if (tid == 0) {
      ks->betacg = beta;
      ks->rz = rz;
    }
    for (int e = tid; e < n; e += nt) p[e] = z[e] + beta * p[e];
    __syncthreads();
  }
}

}  // namespace fde
