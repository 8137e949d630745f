// Batched 1D solves: many independent systems M_i u_i = b_i of different
// sizes n_i and orders alpha_i (Section 1.2) in one persistent launch.
//
// Each workgroup takes instances from a ticket queue and runs the whole
// preconditioned FGMRES solve of one instance by itself: every vector
// operation is a loop of the workgroup's threads over the instance's
// elements, every reduction a fixed-order workgroup reduction, and the small
// dense work (Givens rotations, back substitution) runs in LDS.  Nothing
// synchronises across workgroups, so the instances of a batch proceed
// independently, a large instance never holds back a small one, and an
// instance's result does not depend on the rest of the batch.
//
// Transforms along an instance's line use power-of-two FFTs only:
//  * Toeplitz products T x and T^T x (eq. grunwaldmatrix1/2): T is embedded
//    in a circulant of length 2 Qt, Qt the power of two >= n, zero padded
//    (a circulant of length >= 2n - 1 suffices); the real input is packed into
//    Qt complex values, and both products come back through one two-line
//    inverse FFT of length Qt.
//  * The DST-I S_n (eq. sine_transform): when n + 1 is a power of two, one
//    FFT of length n + 1 of the packed odd extension; otherwise the chirp-z
//    form: sin(pi j k/P) = Im of exp(i pi j^2/2P) exp(i pi k^2/2P)
//    exp(-i pi (k-j)^2/2P), P = n + 1, turns S_n x into a convolution with the
//    chirp exp(-i pi m^2/2P), done with FFTs of length Qs >= 2n - 1.
// An FFT whose data fit the workgroup's LDS runs there (Stockham passes of
// radix RAD); a longer one runs as two passes of LDS-sized FFTs through a
// global scratch buffer (Q = Q1 Q2: columns of length Q1 with the twiddle
// exp(-2 pi i q2 k1/Q), then rows of length Q2).  Inverse FFTs are forward
// FFTs of the conjugate.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/fde.h"
#include "fde_lines.hpp"
#include "fde_reduce.hpp"

namespace fde {
namespace bat {

constexpr int MMAX = 32;                    // longest outer or inner cycle
constexpr int TRI = MMAX * (MMAX + 1) / 2;  // packed upper triangle of a cycle
constexpr int FFT_BYTES = 65536;            // LDS for FFT data
constexpr int FFT_PAD = 64;                 // extra complex slots for padded column blocks

template <typename T>
struct Cap {
  static constexpr int value = FFT_BYTES / (int)sizeof(cx<T>);
  static constexpr int log = sizeof(T) == 8 ? 12 : 13;
};

struct Info {
  int iters, inner_iters, restarts, converged;
  int nonfinite, pad0;
  double relres_true, relres_est;
};

template <typename T>
struct Tab {
  const T *dp, *dm;     // d+, d-
  const T* dinv;        // D^{-1} = 2/(d+ + d-), null when the preconditioner has no D factor
  const T* finv;        // 1/F(theta_j), j = 1..n
  const cx<T>* lam;     // eigenvalues of the circulant embedding of T, k = 0..Qt, over 2 Qt
  const cx<T>* chirp;   // exp(i pi j^2/(2(n+1))), j = 0..n (chirp-z DST)
  const cx<T>* bhat;    // FFT of the chirp filter, times sqrt(2/(n+1))/Qs (chirp-z DST)
  // P_tri (partitioned tridiagonal solve, factors from tri_factor): per row
  // ai, cp, den, sv, sw; per chunk ar, cr, ra, rb, rc; work y (n values)
  const T *ai, *cp, *den, *sv, *sw, *ar, *cr, *ra, *rb, *rc;
  T* ty;
};

struct Inst {
  int n, logQt, logQs, blue;   // blue: chirp-z DST (n + 1 not a power of two)
  int prec, dside, time, precision;
  int kin, m, maxit, tp;       // tp: P_tri chunks (<= 512), chunk starts in tcs
  double tol, nu;
  const int* tcs;
  long off;                    // first element of the instance in the packed vectors
  Tab<double> t64;
  Tab<float> t32;
  double *V, *Z, *b, *t;       // (m+1) n, m n, n, n
  float *Vf, *uf, *zf, *tf;    // (kin+1) n, n, n, n
  cx<double> *fa, *fb;         // global FFT buffers (null when every transform fits in LDS)
};

enum : int {
  MODE_SOLVE = 0,     // solve M x = b for every instance
  MODE_STEP = 1,      // one implicit time step: b = rhs(x), then solve from x
  MODE_MATVEC = 2,    // out = M in
  MODE_TAU = 3,       // out = P^{-1} in (the instance's preconditioner, without an inner solve)
};

struct Args {
  const Inst* inst;
  int count, mode;        // count: instances in the batch (the stride of the per-step info)
  int nq, pad2;           // queue length: the first nq entries of `order` are solved here
  const int* order;       // instances in the order the queue hands them out
  unsigned* queue;        // ticket counter, zero at launch
  const cx<double>* tw64; // exp(-2 pi i m/TW), m < TW = 2^logTW
  const cx<float>* tw32;
  int logTW, pad0;
  const double* bin;      // MODE_SOLVE: packed right-hand sides; MODE_MATVEC / MODE_TAU: inputs
  int single, pad1;       // MODE_MATVEC / MODE_TAU: arithmetic in float32
  double* x;              // packed start vectors / solutions (MODE_STEP: states, advanced in place)
  Info* info;
  const int* step;        // when set, instance i reports to info[*step * count + i]
};

template <int NT>
struct Shm {
  cx<double> fft[FFT_BYTES / 16 + FFT_PAD];
  double red[(NT / 64) * MMAX];
  double tot[MMAX + 1];
  double h[MMAX + 1], c[MMAX + 1], c2[MMAX + 1];
  double R[TRI], cs[MMAX], sn[MMAX], g[MMAX + 1], sc[MMAX + 1], y[MMAX];
  double Ri[TRI], csi[MMAX], sni[MMAX], gi[MMAX + 1], sci[MMAX + 1], yi[MMAX];
  double s[4];
  int ticket;
};

template <typename T, int NT>
__device__ __forceinline__ cx<T>* lds_buf(Shm<NT>& sh) {
  return reinterpret_cast<cx<T>*>(sh.fft);
}

template <typename T>
__device__ __forceinline__ const Tab<T>& tab(const Inst& I);
template <>
__device__ __forceinline__ const Tab<double>& tab<double>(const Inst& I) { return I.t64; }
template <>
__device__ __forceinline__ const Tab<float>& tab<float>(const Inst& I) { return I.t32; }

template <typename T>
__device__ __forceinline__ const cx<T>* twt(const Args& a);
template <>
__device__ __forceinline__ const cx<double>* twt<double>(const Args& a) { return a.tw64; }
template <>
__device__ __forceinline__ const cx<float>* twt<float>(const Args& a) { return a.tw32; }

// ---------------------------------------------------------------------------
// FFTs
// ---------------------------------------------------------------------------

// One Stockham pass of radix R over nl lines of length 2^logL in LDS (line
// stride LS).  Butterfly j of a line reads x[j + r L/R], multiplies element r
// by w^(r k), k = j mod Ls, w = exp(-2 pi i/(Ls R)), applies DFT_R and writes
// y[(j - k) R + k + r Ls].  twsh converts r k into a twiddle-table index.
template <typename T, int NT, int R>
__device__ __forceinline__ void lds_pass(cx<T>* s, int nl, int logL, int LS, int logLs, const cx<T>* tw,
                                         int twsh) {
  constexpr int logR = R == 8 ? 3 : R == 4 ? 2 : 1;
  constexpr int NB = (Cap<T>::value + NT * R - 1) / (NT * R);
  const int logPr = logL - logR;
  const int Pr = 1 << logPr;
  const int nb = nl << logPr;
  const int Ls = 1 << logLs;
  const int tid = threadIdx.x;
  cx<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bf = tid + q * NT;
    if (bf < nb) {
      const cx<T>* src = s + (bf >> logPr) * LS + (bf & (Pr - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * Pr];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bf = tid + q * NT;
    if (bf < nb) {
      const int j = bf & (Pr - 1);
      const int k = j & (Ls - 1);
      if (logLs > 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = mul(v[q][r], tw[(r * k) << twsh]);
      }
      dftR<T, R>(v[q]);
      cx<T>* dst = s + (bf >> logPr) * LS + ((j - k) << logR) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ls] = v[q][r];
    }
  }
  __syncthreads();
}

// Forward FFT of nl lines of length 2^logL held in LDS; nl * 2^logL must not
// exceed Cap<T>.  The caller has synchronised after writing the data.
template <typename T, int NT, int RAD>
__device__ __forceinline__ void lds_fft(cx<T>* s, int nl, int logL, int LS, const cx<T>* tw, int logTW) {
  int logLs = 0;
  while (logLs < logL) {
    const int rem = logL - logLs;
    if (RAD >= 8 && rem >= 3) {
      lds_pass<T, NT, 8>(s, nl, logL, LS, logLs, tw, logTW - logLs - 3);
      logLs += 3;
    } else if (RAD >= 4 && rem >= 2) {
      lds_pass<T, NT, 4>(s, nl, logL, LS, logLs, tw, logTW - logLs - 2);
      logLs += 2;
    } else {
      lds_pass<T, NT, 2>(s, nl, logL, LS, logLs, tw, logTW - logLs - 1);
      logLs += 1;
    }
  }
}

// Forward FFT of length Q = 2^logQ > Cap<T> in global memory `a` (natural
// order in and out), through `tmp` (Q values) and the LDS staging area s.
template <typename T, int NT, int RAD>
__device__ __forceinline__ void staged_fft(cx<T>* a, cx<T>* tmp, int logQ, cx<T>* s, const cx<T>* tw, int logTW) {
  constexpr int LOGCAP = Cap<T>::log;
  const int tid = threadIdx.x;
  const int log1 = (logQ + 1) >> 1, log2 = logQ >> 1;
  const int Q1 = 1 << log1, Q2 = 1 << log2;
  const int tsh = logTW - logQ;
  // columns q2 (length Q1, stride Q2), CB at a time; out of place into tmp
  const int logCB = min(log2, LOGCAP - log1);
  const int CB = 1 << logCB;
  const int LS1 = Q1 + 1;
  for (int c0 = 0; c0 < Q2; c0 += CB) {
    for (int e = tid; e < (CB << log1); e += NT) {
      const int c = e & (CB - 1), q1 = e >> logCB;
      s[c * LS1 + q1] = a[(q1 << log2) + c0 + c];
    }
    __syncthreads();
    lds_fft<T, NT, RAD>(s, CB, log1, LS1, tw, logTW);
    for (int e = tid; e < (CB << log1); e += NT) {
      const int c = e & (CB - 1), k1 = e >> logCB;
      tmp[(k1 << log2) + c0 + c] = mul(s[c * LS1 + k1], tw[((c0 + c) * k1) << tsh]);
    }
    __syncthreads();
  }
  // rows k1 of tmp (length Q2), RB at a time; result k1 + Q1 k2 back into a
  const int logRB = min(log1, LOGCAP - log2);
  const int RB = 1 << logRB;
  const int LS2 = Q2 + 1;
  for (int r0 = 0; r0 < Q1; r0 += RB) {
    for (int e = tid; e < (RB << log2); e += NT) {
      const int r = e >> log2, q2 = e & (Q2 - 1);
      s[r * LS2 + q2] = tmp[((r0 + r) << log2) + q2];
    }
    __syncthreads();
    lds_fft<T, NT, RAD>(s, RB, log2, LS2, tw, logTW);
    for (int e = tid; e < (RB << log2); e += NT) {
      const int r = e & (RB - 1), k2 = e >> logRB;
      a[r0 + r + (k2 << log1)] = s[r * LS2 + k2];
    }
    __syncthreads();
  }
}

// nl lines of length 2^logQ, LS apart: in LDS or through global memory.
template <typename T, int NT, int RAD, bool INLDS>
__device__ __forceinline__ void fft_lines_any(cx<T>* buf, cx<T>* tmp, int nl, int logQ, int LS, Shm<NT>& sh,
                                              const cx<T>* tw, int logTW) {
  if constexpr (INLDS) {
    lds_fft<T, NT, RAD>(buf, nl, logQ, LS, tw, logTW);
  } else {
    for (int l = 0; l < nl; ++l) staged_fft<T, NT, RAD>(buf + (long)l * LS, tmp, logQ, lds_buf<T>(sh), tw, logTW);
  }
}

// ---------------------------------------------------------------------------
// Reductions (fixed order: per-thread strided sums, wavefront butterfly,
// waves in order)
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, Shm<NT>& sh) {
  double a[1] = {v};
  block_multi_sum<1>(a, sh.red, sh.tot);
  return sh.tot[0];
}

// ---------------------------------------------------------------------------
// Line operators
// ---------------------------------------------------------------------------

// y_k = post_k (S_n u)_k, u_j = s pre_j x_j (pre, post may be null), k < n.
template <typename T, int NT, int RAD, bool INLDS, typename Tin, typename Tout>
__device__ __forceinline__ void dst_op(const Inst& I, Shm<NT>& sh, const cx<T>* tw, int logTW, const Tin* x, const T* pre,
                       double s, Tout* y, const T* post) {
  const Tab<T>& tb = tab<T>(I);
  const int n = I.n, tid = threadIdx.x;
  const int logQ = I.logQs, Q = 1 << logQ;
  cx<T>* buf = INLDS ? lds_buf<T>(sh) : reinterpret_cast<cx<T>*>(I.fa);
  cx<T>* tmp = reinterpret_cast<cx<T>*>(I.fb);
  const T ss = (T)s;
  if (!I.blue) {
    // odd extension of length 2P (P = Q = n + 1), packed: z_m = u_2m + i u_2m+1,
    // u_t = x_t (0 < t < P), u_0 = u_P = 0, u_{2P-t} = -u_t
    for (int m = tid; m < Q; m += NT) {
      T v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = 2 * m + h;
        T val = T(0);
        if (t != 0 && t != Q) {
          const int j = t < Q ? t - 1 : 2 * Q - t - 1;
          val = (T)x[j] * ss;
          if (pre) val *= pre[j];
          if (t > Q) val = -val;
        }
        v[h] = val;
      }
      buf[m] = mk(v[0], v[1]);
    }
  } else {
    for (int p = tid; p < Q; p += NT) {
      cx<T> v = mk(T(0), T(0));
      if (p < n) {
        T u = (T)x[p] * ss;
        if (pre) u *= pre[p];
        const cx<T> c = tb.chirp[p + 1];
        v = mk(u * c.x, u * c.y);
      }
      buf[p] = v;
    }
  }
  __syncthreads();
  fft_lines_any<T, NT, RAD, INLDS>(buf, tmp, 1, logQ, Q, sh, tw, logTW);
  if (I.blue) {
    for (int k = tid; k < Q; k += NT) buf[k] = conj(mul(buf[k], tb.bhat[k]));
    __syncthreads();
    fft_lines_any<T, NT, RAD, INLDS>(buf, tmp, 1, logQ, Q, sh, tw, logTW);
    // convolution value k-1 is conj(buf[k-1]); y_k = Im(chirp_k conj(buf[k-1]))
    for (int k = tid; k < n; k += NT) {
      const cx<T> r = buf[k], c = tb.chirp[k + 1];
      T v = c.y * r.x - c.x * r.y;
      if (post) v *= post[k];
      y[k] = (Tout)v;
    }
  } else {
    // U_k = E_k + W_2P^k O_k from bins k and P-k; y_k = -Im(U_k)/sqrt(2P)
    const int sh2 = logTW - logQ - 1;
    const T rs = (T)(1.0 / sqrt(2.0 * (double)Q));
    for (int k = tid; k < n; k += NT) {
      const int kk = k + 1;
      const cx<T> A = buf[kk], B = buf[Q - kk];
      const T dx = A.x - B.x, dy = A.y + B.y;
      const cx<T> w = tw[kk << sh2];
      T v = -T(0.5) * ((A.y - B.y) - w.x * dx + w.y * dy) * rs;
      if (post) v *= post[k];
      y[k] = (Tout)v;
    }
  }
  __syncthreads();
}

// out_i = c0 base_i + c1 x_i + c2 (d+_i (T x)_i + d-_i (T^T x)_i); returns the
// workgroup sum of out_i^2 when want_norm (0 otherwise).  base may be null.
template <typename T, int NT, int RAD, bool INLDS, typename Tio>
__device__ __forceinline__ double toep_op(const Inst& I, Shm<NT>& sh, const cx<T>* tw, int logTW, const Tio* x,
                          const double* base, double c0, double c1, double c2, Tio* out, bool want_norm) {
  const Tab<T>& tb = tab<T>(I);
  const int n = I.n, tid = threadIdx.x;
  const int logQ = I.logQt, Q = 1 << logQ;
  cx<T>* buf = INLDS ? lds_buf<T>(sh) : reinterpret_cast<cx<T>*>(I.fa);
  cx<T>* tmp = reinterpret_cast<cx<T>*>(I.fb);
  cx<T>* buf2 = buf + Q;
  for (int m = tid; m < Q; m += NT) {
    const int i0 = 2 * m, i1 = 2 * m + 1;
    buf[m] = mk(i0 < n ? (T)x[i0] : T(0), i1 < n ? (T)x[i1] : T(0));
  }
  __syncthreads();
  fft_lines_any<T, NT, RAD, INLDS>(buf, tmp, 1, logQ, Q, sh, tw, logTW);
  // bins k and Q-k give X_k and X_{k+Q} of the real 2Q-point input; the two
  // products' spectra are folded back into Q-point packed inverse inputs
  const int shw = logTW - logQ - 1;
  for (int k = tid; k <= (Q >> 1); k += NT) {
    const int k2 = (Q - k) & (Q - 1);
    const cx<T> Zk = buf[k], Zk2 = buf[k2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && k2 == k) break;
      const int kk = side == 0 ? k : k2;
      const cx<T> A = side == 0 ? Zk : Zk2, B = side == 0 ? Zk2 : Zk;
      const cx<T> E = mk(T(0.5) * (A.x + B.x), T(0.5) * (A.y - B.y));
      const cx<T> O = mk(T(0.5) * (A.y + B.y), -T(0.5) * (A.x - B.x));
      const cx<T> W = tw[kk << shw];
      const cx<T> WO = mul(W, O);
      const cx<T> Xa = add(E, WO), Xb = sub(E, WO);
      const cx<T> la = tb.lam[kk], lb = conj(tb.lam[Q - kk]);
      const cx<T> Wc = conj(W);
      const cx<T> y1a = mul(la, Xa), y1b = mul(lb, Xb);
      const cx<T> y2a = mul(conj(la), Xa), y2b = mul(conj(lb), Xb);
      const cx<T> z1 = add(add(y1a, y1b), mul_i(mul(Wc, sub(y1a, y1b))));
      const cx<T> z2 = add(add(y2a, y2b), mul_i(mul(Wc, sub(y2a, y2b))));
      buf[kk] = conj(z1);
      buf2[kk] = conj(z2);
    }
  }
  __syncthreads();
  fft_lines_any<T, NT, RAD, INLDS>(buf, tmp, 2, logQ, Q, sh, tw, logTW);
  double ss = 0.0;
  for (int m = tid; m < Q; m += NT) {
    const cx<T> r1 = buf[m], r2 = buf2[m];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * m + h;
      if (i < n) {
        const T y1 = h == 0 ? r1.x : -r1.y;
        const T y2 = h == 0 ? r2.x : -r2.y;
        T v = (T)c2 * (tb.dp[i] * y1 + tb.dm[i] * y2) + (T)c1 * (T)x[i];
        if (base) v = (T)((double)v + c0 * base[i]);
        out[i] = (Tio)v;
        ss += (double)v * (double)v;
      }
    }
  }
  __syncthreads();
  return want_norm ? block_sum<NT>(ss, sh) : 0.0;
}

template <typename T, int NT, int RAD, typename Tin, typename Tout>
__device__ __forceinline__ void dst_any(const Inst& I, Shm<NT>& sh, const cx<T>* tw, int logTW, const Tin* x,
                                        const T* pre, double s, Tout* y, const T* post) {
  if ((1 << I.logQs) <= Cap<T>::value)
    dst_op<T, NT, RAD, true>(I, sh, tw, logTW, x, pre, s, y, post);
  else
    dst_op<T, NT, RAD, false>(I, sh, tw, logTW, x, pre, s, y, post);
}

template <typename T, int NT, int RAD, typename Tio>
__device__ __forceinline__ double toep_any(const Inst& I, Shm<NT>& sh, const cx<T>* tw, int logTW, const Tio* x,
                                           const double* base, double c0, double c1, double c2, Tio* out,
                                           bool want_norm) {
  if ((2 << I.logQt) <= Cap<T>::value)
    return toep_op<T, NT, RAD, true>(I, sh, tw, logTW, x, base, c0, c1, c2, out, want_norm);
  return toep_op<T, NT, RAD, false>(I, sh, tw, logTW, x, base, c0, c1, c2, out, want_norm);
}

// z = P_tri^{-1}(s v) (Table 2) by the partitioned elimination: chunk k's
// interior is swept with the precomputed pivots (chunks are taken k = tid,
// tid + NT, ..., so any chunk count up to TRI_CHUNKS works with any
// workgroup size), parallel cyclic reduction over the chunk interfaces runs
// in LDS, and every row is then recovered from its interior solution and the
// two neighbouring interfaces.
constexpr int TRI_CHUNKS = MMAX * 16;   // chunk count limit (assembly takes min(TRI_CHUNKS, n/2))

template <typename T, int NT, typename Tin, typename Tout>
__device__ __forceinline__ void tri_wg(const Inst& I, Shm<NT>& sh, const Tin* v, double s, Tout* z) {
  constexpr int KP = (TRI_CHUNKS + NT - 1) / NT;   // chunks per thread
  static_assert(4 * TRI_CHUNKS * sizeof(double) <= FFT_BYTES, "P_tri interface arrays exceed the LDS area");
  const Tab<T>& tb = tab<T>(I);
  const int tid = threadIdx.x, p = I.tp, n = I.n;
  const int* cs = I.tcs;
  T* y = tb.ty;
  T* sA = reinterpret_cast<T*>(sh.fft);
  T* sB = sA + TRI_CHUNKS;
  T* sC = sB + TRI_CHUNKS;
  T* sD = sC + TRI_CHUNKS;
  const T scale = (T)s;
  for (int k = tid; k < p; k += NT) {
    const int s0 = cs[k], r = cs[k + 1] - 1;
    T d = T(0);
    for (int i = s0; i < r; ++i) {
      d = ((T)v[i] * scale - tb.ai[i] * d) * tb.den[i];
      y[i] = d;
    }
    T yn = T(0);
    for (int i = r - 1; i >= s0; --i) {
      yn = y[i] - tb.cp[i] * yn;
      y[i] = yn;
    }
    sD[k] = (T)v[r] * scale - tb.ar[k] * (r > s0 ? y[r - 1] : T(0));
  }
  __syncthreads();
  for (int k = tid; k < p; k += NT) {
    if (k + 1 < p) {
      const int s2 = cs[k + 1], q2 = cs[k + 2] - 1 - s2;
      if (q2 >= 1) sD[k] -= tb.cr[k] * y[s2];
    }
    sA[k] = tb.ra[k];
    sB[k] = tb.rb[k];
    sC[k] = tb.rc[k];
  }
  __syncthreads();
  for (int st = 1; st < p; st <<= 1) {
    T nA[KP], nB[KP], nC[KP], nD[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) {
      const int k = tid + q * NT;
      nA[q] = nB[q] = nC[q] = nD[q] = T(0);
      if (k < p) {
        const int km = k - st, kp = k + st;
        nB[q] = sB[k];
        nD[q] = sD[k];
        if (km >= 0) {
          const T al = -sA[k] / sB[km];
          nA[q] = al * sA[km];
          nB[q] += al * sC[km];
          nD[q] += al * sD[km];
        }
        if (kp < p) {
          const T ga = -sC[k] / sB[kp];
          nC[q] = ga * sC[kp];
          nB[q] += ga * sA[kp];
          nD[q] += ga * sD[kp];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KP; ++q) {
      const int k = tid + q * NT;
      if (k < p) {
        sA[k] = nA[q];
        sB[k] = nB[q];
        sC[k] = nC[q];
        sD[k] = nD[q];
      }
    }
    __syncthreads();
  }
  for (int k = tid; k < p; k += NT) sD[k] = sD[k] / sB[k];   // X_k
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    int k = (int)(((long)i * p) / n);
    while (k + 1 < p && cs[k + 1] <= i) ++k;
    const int r = cs[k + 1] - 1;
    T out;
    if (i == r) {
      out = sD[k];
    } else {
      out = y[i] - sD[k] * tb.sw[i];
      if (k > 0) out -= sD[k - 1] * tb.sv[i];
    }
    z[i] = (Tout)out;
  }
  __syncthreads();
}

// z = P^{-1}(s v) in precision T (eq. prop_1D; Section 3.1 Case I; Table 2):
// left D:  z = S (F^{-1} . S (D^{-1} s v));  right D: z = D^{-1} S (F^{-1} . S (s v)).
// tmp holds the intermediate (n values of T).
template <typename T, int NT, int RAD, typename Tin, typename Tout>
__device__ __forceinline__ void tau_apply(const Inst& I, Shm<NT>& sh, const cx<T>* tw, int logTW, const Tin* v, double s,
                          Tout* z, T* tmp) {
  const Tab<T>& tb = tab<T>(I);
  if (I.prec == FDE_P_NONE) {
    for (int i = threadIdx.x; i < I.n; i += NT) z[i] = (Tout)((T)v[i] * (T)s);
    __syncthreads();
    return;
  }
  if (I.prec == FDE_P_TRI) {
    tri_wg<T, NT>(I, sh, v, s, z);
    return;
  }
  const bool left = I.dside == FDE_D_LEFT;
  dst_any<T, NT, RAD>(I, sh, tw, logTW, v, left ? tb.dinv : (const T*)nullptr, s, tmp, tb.finv);
  dst_any<T, NT, RAD>(I, sh, tw, logTW, (const T*)tmp, (const T*)nullptr, 1.0, z,
                      left ? (const T*)nullptr : tb.dinv);
}

// ---------------------------------------------------------------------------
// Gram-Schmidt over the stored basis V (nk vectors, leading dimension n;
// basis vector q = sc[q] V_q).  A sweep reads w once: with UPD it first
// subtracts sum_{q<nk} coef[q] V_q from w (coef[q] = sc[q] h_q); then it
// forms the dots <V_q, w> for d0 <= q < d0 + KC (q < nk) into tot[q - d0],
// or with NORM the sum of squares into tot[0].  Dots are taken KC at a time
// to bound the accumulators; loads past the last vector re-read vector nk-1
// and carry no weight.
// ---------------------------------------------------------------------------
template <typename T, int NT, int KC, bool UPD, bool NORM>
__device__ __forceinline__ void cgs_sweep(const T* V, int nk, int d0, T* w, int n, const double* coef, Shm<NT>& sh) {
  constexpr int NA = NORM ? 1 : KC;
  double acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  const long ld = n;
  const int nd = NORM ? 0 : min(KC, nk - d0);
  for (int i = threadIdx.x; i < n; i += NT) {
    double u = (double)w[i];
    if (UPD) {
#pragma unroll
      for (int q0 = 0; q0 < MMAX; q0 += 8) {
        if (q0 < nk) {
          T v[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) v[t] = V[(long)min(q0 + t, nk - 1) * ld + i];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (q0 + t < nk) u -= coef[q0 + t] * (double)v[t];
        }
      }
      const T ut = (T)u;
      w[i] = ut;
      u = (double)ut;
    }
    if (NORM) {
      acc[0] += u * u;
    } else {
#pragma unroll
      for (int q0 = 0; q0 < KC; q0 += 8) {
        if (q0 < nd) {
          T v[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) v[t] = V[(long)min(d0 + q0 + t, nk - 1) * ld + i];
#pragma unroll
          for (int t = 0; t < 8; ++t) acc[q0 + t] += (double)v[t] * u;
        }
      }
    }
  }
  block_multi_sum<NA>(acc, sh.red, sh.tot);
}

template <typename T, int NT, bool UPD>
__device__ __forceinline__ void cgs_dots(const T* V, int nk, int d0, T* w, int n, const double* coef, Shm<NT>& sh) {
  if (nk - d0 <= 8) cgs_sweep<T, NT, 8, UPD, false>(V, nk, d0, w, n, coef, sh);
  else cgs_sweep<T, NT, 16, UPD, false>(V, nk, d0, w, n, coef, sh);
}

// CGS2 of w against basis vectors 0..j: h (LDS, j+1 values) and ||w||.
template <typename T, int NT>
__device__ __forceinline__ double cgs2(const T* V, int j, T* w, int n, const double* sc, Shm<NT>& sh) {
  const int nk = j + 1;
  const int tid = threadIdx.x;
  for (int d0 = 0; d0 < nk; d0 += 16) {
    cgs_dots<T, NT, false>(V, nk, d0, w, n, nullptr, sh);
    if (tid < min(16, nk - d0)) {
      const int q = d0 + tid;
      const double hq = sc[q] * sh.tot[tid];
      sh.h[q] = hq;
      sh.c[q] = sc[q] * hq;
    }
    __syncthreads();
  }
  for (int d0 = 0; d0 < nk; d0 += 16) {
    if (d0 == 0) cgs_dots<T, NT, true>(V, nk, 0, w, n, sh.c, sh);
    else cgs_dots<T, NT, false>(V, nk, d0, w, n, nullptr, sh);
    if (tid < min(16, nk - d0)) {
      const int q = d0 + tid;
      const double hq = sc[q] * sh.tot[tid];
      sh.h[q] += hq;
      sh.c2[q] = sc[q] * hq;
    }
    __syncthreads();
  }
  cgs_sweep<T, NT, 1, true, true>(V, nk, 0, w, n, sh.c2, sh);
  return sqrt(sh.tot[0]);
}

// Rotations 0..j-1 applied to column j (h[0..j], hn), rotation j formed,
// g updated; column stored packed in R.  Thread 0; returns |g[j+1]|.
__device__ __forceinline__ double givens_col(const double* h, double hn, int j, double* R, double* cs, double* sn,
                                    double* g) {
  double* col = R + j * (j + 1) / 2;
  for (int i = 0; i <= j; ++i) col[i] = h[i];
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[j];
  const double rho = hypot(a, hn);
  double c = 1.0, s = 0.0;
  if (rho != 0.0) {
    c = a / rho;
    s = hn / rho;
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = rho;
  const double gj = g[j];
  g[j + 1] = -s * gj;
  g[j] = c * gj;
  return fabs(g[j + 1]);
}

// y = R^{-1} g for the leading k x k block (packed columns).  Thread 0.
__device__ __forceinline__ void backsolve(const double* R, const double* g, int k, double* y) {
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= R[l * (l + 1) / 2 + i] * y[l];
    y[i] = s / R[i * (i + 1) / 2 + i];
  }
}

// ---------------------------------------------------------------------------
// Preconditioner of the outer FGMRES: z = P^{-1}(s v), float64 or mixed.
// Mixed: kin float32 GMRES steps on M (right-preconditioned by the float32
// tau solve) from a zero start, then the float32 tau solve of the result;
// kin = 0 is the float32 tau solve alone.
// ---------------------------------------------------------------------------
template <int NT, int RAD>
__device__ __forceinline__ void precondition(const Args& a, const Inst& I, Shm<NT>& sh, const double* v, double s, double* z,
                             int& inner_iters) {
  const int n = I.n, tid = threadIdx.x;
  if (I.precision == FDE_FP64) {
    tau_apply<double, NT, RAD>(I, sh, a.tw64, a.logTW, v, s, z, I.t);
    return;
  }
  const cx<float>* tw = a.tw32;
  if (I.kin == 0) {
    tau_apply<float, NT, RAD>(I, sh, tw, a.logTW, v, s, z, I.tf);
    return;
  }
  float* Vf = I.Vf;
  double ss = 0.0;
  for (int i = tid; i < n; i += NT) {
    const float u = (float)(v[i] * s);
    Vf[i] = u;
    ss += (double)u * (double)u;
  }
  const double nrm = sqrt(block_sum<NT>(ss, sh));
  if (tid == 0) {
    sh.sci[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    sh.gi[0] = nrm;
    for (int i = 1; i <= MMAX; ++i) sh.gi[i] = 0.0;
  }
  __syncthreads();
  int ki = 0;
  if (nrm > 0.0 && isfinite(nrm)) {
    for (int i = 0; i < I.kin; ++i) {
      float* vi = Vf + (long)i * n;
      float* wi = Vf + (long)(i + 1) * n;
      tau_apply<float, NT, RAD>(I, sh, tw, a.logTW, (const float*)vi, sh.sci[i], I.zf, I.tf);
      toep_any<float, NT, RAD>(I, sh, tw, a.logTW, (const float*)I.zf, nullptr, 0.0, I.nu, 1.0, wi, false);
      const double hn = cgs2<float, NT>(Vf, i, wi, n, sh.sci, sh);
      if (tid == 0) {
        givens_col(sh.h, hn, i, sh.Ri, sh.csi, sh.sni, sh.gi);
        sh.sci[i + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
      }
      __syncthreads();
      ki = i + 1;
      if (!(hn > 0.0) || !isfinite(hn)) break;
    }
  }
  inner_iters += ki;
  if (tid == 0) {
    backsolve(sh.Ri, sh.gi, ki, sh.yi);
    for (int i = 0; i < ki; ++i) sh.yi[i] *= sh.sci[i];
  }
  __syncthreads();
  float* u = I.uf;
  for (int e = tid; e < n; e += NT) {
    float acc = 0.0f;
    for (int i = 0; i < ki; ++i) acc += (float)sh.yi[i] * Vf[(long)i * n + e];
    u[e] = acc;
  }
  __syncthreads();
  tau_apply<float, NT, RAD>(I, sh, tw, a.logTW, (const float*)u, 1.0, z, I.tf);
}

// ---------------------------------------------------------------------------
// One instance: right-preconditioned FGMRES(m), CGS2, Givens; cycles end on
// the estimate, breakdown, m steps or maxit, and the float64 true residual
// decides convergence.
// ---------------------------------------------------------------------------
template <int NT, int RAD>
__device__ __forceinline__ void solve_one(const Args& a, const Inst& I, Shm<NT>& sh, Info& res) {
  const int n = I.n, m = I.m, tid = threadIdx.x;
  double* x = a.x + I.off;
  const cx<double>* tw = a.tw64;
  const int logTW = a.logTW;
  const double* b;
  if (a.mode == MODE_STEP) {
    // right-hand side of the time step from the current state (f = 0)
    if (I.time == FDE_T_EULER) {
      for (int i = tid; i < n; i += NT) I.b[i] = I.nu * x[i];
      __syncthreads();
    } else {
      toep_any<double, NT, RAD>(I, sh, tw, logTW, (const double*)x, nullptr, 0.0, I.nu, -1.0, I.b, false);
    }
    b = I.b;
  } else {
    b = a.bin + I.off;
  }
  res = Info{0, 0, 0, 0, 0, 0, 0.0, 0.0};
  double ss = 0.0;
  for (int i = tid; i < n; i += NT) ss += b[i] * b[i];
  const double bnorm = sqrt(block_sum<NT>(ss, sh));
  if (!isfinite(bnorm)) {
    res.nonfinite = 1;
    res.relres_true = bnorm;
    return;
  }
  if (bnorm == 0.0) {
    for (int i = tid; i < n; i += NT) x[i] = 0.0;
    __syncthreads();
    res.converged = 1;
    return;
  }
  const double tolabs = I.tol * bnorm;
  double* V = I.V;
  double* Z = I.Z;
  double beta = sqrt(toep_any<double, NT, RAD>(I, sh, tw, logTW, (const double*)x, b, 1.0, -I.nu, -1.0, V, true));
  res.relres_true = beta / bnorm;
  if (!isfinite(beta)) {
    res.nonfinite = 1;
    return;
  }
  int iters = 0, inner = 0, restarts = 0;
  double est = beta;
  bool conv = beta <= tolabs;
  while (!conv && iters < I.maxit) {
    if (tid == 0) {
      sh.sc[0] = 1.0 / beta;
      sh.g[0] = beta;
      for (int i = 1; i <= MMAX; ++i) sh.g[i] = 0.0;
    }
    __syncthreads();
    int k = 0;
    bool bad = false;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (long)j * n;
      double* w = V + (long)(j + 1) * n;
      double* zj = Z + (long)j * n;
      precondition<NT, RAD>(a, I, sh, vj, sh.sc[j], zj, inner);
      toep_any<double, NT, RAD>(I, sh, tw, logTW, (const double*)zj, nullptr, 0.0, I.nu, 1.0, w, false);
      const double hn = cgs2<double, NT>(V, j, w, n, sh.sc, sh);
      ++iters;
      if (tid == 0) {
        sh.s[0] = givens_col(sh.h, hn, j, sh.R, sh.cs, sh.sn, sh.g);
        sh.sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
      }
      __syncthreads();
      est = sh.s[0];
      k = j + 1;
      bad = !isfinite(est) || !isfinite(hn);
      if (est <= tolabs || hn == 0.0 || bad || iters >= I.maxit) break;
    }
    if (bad) {
      res.nonfinite = 1;
      break;
    }
    if (tid == 0) backsolve(sh.R, sh.g, k, sh.y);
    __syncthreads();
    for (int e = tid; e < n; e += NT) {
      double acc = x[e];
      for (int i = 0; i < k; ++i) acc += sh.y[i] * Z[(long)i * n + e];
      x[e] = acc;
    }
    __syncthreads();
    beta = sqrt(toep_any<double, NT, RAD>(I, sh, tw, logTW, (const double*)x, b, 1.0, -I.nu, -1.0, V, true));
    if (!isfinite(beta)) {
      res.nonfinite = 1;
      break;
    }
    conv = beta <= tolabs;
    if (!conv && iters < I.maxit) ++restarts;
  }
  res.iters = iters;
  res.inner_iters = inner;
  res.restarts = restarts;
  res.converged = conv ? 1 : 0;
  res.relres_true = beta / bnorm;
  res.relres_est = est / bnorm;
}

// One operator application for an instance (matvec or preconditioner), in
// float64 or float32 arithmetic on float64 input and output.
template <int NT, int RAD>
__device__ __forceinline__ void apply_one(const Args& a, const Inst& I, Shm<NT>& sh) {
  const double* in = a.bin + I.off;
  double* out = a.x + I.off;
  if (a.mode == MODE_MATVEC) {
    if (a.single) toep_any<float, NT, RAD>(I, sh, a.tw32, a.logTW, in, nullptr, 0.0, I.nu, 1.0, out, false);
    else toep_any<double, NT, RAD>(I, sh, a.tw64, a.logTW, in, nullptr, 0.0, I.nu, 1.0, out, false);
  } else {
    if (a.single) tau_apply<float, NT, RAD>(I, sh, a.tw32, a.logTW, in, 1.0, out, I.tf);
    else tau_apply<double, NT, RAD>(I, sh, a.tw64, a.logTW, in, 1.0, out, I.t);
  }
}

// Waves per SIMD the kernel is compiled for.  The workgroup's LDS (Shm, about
// 81 KB at 512 threads) admits one workgroup per CU, i.e. two waves per SIMD
// at 512 threads, so the register budget is that of two waves (256 VGPRs):
// asking for more waves would only cap the registers and spill.
constexpr int BATCH_WAVES_PER_EU = 2;

// Persistent kernel: workgroups take instances from the ticket queue until
// it runs dry (every workgroup reaches the exit).  Every device function of
// the engine is inlined into this one kernel: the build with out-of-line
// calls gave wrong float32 results at -O3 (staged chirp-z transforms, radix
// 8) that the same source at -O1, the inlined build and a bounds-checked CPU
// emulation do not show.
template <int NT, int RAD>
__global__ void __launch_bounds__(NT, BATCH_WAVES_PER_EU) batch_kernel(Args a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Shm<NT>& sh = *reinterpret_cast<Shm<NT>*>(smem_raw);
  for (;;) {
    if (threadIdx.x == 0) sh.ticket = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int t = sh.ticket;
    __syncthreads();
    if (t >= a.nq) break;
    const int idx = a.order[t];
    const Inst& I = a.inst[idx];
    if (a.mode >= MODE_MATVEC) {
      apply_one<NT, RAD>(a, I, sh);
      continue;
    }
    Info res;
    solve_one<NT, RAD>(a, I, sh, res);
    if (threadIdx.x == 0) {
      const long slot = a.step ? (long)(*a.step) * a.count + idx : idx;
      a.info[slot] = res;
    }
    __syncthreads();
  }
}

}  // namespace bat
}  // namespace fde
