// Line transforms for the fractional-diffusion solver, gfx950.
//
// A "line" is one row (x direction, contiguous) or one column (y direction,
// stride n1) of the unknowns.  Every transform the method needs along a line
// is built on one power-of-two complex FFT of length P = n + 1 held in LDS:
//
//  * DST-I of length n (the matrix S_n of eq. sine_transform).  The odd
//    extension u of x (length 2P) is real, so its 2P-point DFT is obtained from
//    the P-point FFT of z_j = u_{2j} + i u_{2j+1} and a pairing of bins k and
//    P-k; the DST values are -Im(U_k)/sqrt(2P).
//  * Toeplitz products T z and T^T z (eqs. grunwaldmatrix1/2).  T is embedded
//    in a circulant of length 2P whose eigenvalues lambda are precomputed; the
//    eigenvalues of the circulant that embeds T^T are conj(lambda).  The real,
//    zero-padded z is transformed with one packed P-point FFT, multiplied by
//    lambda and by conj(lambda), and brought back by two packed P-point inverse
//    FFTs (each real 2P-point sequence is recovered from a P-point complex one).
//
// The FFT is a Stockham autosort FFT (radix 8, with one radix-4 or radix-2
// pass when log2 P is not a multiple of 3).  Each workgroup transforms B lines
// at once; every thread owns EPT = 8 elements in the elementwise phases and
// EPT/R butterflies in a radix-R pass, so blockDim = B*P/8.  Twiddles come from
// a host-computed float64 table W2[m] = exp(-2 pi i m/(2P)), m < 2P.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fde {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by i and by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return mk(-a.y, a.x); }
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return mk(a.y, -a.x); }

// ---------------------------------------------------------------------------
// Small forward DFTs (exponent sign -1), natural order in and out.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0];
  v[0] = add(a, v[1]);
  v[1] = sub(a, v[1]);
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& v0, cx<T>& v1, cx<T>& v2, cx<T>& v3) {
  cx<T> a = add(v0, v2), b = sub(v0, v2), c = add(v1, v3), d = mul_mi(sub(v1, v3));
  v0 = add(a, c);
  v2 = sub(a, c);
  v1 = add(b, d);
  v3 = sub(b, d);
}

template <typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T c = T(0.70710678118654752440084436210484903928);
  // even and odd halves
  dft4(v[0], v[2], v[4], v[6]);
  dft4(v[1], v[3], v[5], v[7]);
  cx<T> o1 = v[3], o2 = v[5], o3 = v[7];
  o1 = mk(c * (o1.x + o1.y), c * (o1.y - o1.x));   // * exp(-i pi/4)
  o2 = mul_mi(o2);                                  // * exp(-i pi/2)
  o3 = mk(c * (o3.y - o3.x), -c * (o3.x + o3.y));  // * exp(-3 i pi/4)
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
  v[0] = add(e0, o0);
  v[4] = sub(e0, o0);
  v[1] = add(e1, o1);
  v[5] = sub(e1, o1);
  v[2] = add(e2, o2);
  v[6] = sub(e2, o2);
  v[3] = add(e3, o3);
  v[7] = sub(e3, o3);
}

template <typename T, int R>
__device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 8) dft8(v);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
  else dft2(v);
}

// One Stockham pass of radix R over B lines of length P in LDS (line stride
// LS complex elements).  Ls = product of the radices of earlier passes.
// Butterfly j of a line reads x[j + r P/R], multiplies element r by
// w^(r k) with k = j mod Ls and w = exp(-2 pi i/(Ls R)), applies DFT_R and
// writes y[(j - k) R + k + r Ls].  In place: all reads finish before a
// barrier, then all writes.
template <typename T, int EPT, int R>
__device__ __forceinline__ void fft_pass(cx<T>* buf, int LS, int logPr, int Ls, int logR,
                                         const cx<T>* __restrict__ W2, int twshift) {
  constexpr int NB = EPT / R;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int Pr = 1 << logPr;
  cx<T> v[NB][R];
  int base[NB], jj[NB];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = tid + s * nth;
    const int line = b >> logPr;
    const int j = b & (Pr - 1);
    base[s] = line * LS;
    jj[s] = j;
#pragma unroll
    for (int r = 0; r < R; ++r) v[s][r] = buf[base[s] + j + r * Pr];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int j = jj[s];
    const int k = j & (Ls - 1);
    if (Ls > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[s][r] = mul(v[s][r], W2[(r * k) << twshift]);
    }
    dftR<T, R>(v[s]);
    const int o = base[s] + ((j - k) << logR) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[o + r * Ls] = v[s][r];
  }
  __syncthreads();
}

// Forward FFT of length P = 2^logP on every line in LDS.  The caller has
// synchronised after writing the input; results are visible on return.
template <typename T, int EPT>
__device__ __forceinline__ void fft_lines(cx<T>* buf, int LS, int logP, const cx<T>* __restrict__ W2) {
  int logLs = 0;
  while (logLs < logP) {
    const int rem = logP - logLs;
    const int Ls = 1 << logLs;
    if (rem >= 3) {
      fft_pass<T, EPT, 8>(buf, LS, logP - 3, Ls, 3, W2, logP + 1 - logLs - 3);
      logLs += 3;
    } else if (rem == 2) {
      fft_pass<T, EPT, 4>(buf, LS, logP - 2, Ls, 2, W2, logP + 1 - logLs - 2);
      logLs += 2;
    } else {
      fft_pass<T, EPT, 2>(buf, LS, logP - 1, Ls, 1, W2, logP + 1 - logLs - 1);
      logLs += 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Line programs.
// ---------------------------------------------------------------------------
enum : int {
  LF_DST1 = 1,      // v <- S_n (pre .* sc * in)
  LF_FDST2 = 2,     // v <- S_n (v ./ F)          F(line, m) = fline[line] + felem[m]
  LF_STOREZ = 4,    // zout <- post .* v          (the preconditioned vector)
  LF_TOEP = 8,      // out <- bscale*base + tscale*(cplus .* T v + cminus .* T^T v)
  LF_EXTBASE = 16,  // base is the array `base` (otherwise base = v)
};

template <typename T>
struct LineArgs {
  const T* in;        // input vector
  const T* pre;       // optional elementwise factor applied to the input
  const double* sc;   // optional device scalar factor applied to the input
  const T* fline;     // symbol samples indexed by line (LF_FDST2)
  const T* felem;     // symbol samples indexed by position along the line
  const T* post;      // optional elementwise factor applied after the DSTs
  T* zout;            // LF_STOREZ output
  const T* cplus;     // LF_TOEP coefficients
  const T* cminus;
  const T* base;      // LF_EXTBASE
  T bscale, tscale;
  T* out;             // final output (the DST result when LF_TOEP is off)
  const cx<T>* W2;    // exp(-2 pi i m/(2P)), m < 2P
  const cx<T>* lam;   // circulant eigenvalues, bins 0..P
  const int* skip;    // nonzero: the kernel returns at once
  long ls, es;        // line stride and element stride in the vectors
  int n, P, logP, nlines, B, logB, LS, ntiles;
};

// XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs,
// so workgroup b runs on XCD b % 8.  Consecutive tiles (neighbouring columns
// that share 128-byte lines) are given to workgroups of the same XCD.  The grid
// has 8*ceil(ntiles/8) workgroups; the surplus ones return.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (ntiles + 7) >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

template <typename T, bool COLS, int FL>
__global__ void __launch_bounds__(512) line_kernel(LineArgs<T> a) {
  constexpr int EPT = 8;
  if (a.skip && *a.skip) return;
  const int tile = xcd_tile(a.ntiles);
  if (tile >= a.ntiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);

  const int tid = threadIdx.x, nth = blockDim.x;
  const int P = a.P, logP = a.logP, n = a.n, LS = a.LS;
  const int line0 = tile * a.B;

  int li[EPT], mi[EPT];
  long gi[EPT];
  bool ok[EPT];
  T v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nth;
    int l, m;
    if (COLS) {
      l = e & (a.B - 1);
      m = e >> a.logB;
    } else {
      l = e >> logP;
      m = e & (P - 1);
    }
    li[i] = l;
    mi[i] = m;
    ok[i] = (m < n) && (line0 + l < a.nlines);
    gi[i] = (long)(line0 + l) * a.ls + (long)m * a.es;
  }
  {
    const T s = a.sc ? (T)(*a.sc) : T(1);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      T x = T(0);
      if (ok[i]) {
        x = a.in[gi[i]] * s;
        if (a.pre) x *= a.pre[gi[i]];
      }
      v[i] = x;
    }
  }

  const T rs2P = T(1) / sqrt(T(2 * P));

  // ---- DST-I: v <- S_n v --------------------------------------------------
  auto dst = [&]() {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      T* f = reinterpret_cast<T*>(buf + li[i] * LS);   // f[u] = u_u, u < 2P
      const int m = mi[i];
      if (m < n) {
        f[m + 1] = v[i];
        f[2 * P - m - 1] = -v[i];
      } else {
        f[0] = T(0);
        f[P] = T(0);
      }
    }
    __syncthreads();
    fft_lines<T, EPT>(buf, LS, logP, a.W2);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int m = mi[i];
      if (m < n) {
        const int k = m + 1;
        const cx<T> zk = buf[li[i] * LS + k];
        const cx<T> zn = buf[li[i] * LS + P - k];
        const cx<T> w = a.W2[k];            // cos(pi k/P) - i sin(pi k/P)
        const T imU = T(0.5) * ((zk.y - zn.y) - w.x * (zk.x - zn.x) + w.y * (zk.y + zn.y));
        v[i] = -imU * rs2P;
      }
    }
  };

  if (FL & LF_DST1) dst();
  if (FL & LF_FDST2) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (mi[i] < n) v[i] = v[i] / (a.fline[line0 + li[i] < a.nlines ? line0 + li[i] : 0] + a.felem[mi[i]]);
    dst();
  }
  if (a.post) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (ok[i]) v[i] *= a.post[gi[i]];
  }
  if (FL & LF_STOREZ) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (ok[i]) a.zout[gi[i]] = v[i];
  }
  if (!(FL & LF_TOEP)) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (ok[i]) a.out[gi[i]] = v[i];
    return;
  }

  // ---- Toeplitz: acc = cplus .* T v + cminus .* T^T v -----------------------
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    T* f = reinterpret_cast<T*>(buf + li[i] * LS);   // f[u] = p_u, the zero-padded v
    const int m = mi[i];
    f[m] = (m < n) ? v[i] : T(0);
    f[P + m] = T(0);
  }
  __syncthreads();
  fft_lines<T, EPT>(buf, LS, logP, a.W2);

  // Pair phase: bins k and P-k of the packed spectrum Q give the half
  // spectrum of the real sequence, Pk = E + w O, P(P-k) = conj(E - w O),
  // E = (Qk + conj Q(P-k))/2, O = -i (Qk - conj Q(P-k))/2, w = exp(-i pi k/P).
  // Y1 = lam .* Ph, Y2 = conj(lam) .* Ph; each inverse runs on
  // Wk = (Yk + conj Y(P-k))/2 + i conj(w) (Yk - conj Y(P-k))/2.
  constexpr int NPR = EPT / 2;
  const int logH = logP - 1;
  const int H = 1 << logH;   // P/2 pairs per line
  cx<T> w1[NPR][2], w2[NPR][2];
  int pk[NPR], pl[NPR];
  auto winv = [&](cx<T> yk, cx<T> yn, cx<T> w) -> cx<T> {
    const cx<T> s = scale(add(yk, conj(yn)), T(0.5));
    const cx<T> d = scale(sub(yk, conj(yn)), T(0.5));
    return add(s, mul_i(mul(conj(w), d)));
  };
#pragma unroll
  for (int s = 0; s < NPR; ++s) {
    const int p = tid + s * nth;
    const int l = p >> logH;
    const int k = p & (H - 1);
    pl[s] = l;
    pk[s] = k;
    const cx<T>* q = buf + l * LS;
    if (k == 0) {
      const cx<T> q0 = q[0];
      const T p0 = q0.x + q0.y, pP = q0.x - q0.y;
      const cx<T> l0 = a.lam[0], lP = a.lam[P];
      const cx<T> one = mk(T(1), T(0));
      cx<T> y0 = scale(l0, p0), yP = scale(lP, pP);
      w1[s][0] = winv(y0, yP, one);
      y0 = scale(conj(l0), p0);
      yP = scale(conj(lP), pP);
      w2[s][0] = winv(y0, yP, one);
    } else {
      const cx<T> qk = q[k], qn = q[P - k];
      const cx<T> E = scale(add(qk, conj(qn)), T(0.5));
      const cx<T> O = mul_mi(scale(sub(qk, conj(qn)), T(0.5)));
      const cx<T> w = a.W2[k];
      const cx<T> wO = mul(w, O);
      const cx<T> pkv = add(E, wO);
      const cx<T> pnv = conj(sub(E, wO));
      const cx<T> lk = a.lam[k], ln = a.lam[P - k];
      const cx<T> wn = mk(-w.x, w.y);   // exp(-i pi (P-k)/P) = -conj(w)
      cx<T> yk = mul(lk, pkv), yn = mul(ln, pnv);
      w1[s][0] = winv(yk, yn, w);
      w1[s][1] = winv(yn, yk, wn);
      yk = mul(conj(lk), pkv);
      yn = mul(conj(ln), pnv);
      w2[s][0] = winv(yk, yn, w);
      w2[s][1] = winv(yn, yk, wn);
    }
  }
  // self-paired bin k = P/2 (one per line), w = exp(-i pi/2) = -i; its two
  // spectra go to a side buffer of 2B entries after the line buffers
  cx<T>* sbuf = buf + a.B * LS;
  for (int l = tid; l < a.B; l += nth) {
    const cx<T> q = buf[l * LS + H];
    const cx<T> ph = conj(q);   // E + w O with E = Re q, O = Im q, w = -i
    const cx<T> lh = a.lam[H];
    const cx<T> w = mk(T(0), T(-1));
    cx<T> y = mul(lh, ph);
    sbuf[2 * l] = conj(winv(y, y, w));
    y = mul(conj(lh), ph);
    sbuf[2 * l + 1] = conj(winv(y, y, w));
  }
  __syncthreads();
  auto put = [&](cx<T> (*wr)[2], int which) {
#pragma unroll
    for (int s = 0; s < NPR; ++s) {
      cx<T>* q = buf + pl[s] * LS;
      const int k = pk[s];
      q[k] = conj(wr[s][0]);
      if (k != 0) q[P - k] = conj(wr[s][1]);
    }
    for (int l = tid; l < a.B; l += nth) buf[l * LS + H] = sbuf[2 * l + which];
  };
  put(w1, 0);
  __syncthreads();
  fft_lines<T, EPT>(buf, LS, logP, a.W2);
  const T invP = T(1) / T(P);
  T acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    acc[i] = T(0);
    const int m = mi[i];
    if (ok[i]) {
      const cx<T> r = buf[li[i] * LS + (m >> 1)];
      const T y = ((m & 1) ? -r.y : r.x) * invP;
      acc[i] = a.cplus[gi[i]] * y;
    }
  }
  __syncthreads();
  put(w2, 1);
  __syncthreads();
  fft_lines<T, EPT>(buf, LS, logP, a.W2);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int m = mi[i];
    if (ok[i]) {
      const cx<T> r = buf[li[i] * LS + (m >> 1)];
      const T y = ((m & 1) ? -r.y : r.x) * invP;
      acc[i] += a.cminus[gi[i]] * y;
      const T b = (FL & LF_EXTBASE) ? a.base[gi[i]] : v[i];
      a.out[gi[i]] = a.bscale * b + a.tscale * acc[i];
    }
  }
}

}  // namespace fde
