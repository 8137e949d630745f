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
// pass when log2 P is not a multiple of 3) in a padded LDS layout.  Each
// workgroup transforms B lines at once (rows: one line from P = 512 up;
// columns: up to four neighbouring columns); every thread owns EPT = 8
// elements in the elementwise phases and EPT/R butterflies in a radix-R pass,
// so blockDim = B*P/8.  Twiddles come from a host-computed float64 table
// W2[m] = exp(-2 pi i m/(2P)), m < 2P; a butterfly reads one and forms the
// powers it needs by products.
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

// LDS layout of a line: element i at offset i + i/8.  The first two radix-8
// Stockham passes write elements 8 and 64 apart from neighbouring lanes;
// unpadded, those writes fall into a handful of banks (16- and 8-way
// conflicts), padded they spread over all of them.
__host__ __device__ constexpr int pidx(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }
// Lines of a row tile are pidx(P) + 1 elements apart.
__host__ __device__ constexpr int line_stride(int P) { return pidx(P) + 1; }
// Column tiles: a wavefront's elementwise accesses cover 4 lines x 16
// positions; lines 2(pidx(P) + 8) words apart put those 64 accesses in
// distinct banks (64 banks of 4 bytes) when pidx(P) is a multiple of 32.
__host__ __device__ constexpr int cols_line_stride(int P) { return pidx(P) + 8; }
// Lines per workgroup: rows (contiguous lines) fill one wavefront at least;
// columns (lines of stride n1) take up to four neighbouring columns, so that
// every row of the tile is one 16- or 32-byte segment, within 512 threads.
__host__ __device__ constexpr int rows_per_tile(int P) { return P >= 512 ? 1 : 512 / P; }
__host__ __device__ constexpr int cols_per_tile(int P) {
  return rows_per_tile(P) > (4096 / P < 4 ? 4096 / P : 4) ? rows_per_tile(P) : (4096 / P < 4 ? 4096 / P : 4);
}

// One Stockham pass of radix R over B lines of length P in LDS (line stride
// LS complex elements).  Ls = product of the radices of earlier passes.
// Butterfly j of a line reads x[j + r P/R], multiplies element r by
// w^(r k) with k = j mod Ls and w = exp(-2 pi i/(Ls R)), applies DFT_R and
// writes y[(j - k) R + k + r Ls].  In place: all reads finish before a
// barrier, then all writes.  tw holds exp(-i pi m/P), m < P, in LDS.

template <typename T, int EPT, int R>
__device__ __forceinline__ void fft_pass(cx<T>* buf, int LS, int logPr, int Ls, int logR,
                                         const cx<T>* tw, int twshift) {
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
    for (int r = 0; r < R; ++r) v[s][r] = buf[base[s] + pidx(j + r * Pr)];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int j = jj[s];
    const int k = j & (Ls - 1);
    if (Ls > 1) {
      // w^k from the table (k << twshift < P), its powers by products of
      // depth at most 3: one LDS read per butterfly instead of R - 1
      cx<T> w[R];
      w[1] = tw[k << twshift];
      if constexpr (R >= 4) {
        w[2] = mul(w[1], w[1]);
        w[3] = mul(w[2], w[1]);
      }
      if constexpr (R == 8) {
        w[4] = mul(w[2], w[2]);
        w[5] = mul(w[4], w[1]);
        w[6] = mul(w[3], w[3]);
        w[7] = mul(w[4], w[3]);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[s][r] = mul(v[s][r], w[r]);
    }
    dftR<T, R>(v[s]);
    const int o = ((j - k) << logR) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[base[s] + pidx(o + r * Ls)] = v[s][r];
  }
  __syncthreads();
}

// Compile-time pass sequence (radix 8, then 4 or 2) for P = 2^LOGP.
template <typename T, int EPT, int LOGP, int LOGLS>
__device__ __forceinline__ void fft_lines_ct(cx<T>* buf, int LS, const cx<T>* tw) {
  if constexpr (LOGLS < LOGP) {
    constexpr int REM = LOGP - LOGLS;
    constexpr int LOGE = ilog2c(EPT);   // a pass's radix is at most EPT
    constexpr int LOGR0 = REM >= 3 ? 3 : REM;
    constexpr int LOGR = LOGR0 < LOGE ? LOGR0 : LOGE;
    fft_pass<T, EPT, (1 << LOGR)>(buf, LS, LOGP - LOGR, 1 << LOGLS, LOGR, tw, LOGP + 1 - LOGLS - LOGR);
    fft_lines_ct<T, EPT, LOGP, LOGLS + LOGR>(buf, LS, tw);
  }
}

// Forward FFT of length P = 2^logP on every line in LDS.  The caller has
// synchronised after writing the input; results are visible on return.
template <typename T, int EPT>
__device__ __forceinline__ void fft_lines(cx<T>* buf, int LS, int logP, const cx<T>* tw) {
  int logLs = 0;
  while (logLs < logP) {
    const int rem = logP - logLs;
    const int Ls = 1 << logLs;
    if (rem >= 3) {
      fft_pass<T, EPT, 8>(buf, LS, logP - 3, Ls, 3, tw, logP + 1 - logLs - 3);
      logLs += 3;
    } else if (rem == 2) {
      fft_pass<T, EPT, 4>(buf, LS, logP - 2, Ls, 2, tw, logP + 1 - logLs - 2);
      logLs += 2;
    } else {
      fft_pass<T, EPT, 2>(buf, LS, logP - 1, Ls, 1, tw, logP + 1 - logLs - 1);
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
  const int* skip2;   // second flag with the same meaning
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

// LOGP > 0: transform size fixed at compile time (P = 2^LOGP, B =
// rows_per_tile(P) or cols_per_tile(P) lines per workgroup), so that pass
// radices, strides, twiddle indices and LDS offsets are constants; LOGP = 0
// reads them from `a`.  COLS: the B lines of a tile are neighbouring columns
// (line stride 1, element stride n1), and consecutive threads take the B
// entries of one row, so that the global accesses of a wavefront are row
// segments rather than single elements.
// The program on tile `tile` (B lines): the body of line_kernel, also run
// by the single-workgroup PCG kernel.  Every thread of the workgroup calls
// it; it reads its operands from global memory and writes its results there.
// EPT: elements per thread (8; 4 takes twice the threads, radix-4 passes).
template <typename T, bool COLS, int FL, int LOGP, int EPT = 8>
__device__ __forceinline__ void line_body(const LineArgs<T>& a, int tile) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);

  constexpr int CP = LOGP > 0 ? (1 << LOGP) : 0;
  constexpr int CB = LOGP > 0 ? (COLS ? cols_per_tile(CP) : rows_per_tile(CP)) : 0;
  const int logP = LOGP > 0 ? LOGP : a.logP;
  const int P = LOGP > 0 ? CP : a.P;
  const int B = LOGP > 0 ? CB : a.B;
  const int logB = LOGP > 0 ? ilog2c(CB) : a.logB;
  const int LS = LOGP > 0 ? (COLS ? cols_line_stride(CP) : line_stride(CP)) : a.LS;
  const int nth = LOGP > 0 ? CB * CP / EPT : (int)blockDim.x;
  const int tid = threadIdx.x;
  const int n = a.n;
  const int line0 = tile * B;
  // LDS: B line buffers, 2B side entries, P twiddle slots
  cx<T>* tw = buf + B * LS + 2 * B;
  // twiddle loads per thread: ceil(P / nth) = ceil(EPT / B) (all of them for
  // the generic form)
  constexpr int TWK = LOGP > 0 ? (EPT / CB > 1 ? EPT / CB : 1) : EPT;

  int li[EPT], mi[EPT];
  int gi[EPT];   // element offsets (N < 2^31); 0 for padding/out-of-range slots
  bool ok[EPT];
  T v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * nth;
    int l, m;
    if (COLS) {
      l = e & (B - 1);
      m = e >> logB;
    } else {
      l = e >> logP;
      m = e & (P - 1);
    }
    li[i] = l;
    mi[i] = m;
    ok[i] = (m < n) && (line0 + l < a.nlines);
    gi[i] = ok[i] ? (line0 + l) * (int)a.ls + m * (int)a.es : 0;
  }
  // Every global operand of this thread is loaded here, unconditionally (at
  // a valid offset) and before any use, so that all loads are in flight
  // together and their latency overlaps the transforms below.
  T xpre[EPT], xpost[EPT], xcp[EPT], xcm[EPT], xb[EPT], xf[EPT];
  T twr[TWK], twi[TWK];
#pragma unroll
  for (int k = 0; k < TWK; ++k) {
    const cx<T> t = a.W2[(tid + k * nth) & (P - 1)];
    twr[k] = t.x;
    twi[k] = t.y;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    v[i] = a.in[gi[i]];
    if (a.pre) xpre[i] = a.pre[gi[i]];
    if (a.post) xpost[i] = a.post[gi[i]];
    if (FL & LF_FDST2) {
      const int ln = line0 + li[i] < a.nlines ? line0 + li[i] : 0;
      xf[i] = a.fline[ln] + a.felem[mi[i] < n ? mi[i] : 0];
    }
    if (FL & LF_TOEP) {
      xcp[i] = a.cplus[gi[i]];
      xcm[i] = a.cminus[gi[i]];
    }
    if (FL & LF_EXTBASE) xb[i] = a.base[gi[i]];
  }
  // keep the scheduler from interleaving the LDS stores (which wait for
  // their load) with the loads above
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < TWK; ++k)
    if (tid + k * nth < P) tw[tid + k * nth] = mk(twr[k], twi[k]);
  {
    const T sc = a.sc ? (T)(*a.sc) : T(1);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      T x = v[i] * sc;
      if (a.pre) x *= xpre[i];
      v[i] = ok[i] ? x : T(0);
    }
  }

  const T rs2P = T(1) / sqrt(T(2 * P));
  auto FFT = [&]() {
    if constexpr (LOGP > 0) fft_lines_ct<T, EPT, LOGP, 0>(buf, LS, tw);
    else fft_lines<T, EPT>(buf, LS, logP, tw);
  };
  T* bufr = reinterpret_cast<T*>(buf);
  // real view: f_u of line l is component (u & 1) of complex element u >> 1
  auto rset = [&](int l, int u, T val) { bufr[2 * (l * LS + pidx(u >> 1)) + (u & 1)] = val; };
  auto cget = [&](int l, int i) -> cx<T> { return buf[l * LS + pidx(i)]; };

  // ---- DST-I: v <- S_n v --------------------------------------------------
  auto dst = [&]() {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int m = mi[i];   // f_u = u_u, the odd extension, u < 2P
      if (m < n) {
        rset(li[i], m + 1, v[i]);
        rset(li[i], 2 * P - m - 1, -v[i]);
      } else {
        rset(li[i], 0, T(0));
        rset(li[i], P, T(0));
      }
    }
    __syncthreads();
    FFT();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int m = mi[i];
      if (m < n) {
        const int k = m + 1;
        const cx<T> zk = cget(li[i], k);
        const cx<T> zn = cget(li[i], P - k);
        const cx<T> w = tw[k];              // cos(pi k/P) - i sin(pi k/P)
        const T imU = T(0.5) * ((zk.y - zn.y) - w.x * (zk.x - zn.x) + w.y * (zk.y + zn.y));
        v[i] = -imU * rs2P;
      }
    }
  };

  if (FL & LF_DST1) dst();
  if (FL & LF_FDST2) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (mi[i] < n) v[i] = v[i] / xf[i];
    dst();
  }
  if (a.post) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (ok[i]) v[i] *= xpost[i];
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
    const int m = mi[i];   // f_u = p_u, the zero-padded v, u < 2P
    rset(li[i], m, (m < n) ? v[i] : T(0));
    rset(li[i], P + m, T(0));
  }
  __syncthreads();
  FFT();

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
    if (k == 0) {
      const cx<T> q0 = cget(l, 0);
      const T p0 = q0.x + q0.y, pP = q0.x - q0.y;
      const cx<T> l0 = a.lam[0], lP = a.lam[P];
      const cx<T> one = mk(T(1), T(0));
      cx<T> y0 = scale(l0, p0), yP = scale(lP, pP);
      w1[s][0] = winv(y0, yP, one);
      y0 = scale(conj(l0), p0);
      yP = scale(conj(lP), pP);
      w2[s][0] = winv(y0, yP, one);
    } else {
      const cx<T> qk = cget(l, k), qn = cget(l, P - k);
      const cx<T> E = scale(add(qk, conj(qn)), T(0.5));
      const cx<T> O = mul_mi(scale(sub(qk, conj(qn)), T(0.5)));
      const cx<T> w = tw[k];
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
  cx<T>* sbuf = buf + B * LS;
  for (int l = tid; l < B; l += nth) {
    const cx<T> q = cget(l, H);
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
      q[pidx(k)] = conj(wr[s][0]);
      if (k != 0) q[pidx(P - k)] = conj(wr[s][1]);
    }
    for (int l = tid; l < B; l += nth) buf[l * LS + pidx(H)] = sbuf[2 * l + which];
  };
  put(w1, 0);
  __syncthreads();
  FFT();
  const T invP = T(1) / T(P);
  T acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    acc[i] = T(0);
    const int m = mi[i];
    if (ok[i]) {
      const cx<T> r = cget(li[i], m >> 1);
      const T y = ((m & 1) ? -r.y : r.x) * invP;
      acc[i] = xcp[i] * y;
    }
  }
  __syncthreads();
  put(w2, 1);
  __syncthreads();
  FFT();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int m = mi[i];
    if (ok[i]) {
      const cx<T> r = cget(li[i], m >> 1);
      const T y = ((m & 1) ? -r.y : r.x) * invP;
      acc[i] += xcm[i] * y;
      const T b = (FL & LF_EXTBASE) ? xb[i] : v[i];
      a.out[gi[i]] = a.bscale * b + a.tscale * acc[i];
    }
  }
}

template <typename T, bool COLS, int FL, int LOGP>
__global__ void __launch_bounds__(512) line_kernel(LineArgs<T> a) {
  if ((a.skip && *a.skip) || (a.skip2 && *a.skip2)) return;
  const int tile = xcd_tile(a.ntiles);
  if (tile >= a.ntiles) return;
  line_body<T, COLS, FL, LOGP>(a, tile);
}

}  // namespace fde
