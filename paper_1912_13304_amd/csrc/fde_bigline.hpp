// Transforms of one 1D line longer than a workgroup holds (P = n + 1 > 4096).
//
// The complex P-point FFT is a four-step FFT in two kernels, P = P1 * P2
// with both factors <= 4096: view x (j = j1 P2 + j2) as a P1 x P2 array;
// the first pass transforms its P2 columns (length P1, read and written in
// place with stride P2) and multiplies entry (k1, j2) by
// exp(-2 pi i j2 k1 / P); the second transforms the P1 rows (length P2) and
// writes X[k1 + P1 k2] to position k1 + P1 k2, the natural order.  A
// workgroup takes neighbouring columns (rows), so that the strided accesses
// of a wavefront are segments of neighbouring elements.
//
// The DST-I and Toeplitz programs use the same packings as the one-workgroup
// line kernels (odd extension / zero padding packed into P complex points,
// bins k and P - k paired), here as elementwise kernels around the big FFT;
// the division by the symbol between the two DSTs of the preconditioner is
// fused with the unpacking of the first and the packing of the second.
#pragma once

#include <hip/hip_runtime.h>

#include "fde_krylov.hpp"
#include "fde_lines.hpp"

namespace fde {

__device__ __forceinline__ bool skip2f(const int* a, const int* b) { return (a && *a) || (b && *b); }

// Elements per thread and lines per workgroup of a four-step pass.  A
// 65536-point FFT has only P / 8 = 8192 threads at 8 elements each, too few
// wavefronts for the CUs, so the passes take 4 elements (radix-4 passes) and
// one line per workgroup from L = 256 up (measured 9 % faster per 1D
// iteration at n = 65535).
__host__ __device__ constexpr int fourstep_ept(int) { return 4; }
__host__ __device__ constexpr int fourstep_lines(int L) { return L >= 256 ? 1 : 256 / L; }

// One pass of the four-step FFT: FFTs of length L = 2^LOGL on lines of a
// batch of P-point arrays; line g (item z = g / npl, q = g mod npl) takes
// its elements from the loader, in(z, q ils + m ies) (an array, or one of
// the packings below computed on the fly), and writes them to
// out[z P + q ols + k oes].  CIN / COUT: the lines are 1 element apart
// (ils == 1 / ols == 1), so neighbouring threads take neighbouring lines
// there.  apply_tw multiplies entry (q, k) by Wbig[2 q k] =
// exp(-2 pi i q k / P).  B = fourstep_lines(L) lines per workgroup (B divides
// npl), B L / fourstep_ept(L) threads.
template <typename T, int LOGL, bool CIN, bool COUT, class LD>
__global__ void __launch_bounds__(512)
fourstep_kernel(LD in, cx<T>* __restrict__ out, long P, int npl, long ils, long ies, long ols, long oes,
                const cx<T>* __restrict__ Wsub, const cx<T>* __restrict__ Wbig, int apply_tw, const int* skip,
                const int* skip2) {
  constexpr int EPT = fourstep_ept(1 << LOGL);
  constexpr int L = 1 << LOGL;
  constexpr int B = fourstep_lines(L);
  constexpr int LOGB = ilog2c(B);
  constexpr int NTH = B * L / EPT;
  constexpr int LS = line_stride(L);
  if (skip2f(skip, skip2)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + B * LS;
  const int tid = threadIdx.x;
  const long g0 = (long)blockIdx.x * B;
  const long z = g0 / npl;
  const int q0 = (int)(g0 - z * npl);
  cx<T>* dst = out + z * P;
  cx<T> v[EPT];
  T twr[EPT], twi[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const cx<T> t = Wsub[(tid + k * NTH) & (L - 1)];
    twr[k] = t.x;
    twi[k] = t.y;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NTH;
    const int l = CIN ? (e & (B - 1)) : (e >> LOGL);
    const int m = CIN ? (e >> LOGB) : (e & (L - 1));
    v[i] = in(z, (long)(q0 + l) * ils + (long)m * ies);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < EPT; ++k) tw[tid + k * NTH] = mk(twr[k], twi[k]);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NTH;
    const int l = CIN ? (e & (B - 1)) : (e >> LOGL);
    const int m = CIN ? (e >> LOGB) : (e & (L - 1));
    buf[l * LS + pidx(m)] = v[i];
  }
  __syncthreads();
  fft_lines_ct<T, EPT, LOGL, 0>(buf, LS, tw);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NTH;
    const int l = COUT ? (e & (B - 1)) : (e >> LOGL);
    const int k = COUT ? (e >> LOGB) : (e & (L - 1));
    cx<T> x = buf[l * LS + pidx(k)];
    if (apply_tw) x = mul(x, Wbig[2 * (long)(q0 + l) * k]);
    dst[(long)(q0 + l) * ols + (long)k * oes] = x;
  }
}

// Loaders of the column pass.  Each returns entry j of item z of the array
// the pass transforms.

// The array itself.
template <typename T>
struct LdArray {
  const cx<T>* a;
  long P;
  __device__ cx<T> operator()(long z, long j) const { return a[z * P + j]; }
};

// DST packing: z_j = u_{2j} + i u_{2j+1}, u the odd extension (length 2P) of
// x_m = sc * pre_m * in_{m-1}, m = 1..n (u_0 = u_P = 0, u_{2P-m} = -x_m).
// The input may be of a wider type TI (a float64 vector into the float32
// transform): then x_m = (T)(in_{m-1} sc) is formed in TI, as a separate
// scale-and-cast kernel would.
template <typename T, typename TI = T>
struct LdPackDst {
  const TI* in;
  const T* pre;
  const double* sc;
  int P;
  __device__ T u(int m, double s) const {
    if (m == 0 || m == P) return T(0);
    const int mm = m < P ? m : 2 * P - m;
    T x;
    if constexpr (sizeof(TI) == sizeof(T)) x = in[mm - 1] * (T)s;
    else x = (T)((double)in[mm - 1] * s);
    if (pre) x *= pre[mm - 1];
    return m < P ? x : -x;
  }
  __device__ cx<T> operator()(long, long j) const {
    const double s = sc ? *sc : 1.0;
    return mk(u(2 * (int)j, s), u(2 * (int)j + 1, s));
  }
};

// DST value y_k (k = 1..n) from the P-point FFT Z of the packed odd extension.
template <typename T>
__device__ __forceinline__ T dst_value(const cx<T>* Z, const cx<T>* W, int k, int P) {
  const cx<T> zk = Z[k], zn = Z[P - k], w = W[k];
  const T imU = T(0.5) * ((zk.y - zn.y) - w.x * (zk.x - zn.x) + w.y * (zk.y + zn.y));
  return -imU / sqrt(T(2 * P));
}

// y_{m+1} -> out[m] (times post_m when post), m < n.
template <typename T>
__global__ void unpack_dst_kernel(const cx<T>* Z, const cx<T>* W, const T* post, T* out, T* out2, int n, int P,
                                  const int* skip, const int* skip2) {
  if (skip2f(skip, skip2)) return;
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n; m += gridDim.x * blockDim.x) {
    T y = dst_value(Z, W, m + 1, P);
    if (post) y *= post[m];
    out[m] = y;
    if (out2) out2[m] = y;
  }
}

// Between the two DSTs of the preconditioner: y = DST(x) from Z, divide by F
// (F_m = f[m - 1]), and the packed odd extension of y / F for the second DST.
template <typename T>
struct LdFRepack {
  const cx<T>* Z;
  const cx<T>* W;
  const T* f;
  int P;
  __device__ T u(int m) const {
    if (m == 0 || m == P) return T(0);
    const int mm = m < P ? m : 2 * P - m;
    const T y = dst_value(Z, W, mm, P) / f[mm - 1];
    return m < P ? y : -y;
  }
  __device__ cx<T> operator()(long, long j) const { return mk(u(2 * (int)j), u(2 * (int)j + 1)); }
};

// Toeplitz packing: q_j = p_{2j} + i p_{2j+1}, p = (z_0..z_{n-1}, 0, ..., 0) of length 2P.
template <typename T>
struct LdPackToep {
  const T* zin;
  int n;
  __device__ cx<T> operator()(long, long j) const {
    const long a = 2 * j, b = 2 * j + 1;
    return mk(a < n ? zin[a] : T(0), b < n ? zin[b] : T(0));
  }
};

// The preconditioner's last step and the Toeplitz packing in one loader: the
// DST values y_{m+1} (times post_m) from the FFT Z of the second DST, written
// to zout (the stored z = P^{-1} v) and packed as LdPackToep packs them.
// Every index j is loaded once per pass, so each z_m is written once.
// TZ: the preconditioner's precision (float32 in the mixed form, whose z
// is stored and multiplied in float64: y is then rounded once, to T).
template <typename T, typename TZ = T>
struct LdDstPackToep {
  const cx<TZ>* Z;
  const cx<TZ>* W;
  const TZ* post;
  T* zout;
  int n, P;
  __device__ T zval(long m) const {
    if (m >= n) return T(0);
    TZ y = dst_value(Z, W, (int)m + 1, P);
    if (post) y *= post[m];
    const T yt = (T)y;
    zout[m] = yt;
    return yt;
  }
  __device__ cx<T> operator()(long, long j) const { return mk(zval(2 * j), zval(2 * j + 1)); }
};

// Pair phase of the Toeplitz product: from Q (FFT of the packed zero-padded
// input) the half spectrum Ph, Y1 = lam Ph (item 0) or Y2 = conj(lam) Ph
// (item 1), and bin k of the conjugated packed inverse input conj(W1) or
// conj(W2); bins k and P - k come from the same pair of Q bins.
template <typename T>
struct LdPairToep {
  const cx<T>* Q;
  const cx<T>* lam;
  const cx<T>* W;
  int P;
  __device__ static cx<T> winv(cx<T> yk, cx<T> yn, cx<T> w) {
    const cx<T> s = scale(add(yk, conj(yn)), T(0.5));
    const cx<T> d = scale(sub(yk, conj(yn)), T(0.5));
    return add(s, mul_i(mul(conj(w), d)));
  }
  __device__ cx<T> operator()(long z, long jl) const {
    const int k = (int)jl, H = P / 2;
    const bool second = z != 0;
    auto L = [&](cx<T> l) { return second ? conj(l) : l; };
    if (k == 0) {
      const cx<T> q0 = Q[0];
      const T p0 = q0.x + q0.y, pP = q0.x - q0.y;
      return conj(winv(scale(L(lam[0]), p0), scale(L(lam[P]), pP), mk(T(1), T(0))));
    }
    if (k == H) {
      const cx<T> y = mul(L(lam[H]), conj(Q[H]));
      return conj(winv(y, y, mk(T(0), T(-1))));
    }
    const int kk = k < H ? k : P - k;   // the pair (kk, P - kk), 0 < kk < H
    const cx<T> qk = Q[kk], qn = Q[P - kk];
    const cx<T> E = scale(add(qk, conj(qn)), T(0.5));
    const cx<T> O = mul_mi(scale(sub(qk, conj(qn)), T(0.5)));
    const cx<T> w = W[kk];
    const cx<T> wO = mul(w, O);
    const cx<T> pk = add(E, wO), pn = conj(sub(E, wO));
    const cx<T> yk = mul(L(lam[kk]), pk), yn = mul(L(lam[P - kk]), pn);
    if (k < H) return conj(winv(yk, yn, w));
    return conj(winv(yn, yk, mk(-w.x, w.y)));
  }
};

// ---------------------------------------------------------------------------
// DST-I of a line whose n + 1 is not a power of two (chirp-z form).  With
// P = n + 1 and c_j = exp(i pi j^2 / (2P)), jk = (j^2 + k^2 - (k-j)^2)/2 turns
// sum_j x_j sin(pi jk/P) into Im(c_k sum_j (x_j c_j) conj(c_{k-j})): a
// convolution with the chirp, done with power-of-two FFTs of length Q >= 2n - 1
// (the chirp filter's spectrum bhat is precomputed, with the factor
// sqrt(2/P)/Q).  Index j of the FFT input holds entry j + 1 of the line.
// ---------------------------------------------------------------------------

// First FFT input: a_j = sc pre_j in_j c_{j+1} (j < n), zero beyond.
template <typename T, typename TI = T>
struct LdChirpIn {
  const TI* in;
  const T* pre;
  const double* sc;
  const cx<T>* chirp;
  int n;
  __device__ cx<T> operator()(long, long j) const {
    if (j >= n) return mk(T(0), T(0));
    T u;
    if constexpr (sizeof(TI) == sizeof(T)) {
      u = in[j];
      if (sc) u *= (T)(*sc);
    } else {
      u = (T)((double)in[j] * (sc ? *sc : 1.0));
    }
    if (pre) u *= pre[j];
    const cx<T> c = chirp[j + 1];
    return mk(u * c.x, u * c.y);
  }
};

// Second FFT input: conj(A_k bhat_k) (an inverse FFT as a forward one).
template <typename T>
struct LdChirpMul {
  const cx<T>* A;
  const cx<T>* bhat;
  __device__ cx<T> operator()(long, long k) const { return conj(mul(A[k], bhat[k])); }
};

// DST value y_{k+1} = Im(c_{k+1} conj(R_k)) from the second FFT's output R.
template <typename T>
__device__ __forceinline__ T chirp_value(const cx<T>* R, const cx<T>* chirp, long k) {
  const cx<T> r = R[k], c = chirp[k + 1];
  return c.y * r.x - c.x * r.y;
}

// Between the two DSTs of the preconditioner: y / F, chirped for the next DST.
template <typename T>
struct LdChirpMid {
  const cx<T>* R;
  const cx<T>* chirp;
  const T* f;
  int n;
  __device__ cx<T> operator()(long, long j) const {
    if (j >= n) return mk(T(0), T(0));
    const T u = chirp_value(R, chirp, j) / f[j];
    const cx<T> c = chirp[j + 1];
    return mk(u * c.x, u * c.y);
  }
};

// out[m] = post_m y_{m+1}, m < n (and a second copy when out2).
template <typename T>
__global__ void unpack_chirp_kernel(const cx<T>* R, const cx<T>* chirp, const T* post, T* out, T* out2, int n,
                                    const int* skip, const int* skip2) {
  if (skip2f(skip, skip2)) return;
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n; m += gridDim.x * blockDim.x) {
    T y = chirp_value(R, chirp, m);
    if (post) y *= post[m];
    out[m] = y;
    if (out2) out2[m] = y;
  }
}

// The chirp-z preconditioner's last step and the Toeplitz packing in one
// loader (as LdDstPackToep): y_{m+1} (times post_m) from the second FFT's
// output R, written to zout and packed.
template <typename T, typename TZ = T>
struct LdChirpPackToep {
  const cx<TZ>* R;
  const cx<TZ>* chirp;
  const TZ* post;
  T* zout;
  int n;
  __device__ T zval(long m) const {
    if (m >= n) return T(0);
    TZ y = chirp_value(R, chirp, m);
    if (post) y *= post[m];
    const T yt = (T)y;
    zout[m] = yt;
    return yt;
  }
  __device__ cx<T> operator()(long, long j) const { return mk(zval(2 * j), zval(2 * j + 1)); }
};

// out_m = bscale * base_m + tscale * (cplus_m y1_m + cminus_m y2_m), where
// y_{2j} = Re R_j / P and y_{2j+1} = -Im R_j / P for R = FFT(conj W).
template <typename T>
__global__ void extract_toep_kernel(const cx<T>* R1, const cx<T>* R2, const T* cplus, const T* cminus,
                                    const T* base, T bscale, T tscale, T* out, int n, int P, const int* skip,
                                    const int* skip2) {
  if (skip2f(skip, skip2)) return;
  const T invP = T(1) / T(P);
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n; m += gridDim.x * blockDim.x) {
    const cx<T> r1 = R1[m >> 1], r2 = R2[m >> 1];
    const T y1 = ((m & 1) ? -r1.y : r1.x) * invP;
    const T y2 = ((m & 1) ? -r2.y : r2.x) * invP;
    out[m] = bscale * base[m] + tscale * (cplus[m] * y1 + cminus[m] * y2);
  }
}

}  // namespace fde
