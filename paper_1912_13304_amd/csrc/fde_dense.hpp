// Line operators of small 2D grids as dense matrix products on the matrix
// cores (gfx950 MFMA), for any n (n + 1 need not be a power of two).
//
// With the unknowns X stored as an n2 x n1 row-major array (x fastest), an
// operator along x acts on every row: X -> X A^T, and one along y on every
// column: X -> A X, A the n x n matrix of the direction.  The matrices are
// generated element by element, never stored:
//  * DST-I (eq. sine_transform): S[j][k] = sqrt(2/(n+1)) sin(pi (j+1)(k+1)/(n+1)),
//    read from a table of sqrt(2/(n+1)) sin(pi m/(n+1)), m < 2(n+1);
//  * the Toeplitz matrix T = -[g_{i-j+1}] (eq. grunwaldmatrix1/2), from the
//    weights g_0..g_n.
// One wavefront computes a 16 x 16 output tile with the 16x16x4 MFMA
// (float64 or float32): step k0 takes A[i][k0 + l/16] (i = l mod 16) and
// B[k0 + l/16][j] (j = l mod 16) from lane l and accumulates D = A B.  Lane l
// holds column l mod 16 of D, item q < 4 of it being row 4 (l/16) + q for the
// float32 instruction and row 4 q + l/16 for the float64 one (both measured
// on gfx950 with one-hot operands).  A workgroup of
// four wavefronts covers a 32 x 32 tile.  Operands outside the matrix are
// zero, so any n works.  The epilogues fuse what the line kernels fuse: the
// input scaling (D^{-1}, a device scalar), the division by the symbol samples
// F(r, c) = fx[c] + fy[r] between the two y-direction DSTs, the D^{-1} after
// the last DST, and the coefficient-weighted sum of the Toeplitz pair.
#pragma once

#include <hip/hip_runtime.h>

namespace fde {

enum : int {
  DM_ROW_DST = 0,    // C = (sc pre .* X) S1
  DM_COL_DST = 1,    // C = S2 X
  DM_ROW_TOEP = 2,   // C1 = X T1^T (T1 along each row), C2 = X T1 (T1^T along each row)
  DM_COL_TOEP = 3,   // C1 = T2 X, C2 = T2^T X
};

template <typename T>
struct DenseArgs {
  const T* in;        // X, n2 x n1
  const T* pre;       // DM_ROW_DST: elementwise factor on the input (or null)
  const double* sc;   // DM_ROW_DST: device scalar on the input (or null)
  const T* post;      // DST: elementwise factor on the output (or null)
  const T* fx;        // DM_COL_DST: divide by fx[c] + fy[r] (null: no division)
  const T* fy;
  const T* stab;      // DST: sine table of the direction, 2(n+1) entries
  const T* g;         // TOEP: weights g_0..g_n of the direction
  const T* cp;        // TOEP: coefficient of the T product (C1)
  const T* cm;        // TOEP: coefficient of the T^T product (C2)
  const T* base;      // TOEP: out = bscale base + tscale (cp C1 + cm C2); null: base = X
  T bscale, tscale;
  T* out;
  const int* skip;    // nonzero: return at once
  const int* skip2;
  int n1, n2;
};

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 step(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int q) { return 4 * q + lk; }   // row of item q in lane group lk
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 step(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int q) { return 4 * lk + q; }
};

// Element (j, k) of the DST matrix of a direction with n points: the table
// holds sqrt(2/P) sin(pi m/P), m < 2P, P = n + 1; sin(pi (j+1)(k+1)/P) has
// period 2P in (j+1)(k+1).
template <typename T>
__device__ __forceinline__ T dst_elem(const T* stab, int j, int k, int n) {
  if (j >= n || k >= n) return T(0);
  const int P2 = 2 * (n + 1);
  return stab[((j + 1) * (k + 1)) % P2];
}

// Element (i, j) of T = -[g_{i-j+1}] (zero above the first superdiagonal).
template <typename T>
__device__ __forceinline__ T toep_elem(const T* g, int i, int j, int n) {
  const int d = i - j + 1;
  return (i < n && j < n && d >= 0) ? -g[d] : T(0);
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) dense_kernel(DenseArgs<T> a) {
  if ((a.skip && *a.skip) || (a.skip2 && *a.skip2)) return;
  typedef typename Mfma<T>::v4 v4;
  const int n1 = a.n1, n2 = a.n2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 32 + (wave >> 1) * 16;   // output rows (y index)
  const int c0 = blockIdx.x * 32 + (wave & 1) * 16;    // output columns (x index)
  const int li = lane & 15, lk = lane >> 4;
  const int ra = r0 + li;   // row of the A operand this lane supplies
  const int cb = c0 + li;   // column of the B operand this lane supplies
  constexpr bool ROWS = MODE == DM_ROW_DST || MODE == DM_ROW_TOEP;
  constexpr bool TOEP = MODE == DM_ROW_TOEP || MODE == DM_COL_TOEP;
  const int K = ROWS ? n1 : n2;
  const T s = (MODE == DM_ROW_DST && a.sc) ? (T)(*a.sc) : T(1);
  v4 acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    T av[4], bv[4], av2[4], bv2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + lk;
      if (ROWS) {
        // A = X (row ra, column k); B = the x-direction matrix
        T x = T(0);
        if (ra < n2 && k < n1) {
          x = a.in[(long)ra * n1 + k];
          if (MODE == DM_ROW_DST) {
            x *= s;
            if (a.pre) x *= a.pre[(long)ra * n1 + k];
          }
        }
        av[u] = x;
        if (MODE == DM_ROW_DST) {
          bv[u] = dst_elem(a.stab, k, cb, n1);   // S1[k][c] (S symmetric)
        } else {
          bv[u] = toep_elem(a.g, cb, k, n1);      // (T1^T)[k][c] = T1[c][k]
          bv2[u] = toep_elem(a.g, k, cb, n1);     // T1[k][c]
        }
      } else {
        // A = the y-direction matrix (row ra, column k); B = X (row k, column cb)
        bv[u] = (k < n2 && cb < n1) ? a.in[(long)k * n1 + cb] : T(0);
        if (MODE == DM_COL_DST) {
          av[u] = dst_elem(a.stab, ra, k, n2);
        } else {
          av[u] = toep_elem(a.g, ra, k, n2);      // T2[r][k]
          av2[u] = toep_elem(a.g, k, ra, n2);     // (T2^T)[r][k]
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (MODE == DM_ROW_TOEP) {
        acc1 = Mfma<T>::step(av[u], bv[u], acc1);
        acc2 = Mfma<T>::step(av[u], bv2[u], acc2);
      } else if (MODE == DM_COL_TOEP) {
        acc1 = Mfma<T>::step(av[u], bv[u], acc1);
        acc2 = Mfma<T>::step(av2[u], bv[u], acc2);
      } else {
        acc1 = Mfma<T>::step(av[u], bv[u], acc1);
      }
    }
  }
  const int c = c0 + li;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + Mfma<T>::row(lk, q);
    if (r >= n2 || c >= n1) continue;
    const long e = (long)r * n1 + c;
    T v;
    if (TOEP) {
      const T b = a.base ? a.base[e] : a.in[e];
      v = a.bscale * b + a.tscale * (a.cp[e] * acc1[q] + a.cm[e] * acc2[q]);
    } else {
      v = acc1[q];
      if (MODE == DM_COL_DST && a.fx) v = v / (a.fx[c] + a.fy[r]);
      if (a.post) v *= a.post[e];
    }
    a.out[e] = v;
  }
}

}  // namespace fde
