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
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int R0 = blockIdx.y * 32, C0 = blockIdx.x * 32;   // the workgroup's 32 x 32 output tile
  const int r0 = R0 + wr * 16;   // this wave's 16 x 16 part
  const int c0 = C0 + wc * 16;
  const int li = lane & 15, lk = lane >> 4;
  constexpr bool ROWS = MODE == DM_ROW_DST || MODE == DM_ROW_TOEP;
  constexpr bool TOEP = MODE == DM_ROW_TOEP || MODE == DM_COL_TOEP;
  const int K = ROWS ? n1 : n2;
  const T s = (MODE == DM_ROW_DST && a.sc) ? (T)(*a.sc) : T(1);
  // The operands of one step of 16 along k, staged in LDS by the whole
  // workgroup: the A panel (32 output rows x 16) and the B panel (16 x 32
  // output columns), a second A (column Toeplitz pair) or B (row Toeplitz
  // pair) panel.  X is loaded (rows: 16 neighbouring elements of a row,
  // columns: 32 of a row of X), the direction's matrix generated.  Rows are
  // padded by one element against bank conflicts.
  constexpr int AS = 17, BS = 33;
  __shared__ T Ap[32 * AS], Bp[16 * BS], P2[TOEP ? (ROWS ? 16 * BS : 32 * AS) : 1];
  // thread t stages elements e = t and t + 256 of each panel:
  // A panel (row e >> 4, k e & 15), B panel (k e >> 5, column e & 31)
  T ra[2], rb[2], r2[2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + 256 * h;
      const int ar = R0 + (e >> 4), ak = k0 + (e & 15);   // A panel element
      const int bk = k0 + (e >> 5), bc = C0 + (e & 31);   // B panel element
      if (ROWS) {
        T x = T(0);
        if (ar < n2 && ak < n1) {
          x = a.in[(long)ar * n1 + ak];
          if (MODE == DM_ROW_DST) {
            x *= s;
            if (a.pre) x *= a.pre[(long)ar * n1 + ak];
          }
        }
        ra[h] = x;
        if (MODE == DM_ROW_DST) {
          rb[h] = dst_elem(a.stab, bk, bc, n1);   // S1[k][c] (S symmetric)
        } else {
          rb[h] = toep_elem(a.g, bc, bk, n1);     // (T1^T)[k][c] = T1[c][k]
          r2[h] = toep_elem(a.g, bk, bc, n1);     // T1[k][c]
        }
      } else {
        rb[h] = (bk < n2 && bc < n1) ? a.in[(long)bk * n1 + bc] : T(0);
        if (MODE == DM_COL_DST) {
          ra[h] = dst_elem(a.stab, ar, ak, n2);   // S2[r][k]
        } else {
          ra[h] = toep_elem(a.g, ar, ak, n2);     // T2[r][k]
          r2[h] = toep_elem(a.g, ak, ar, n2);     // (T2^T)[r][k]
        }
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + 256 * h;
      Ap[(e >> 4) * AS + (e & 15)] = ra[h];
      Bp[(e >> 5) * BS + (e & 31)] = rb[h];
      if (TOEP) {
        if (ROWS) P2[(e >> 5) * BS + (e & 31)] = r2[h];
        else P2[(e >> 4) * AS + (e & 15)] = r2[h];
      }
    }
  };
  v4 acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0};
  fetch(0);
  stage();
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bool more = k0 + 16 < K;   // (the same in every thread)
    if (more) fetch(k0 + 16);        // the next step's loads, in flight during the products
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = 4 * u + lk;
      const T av = Ap[(wr * 16 + li) * AS + kk];
      const T bv = Bp[kk * BS + wc * 16 + li];
      acc1 = Mfma<T>::step(av, bv, acc1);
      if (MODE == DM_ROW_TOEP) acc2 = Mfma<T>::step(av, P2[kk * BS + wc * 16 + li], acc2);
      if (MODE == DM_COL_TOEP) acc2 = Mfma<T>::step(P2[(wr * 16 + li) * AS + kk], bv, acc2);
    }
    if (more) {
      __syncthreads();   // every wave has read this step's panels
      stage();
      __syncthreads();
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
