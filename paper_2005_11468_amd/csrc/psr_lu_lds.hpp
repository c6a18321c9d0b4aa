// Blocked FP32 LU of one matrix held entirely in LDS (gfx950: up to n = 201,
// 160 KB per workgroup), for the batched factorisation of large Jacobians.
//
// Right-looking blocked LU with partial pivoting (first index of the largest
// |a| in the column), panel width 16:
//   * the panel A[k0:n, k0:k0+16] is factored in LDS by wavefront 0 alone
//     (lane l handles rows l, l+64, l+128, l+192), the pivot from a
//     wavefront argmax (DPP within rows of 16 lanes, then the four row
//     results from scalar registers): no block barrier per column, and a
//     compact column loop (a fully unrolled register panel overflows the
//     instruction cache);
//   * the panel's row interchanges are applied to the other columns and
//     U12 = L11^-1 A12 is formed by forward substitution (one column per
//     thread);
//   * A22 -= L21 U12 runs on the matrix cores (v_mfma_f32_16x16x4f32, four
//     K-steps per 16 x 16 tile), tiles dealt to the wavefronts round robin.
// Operand layouts of the 16x16x4 instruction: A lane l -> (row l % 16,
// k l / 16); B lane l -> (k l / 16, column l % 16); D register v ->
// (row 4 (l / 16) + v, column l % 16).
// Rows are physically interchanged (LAPACK getrf convention for piv).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>


namespace psr {
namespace lulds {

typedef float v4f __attribute__((ext_vector_type(4)));

// 64-bit DPP move within rows of 16 lanes: quad_perm [1,0,3,2], quad_perm
// [2,3,0,1], row_ror 4, row_ror 8 for sel = 0..3.
template <int SEL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
  constexpr int ctrl = SEL == 0 ? 0xB1 : (SEL == 1 ? 0x4E : (SEL == 2 ? 0x124 : 0x128));
  const int lo = (int)(v & 0xffffffffull), hi = (int)(v >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned int)h2 << 32) | (unsigned int)l2;
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int lane) {
  const unsigned int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffull), lane);
  const unsigned int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

// Order wavefront-local LDS traffic: writes by some lanes must be visible to
// later reads by other lanes of the same wavefront.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Factor a rows x kb panel (rows <= 256, kb <= 16) in LDS by one wavefront:
// element (t, j) at P[t * ld + j]; lane l handles rows l + 64 q.  Per
// column: wavefront argmax (key = |a| bits above the complemented row index,
// so the largest |a| and, among equal values, the lowest row wins; DPP within
// rows of 16 lanes, then the four row results), interchange of the two rows
// inside the panel, then the multipliers and the rank-one update of the rows
// below with whole 16-column rows loaded at once.  A compact runtime column
// loop: a panel unrolled over its 16 columns overflows the instruction cache,
// and one that keeps the rows in registers and shifts them after each column
// measured no faster.  piv[k0 + j] receives k0 + the pivot row of column j;
// returns 0 or k0 + j + 1 for a zero pivot column j.
__device__ __forceinline__ int panel(float *P, int ld, int rows, int kb, int k0, int *piv) {
  const int lane = threadIdx.x & 63;
  const int nq = (rows + 63) >> 6;
#pragma unroll 1
  for (int jj = 0; jj < kb; jj++) {
    unsigned long long key = 0ull;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int t = lane + 64 * q;
      if (q < nq && t < rows && t >= jj) {
        const float a = fabsf(P[t * ld + jj]);
        const unsigned long long kq = ((unsigned long long)(unsigned int)__float_as_int(a) << 32) |
                                      (unsigned int)(0xffffffffu - (unsigned int)t);
        key = kq > key ? kq : key;
      }
    }
    unsigned long long o;
    o = dpp64<0>(key); key = o > key ? o : key;
    o = dpp64<1>(key); key = o > key ? o : key;
    o = dpp64<2>(key); key = o > key ? o : key;
    o = dpp64<3>(key); key = o > key ? o : key;
    unsigned long long best = readlane64(key, 0);
    o = readlane64(key, 16); best = o > best ? o : best;
    o = readlane64(key, 32); best = o > best ? o : best;
    o = readlane64(key, 48); best = o > best ? o : best;
    if ((best >> 32) == 0ull) return k0 + jj + 1;
    const int pr = (int)(0xffffffffu - (unsigned int)(best & 0xffffffffull));
    if (lane == 0) piv[k0 + jj] = k0 + pr;
    if (pr != jj && lane < kb) {
      const float x = P[jj * ld + lane], y = P[pr * ld + lane];
      P[jj * ld + lane] = y;
      P[pr * ld + lane] = x;
    }
    wave_lds_sync();
    // (columns j >= kb lie outside the panel: never read or written)
    float pr16[16];
#pragma unroll
    for (int j = 0; j < 16; j++) pr16[j] = j < kb ? P[jj * ld + j] : 0.f;
    const float inv = 1.0f / P[jj * ld + jj];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int t = lane + 64 * q;
      if (q < nq && t < rows && t > jj) {
        float r[16];
#pragma unroll
        for (int j = 0; j < 16; j++) r[j] = j < kb ? P[t * ld + j] : 0.f;
        const float l = P[t * ld + jj] * inv;
#pragma unroll
        for (int j = 0; j < 16; j++)
          if (j > jj && j < kb) P[t * ld + j] = r[j] - l * pr16[j];
        P[t * ld + jj] = l;
      }
    }
    wave_lds_sync();
  }
  return 0;
}

// The panel's row interchanges applied to the columns outside it (in
// order), then U12 = L11^-1 A12 for the trailing columns by forward
// substitution; one column per thread (n <= NT).
template <int NT>
__device__ __forceinline__ void swaps_u12(float *A, int n, int lda, int k0, int kb, const int *piv) {
  const int c = threadIdx.x, R0 = k0 + kb;
  if (c >= n || (c >= k0 && c < R0)) return;
  int pr[16];
#pragma unroll
  for (int jj = 0; jj < 16; jj++) pr[jj] = jj < kb ? piv[k0 + jj] : k0 + jj;
#pragma unroll
  for (int jj = 0; jj < 16; jj++) {
    if (jj < kb && pr[jj] != k0 + jj) {
      const float t = A[(k0 + jj) * lda + c];
      A[(k0 + jj) * lda + c] = A[pr[jj] * lda + c];
      A[pr[jj] * lda + c] = t;
    }
  }
  if (c >= R0) {
    float u[16];
#pragma unroll
    for (int i = 0; i < 16; i++) u[i] = i < kb ? A[(k0 + i) * lda + c] : 0.f;
#pragma unroll
    for (int i = 1; i < 16; i++) {
      float acc = u[i];
#pragma unroll
      for (int q = 0; q < 16; q++)
        if (q < i) acc -= (i < kb ? A[(k0 + i) * lda + k0 + q] : 0.f) * u[q];
      u[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < 16; i++)
      if (i < kb) A[(k0 + i) * lda + c] = u[i];
  }
}

// A22 -= L21 U12 (rows and columns from R0 = k0 + kb) on the matrix cores:
// each wavefront takes every NW-th 16-row tile row, keeps its L21 fragment in
// registers and sweeps the tile columns four at a time (four independent
// accumulation chains; all operand loads of a group issued together).
template <int NT>
__device__ __forceinline__ void update_mfma(float *A, int n, int lda, int k0, int kb) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int R0 = k0 + kb, m = n - R0, nt = (m + 15) >> 4;
  const int lr = lane & 15, lk = lane >> 4;
  for (int ti = wv; ti < nt; ti += NW) {
    const int arow = R0 + 16 * ti + lr, crow = R0 + 16 * ti + 4 * lk;
    float aq[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int k = 4 * q + lk;
      aq[q] = (arow < n && k < kb) ? -A[arow * lda + k0 + k] : 0.f;
    }
    for (int tj0 = 0; tj0 < nt; tj0 += 4) {
      float bq[4][4];
      v4f acc[4];
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int col = R0 + 16 * (tj0 + t) + lr;
        const bool cin = (tj0 + t) < nt && col < n;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int k = 4 * q + lk;
          bq[t][q] = (cin && k < kb) ? A[(k0 + k) * lda + col] : 0.f;
        }
#pragma unroll
        for (int v = 0; v < 4; v++) acc[t][v] = (cin && crow + v < n) ? A[(crow + v) * lda + col] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int t = 0; t < 4; t++) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[q], bq[t][q], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int col = R0 + 16 * (tj0 + t) + lr;
        if ((tj0 + t) < nt && col < n) {
#pragma unroll
          for (int v = 0; v < 4; v++)
            if (crow + v < n) A[(crow + v) * lda + col] = acc[t][v];
        }
      }
    }
  }
}

// In-place LU of the n x n matrix A (LDS, leading dimension lda, n <= NT and
// n <= 256) by a workgroup of NT threads.  piv (LDS, n ints) receives the
// pivot rows; s_info is one LDS int of scratch.  Returns 0 or k + 1 for the
// first zero pivot column k (the factorisation stops there).
template <int NT>
__device__ __forceinline__ int factor(float *A, int n, int lda, int *piv, int *s_info) {
  static_assert(NT % 64 == 0 && NT >= 256, "one column per thread");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k0 = 0; k0 < n; k0 += 16) {
    const int kb = n - k0 < 16 ? n - k0 : 16;
    if (wv == 0) {
      const int r = panel(A + k0 * lda + k0, lda, n - k0, kb, k0, piv);
      if (lane == 0) *s_info = r;
    }
    __syncthreads();
    const int pinfo = *s_info;
    __syncthreads();
    if (pinfo != 0) return pinfo;
    swaps_u12<NT>(A, n, lda, k0, kb, piv);
    __syncthreads();
    if (k0 + kb >= n) break;
    update_mfma<NT>(A, n, lda, k0, kb);
    __syncthreads();
  }
  return 0;
}

// Copy an n x n row-major double matrix g into the float LDS matrix M
// (leading dimension lda), eight rows in flight per thread; thread c takes
// column c (n <= NT).
template <int NT>
__device__ __forceinline__ void load_f32(float *M, int n, int lda, const double *g) {
  const int c = threadIdx.x;
  if (c >= n) return;
  for (int r0 = 0; r0 < n; r0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = r0 + u < n ? g[(int64_t)(r0 + u) * n + c] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (r0 + u < n) M[(r0 + u) * lda + c] = (float)v[u];
  }
}

// The factors back to double, row-major.
template <int NT>
__device__ __forceinline__ void store_f64(const float *M, int n, int lda, double *g) {
  const int c = threadIdx.x;
  if (c >= n) return;
  for (int r = 0; r < n; r++) g[(int64_t)r * n + c] = (double)M[r * lda + c];
}

}  // namespace lulds
}  // namespace psr
