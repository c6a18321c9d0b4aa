// Batched float LU with partial pivoting, one wavefront per matrix, for
// 64 < n <= 256 (the standalone psr_lu_factor_batch entry, PSR_MIXED): the
// LU decomposition of the paper's Newton step (Sec. 3) on the matrix cores.
//
// Each wavefront factors its matrices one after another with no barrier and
// no other wavefront involved:
//   * the working copy is a float matrix in a per-wavefront HBM area whose
//     rows are never moved: a logical -> physical row map in LDS stands for
//     the row interchanges, and the factors are written to the caller's
//     double matrix in logical order at the end;
//   * a 16-column panel lives in registers, rows spread over the lanes (lane
//     l holds the rows k0 + l + 64 j, j < 4); each column's pivot is found by
//     one DPP wavefront maximum over a key that packs |a|, the logical row
//     (lowest wins a tie, as LAPACK) and the row's register position; the
//     interchange only relabels rows, and the pivot row reaches every lane by
//     readlane;
//   * U12 = L11^-1 A12 with one column per lane, then A22 -= L21 U12 on
//     v_mfma_f32_16x16x4f32 with both operands from LDS and the C tiles
//     streamed from and to the float copy.
// The first panel reads the caller's double matrix directly (rounding each
// element to float once), so no separate conversion pass is made.
#pragma once

namespace psr {
namespace luw {

constexpr int kPS = 17;   // row stride (floats) of the LDS panel copy
constexpr int kUS = 272;  // row stride (floats) of the LDS U12 copy: the four
                          // rows a B operand load touches fall in disjoint banks
constexpr int kW = 4;     // wavefronts per workgroup

struct WaveLds {
  float L[256 * kPS];  // panel columns of logical rows k0..n-1 (row r - k0)
  float U[16 * kUS];   // U12 of the current panel (column c - R0)
  int perm[256];       // logical row -> physical row of the float copy
};

typedef float v4f_t __attribute__((ext_vector_type(4)));

// Float working copy: rows and columns rounded up to whole tiles of 16.
__host__ __device__ constexpr int pad_rows(int n) { return (n + 15) & ~15; }
__host__ __device__ constexpr int pad_ld(int n) { return (n + 15) & ~15; }

__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// Maximum over the wavefront of a double (every lane active), the same bits
// in every lane: DPP within rows of 16, then the four row maxima.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double rdlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wmax(double v) {
  v = fmax(v, dpp_mov<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_mov<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_mov<0x124>(v));  // row_ror 4
  v = fmax(v, dpp_mov<0x128>(v));  // row_ror 8
  return fmax(fmax(rdlane_d(v, 0), rdlane_d(v, 16)), fmax(rdlane_d(v, 32), rdlane_d(v, 48)));
}
// Orders this wavefront's earlier global-memory writes before its later
// reads of the same addresses by other lanes.
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}
// LDS operations of one wavefront take effect in issue order, so between
// LDS writes and other lanes' reads only the compiler must keep the order.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Element (r, c) of the matrix being factored: the caller's double matrix
// before the first panel has written the float copy, the float copy after.
template <bool FIRST>
__device__ __forceinline__ float ld_elem(const double *g, const float *M, int n, int ld, int r, int c) {
  return FIRST ? (float)g[(int64_t)r * n + c] : M[(int64_t)r * ld + c];
}

// A22 -= L21 U12 for the trailing block at logical row and column R0 (a
// multiple of 16), NT x NT tiles of 16: one row of tiles at a time in the MFMA result layout
// (register v of lane l holds row 4 (l / 16) + v, column l mod 16), the loads
// of the next row issued before the products of the current one.  Tiles
// reaching past n read and write the padding rows and columns of the float
// copy, so no access is predicated; the zero rows of the A operand and zero
// columns of U12 keep the padding out of the real elements.
template <bool FIRST, int NT>
__device__ __forceinline__ void trailing(int n, int ld, int k0, int kb, int R0, const double *g, float *M,
                                         const WaveLds &S, int lane) {
  constexpr int nt = NT;
  const int lr = lane & 15, lk = lane >> 4;
  float bq[NT][4];
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int q = 0; q < 4; q++) bq[t][q] = S.U[(4 * q + lk) * kUS + 16 * t + lr];
  v4f_t cur[NT], nxt[NT];
  auto load_row = [&](v4f_t *c, int ti) {
    int pr[4];
#pragma unroll
    for (int v = 0; v < 4; v++) pr[v] = S.perm[R0 + 16 * ti + 4 * lk + v];
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const int col = R0 + 16 * t + lr;
#pragma unroll
      for (int v = 0; v < 4; v++)
        c[t][v] = FIRST ? (float)g[(int64_t)(pr[v] < n ? pr[v] : n - 1) * n + (col < n ? col : n - 1)]
                        : M[(int64_t)pr[v] * ld + col];
    }
  };
  load_row(cur, 0);
  for (int ti = 0; ti < nt; ti++) {
    if (ti + 1 < nt) load_row(nxt, ti + 1);
    const int arow = R0 + 16 * ti + lr;  // A operand row of this lane
    float aq[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int kq = 4 * q + lk;
      const float v = S.L[((arow < n ? arow : n - 1) - k0) * kPS + kq];
      aq[q] = (arow < n && kq < kb) ? -v : 0.f;
    }
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int q = 0; q < 4; q++) cur[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[q], bq[t][q], cur[t], 0, 0, 0);
    int pr[4];
#pragma unroll
    for (int v = 0; v < 4; v++) pr[v] = S.perm[R0 + 16 * ti + 4 * lk + v];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int v = 0; v < 4; v++) M[(int64_t)pr[v] * ld + R0 + 16 * t + lr] = cur[t][v];
#pragma unroll
    for (int t = 0; t < NT; t++) cur[t] = nxt[t];
  }
}

// One panel step at column k0: factor columns k0..k0+kb-1 of the logical rows
// k0..n-1, then U12 and the trailing update.  Loads are unconditional at
// clamped in-range addresses, so the compiler can issue them together.
template <bool FIRST>
__device__ __forceinline__ void panel_step(int n, int ld, int k0, double *g, float *M, int *piv, WaveLds &S,
                                           int lane, int &info) {
  const int lr = lane & 15, lk = lane >> 4;
  const int kb = n - k0 < 16 ? n - k0 : 16;
  const int R0 = k0 + kb;
  // ---- panel: logical rows k0 + lane + 64 j, columns k0..k0+15
  float a[4][16];
  int phys[4], pos[4];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int t = k0 + lane + 64 * j;
    const bool ok = t < n;
    pos[j] = ok ? t : (1 << 20);
    phys[j] = S.perm[ok ? t : n - 1];
    if (FIRST) {
      const double *src = g + (int64_t)phys[j] * n;  // n > 64: columns 0..15 exist
#pragma unroll
      for (int c = 0; c < 16; c++) {
        const float v = (float)src[c];
        a[j][c] = ok ? v : 0.f;
      }
    } else {
      const float *src = M + (int64_t)phys[j] * ld;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // a chunk of four columns lies inside the row (ld is a multiple of 4)
        const int c0 = k0 + 4 * q < ld ? k0 + 4 * q : k0;
        const v4f_t v = *reinterpret_cast<const v4f_t *>(src + c0);
#pragma unroll
        for (int e = 0; e < 4; e++) a[j][4 * q + e] = (ok && k0 + 4 * q + e < n) ? v[e] : 0.f;
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < 16; jj++) {
    // a constant trip count keeps the loop unrolled, so every register
    // index is a compile-time constant
    if (jj >= kb) continue;
    const int k = k0 + jj;
    // key: |a| bits (31), 511 - logical row (9), lane * 4 + slot (8)
    double key = -1.0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const unsigned long long bits = __float_as_uint(fabsf(a[j][jj]));
      const double kj = (double)((bits << 17) | ((unsigned long long)(511 - (pos[j] & 511)) << 8) |
                                 (unsigned long long)(lane * 4 + j));
      key = (pos[j] >= k && pos[j] < n) ? fmax(key, kj) : key;
    }
    const unsigned long long kk = (unsigned long long)wmax(key);
    const int tp = 511 - (int)((kk >> 8) & 511);
    const int lp = (int)((kk & 255) >> 2), sp = (int)(kk & 3);
    float pr[16];
    switch (sp) {
#define PSR_LUW_ROW(J)                                                                        \
  case J:                                                                                     \
    _Pragma("unroll") for (int c = 0; c < 16; c++) if (c >= jj) pr[c] = rdlane(a[J][c], lp); \
    break;
      PSR_LUW_ROW(0)
      PSR_LUW_ROW(1)
      PSR_LUW_ROW(2)
      default:
        PSR_LUW_ROW(3)
#undef PSR_LUW_ROW
    }
    if (lane == 0) piv[k] = tp;
    // the interchange of logical rows k and tp relabels two rows
#pragma unroll
    for (int j = 0; j < 4; j++) pos[j] = pos[j] == k ? tp : (pos[j] == tp ? k : pos[j]);
    const float pv = pr[jj];
    float rcp = 0.f;
    if (pv != 0.f) rcp = 1.0f / pv;
    else if (info == 0) info = k + 1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const bool act = pos[j] > k && pos[j] < n;
      // |l| <= 1 by the choice of the pivot; the clamp keeps it so under the
      // rounding of the reciprocal
      const float l = act ? fminf(1.f, fmaxf(-1.f, a[j][jj] * rcp)) : 0.f;
      a[j][jj] = act ? l : a[j][jj];
#pragma unroll
      for (int c = 0; c < 16; c++)
        if (c > jj) a[j][c] = fmaf(-l, pr[c], a[j][c]);
    }
  }
  // ---- panel back to the float copy (physical rows) and to LDS (logical)
#pragma unroll
  for (int j = 0; j < 4; j++) {
    if (pos[j] < n) {
      float *dst = M + (int64_t)phys[j] * ld + k0;
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (k0 + 4 * q < ld) {
          const v4f_t v = {a[j][4 * q], a[j][4 * q + 1], a[j][4 * q + 2], a[j][4 * q + 3]};
          *reinterpret_cast<v4f_t *>(dst + 4 * q) = v;
        }
      float *l = S.L + (pos[j] - k0) * kPS;
#pragma unroll
      for (int c = 0; c < 16; c++) l[c] = a[j][c];
      S.perm[pos[j]] = phys[j];
    }
  }
  lds_order();
  const int m = n - R0;
  if (m <= 0) return;
  // ---- U12 = L11^-1 A12, columns R0 + lane + 64 g (m > 0, so kb = 16)
  float u[4][16];
  int prow[16];
#pragma unroll
  for (int i = 0; i < 16; i++) prow[i] = S.perm[k0 + i];
#pragma unroll
  for (int gq = 0; gq < 4; gq++) {
    const int c = R0 + lane + 64 * gq;
    const int cc = c < n ? c : n - 1;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const float v = ld_elem<FIRST>(g, M, n, ld, prow[i], cc);
      u[gq][i] = c < n ? v : 0.f;
    }
  }
  // L11 row l in lane l (l < 16); its elements reach every lane by readlane
  float lrow[16];
#pragma unroll
  for (int t = 0; t < 16; t++) lrow[t] = S.L[(lane & 15) * kPS + t];
#pragma unroll
  for (int i = 1; i < 16; i++) {
#pragma unroll
    for (int t = 0; t < i; t++) {
      const float lit = rdlane(lrow[t], i);
#pragma unroll
      for (int gq = 0; gq < 4; gq++) u[gq][i] = fmaf(-lit, u[gq][t], u[gq][i]);
    }
  }
#pragma unroll
  for (int gq = 0; gq < 4; gq++) {
    const int c = R0 + lane + 64 * gq;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (c < ld) M[(int64_t)prow[i] * ld + c] = u[gq][i];  // columns past n: padding
      S.U[i * kUS + lane + 64 * gq] = u[gq][i];           // zero past n
    }
  }
  lds_order();
  // ---- A22 -= L21 U12 on the matrix cores
  switch ((m + 15) >> 4) {
#define PSR_LUW_NT(T) \
  case T: trailing<FIRST, T>(n, ld, k0, kb, R0, g, M, S, lane); break;
    PSR_LUW_NT(1) PSR_LUW_NT(2) PSR_LUW_NT(3) PSR_LUW_NT(4) PSR_LUW_NT(5)
    PSR_LUW_NT(6) PSR_LUW_NT(7) PSR_LUW_NT(8) PSR_LUW_NT(9) PSR_LUW_NT(10)
    PSR_LUW_NT(11) PSR_LUW_NT(12) PSR_LUW_NT(13) PSR_LUW_NT(14)
    default: trailing<FIRST, 15>(n, ld, k0, kb, R0, g, M, S, lane); break;
#undef PSR_LUW_NT
  }
  wave_fence();
}

// Factor one n x n matrix g (row-major doubles, 64 < n <= 256) in place; M is
// this wavefront's float area, pad_rows(n) rows of ld floats, ld = pad_ld(n).
// Writes piv[0..n) (LAPACK convention) and returns info (0, or k + 1 of the
// first column without a nonzero pivot; the factorisation then continues as
// LAPACK's does, with no elimination in that column).
__device__ __forceinline__ int factor(int n, int ld, double *g, float *M, int *piv, WaveLds &S, int lane) {
  for (int i = lane; i < 256; i += 64) S.perm[i] = i;  // rows past n: padding
  lds_order();
  int info = 0;
  panel_step<true>(n, ld, 0, g, M, piv, S, lane, info);
  for (int k0 = 16; k0 < n; k0 += 16) panel_step<false>(n, ld, k0, g, M, piv, S, lane, info);
  wave_fence();
  // ---- factors to the caller's matrix in logical row order
  for (int i0 = 0; i0 < n; i0 += 32) {
    float v[32][4];
#pragma unroll
    for (int r = 0; r < 32; r++) {
      const int i = i0 + r;
      const int pr = S.perm[i < n ? i : n - 1];
#pragma unroll
      for (int gq = 0; gq < 4; gq++) {
        const int c = lane + 64 * gq;
        v[r][gq] = M[(int64_t)pr * ld + (c < n ? c : n - 1)];
      }
    }
#pragma unroll
    for (int r = 0; r < 32; r++) {
      const int i = i0 + r;
#pragma unroll
      for (int gq = 0; gq < 4; gq++) {
        const int c = lane + 64 * gq;
        if (i < n && c < n) g[(int64_t)i * n + c] = (double)v[r][gq];
      }
    }
  }
  return info;
}

}  // namespace luw
}  // namespace psr
