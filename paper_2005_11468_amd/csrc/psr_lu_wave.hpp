// Batched LU with partial pivoting, one wavefront per matrix, for the
// standalone psr_lu_factor_batch entry: float factors for 64 < n <= 256
// (PSR_MIXED) and FP64 factors for 64 < n <= 128 (PSR_FP64) -- the LU
// decomposition of the paper's Newton step (Sec. 3) on the matrix cores.
//
// Each wavefront factors its matrices one after another with no barrier and
// no other wavefront involved:
//   * the working copy is a matrix in a per-wavefront HBM area whose
//     rows are never moved: a logical -> physical row map in LDS stands for
//     the row interchanges, and the factors are written to the caller's
//     double matrix in logical order at the end;
//   * a 16-column panel lives in registers, rows spread over the lanes (lane
//     l holds the rows k0 + l + 64 j); in float each column's pivot is one DPP
//     wavefront maximum over a key that packs |a|, the logical row (lowest
//     wins a tie, as LAPACK) and the row's register position, in FP64 a
//     maximum of |a| and then a minimum of the logical row among the lanes
//     that hold it; the interchange only relabels rows, and the pivot row
//     reaches every lane by readlane;
//   * U12 = L11^-1 A12 with one column per lane, then A22 -= L21 U12 on
//     v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64 with both operands from
//     LDS and the C tiles streamed from and to the working copy.
// The first panel reads the caller's double matrix directly (in float
// rounding each element once), so no separate conversion pass is made.
#pragma once

namespace psr {
namespace luw {

constexpr int kPS = 17;  // row stride of the LDS panel copy
constexpr int kW = 4;    // wavefronts per workgroup

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v4d_t __attribute__((ext_vector_type(4)));

// Per precision: largest n, row slots per lane, LDS U12 row stride (the four
// rows a B operand load touches fall in different banks), accumulator tile.
template <typename T>
struct Prec;
template <>
struct Prec<float> {
  static constexpr int NMAX = 256, NS = 4, US = 272;
  typedef v4f_t acc_t;
  // MFMA result layout: register v of lane l holds row 4 (l / 16) + v
  static __device__ __forceinline__ int drow(int lk, int v) { return 4 * lk + v; }
  static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Prec<double> {
  static constexpr int NMAX = 128, NS = 2, US = 144;
  typedef v4d_t acc_t;
  // MFMA result layout: register v of lane l holds row l / 16 + 4 v
  static __device__ __forceinline__ int drow(int lk, int v) { return lk + 4 * v; }
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T>
struct WaveLds {
  T L[Prec<T>::NMAX * kPS];  // panel columns of logical rows k0..n-1 (row r - k0)
  T U[16 * Prec<T>::US];     // U12 of the current panel (column c - R0)
  int perm[256];             // logical row -> physical row of the working copy
};

// Working copy: rows and columns rounded up to whole tiles of 16.
__host__ __device__ constexpr int pad_rows(int n) { return (n + 15) & ~15; }
__host__ __device__ constexpr int pad_ld(int n) { return (n + 15) & ~15; }

__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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
__device__ __forceinline__ double wmax(double v) {
  v = fmax(v, dpp_mov<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_mov<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_mov<0x124>(v));  // row_ror 4
  v = fmax(v, dpp_mov<0x128>(v));  // row_ror 8
  return fmax(fmax(rdlane(v, 0), rdlane(v, 16)), fmax(rdlane(v, 32), rdlane(v, 48)));
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

// The caller's matrix is read once and written once: streaming accesses,
// which leave the caches to the working copies.
__device__ __forceinline__ double ld_once(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_once(double v, double *p) { __builtin_nontemporal_store(v, p); }

// Element (r, c) of the matrix being factored: the caller's double matrix
// before the first panel has written the working copy, the copy after.
template <typename T, bool FIRST>
__device__ __forceinline__ T ld_elem(const double *g, const T *M, int n, int ld, int r, int c) {
  return FIRST ? (T)ld_once(g + (int64_t)r * n + c) : M[(int64_t)r * ld + c];
}

// Pivot of column jj among the rows this lane holds (logical rows pos[j],
// candidates those >= k and < n): returns the logical row tp, the lane lp
// and slot sp that hold it.  The largest |a| wins, the lowest logical row
// among equals.
template <typename T, int NS>
__device__ __forceinline__ void pivot(const T (&a)[NS][16], int jj, const int (&pos)[NS], int k, int n, int lane,
                                      int &tp, int &lp, int &sp);
template <>
__device__ __forceinline__ void pivot<float, 4>(const float (&a)[4][16], int jj, const int (&pos)[4], int k, int n,
                                                int lane, int &tp, int &lp, int &sp) {
  // key: |a| bits (31), 511 - logical row (9), lane * 4 + slot (8), exact in a double
  double key = -1.0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const unsigned long long bits = __float_as_uint(fabsf(a[j][jj]));
    const double kj = (double)((bits << 17) | ((unsigned long long)(511 - (pos[j] & 511)) << 8) |
                               (unsigned long long)(lane * 4 + j));
    key = (pos[j] >= k && pos[j] < n) ? fmax(key, kj) : key;
  }
  const unsigned long long kk = (unsigned long long)wmax(key);
  tp = 511 - (int)((kk >> 8) & 511);
  lp = (int)((kk & 255) >> 2);
  sp = (int)(kk & 3);
}
template <>
__device__ __forceinline__ void pivot<double, 2>(const double (&a)[2][16], int jj, const int (&pos)[2], int k, int n,
                                                 int lane, int &tp, int &lp, int &sp) {
  double best = -1.0;
#pragma unroll
  for (int j = 0; j < 2; j++) best = (pos[j] >= k && pos[j] < n) ? fmax(best, fabs(a[j][jj])) : best;
  const double mx = wmax(best);
  // the lowest logical row holding the maximum: a maximum of -row
  double cand = -1024.0;
#pragma unroll
  for (int j = 0; j < 2; j++)
    cand = (pos[j] >= k && pos[j] < n && fabs(a[j][jj]) == mx) ? fmax(cand, (double)-pos[j]) : cand;
  tp = -(int)wmax(cand);
  lp = 0;
  sp = 0;
#pragma unroll
  for (int j = 0; j < 2; j++) {
    const unsigned long long m = __ballot(pos[j] == tp);
    if (m) {
      lp = __ffsll((long long)m) - 1;
      sp = j;
    }
  }
}

// A22 -= L21 U12 for the trailing block at logical row and column R0 (a
// multiple of 16), NT x NT tiles of 16: one row of tiles at a time in the
// MFMA result layout, the loads of the next row issued before the products of
// the current one.  Tiles reaching past n read and write the padding rows and
// columns of the working copy, so no access is predicated; the zero rows of
// the A operand and zero columns of U12 keep the padding out of the real
// elements.
template <typename T, int NT, bool FIRST>
__device__ __forceinline__ void trailing(int n, int ld, int k0, int kb, int R0, const double *g, T *M,
                                         const WaveLds<T> &S, int lane) {
  typedef Prec<T> P;
  constexpr int nt = NT;
  const int lr = lane & 15, lk = lane >> 4;
  T bq[NT][4];
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int q = 0; q < 4; q++) bq[t][q] = S.U[(4 * q + lk) * P::US + 16 * t + lr];
  typename P::acc_t cur[NT], nxt[NT];
  auto load_row = [&](typename P::acc_t *c, int ti) {
    int pr[4];
#pragma unroll
    for (int v = 0; v < 4; v++) pr[v] = S.perm[R0 + 16 * ti + P::drow(lk, v)];
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const int col = R0 + 16 * t + lr;
#pragma unroll
      for (int v = 0; v < 4; v++)
        c[t][v] = FIRST ? (T)ld_once(g + (int64_t)(pr[v] < n ? pr[v] : n - 1) * n + (col < n ? col : n - 1))
                        : M[(int64_t)pr[v] * ld + col];
    }
  };
  load_row(cur, 0);
  for (int ti = 0; ti < nt; ti++) {
    if (ti + 1 < nt) load_row(nxt, ti + 1);
    const int arow = R0 + 16 * ti + lr;  // A operand row of this lane
    T aq[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int kq = 4 * q + lk;
      const T v = S.L[((arow < n ? arow : n - 1) - k0) * kPS + kq];
      aq[q] = (arow < n && kq < kb) ? -v : (T)0;
    }
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int q = 0; q < 4; q++) cur[t] = P::mfma(aq[q], bq[t][q], cur[t]);
    int pr[4];
#pragma unroll
    for (int v = 0; v < 4; v++) pr[v] = S.perm[R0 + 16 * ti + P::drow(lk, v)];
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
template <typename T, bool FIRST>
__device__ __forceinline__ void panel_step(int n, int ld, int k0, double *g, T *M, int *piv, WaveLds<T> &S, int lane,
                                           int &info) {
  typedef Prec<T> P;
  constexpr int NS = P::NS, GQ = P::NMAX / 64;
  const int kb = n - k0 < 16 ? n - k0 : 16;
  const int R0 = k0 + kb;
  // ---- panel: logical rows k0 + lane + 64 j, columns k0..k0+15
  T a[NS][16];
  int phys[NS], pos[NS];
#pragma unroll
  for (int j = 0; j < NS; j++) {
    const int t = k0 + lane + 64 * j;
    const bool ok = t < n;
    pos[j] = ok ? t : (1 << 20);
    phys[j] = S.perm[ok ? t : n - 1];
    if (FIRST) {
      const double *src = g + (int64_t)phys[j] * n;  // n > 64: columns 0..15 exist
#pragma unroll
      for (int c = 0; c < 16; c++) {
        const T v = (T)ld_once(src + c);
        a[j][c] = ok ? v : (T)0;
      }
    } else if constexpr (sizeof(T) == 4) {
      // columns k0..k0+15 lie inside the padded row, 64-byte aligned
      const v4f_t *src = reinterpret_cast<const v4f_t *>(M + (int64_t)phys[j] * ld + k0);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const v4f_t v = src[q];
#pragma unroll
        for (int e = 0; e < 4; e++) a[j][4 * q + e] = (ok && k0 + 4 * q + e < n) ? v[e] : (T)0;
      }
    } else {
      const T *src = M + (int64_t)phys[j] * ld + k0;
#pragma unroll
      for (int c = 0; c < 16; c++) {
        const T v = src[c];
        a[j][c] = (ok && k0 + c < n) ? v : (T)0;
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < 16; jj++) {
    // a constant trip count keeps the loop unrolled, so every register
    // index is a compile-time constant
    if (jj >= kb) continue;
    const int k = k0 + jj;
    int tp, lp, sp;
    pivot<T, NS>(a, jj, pos, k, n, lane, tp, lp, sp);
    T pr[16];
    switch (sp) {
#define PSR_LUW_ROW(J)                                                                        \
  case J:                                                                                     \
    _Pragma("unroll") for (int c = 0; c < 16; c++) if (c >= jj) pr[c] = rdlane(a[J][c], lp); \
    break;
      PSR_LUW_ROW(0)
      default:
        if constexpr (NS == 2) {
          _Pragma("unroll") for (int c = 0; c < 16; c++) if (c >= jj) pr[c] = rdlane(a[1][c], lp);
        } else {
          switch (sp) {
            PSR_LUW_ROW(1)
            PSR_LUW_ROW(2)
            default:
              _Pragma("unroll") for (int c = 0; c < 16; c++) if (c >= jj) pr[c] = rdlane(a[3][c], lp);
          }
        }
        break;
#undef PSR_LUW_ROW
    }
    if (lane == 0) piv[k] = tp;
    // the interchange of logical rows k and tp relabels two rows
#pragma unroll
    for (int j = 0; j < NS; j++) pos[j] = pos[j] == k ? tp : (pos[j] == tp ? k : pos[j]);
    const T pv = pr[jj];
    T rcp = 0;
    if (pv != (T)0) rcp = (T)1 / pv;
    else if (info == 0) info = k + 1;
#pragma unroll
    for (int j = 0; j < NS; j++) {
      const bool act = pos[j] > k && pos[j] < n;
      // |l| <= 1 by the choice of the pivot; the clamp keeps it so under the
      // rounding of the reciprocal
      const T l = act ? fmin((T)1, fmax((T)-1, a[j][jj] * rcp)) : (T)0;
      a[j][jj] = act ? l : a[j][jj];
#pragma unroll
      for (int c = 0; c < 16; c++)
        if (c > jj) a[j][c] = fma(-l, pr[c], a[j][c]);
    }
  }
  // ---- panel back to the working copy (physical rows) and to LDS (logical)
#pragma unroll
  for (int j = 0; j < NS; j++) {
    if (pos[j] < n) {
      T *dst = M + (int64_t)phys[j] * ld + k0;
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const v4f_t v = {a[j][4 * q], a[j][4 * q + 1], a[j][4 * q + 2], a[j][4 * q + 3]};
          reinterpret_cast<v4f_t *>(dst)[q] = v;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 16; c++) dst[c] = a[j][c];
      }
      T *l = S.L + (pos[j] - k0) * kPS;
#pragma unroll
      for (int c = 0; c < 16; c++) l[c] = a[j][c];
      S.perm[pos[j]] = phys[j];
    }
  }
  lds_order();
  const int m = n - R0;
  if (m <= 0) return;
  // ---- U12 = L11^-1 A12, columns R0 + lane + 64 g (m > 0, so kb = 16)
  T u[GQ][16];
  int prow[16];
#pragma unroll
  for (int i = 0; i < 16; i++) prow[i] = S.perm[k0 + i];
#pragma unroll
  for (int gq = 0; gq < GQ; gq++) {
    const int c = R0 + lane + 64 * gq;
    const int cc = c < n ? c : n - 1;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const T v = ld_elem<T, FIRST>(g, M, n, ld, prow[i], cc);
      u[gq][i] = c < n ? v : (T)0;
    }
  }
  // L11 row l in lane l (l < 16); its elements reach every lane by readlane
  T lrow[16];
#pragma unroll
  for (int t = 0; t < 16; t++) lrow[t] = S.L[(lane & 15) * kPS + t];
#pragma unroll
  for (int i = 1; i < 16; i++) {
#pragma unroll
    for (int t = 0; t < i; t++) {
      const T lit = rdlane(lrow[t], i);
#pragma unroll
      for (int gq = 0; gq < GQ; gq++) u[gq][i] = fma(-lit, u[gq][t], u[gq][i]);
    }
  }
#pragma unroll
  for (int gq = 0; gq < GQ; gq++) {
    const int c = R0 + lane + 64 * gq;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      if (c < ld) M[(int64_t)prow[i] * ld + c] = u[gq][i];  // columns past n: padding
      S.U[i * P::US + lane + 64 * gq] = u[gq][i];           // zero past n
    }
  }
  lds_order();
  // ---- A22 -= L21 U12 on the matrix cores
  switch ((m + 15) >> 4) {
#define PSR_LUW_NT(T_) \
  case T_: trailing<T, T_, FIRST>(n, ld, k0, kb, R0, g, M, S, lane); break;
    PSR_LUW_NT(1) PSR_LUW_NT(2) PSR_LUW_NT(3) PSR_LUW_NT(4) PSR_LUW_NT(5) PSR_LUW_NT(6)
    default:
      if constexpr (P::NMAX > 128) {
        switch ((m + 15) >> 4) {
          PSR_LUW_NT(7) PSR_LUW_NT(8) PSR_LUW_NT(9) PSR_LUW_NT(10)
          PSR_LUW_NT(11) PSR_LUW_NT(12) PSR_LUW_NT(13) PSR_LUW_NT(14)
          default: trailing<T, 15, FIRST>(n, ld, k0, kb, R0, g, M, S, lane); break;
        }
      } else {
        trailing<T, 7, FIRST>(n, ld, k0, kb, R0, g, M, S, lane);
      }
      break;
#undef PSR_LUW_NT
  }
  wave_fence();
}

// Factor one n x n matrix g (row-major doubles, 64 < n <= Prec<T>::NMAX) in
// place; M is this wavefront's area, pad_rows(n) rows of ld = pad_ld(n)
// elements.  Writes piv[0..n) (LAPACK convention) and returns info (0, or
// k + 1 of the first column without a nonzero pivot; the factorisation then
// continues as LAPACK's does, with no elimination in that column).
template <typename T>
__device__ __forceinline__ int factor(int n, int ld, double *g, T *M, int *piv, WaveLds<T> &S, int lane) {
  constexpr int GQ = Prec<T>::NMAX / 64;
  for (int i = lane; i < 256; i += 64) S.perm[i] = i;  // rows past n: padding
  lds_order();
  int info = 0;
  panel_step<T, true>(n, ld, 0, g, M, piv, S, lane, info);
  for (int k0 = 16; k0 < n; k0 += 16) panel_step<T, false>(n, ld, k0, g, M, piv, S, lane, info);
  wave_fence();
  // ---- factors to the caller's matrix in logical row order
  for (int i0 = 0; i0 < n; i0 += 32) {
    T v[32][GQ];
#pragma unroll
    for (int r = 0; r < 32; r++) {
      const int i = i0 + r;
      const int pr = S.perm[i < n ? i : n - 1];
#pragma unroll
      for (int gq = 0; gq < GQ; gq++) {
        const int c = lane + 64 * gq;
        v[r][gq] = M[(int64_t)pr * ld + (c < n ? c : n - 1)];
      }
    }
#pragma unroll
    for (int r = 0; r < 32; r++) {
      const int i = i0 + r;
#pragma unroll
      for (int gq = 0; gq < GQ; gq++) {
        const int c = lane + 64 * gq;
        if (i < n && c < n) st_once((double)v[r][gq], g + (int64_t)i * n + c);
      }
    }
  }
  return info;
}

}  // namespace luw
}  // namespace psr
