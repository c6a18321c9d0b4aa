// Wavefront-per-reactor engine for systems of up to NP <= 64 unknowns.
//
// A workgroup holds RPW wavefronts; every wavefront owns one reactor and
// advances it independently (wavefront-level synchronisation only).  The
// mechanism tables are staged once per workgroup in LDS and shared by its
// wavefronts.  Per reactor:
//   * vectors of length n (x, Newton step, ...): one element per lane, in VGPRs;
//   * species scratch for the residual and Jacobian: LDS;
//   * reactions are spread over the lanes; each lane scatters its reactions'
//     contributions into per-species LDS accumulators with LDS atomic adds
//     (one wavefront owns the area, so the order of the adds is fixed);
//   * the Jacobian is assembled in LDS (row i = equation i), then lane i loads
//     row i into VGPRs and the LU runs in registers: the pivot column is found
//     with a wave reduction, the pivot row is broadcast with readlane, rows do
//     not move during the elimination; afterwards pivot row k is moved to lane
//     k once and L, U are scaled to unit diagonals for the solves.
// Paper: Section 2 (Eqs. 1-3) and Section 3 (Eqs. 4-9, hybrid method).
#pragma once

#include "psr_device.hpp"

namespace psr {
namespace wave {

constexpr int WS = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WS - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / WS; }
__device__ __forceinline__ void wsync() { __syncwarp(); }

// Row-local data movement with DPP (no LDS round trip).  CTRL: 0xB1 swaps
// neighbouring lanes, 0x4E lanes two apart, 0x124 / 0x128 rotate each row of
// 16 lanes by 4 / 8.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int bcast(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Wavefront reductions (call with every lane active).  Each row of 16 lanes
// is reduced with DPP, the four row results are combined in a fixed order
// from scalar registers, so every lane gets the same bits.
__device__ __forceinline__ double wsum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x124>(v);
  v += dpp_mov<0x128>(v);
  return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}
__device__ __forceinline__ double wmax(double v) {  // NaN counts as +inf
  if (v != v) v = __builtin_inf();
  v = fmax(v, dpp_mov<0xB1>(v));
  v = fmax(v, dpp_mov<0x4E>(v));
  v = fmax(v, dpp_mov<0x124>(v));
  v = fmax(v, dpp_mov<0x128>(v));
  return fmax(fmax(bcast(v, 0), bcast(v, 16)), fmax(bcast(v, 32), bcast(v, 48)));
}
__device__ __forceinline__ bool wany(bool p) { return __ballot(p) != 0ull; }

constexpr double kThird = 1.0 / 3.0;

// c^m for a stoichiometric coefficient m >= 1: straight-line for m <= 3 (every
// elementary reaction here), a loop beyond.
__device__ __forceinline__ double ipow(double c, int m) {
  double p = c;
  if (m >= 2) p *= c;
  if (m >= 3) p *= c;
  for (int e = 3; e < m; e++) p *= c;
  return p;
}

// ----------------------------------------------------------------- tables

// Packed mechanism tables in LDS (shared by the workgroup's wavefronts).
// Reaction k: slots packed in three words
//   w0 = r0 | r1 << 8 | r2 << 16          reactant species (0xff: unused)
//   w1 = p0 | p1 << 8 | p2 << 16          product species
//   w2 = rnu0 | rnu1 << 4 | rnu2 << 8 | pnu0 << 12 | pnu1 << 16 | pnu2 << 20 | (dnu + 16) << 24
// CSR entry of species i: k << 8 | (net nu + 128).
struct Tables {
  int N, I, nnz;
  const double *lnA, *beta, *EoR, *W, *nasa;
  const int *w0, *w1, *w2, *sp_ptr, *sp_ent;
};

__host__ __device__ inline size_t tables_bytes(int N, int I, int nnz) {
  return (size_t)8 * (3 * I + N + 7 * N) + (size_t)4 * (3 * I + N + 1 + nnz);
}

// Stage the tables of `m` into LDS at `base` (all threads of the block).
__device__ __forceinline__ Tables stage_tables(const MechDev &m, char *base, const int *packed) {
  Tables t;
  t.N = m.N; t.I = m.I; t.nnz = m.nnz;
  double *d = reinterpret_cast<double *>(base);
  double *lnA = d, *beta = d + m.I, *EoR = d + 2 * m.I, *W = d + 3 * m.I, *nasa = W + m.N;
  int *ib = reinterpret_cast<int *>(nasa + 7 * m.N);
  int *w0 = ib, *w1 = ib + m.I, *w2 = ib + 2 * m.I, *ptr = ib + 3 * m.I, *ent = ptr + m.N + 1;
  for (int k = threadIdx.x; k < m.I; k += blockDim.x) {
    lnA[k] = m.lnA[k]; beta[k] = m.beta[k]; EoR[k] = m.EoR[k];
    w0[k] = packed[k]; w1[k] = packed[m.I + k]; w2[k] = packed[2 * m.I + k];
  }
  for (int i = threadIdx.x; i < m.N; i += blockDim.x) W[i] = m.W[i];
  for (int e = threadIdx.x; e < 7 * m.N; e += blockDim.x) nasa[e] = m.nasa[e];
  for (int i = threadIdx.x; i <= m.N; i += blockDim.x) ptr[i] = m.sp_ptr[i];
  for (int e = threadIdx.x; e < m.nnz; e += blockDim.x) ent[e] = packed[3 * m.I + e];
  t.lnA = lnA; t.beta = beta; t.EoR = EoR; t.W = W; t.nasa = nasa;
  t.w0 = w0; t.w1 = w1; t.w2 = w2; t.sp_ptr = ptr; t.sp_ent = ent;
  return t;
}

// ------------------------------------------------------------ reactor LDS

// Per-reactor LDS area (doubles): Jacobian rows [n][ldj] (ldj = n | 1),
// species scratch, column scales and a two-slot-per-lane area zs used as
// per-species accumulators by the residual and Jacobian and as a broadcast
// vector by the solves.
template <int NP>
struct WArea {
  static __host__ __device__ int ldj_of(int n) { return n | 1; }
  static __host__ __device__ int doubles(int n) { return n * ldj_of(n) + 8 * WS; }
  int ldj;
  double *J, *Cs, *gs, *hs, *iSW, *rW, *cs, *zs;
  __device__ void at(double *p, int n) {
    ldj = ldj_of(n);
    J = p; p += n * ldj;
    Cs = p; p += WS; gs = p; p += WS; hs = p; p += WS; iSW = p; p += WS; rW = p; p += WS;
    cs = p; p += WS; zs = p;
  }
  // Species scratch of a residual evaluation only (C, g, H/RT and the two
  // accumulators; no Jacobian rows or Jacobian scratch).
  static __host__ __device__ int species_doubles() { return 5 * WS; }
  __device__ void at_species(double *p) {
    ldj = 0;
    J = nullptr;
    iSW = rW = cs = nullptr;
    Cs = p; p += WS; gs = p; p += WS; hs = p; p += WS; zs = p;
  }
};

// Per-reactor values of the last residual evaluation.
struct Eval {
  double T, S, rho, mdot;
  double cpR, hRT, wdot, C;  // lane i < N: species i
};

struct WCtx {
  Tables t;
  int N, n, energy;
  double P, tau, Tin;
  double Yin, Hin;  // lane i < N
};

// Residual F (lane i holds F_i; lane N holds F_T) of Eq. 2 and Eq. 3 times
// -rho V, rates from Eqs. 4-9.  Leaves C, g = S/R - H/RT and H/RT in LDS;
// reaction k is handled by lane k mod 64, which adds nu_ik q_k into species
// i's production-rate accumulator.  Returns the scaled
// residual when asked (each equation's |F| over the sum of its terms'
// magnitudes).
template <int NP>
__device__ __forceinline__ double w_residual(const WCtx &c, const WArea<NP> &a, double x, double &F, Eval &ev,
                             bool want_sres) {
  const Tables &t = c.t;
  const int lane = lane_id(), N = c.N;
  const double T = c.energy ? bcast(x, N) : c.Tin;
  const bool sp = lane < N;
  const double Wl = sp ? t.W[lane] : 1.0;
  const double S = wsum(sp ? x / Wl : 0.0);
  const double rho = c.P * 1.0e-6 / (kR * T * S);
  const double mdot = rho * kV / c.tau;
  const double lnT = log(T), invT = 1.0 / T;
  const double lnc = log(kPatm * 1.0e-6 / (kR * T));
  ev.T = T; ev.S = S; ev.rho = rho; ev.mdot = mdot;
  if (sp) {
    const double *n7 = t.nasa + 7 * lane;
    const double C = rho * x / Wl;
    const double cp = n7[0] + T * (n7[1] + T * (n7[2] + T * (n7[3] + T * n7[4])));
    // constant reciprocals instead of divisions (an FP64 division is ~10 instructions)
    const double h = n7[0] + T * (n7[1] * 0.5 + T * (n7[2] * kThird + T * (n7[3] * 0.25 + T * n7[4] * 0.2)))
                     + n7[5] * invT;
    const double s = n7[0] * lnT + T * (n7[1] + T * (n7[2] * 0.5 + T * (n7[3] * kThird + T * n7[4] * 0.25)))
                     + n7[6];
    a.Cs[lane] = C; a.gs[lane] = s - h; a.hs[lane] = h;
    ev.C = C; ev.cpR = cp; ev.hRT = h;
  } else {
    ev.C = 0.0; ev.cpR = 0.0; ev.hRT = 0.0;
  }
  double *wd = a.zs, *gq = a.zs + WS;  // per-species net and gross rates
  wd[lane] = 0.0;
  gq[lane] = 0.0;
  wsync();
#pragma unroll 2
  for (int k = lane; k < t.I; k += WS) {
    const int w0 = t.w0[k], w1 = t.w1[k], w2 = t.w2[k];
    double g = 0.0, fwd = 1.0, rev = 1.0;
#pragma unroll
    for (int sl = 0; sl < 3; sl++) {
      const int ir = (w0 >> (8 * sl)) & 0xff, ip = (w1 >> (8 * sl)) & 0xff;
      if (ir != 0xff) {
        const int nu = (w2 >> (4 * sl)) & 0xf;
        const double Cj = a.Cs[ir];
        g -= nu * a.gs[ir];
        fwd *= ipow(Cj, nu);
      }
      if (ip != 0xff) {
        const int nu = (w2 >> (12 + 4 * sl)) & 0xf;
        const double Cj = a.Cs[ip];
        g += nu * a.gs[ip];
        rev *= ipow(Cj, nu);
      }
    }
    const int dnu = ((w2 >> 24) & 0xff) - 16;
    const double lnkf = t.lnA[k] + t.beta[k] * lnT - t.EoR[k] * invT;
    const double lnKc = g + dnu * lnc;
    const double rf = exp(lnkf) * fwd, rr = exp(lnkf - lnKc) * rev;
    const double q = rf - rr, qa = fabs(rf) + fabs(rr);
#pragma unroll
    for (int sl = 0; sl < 3; sl++) {
      const int ir = (w0 >> (8 * sl)) & 0xff, ip = (w1 >> (8 * sl)) & 0xff;
      if (ir != 0xff) {
        const double nu = (double)((w2 >> (4 * sl)) & 0xf);
        atomicAdd(&wd[ir], -nu * q);
        if (want_sres) atomicAdd(&gq[ir], nu * qa);
      }
      if (ip != 0xff) {
        const double nu = (double)((w2 >> (12 + 4 * sl)) & 0xf);
        atomicAdd(&wd[ip], nu * q);
        if (want_sres) atomicAdd(&gq[ip], nu * qa);
      }
    }
  }
  wsync();
  double Fl = 0.0, w = 0.0, gr = 0.0;
  if (sp) {
    w = wd[lane];
    gr = gq[lane];
    Fl = mdot * (x - c.Yin) - kV * Wl * w;
  }
  ev.wdot = w;
  double sres = 0.0;
  if (c.energy) {
    const double H = kR * T * ev.hRT;
    const double inflow = wsum(sp ? c.Yin * (H - c.Hin) / Wl : 0.0);
    const double chem = wsum(sp ? H * w : 0.0);
    const double FT = mdot * inflow + kV * chem;
    if (lane == N) Fl = FT;
    if (want_sres) {
      const double den = wsum(sp ? mdot * fabs(c.Yin * (H - c.Hin) / Wl) + kV * fabs(H) * gr : 0.0);
      double r = (den > 0.0) ? fabs(FT) / den : 0.0;
      if (FT != FT) r = __builtin_inf();
      sres = r;
    }
  }
  if (want_sres) {
    double r = 0.0;
    if (sp) {
      const double den = mdot * (fabs(x) + fabs(c.Yin)) + kV * Wl * gr;
      r = (den > 0.0) ? fabs(Fl) / den : 0.0;
      if (!(den >= 0.0) || Fl != Fl) r = __builtin_inf();
    }
    sres = fmax(sres, wmax(r));
  }
  F = Fl;
  return sres;
}

// Analytic Jacobian of w_residual at the same x, into the LDS rows a.J.
// Lane k mod 64 re-evaluates k_f, k_r of reaction k and the derivatives
// dq_k/dC_m for the (at most six) species m of the reaction, and adds
// nu_ik dq_k/dC_m into D_im (held in the rows of a.J) for every species i of
// the reaction, together with the reaction's terms of E_i = sum_k nu_ik
// sum_m C_m dq_k/dC_m and of the temperature derivative at constant C.  The
// density and temperature chain rule then turns D into dF/dx (the same
// formulas as jacobian() in psr_device.hpp).
template <int NP>
__device__ __forceinline__ void w_jacobian(const WCtx &c, const WArea<NP> &a, double x, const Eval &ev) {
  const int LDJ = a.ldj;
  const Tables &t = c.t;
  const int lane = lane_id(), N = c.N, n = c.n;
  const bool sp = lane < N;
  const double T = ev.T, S = ev.S, rho = ev.rho, mdot = ev.mdot, invT = 1.0 / T, lnT = log(T);
  const double lnc = log(kPatm * 1.0e-6 / (kR * T));
  double *Ea = a.zs, *dTa = a.zs + WS;
#pragma unroll 4
  for (int e = lane; e < n * LDJ; e += WS) a.J[e] = 0.0;
  Ea[lane] = 0.0;
  dTa[lane] = 0.0;
  if (sp) {
    const double Wl = t.W[lane];
    a.iSW[lane] = 1.0 / (S * Wl);
    a.rW[lane] = rho / Wl;
  }
  wsync();
  for (int k = lane; k < t.I; k += WS) {
    const int w0 = t.w0[k], w1 = t.w1[k], w2 = t.w2[k];
    // slots 0-2: reactants, 3-5: products; idx 0xff marks an unused slot
    int idx[6];
    double nu[6], Cv[6], pw[6], dpw[6];
    double g = 0.0, sh = 0.0;
#pragma unroll
    for (int q = 0; q < 6; q++) {
      const int sl = q % 3;
      const bool prod = q >= 3;
      const int i = ((prod ? w1 : w0) >> (8 * sl)) & 0xff;
      const int m = (w2 >> (prod ? 12 + 4 * sl : 4 * sl)) & 0xf;
      idx[q] = i;
      double C = 0.0, p = 1.0, dp = 0.0, v = 0.0;
      if (i != 0xff) {
        C = a.Cs[i];
        const double sgn = prod ? 1.0 : -1.0;
        g += sgn * m * a.gs[i];
        sh += sgn * m * a.hs[i];
        const double pm1 = m >= 2 ? ipow(C, m - 1) : 1.0;  // C^(m-1)
        dp = m * pm1;
        p = pm1 * C;
        v = sgn * m;
      }
      nu[q] = v; Cv[q] = C; pw[q] = p; dpw[q] = dp;
    }
    const int dnu = ((w2 >> 24) & 0xff) - 16;
    const double lnkf = t.lnA[k] + t.beta[k] * lnT - t.EoR[k] * invT;
    const double kf = exp(lnkf), kr = exp(lnkf - (g + dnu * lnc));
    double dq[6];
    dq[0] = kf * dpw[0] * pw[1] * pw[2];
    dq[1] = kf * pw[0] * dpw[1] * pw[2];
    dq[2] = kf * pw[0] * pw[1] * dpw[2];
    dq[3] = -kr * dpw[3] * pw[4] * pw[5];
    dq[4] = -kr * pw[3] * dpw[4] * pw[5];
    dq[5] = -kr * pw[3] * pw[4] * dpw[5];
    const double Rf = kf * pw[0] * pw[1] * pw[2], Rr = kr * pw[3] * pw[4] * pw[5];
    double sumC = 0.0;
#pragma unroll
    for (int q = 0; q < 6; q++) sumC += Cv[q] * dq[q];
    const double dlnkf = t.beta[k] * invT + t.EoR[k] * invT * invT;
    const double dlnKc = sh * invT - dnu * invT;
    const double tq = Rf * dlnkf - Rr * (dlnkf - dlnKc) - sumC * invT;
#pragma unroll
    for (int q = 0; q < 6; q++) {
      if (idx[q] == 0xff) continue;
      const int i = idx[q];
      atomicAdd(&Ea[i], nu[q] * sumC);
      atomicAdd(&dTa[i], nu[q] * tq);
      double *Di = a.J + i * LDJ;
#pragma unroll
      for (int r = 0; r < 6; r++)
        if (idx[r] != 0xff) atomicAdd(&Di[idx[r]], nu[q] * dq[r]);
    }
  }
  wsync();
  const double E = sp ? Ea[lane] : 0.0, dT = sp ? dTa[lane] : 0.0;
  double *row = a.J + (lane < n ? lane : 0) * LDJ;
  if (c.energy) {
    const double Wl = sp ? t.W[lane] : 1.0;
    const double H = kR * T * ev.hRT;
    const double Qin = wsum(sp ? c.Yin * (H - c.Hin) / Wl : 0.0);
    const double dQin = wsum(sp ? c.Yin * kR * ev.cpR / Wl : 0.0);
    const double TT = wsum(sp ? kV * (kR * ev.cpR * ev.wdot + H * dT) : 0.0);
    const double HE = wsum(sp ? H * E : 0.0);
    double v = 0.0;
    if (sp) {
#pragma unroll 8
      for (int i = 0; i < N; i++) v += a.hs[i] * a.J[i * LDJ + lane];
      v *= kR * T;
      a.J[N * LDJ + lane] = -mdot * Qin * a.iSW[lane] + kV * (v * a.rW[lane] - HE * a.iSW[lane]);
    }
    if (lane == N) a.J[N * LDJ + N] = -mdot * invT * Qin + mdot * dQin + TT;
    wsync();
  }
  if (sp) {
    const double yd = x - c.Yin, Wl = t.W[lane];
#pragma unroll 8
    for (int m = 0; m < N; m++) {
      const double is = a.iSW[m];
      double v = -mdot * is * yd - kV * Wl * (row[m] * a.rW[m] - E * is);
      if (m == lane) v += mdot;
      row[m] = v;
    }
    if (c.energy) row[N] = -mdot * invT * yd - kV * Wl * dT;
  }
  wsync();
}

// ------------------------------------------------------------ register LU

// A matrix row lives in lane r's VGPRs as T a[NP].  Inside the LU and the
// solves it is held as four local 16-element vectors (they must be function
// locals: wrapped in a struct they are placed in scratch memory).  Column k
// is read from vector k / 16 with a relative register move; every loop over
// k is split by that vector at compile time, so all other accesses use
// compile-time indices.
template <typename T>
struct V16 {
  typedef T type __attribute__((ext_vector_type(16)));
};

template <int Q, typename VT>
__device__ __forceinline__ VT &chunk(VT &c0, VT &c1, VT &c2, VT &c3) {
  if constexpr (Q == 0) return c0;
  else if constexpr (Q == 1) return c1;
  else if constexpr (Q == 2) return c2;
  else return c3;
}

template <int NP, typename T, typename VT>
__device__ __forceinline__ void row_to_vec(const T (&a)[NP], VT &c0, VT &c1, VT &c2, VT &c3) {
  static_assert(NP % 16 == 0 && NP <= 64, "row length must be 16, 32, 48 or 64");
#pragma unroll
  for (int j = 0; j < 16; j++) {
    c0[j] = a[j];
    c1[j] = NP > 16 ? a[(NP > 16 ? 16 : 0) + j] : T(0);
    c2[j] = NP > 32 ? a[(NP > 32 ? 32 : 0) + j] : T(0);
    c3[j] = NP > 48 ? a[(NP > 48 ? 48 : 0) + j] : T(0);
  }
}

template <int NP, typename T, typename VT>
__device__ __forceinline__ void vec_to_row(const VT &c0, const VT &c1, const VT &c2, const VT &c3, T (&a)[NP]) {
#pragma unroll
  for (int j = 0; j < 16; j++) {
    a[j] = c0[j];
    if (NP > 16) a[(NP > 16 ? 16 : 0) + j] = c1[j];
    if (NP > 32) a[(NP > 32 ? 32 : 0) + j] = c2[j];
    if (NP > 48) a[(NP > 48 ? 48 : 0) + j] = c3[j];
  }
}

// Rank-one update of vectors Q.. at elimination step k (column kk = k mod 16
// of vector KC): c[j] -= l * u[j] with u the pivot row (lane p), read with
// readlane a whole vector at a time; columns <= k keep their values.
template <int NP, int KC, int Q, typename T, typename VT>
__device__ __forceinline__ void lu_update(VT &c0, VT &c1, VT &c2, VT &c3, int kk, int p, T l) {
  if constexpr (Q < NP / 16) {
    VT &cq = chunk<Q>(c0, c1, c2, c3);
    T u[16];
#pragma unroll
    for (int j = 0; j < 16; j++) {
      u[j] = bcast(cq[j], p);
      if (Q == KC) u[j] = j > kk ? u[j] : T(0);
    }
#pragma unroll
    for (int j = 0; j < 16; j++) cq[j] -= l * u[j];
    lu_update<NP, KC, Q + 1, T>(c0, c1, c2, c3, kk, p, l);
  }
}

// Elimination steps k = 16 KC .. min(n, 16 KC + 16) - 1.  Returns false on a
// zero pivot column (info = k + 1).
template <int NP, int KC, typename T, typename VT>
__device__ __forceinline__ bool lu_steps(VT &c0, VT &c1, VT &c2, VT &c3, int n, int &pos, int &permk, T &pivk,
                                         int &info) {
  if constexpr (KC < NP / 16) {
    const int lane = lane_id();
    VT &ck = chunk<KC>(c0, c1, c2, c3);
    const int kend = n < 16 * KC + 16 ? n : 16 * KC + 16;
    for (int k = 16 * KC; k < kend; k++) {
      const int kk = k & 15;
      const T ak = ck[kk];
      const double v = (pos == NP) ? fabs((double)ak) : -1.0;
      const double vmax = wmax(v);
      const unsigned long long m = __ballot(v == vmax);
      if (!(vmax > 0.0) || m == 0ull) {
        info = k + 1;
        return false;
      }
      const int p = __builtin_ctzll(m);
      const T piv = bcast(ak, p);
      if (lane == k) {
        permk = p;
        pivk = piv;
      }
      const T l = (pos == NP && lane != p) ? ak / piv : T(0);
      lu_update<NP, KC, KC, T>(c0, c1, c2, c3, kk, p, l);
      if (lane == p) pos = k;
    }
    if (kend < 16 * KC + 16) return true;
    return lu_steps<NP, KC + 1, T>(c0, c1, c2, c3, n, pos, permk, pivk, info);
  }
  return true;
}

// LU with partial pivoting of the n x n matrix whose row r sits in lane r's
// registers a[0..NP-1] (rows >= n are zero).  Rows are not moved: pos is the
// step at which the lane's row became the pivot row (NP while not yet
// pivoted, -1 for padding lanes); lane k's permk records the lane of pivot
// row k and its pivk the pivot U_kk.  After the call the lane whose row was
// pivot row `pos` holds U in columns pos..n-1 and, in columns k < pos, the
// value a_rk the row had when column k was eliminated (its L multiplier is
// a_rk / U_kk).  Pivot = first lane index among the largest |a_rk| of the
// not-yet-pivoted rows.  Returns 0, or k+1 if column k has no nonzero pivot.
template <int NP, typename T>
__device__ __forceinline__ int lu_regs(T (&a)[NP], int n, int &pos, int &permk, T &pivk) {
  typedef typename V16<T>::type VT;
  VT c0, c1, c2, c3;
  row_to_vec<NP, T>(a, c0, c1, c2, c3);
  pos = (lane_id() < n) ? NP : -1;
  permk = 0;
  pivk = T(1);
  int info = 0;
  lu_steps<NP, 0, T>(c0, c1, c2, c3, n, pos, permk, pivk, info);
  vec_to_row<NP, T>(c0, c1, c2, c3, a);
  return info;
}

// Lane `src`'s value, for every lane (ds_bpermute; no LDS storage is used).
__device__ __forceinline__ double bperm(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int NP, int Q, typename VD>
__device__ __forceinline__ void permute_scale(VD &c0, VD &c1, VD &c2, VD &c3, int src, double pinv) {
  if constexpr (Q < NP / 16) {
    const int lane = lane_id();
    VD &cq = chunk<Q>(c0, c1, c2, c3);
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const double v = bperm(cq[j], src);
      const double pj = bcast(pinv, 16 * Q + j);
      cq[j] = v * ((16 * Q + j) < lane ? pj : pinv);
    }
    permute_scale<NP, Q + 1>(c0, c1, c2, c3, src, pinv);
  }
}

// Turn the register factors of lu_regs into the form the solves use: lane k
// (k < n) receives pivot row k (moved with ds_bpermute), its L part
// (columns j < k) is divided by U_jj and its U part by U_kk, so L and U both
// have unit diagonals; pinv (lane k) = 1 / U_kk.  Rows of lanes >= n stay 0.
template <int NP, typename T>
__device__ __forceinline__ void lu_finish(const T (&f)[NP], double (&a)[NP], int n, int permk, T pivk,
                                          double &pinv) {
  typedef typename V16<double>::type VD;
  VD c0, c1, c2, c3;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    c0[j] = (double)f[j];
    c1[j] = NP > 16 ? (double)f[(NP > 16 ? 16 : 0) + j] : 0.0;
    c2[j] = NP > 32 ? (double)f[(NP > 32 ? 32 : 0) + j] : 0.0;
    c3[j] = NP > 48 ? (double)f[(NP > 48 ? 48 : 0) + j] : 0.0;
  }
  const int lane = lane_id();
  pinv = 1.0 / (double)pivk;
  permute_scale<NP, 0>(c0, c1, c2, c3, lane < n ? permk : lane, pinv);
  vec_to_row<NP, double>(c0, c1, c2, c3, a);
}

// The substitution loops are unrolled (compile-time column index, no
// relative register moves); a uniform guard stops at column n.
template <int NP, int KC, typename VD>
__device__ __forceinline__ double solve_lower(const VD &c0, const VD &c1, const VD &c2, const VD &c3, int n,
                                              double y) {
  if constexpr (KC < NP / 16) {
    const int lane = lane_id();
    const VD &ck = chunk<KC>(const_cast<VD &>(c0), const_cast<VD &>(c1), const_cast<VD &>(c2), const_cast<VD &>(c3));
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      const int k = 16 * KC + kk;
      if (k >= n) return y;
      const double l = lane > k ? ck[kk] : 0.0;  // masked operand keeps y off the select
      y = fma(-l, bcast(y, k), y);
    }
    return solve_lower<NP, KC + 1>(c0, c1, c2, c3, n, y);
  }
  return y;
}

template <int NP, int KC, typename VD>
__device__ __forceinline__ double solve_upper(const VD &c0, const VD &c1, const VD &c2, const VD &c3, int n,
                                              double y) {
  if constexpr (KC >= 0) {
    const int lane = lane_id();
    const VD &ck = chunk<KC>(const_cast<VD &>(c0), const_cast<VD &>(c1), const_cast<VD &>(c2), const_cast<VD &>(c3));
#pragma unroll
    for (int kk = 15; kk >= 0; kk--) {
      const int k = 16 * KC + kk;
      if (k < n) {
        const double u = lane < k ? ck[kk] : 0.0;
        y = fma(-u, bcast(y, k), y);
      }
    }
    return solve_upper<NP, KC - 1>(c0, c1, c2, c3, n, y);
  }
  return y;
}

// Solve (P L U) z = b with the factors of lu_finish; b, z: lane i holds
// element i.  y = P b (gathered with ds_bpermute), unit-lower forward
// substitution, scaling by 1 / U_kk, unit-upper back substitution.  Each step
// is one readlane of the newly final element and one FMA.
template <int NP>
__device__ __forceinline__ double lu_solve_w(const double (&a)[NP], int n, int perm, double pinv, double b) {
  typedef typename V16<double>::type VD;
  VD c0, c1, c2, c3;
  row_to_vec<NP, double>(a, c0, c1, c2, c3);
  const int lane = lane_id();
  double y = bperm(b, lane < n ? perm : lane);
  y = solve_lower<NP, 0>(c0, c1, c2, c3, n, y);
  y *= pinv;
  return solve_upper<NP, NP / 16 - 1>(c0, c1, c2, c3, n, y);
}

}  // namespace wave
}  // namespace psr
