// Device building blocks of the batched PSR solver (gfx950).
//
// One workgroup of BS threads owns one reactor at a time.  Every per-reactor
// array lives in LDS (or, for the host-driven scheduler, in global memory
// reached through the same flat pointers).  Threads stride over species,
// reactions, matrix rows and elements; block reductions broadcast scalars.
//
// Paper: Section 2 (Eqs. 1-3, the PSR balances), Section 3 (Eqs. 4-9, the
// rates and the hybrid Newton / time-integration method).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psr {

constexpr double kR = 8.314462618;  // J/(mol K)
constexpr double kPatm = 101325.0;  // Pa, standard state of Eq. 8
constexpr double kV = 1.0;          // cm^3
constexpr double kGamma = 1.7071067811865475244;  // ROS2: 1 + 1/sqrt(2)

// Mechanism tables in device memory (by value in kernel arguments).
struct MechDev {
  int N, I, nnz;
  const double *W;     // [N] g/mol
  const double *nasa;  // [N*7]
  const double *lnA, *beta, *EoR;  // [I]; E/R in K
  const int *dnu;                  // [I] sum of net coefficients
  const int *r_idx, *r_nu, *p_idx, *p_nu;  // [I*3], -1 pads
  const int *sp_ptr, *sp_rx, *sp_nu;       // species -> (reaction, net nu), CSR
  const int *packed;  // wavefront engine: w0[I], w1[I], w2[I], CSR entries[nnz]; null if unusable
  // soot moments (MOMIC); soot == 0: gas phase only
  int soot, sP, sG;                 // precursor and growth species
  double Cmin, D;                   // carbon atoms per nucleus and per growth step
  double An, bn, EnR, As, bs, EsR;  // k_n, k_s = A T^b exp(-(E/R)/T), E/R in K
  double KW;                        // chi pi d^2 (d: diameter of one carbon atom's soot volume)
  double KF0;                       // free-molecular coagulation kernel / sqrt(T)
  const double *frac;               // [kSootOrders][6] d ln mu_p / d ln M_j, then [4] L_l(1/2)
};

// Unknowns per reactor: Y[, T][, ln M_0..ln M_5].
__host__ __device__ inline int n_unknowns(const MechDev &m, int energy) {
  return m.N + (energy ? 1 + (m.soot ? 6 : 0) : 0);
}

// Fractional orders of the soot closure: index 3 j + t is order j + 1/6
// (t = 0), j - 1/6 (t = 1), j - 1/2 (t = 2) for j = 0..7 (coagulation); 24 + l
// is order l + 2/3 for l = 0..4 (surface growth).
constexpr int kSootOrders = 29;
constexpr int kSootPairs = 11;  // (x, y) of the coagulation interpolants f_{x,y}
constexpr int kSootScratch = 7 * (kSootOrders + 4 * kSootPairs + kSootPairs) + 12 * 6 + 16;

struct Opts {
  int precision, scheduler;
  double rtol, atol_Y, atol_T, ftol, lambda_min, T_min, T_max;
  double ts_rtol, ts_atol_Y, ts_atol_T, ts_neg_tol, h0, h_max, h_min, nw_h_ratio;
  int nw_max_it, nw_every, max_lin, max_refine;
  double refine_tol;
  double atol_lnM, ts_atol_lnM;  // soot moments
  double lnM_step;               // largest |d ln M_r| of one Newton step
  double ct_ratio, ct_tau_min, ct_min_step;  // continuation in tau
  int mixed_max_n;  // mixed precision: largest system factored in FP32 first
};

// Mixed precision: refinement target of the solve whose Newton step ends a
// reactor's solve (the loose opts.refine_tol only steers the iteration).
constexpr double kFinalRefine = 1e-10;
// Mixed precision: after a matrix needed the FP64 fallback, the following
// linearisations of the reactor are factored in FP64 directly (the float
// attempt on a matrix that ill-conditioned would be wasted): kStickFP64 of
// them after a first fallback, twice as many after each further fallback of
// a float attempt (up to kStickMax), back to none once a float attempt goes
// through without one.  The FP32 factors only help while cond(A) stays well
// below 1 / eps_float; the Jacobians of the 100- to 201-unknown mechanisms
// often do not.
constexpr int kStickFP64 = 4;
constexpr int kStickMax = 256;

enum Phase : int { PH_NW_BASE = 0, PH_NW_TRIAL = 1, PH_TS1 = 2, PH_TS2 = 3, PH_DONE = 4 };
// Continuation in tau: first attempt at the reactor's tau, down search,
// walk back up, or not (any more) in use.
enum CtMode : int { CT_OFF = 0, CT_FIRST = 1, CT_DOWN = 2, CT_WALK = 3 };
enum RStatus : int { RS_CONVERGED = 0, RS_MAXITER = 1, RS_TS_FAILED = 2, RS_NONFINITE = 3, RS_SINGULAR = 4,
                     RS_RUNNING = 9 };

// Per-reactor controller state of the hybrid method.
struct RState {
  int phase, status, n_lin, n_jac, n_ts, n_att, nw_it, accepted;
  int fb64;      // mixed mode: current matrix refactored in FP64
  int n_fb64;    // mixed mode: FP64 fallbacks so far
  int stick;     // mixed mode: linearisations still to factor in FP64 directly
  int stick_len; // mixed mode: length of the current run of FP64 linearisations
  int sing, fin; // matrix flags of this round
  int ct, ct_k;  // continuation mode, down-search rung
  double nd, lam, h, sres;
  double tau_c;                // residence time of the current Newton attempt
  double ct_lc, ct_ln, ct_step; // continuation: ln tau of the last root, of
                                // the current attempt, step in ln tau
};

// Mixed precision: a float attempt fell back to FP64 (see kStickFP64).
__host__ __device__ inline void note_fallback(RState &s) {
  s.stick_len = s.stick_len > 0 ? (2 * s.stick_len < kStickMax ? 2 * s.stick_len : kStickMax) : kStickFP64;
  s.stick = s.stick_len;
}

// LDS / workspace layout of one reactor, in doubles (8-byte units).  The
// first `persist` doubles (inlet data, vectors, matrices, pivots) carry the
// controller's state from one round to the next; the rest is scratch that
// every residual evaluation rebuilds.
struct Layout {
  int N, I, n, lda;
  int Yin, Hin;                                       // inlet data
  int x, xnw, xev, d, t, M, G, rs, cs, rb, rr;        // vectors
  int A64, A32, piv, persist;                         // matrices
  int split, mat_total;  // split: matrices in a separate (HBM) area of mat_total doubles
  int C, hRT, sR, cpR, wdot, gross, Erow, dwdT;       // species scratch
  int kf, kr, Rf, Rr, sumC, dqdT, dqdC;               // reaction scratch
  int soot;                                           // soot-closure scratch (n = N + 7 only)
  int red, total;
  // lean: a residual evaluation alone (x, G and the residual's scratch; the
  // solver vectors, the Jacobian scratch and the matrices get no space)
  __host__ __device__ void make(int N_, int I_, int n_, bool mixed, int BS, bool split_ = false, bool lean = false) {
    N = N_; I = I_; n = n_;
    lda = (n % 2 == 0) ? n + 1 : n;
    split = (split_ || lean) ? 1 : 0;
    const int nv = lean ? 0 : n;  // size of a solver vector
    int o = 0;
    Yin = o; o += N; Hin = o; o += N;
    x = o; o += n; G = o; o += n;
    xnw = o; o += nv; xev = o; o += nv; d = o; o += nv; t = o; o += nv;
    M = o; o += nv; rs = o; o += nv; cs = o; o += nv; rb = o; o += nv; rr = o; o += nv;
    int m = split ? 0 : o;  // matrices follow the vectors, or start their own area
    A64 = m; m += n * lda;
    A32 = m; m += mixed ? (n * lda + 1) / 2 : 0;
    piv = m; m += (n + 1) / 2;
    if (split) mat_total = m;
    else { mat_total = 0; o = m; }
    persist = o;
    C = o; o += N; hRT = o; o += N; sR = o; o += N; cpR = o; o += N; wdot = o; o += N;
    gross = o; o += N; Erow = o; o += lean ? 0 : N; dwdT = o; o += lean ? 0 : N;
    kf = o; o += I; kr = o; o += I; Rf = o; o += I; Rr = o; o += I;
    sumC = o; o += lean ? 0 : I; dqdT = o; o += lean ? 0 : I; dqdC = o; o += lean ? 0 : 6 * I;
    soot = o; o += (n == N + 7) ? kSootScratch : 0;
    red = o; o += BS + 8;
    total = o;
  }
};

// ---------------------------------------------------------------- reductions

// Data movement inside a wavefront: DPP within rows of 16 lanes (CTRL 0xB1
// swaps neighbouring lanes, 0x4E lanes two apart, 0x124 / 0x128 rotate the
// row by 4 / 8), readlane of one lane for all.
template <int CTRL>
__device__ __forceinline__ double dpp_row_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the wavefront (every lane active) in a fixed order, the same bits
// in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_row_mov<0xB1>(v);
  v += dpp_row_mov<0x4E>(v);
  v += dpp_row_mov<0x124>(v);
  v += dpp_row_mov<0x128>(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}
// Maximum over the wavefront (every lane active), the same bits in every lane.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_row_mov<0xB1>(v));
  v = fmax(v, dpp_row_mov<0x4E>(v));
  v = fmax(v, dpp_row_mov<0x124>(v));
  v = fmax(v, dpp_row_mov<0x128>(v));
  return fmax(fmax(lane_read(v, 0), lane_read(v, 16)), fmax(lane_read(v, 32), lane_read(v, 48)));
}

template <int BS>
__device__ inline double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < BS / 64; w++) s += red[w];
  return s;
}

// Max with NaN treated as +inf.
template <int BS>
__device__ inline double block_max(double v, double *red) {
  if (v != v) v = __builtin_inf();
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < BS / 64; w++) s = fmax(s, red[w]);
  return s;
}

template <int BS>
__device__ inline int block_or(int v, double *red) {
  double s = block_max<BS>(v ? 1.0 : 0.0, red);
  return s > 0.0;
}

// ------------------------------------------------------- reactor evaluation

// Per-reactor context: pointers into the reactor's LDS (or workspace) area.
struct Ctx {
  MechDev m;
  int N, n, energy;
  double P, tau, Tin;
  double *base;  // start of the reactor's area (doubles)
  double *mat;   // split layout: start of the reactor's matrix area (HBM), else null
  Layout L;
  // scalars of the last residual evaluation
  double T, S, rho, mdot;
  __device__ double *p(int off) const { return base + off; }
  __device__ double *A64() const { return (mat ? mat : base) + L.A64; }
  __device__ float *A32() const { return reinterpret_cast<float *>((mat ? mat : base) + L.A32); }
  __device__ int *piv() const { return reinterpret_cast<int *>((mat ? mat : base) + L.piv); }
};

// Set up a reactor: inlet composition and molar inlet enthalpies H_i(T_in).
template <int BS>
__device__ void load_inlet(Ctx &c, const double *Yin_soa, int64_t B, int64_t b) {
  double *Yin = c.p(c.L.Yin), *Hin = c.p(c.L.Hin);
  const double Tin = c.Tin;
  for (int i = threadIdx.x; i < c.N; i += BS) {
    Yin[i] = Yin_soa[(int64_t)i * B + b];
    const double *a = c.m.nasa + 7 * i;
    double hRT = a[0] + Tin * (a[1] / 2.0 + Tin * (a[2] / 3.0 + Tin * (a[3] / 4.0 + Tin * a[4] / 5.0)))
                 + a[5] / Tin;
    Hin[i] = kR * Tin * hRT;
  }
}

// ------------------------------------------------------------- soot (MOMIC)
//
// Frenklach's method of moments with interpolative closure for the soot
// particles of a sooting reactor (the paper couples it to the gas phase,
// Sections 1-2 and 6).  The closure needs reduced moments mu_p = M_p/M_0 of
// fractional order p; ln mu_p is a fixed linear combination of the ln M_j
// (Lagrange interpolation over the integer orders, coefficients tabulated
// at mechanism creation), so every quantity below carries its value and its
// six derivatives with respect to ln M_0..ln M_5 (index 0 and 1..6 of a
// 7-double record).  Stages run on a few threads each, separated by block
// barriers; all threads of the workgroup must call soot_eval.

namespace soot {
constexpr double kNA = 6.02214076e23;  // 1/mol
constexpr int MU = 0, FL = MU + 7 * kSootOrders, FX = FL + 7 * 4 * kSootPairs;
constexpr int OUT = FX + 7 * kSootPairs;  // per r: R, W, G, dsrc/dlnM[6], dsrc/dCP, dsrc/dCG, dsrc/dT|C
constexpr int W1 = OUT + 12 * 6;           // W_1, dW_1/dlnM[6], dW_1/dCG, dW_1/dT|C
constexpr int SK = W1 + 9;                 // s_P = 2 I, ds_P/dCP, ds_P/dT|C
static_assert(SK + 3 <= kSootScratch, "soot scratch");
// coagulation pairs (x, y): (0,0), then x + y = 2, 3, 4, 5 with x = 1..r-1
__device__ constexpr int kPairX[kSootPairs] = {0, 1, 1, 2, 1, 2, 3, 1, 2, 3, 4};
__device__ constexpr int kPairY[kSootPairs] = {0, 1, 2, 1, 3, 2, 1, 4, 3, 2, 1};
__device__ constexpr int kPairBase[6] = {0, 0, 1, 2, 4, 7};  // first pair with x + y = r
__device__ constexpr double kBinom[6][6] = {{1, 0, 0, 0, 0, 0}, {1, 1, 0, 0, 0, 0}, {1, 2, 1, 0, 0, 0},
                                            {1, 3, 3, 1, 0, 0}, {1, 4, 6, 4, 1, 0}, {1, 5, 10, 10, 5, 1}};
}  // namespace soot

// Sources of the six moments and the gas sinks at (T, CP, CG, ln M), with
// derivatives (results in the OUT / W1 / SK records of `w`):
//   R_r = N_A k_n CP^2 Cmin^r                      nucleation
//   W_r = k_s CG chi pi d^2 M_0 sum_{l<r} C(r,l) D^(r-l) mu_{l+2/3}   growth
//   G_0 = -K_f M_0^2 f_00 / 2, G_1 = 0, G_r = K_f M_0^2 sum_k C(r,k) f_{k,r-k} / 2
// Growth and coagulation are off while M_0 < 1 per cm^3.
template <int BS>
__device__ void soot_eval(const MechDev &m, double T, double CP, double CG, const double *lnM, double *w) {
  const int t = threadIdx.x;
  if (t < kSootOrders) {  // fractional moments
    const double *cf = m.frac + 6 * t;
    double l = 0.0;
    for (int j = 0; j < 6; j++) l += cf[j] * lnM[j];
    const double mu = exp(l);
    double *o = w + soot::MU + 7 * t;
    o[0] = mu;
    for (int j = 0; j < 6; j++) o[1 + j] = mu * cf[j];
  }
  __syncthreads();
  if (t < 4 * kSootPairs) {  // coagulation grid functions f_l of pair q
    const int q = t >> 2, l = t & 3, x = soot::kPairX[q], y = soot::kPairY[q];
    double f[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k <= l; k++) {
      const double b = soot::kBinom[l][k];
      const double *a0 = w + soot::MU + 7 * (3 * (k + x) + 0), *a1 = w + soot::MU + 7 * (3 * (k + x) + 1);
      const double *a2 = w + soot::MU + 7 * (3 * (k + x) + 2);
      const int jb = l - k + y;
      const double *b0 = w + soot::MU + 7 * (3 * jb + 0), *b1 = w + soot::MU + 7 * (3 * jb + 1);
      const double *b2 = w + soot::MU + 7 * (3 * jb + 2);
      // mu_{j+1/6} mu_{j'-1/2} + 2 mu_{j-1/6} mu_{j'-1/6} + mu_{j-1/2} mu_{j'+1/6}
      f[0] += b * (a0[0] * b2[0] + 2.0 * a1[0] * b1[0] + a2[0] * b0[0]);
      for (int j = 1; j < 7; j++)
        f[j] += b * (a0[j] * b2[0] + a0[0] * b2[j] + 2.0 * (a1[j] * b1[0] + a1[0] * b1[j]) +
                     a2[j] * b0[0] + a2[0] * b0[j]);
    }
    double *o = w + soot::FL + 7 * t;
    for (int j = 0; j < 7; j++) o[j] = f[j];
  }
  __syncthreads();
  if (t < kSootPairs) {  // f_{x,y}: log-Lagrange value at l = 1/2
    const double *L4 = m.frac + 6 * kSootOrders;
    const double *fl = w + soot::FL + 7 * 4 * t;
    double lf = 0.0, d[6] = {0, 0, 0, 0, 0, 0};
    for (int l = 0; l < 4; l++) {
      lf += L4[l] * log(fl[7 * l]);
      const double inv = L4[l] / fl[7 * l];
      for (int j = 0; j < 6; j++) d[j] += inv * fl[7 * l + 1 + j];
    }
    const double v = exp(lf);
    double *o = w + soot::FX + 7 * t;
    o[0] = v;
    for (int j = 0; j < 6; j++) o[1 + j] = v * d[j];
  }
  __syncthreads();
  if (t < 7) {
    const double lnT = log(T), invT = 1.0 / T;
    const double kn = m.An * exp(m.bn * lnT - m.EnR * invT), dlkn = (m.bn + m.EnR * invT) * invT;
    const double ks = m.As * exp(m.bs * lnT - m.EsR * invT), dlks = (m.bs + m.EsR * invT) * invT;
    if (t == 6) {
      w[soot::SK] = 2.0 * kn * CP * CP;
      w[soot::SK + 1] = 4.0 * kn * CP;
      w[soot::SK + 2] = 2.0 * kn * CP * CP * dlkn;
    } else {
      const int r = t;
      double cr = 1.0;
      for (int i = 0; i < r; i++) cr *= m.Cmin;
      const double Rv = soot::kNA * kn * CP * CP * cr;
      const double M0 = exp(lnM[0]);
      const bool on = M0 >= 1.0;
      // growth
      double S = 0.0, dS[6] = {0, 0, 0, 0, 0, 0};
      for (int l = 0; l < r; l++) {
        double dp = 1.0;
        for (int i = 0; i < r - l; i++) dp *= m.D;
        const double cw = soot::kBinom[r][l] * dp;
        const double *mu = w + soot::MU + 7 * (24 + l);
        S += cw * mu[0];
        for (int j = 0; j < 6; j++) dS[j] += cw * mu[1 + j];
      }
      const double kw = on ? m.KW * ks * M0 : 0.0;
      const double Wv = kw * CG * S;
      double dW[6];
      for (int j = 0; j < 6; j++) dW[j] = kw * CG * (dS[j] + (j == 0 ? S : 0.0));
      // coagulation
      double Gs = 0.0, dG[6] = {0, 0, 0, 0, 0, 0};
      if (r == 0) {
        const double *f = w + soot::FX;
        Gs = -0.5 * f[0];
        for (int j = 0; j < 6; j++) dG[j] = -0.5 * f[1 + j];
      } else if (r >= 2) {
        for (int k = 1; k < r; k++) {
          const double *f = w + soot::FX + 7 * (soot::kPairBase[r] + k - 1);
          const double cb = 0.5 * soot::kBinom[r][k];
          Gs += cb * f[0];
          for (int j = 0; j < 6; j++) dG[j] += cb * f[1 + j];
        }
      }
      const double kg = on ? m.KF0 * sqrt(T) * M0 * M0 : 0.0;
      const double Gv = kg * Gs;
      double *o = w + soot::OUT + 12 * r;
      o[0] = Rv; o[1] = Wv; o[2] = Gv;
      for (int j = 0; j < 6; j++) o[3 + j] = dW[j] + kg * (dG[j] + (j == 0 ? 2.0 * Gs : 0.0));
      o[9] = 2.0 * soot::kNA * kn * CP * cr;
      o[10] = kw * S;
      o[11] = Rv * dlkn + Wv * dlks + 0.5 * Gv * invT;
      if (r == 1) {
        double *q = w + soot::W1;
        q[0] = Wv;
        for (int j = 0; j < 6; j++) q[1 + j] = dW[j];
        q[7] = kw * S;
        q[8] = Wv * dlks;
      }
    }
  }
  __syncthreads();
}

// Steady residual F(x) (Eq. 2 and Eq. 3 times -rho V) with the rates of
// Eqs. 4-9.  Leaves C, thermo, k_f, k_r, forward/reverse terms and wdot in
// the context for the Jacobian.  Returns the scaled residual if asked for
// (each equation's residual over the sum of the magnitudes of its terms).
template <int BS>
__device__ double residual(Ctx &c, const double *x, double *F, bool want_sres) {
  const MechDev &m = c.m;
  const int N = c.N, I = m.I, tid = threadIdx.x;
  double *red = c.p(c.L.red);
  double *C = c.p(c.L.C), *hRT = c.p(c.L.hRT), *sR = c.p(c.L.sR), *cpR = c.p(c.L.cpR);
  double *wdot = c.p(c.L.wdot), *gross = c.p(c.L.gross);
  double *kf = c.p(c.L.kf), *kr = c.p(c.L.kr), *Rf = c.p(c.L.Rf), *Rr = c.p(c.L.Rr);
  const double *Yin = c.p(c.L.Yin), *Hin = c.p(c.L.Hin);

  const double T = c.energy ? x[N] : c.Tin;
  double s = 0.0;
  for (int i = tid; i < N; i += BS) s += x[i] / m.W[i];
  const double S = block_sum<BS>(s, red);
  const double rho = c.P * 1.0e-6 / (kR * T * S);
  const double mdot = rho * kV / c.tau;
  c.T = T; c.S = S; c.rho = rho; c.mdot = mdot;
  const double lnT = log(T), invT = 1.0 / T;
  const double lnc = log(kPatm * 1.0e-6 / (kR * T));

  // species: concentrations and NASA-7 thermo (the S, H of Eq. 9)
  for (int i = tid; i < N; i += BS) {
    C[i] = rho * x[i] / m.W[i];
    const double *a = m.nasa + 7 * i;
    cpR[i] = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
    hRT[i] = a[0] + T * (a[1] / 2.0 + T * (a[2] / 3.0 + T * (a[3] / 4.0 + T * a[4] / 5.0))) + a[5] * invT;
    sR[i] = a[0] * lnT + T * (a[1] + T * (a[2] / 2.0 + T * (a[3] / 3.0 + T * a[4] / 4.0))) + a[6];
  }
  __syncthreads();
  // reactions: Eq. 6 (k_f), Eqs. 8-9 (K_c), Eq. 7 (k_r), Eq. 5 (q)
  for (int k = tid; k < I; k += BS) {
    double g = 0.0, fwd = 1.0, rev = 1.0;
    for (int sl = 0; sl < 3; sl++) {
      const int ir = m.r_idx[3 * k + sl];
      if (ir >= 0) {
        const int nu = m.r_nu[3 * k + sl];
        g -= nu * (sR[ir] - hRT[ir]);
        for (int e = 0; e < nu; e++) fwd *= C[ir];
      }
      const int ip = m.p_idx[3 * k + sl];
      if (ip >= 0) {
        const int nu = m.p_nu[3 * k + sl];
        g += nu * (sR[ip] - hRT[ip]);
        for (int e = 0; e < nu; e++) rev *= C[ip];
      }
    }
    const double lnkf = m.lnA[k] + m.beta[k] * lnT - m.EoR[k] * invT;
    const double lnKc = g + m.dnu[k] * lnc;
    const double kfk = exp(lnkf), krk = exp(lnkf - lnKc);
    kf[k] = kfk; kr[k] = krk;
    fwd *= kfk; rev *= krk;
    Rf[k] = fwd; Rr[k] = rev;
  }
  __syncthreads();
  // soot moments: sources and the precursor / growth-species sinks
  const bool soot = m.soot && c.energy;
  double *sw = soot ? c.p(c.L.soot) : nullptr;
  if (soot) soot_eval<BS>(m, T, C[m.sP], C[m.sG], x + N + 1, sw);
  // molar consumption rate of species i by soot formation
  auto sink = [&](int i) -> double {
    if (!soot) return 0.0;
    if (i == m.sP) return sw[soot::SK];
    if (i == m.sG) return sw[soot::W1] / (m.D * soot::kNA);
    return 0.0;
  };
  // species: Eq. 4 and the species residual
  double inflow = 0.0, chem = 0.0, sr = 0.0;
  for (int i = tid; i < N; i += BS) {
    double w = 0.0, gr = 0.0;
    for (int p = m.sp_ptr[i]; p < m.sp_ptr[i + 1]; p++) {
      const int k = m.sp_rx[p];
      w += m.sp_nu[p] * (Rf[k] - Rr[k]);
      if (want_sres) gr += fabs((double)m.sp_nu[p]) * (fabs(Rf[k]) + fabs(Rr[k]));
    }
    wdot[i] = w;
    gross[i] = gr;
    const double sk = sink(i);
    const double Fi = mdot * (x[i] - Yin[i]) - kV * m.W[i] * (w - sk);
    F[i] = Fi;
    if (c.energy == 1) {
      const double H = kR * T * hRT[i];
      inflow += Yin[i] * (H - Hin[i]) / m.W[i];
      chem += H * (w - sk);
    }
    if (want_sres) {
      const double den = mdot * (fabs(x[i]) + fabs(Yin[i])) + kV * m.W[i] * (gr + sk);
      double r = (den > 0.0) ? fabs(Fi) / den : 0.0;
      if (!(den >= 0.0) || Fi != Fi) r = __builtin_inf();
      sr = fmax(sr, r);
    }
  }
  double FT = 0.0;
  if (c.energy == 2) {  // prescribed reactor temperature: T pinned to T_in
    FT = kV * (T - c.Tin) / c.tau;
    if (tid == 0) F[N] = FT;
    if (want_sres && tid == 0) {
      double r = fabs(FT) / (kV * (fabs(T) + fabs(c.Tin)) / c.tau);
      if (FT != FT) r = __builtin_inf();
      sr = fmax(sr, r);
    }
  } else if (c.energy) {
    const double in_s = block_sum<BS>(inflow, red);
    const double ch_s = block_sum<BS>(chem, red);
    FT = mdot * in_s + kV * ch_s;
    if (tid == 0) F[N] = FT;
  }
  double sres = 0.0;
  if (want_sres) {
    if (c.energy == 1) {
      double den = 0.0;
      for (int i = tid; i < N; i += BS) {
        const double H = kR * T * hRT[i];
        den += mdot * fabs(Yin[i] * (H - Hin[i]) / m.W[i]) + kV * fabs(H) * (gross[i] + sink(i));
      }
      den = block_sum<BS>(den, red);
      if (tid == 0) {
        double r = (den > 0.0) ? fabs(FT) / den : 0.0;
        if (FT != FT) r = __builtin_inf();
        sr = fmax(sr, r);
      }
    }
  }
  // moment rows: V (M_r/tau - R_r - W_r - G_r), relative to outflow plus
  // the magnitudes of the sources
  if (soot && tid < 6) {
    const double *o = sw + soot::OUT + 12 * tid;
    const double Mr = exp(x[N + 1 + tid]);
    const double Fr = kV * (Mr / c.tau - (o[0] + o[1] + o[2]));
    F[N + 1 + tid] = Fr;
    if (want_sres) {
      const double den = kV * (Mr / c.tau + fabs(o[0]) + fabs(o[1]) + fabs(o[2]));
      double r = fabs(Fr) / den;
      if (!(r == r)) r = __builtin_inf();
      sr = fmax(sr, r);
    }
  }
  if (want_sres) sres = block_max<BS>(sr, red);
  __syncthreads();
  return sres;
}

// Mass-matrix diagonal of the transient form: rho V (species), rho V cp_mix
// (energy; V for a prescribed temperature, relaxed to T_in over tau).  Uses
// the state of the last residual() call at the same x.
template <int BS>
__device__ void mass_diag(Ctx &c, const double *x, double *M) {
  const int N = c.N, tid = threadIdx.x;
  double *red = c.p(c.L.red);
  const double *cpR = c.p(c.L.cpR);
  double cp = 0.0;
  if (c.energy)
    for (int i = tid; i < N; i += BS) cp += x[i] * kR * cpR[i] / c.m.W[i];
  const double cpmix = c.energy ? block_sum<BS>(cp, red) : 0.0;
  for (int i = tid; i < N; i += BS) M[i] = c.rho * kV;
  if (c.energy && tid == 0) M[N] = c.energy == 2 ? kV : c.rho * kV * cpmix;
  // soot: d M_r/dt = M_r d ln M_r/dt
  if (c.energy && c.m.soot && tid < 6) M[N + 1 + tid] = kV * exp(x[N + 1 + tid]);
  __syncthreads();
}

// Soot terms of the Jacobian, added to A after the gas-phase part: rows of
// the precursor, the growth species, the energy equation and the moments.
// The concentrations depend on every Y and on T through rho:
//   dC_j/dY_m = rho delta_jm / W_j - C_j/(S W_m),  dC_j/dT = -C_j/T.
// Uses the soot records of the residual() call at the same x.
template <int BS>
__device__ void soot_jacobian(Ctx &c, const double *x, double *A, int lda) {
  const MechDev &m = c.m;
  const int N = c.N, tid = threadIdx.x, P = m.sP, Gs = m.sG;
  const double *C = c.p(c.L.C), *hRT = c.p(c.L.hRT), *cpR = c.p(c.L.cpR);
  const double *w = c.p(c.L.soot);
  const double T = c.T, S = c.S, rho = c.rho, invT = 1.0 / T;
  const double gD = 1.0 / (m.D * soot::kNA);  // mol of G per carbon atom of growth
  const double HP = kR * T * hRT[P], HG = kR * T * hRT[Gs];
  const double *sk = w + soot::SK, *w1 = w + soot::W1;
  for (int mm = tid; mm < N; mm += BS) {  // species columns
    const double SW = S * m.W[mm];
    const double dCP = (mm == P ? rho / m.W[P] : 0.0) - C[P] / SW;
    const double dCG = (mm == Gs ? rho / m.W[Gs] : 0.0) - C[Gs] / SW;
    const double dsP = sk[1] * dCP, dsG = w1[7] * dCG * gD;
    A[(int64_t)P * lda + mm] += kV * m.W[P] * dsP;
    A[(int64_t)Gs * lda + mm] += kV * m.W[Gs] * dsG;
    if (c.energy == 1) A[(int64_t)N * lda + mm] -= kV * (HP * dsP + HG * dsG);
    for (int r = 0; r < 6; r++) {
      const double *o = w + soot::OUT + 12 * r;
      A[(int64_t)(N + 1 + r) * lda + mm] -= kV * (o[9] * dCP + o[10] * dCG);
    }
  }
  if (tid >= BS - 7) {  // temperature and ln M columns, one per thread
    const int col = N + (tid - (BS - 7));
    if (col == N) {
      const double dCP = -C[P] * invT, dCG = -C[Gs] * invT;
      const double dsP = sk[2] + sk[1] * dCP, dsG = (w1[8] + w1[7] * dCG) * gD;
      A[(int64_t)P * lda + N] += kV * m.W[P] * dsP;
      A[(int64_t)Gs * lda + N] += kV * m.W[Gs] * dsG;
      if (c.energy == 1)
        A[(int64_t)N * lda + N] -= kV * (kR * cpR[P] * sk[0] + HP * dsP + kR * cpR[Gs] * w1[0] * gD + HG * dsG);
      for (int r = 0; r < 6; r++) {
        const double *o = w + soot::OUT + 12 * r;
        A[(int64_t)(N + 1 + r) * lda + N] -= kV * (o[11] + o[9] * dCP + o[10] * dCG);
      }
    } else {
      const int j = col - N - 1;
      A[(int64_t)Gs * lda + col] += kV * m.W[Gs] * w1[1 + j] * gD;
      if (c.energy == 1) A[(int64_t)N * lda + col] -= kV * HG * w1[1 + j] * gD;
      for (int r = 0; r < 6; r++) {
        const double *o = w + soot::OUT + 12 * r;
        A[(int64_t)(N + 1 + r) * lda + col] += kV * ((r == j ? exp(x[N + 1 + r]) / c.tau : 0.0) - o[3 + j]);
      }
    }
  }
  __syncthreads();
}

// Analytic Jacobian of residual() at the same x, into A (row-major, lda).
// Chain rule through rho(Y,T), C(Y,T), k_f(T), K_c(T):
//   dC_j/dY_m = rho delta_jm / W_j - C_j/(S W_m),  dC_j/dT = -C_j/T
//   d ln k_f/dT = beta/T + E/(R T^2),  d ln K_c/dT = sum nu_i (H_i/RT)/T - dnu/T
// D_im = sum_k nu_ik dq_k/dC_m is gathered row by row (row i owned by one
// thread, so the accumulation order is fixed), then the rank-one density
// terms are applied.
template <int BS>
__device__ void jacobian(Ctx &c, const double *x, double *A, int lda) {
  const MechDev &m = c.m;
  const int N = c.N, n = c.n, I = m.I, tid = threadIdx.x;
  double *red = c.p(c.L.red);
  const double *C = c.p(c.L.C), *hRT = c.p(c.L.hRT), *cpR = c.p(c.L.cpR), *wdot = c.p(c.L.wdot);
  const double *kf = c.p(c.L.kf), *kr = c.p(c.L.kr), *Rf = c.p(c.L.Rf), *Rr = c.p(c.L.Rr);
  double *sumC = c.p(c.L.sumC), *dqdT = c.p(c.L.dqdT), *dqdC = c.p(c.L.dqdC);
  double *Erow = c.p(c.L.Erow), *dwdT = c.p(c.L.dwdT);
  const double *Yin = c.p(c.L.Yin), *Hin = c.p(c.L.Hin);
  const double T = c.T, S = c.S, rho = c.rho, mdot = c.mdot, invT = 1.0 / T;

  for (int k = tid; k < I; k += BS) {
    double sc = 0.0, sh = 0.0;
    for (int sl = 0; sl < 3; sl++) {
      const int ir = m.r_idx[3 * k + sl];
      double dr = 0.0;
      if (ir >= 0) {
        dr = kf[k] * m.r_nu[3 * k + sl];
        for (int e = 0; e < m.r_nu[3 * k + sl] - 1; e++) dr *= C[ir];
        for (int s2 = 0; s2 < 3; s2++) {
          const int j = m.r_idx[3 * k + s2];
          if (s2 != sl && j >= 0)
            for (int e = 0; e < m.r_nu[3 * k + s2]; e++) dr *= C[j];
        }
        sc += C[ir] * dr;
        sh -= m.r_nu[3 * k + sl] * hRT[ir];
      }
      dqdC[6 * k + sl] = dr;
      const int ip = m.p_idx[3 * k + sl];
      double dp = 0.0;
      if (ip >= 0) {
        dp = kr[k] * m.p_nu[3 * k + sl];
        for (int e = 0; e < m.p_nu[3 * k + sl] - 1; e++) dp *= C[ip];
        for (int s2 = 0; s2 < 3; s2++) {
          const int j = m.p_idx[3 * k + s2];
          if (s2 != sl && j >= 0)
            for (int e = 0; e < m.p_nu[3 * k + s2]; e++) dp *= C[j];
        }
        dp = -dp;
        sc += C[ip] * dp;
        sh += m.p_nu[3 * k + sl] * hRT[ip];
      }
      dqdC[6 * k + 3 + sl] = dp;
    }
    const double dlnkf = m.beta[k] * invT + m.EoR[k] * invT * invT;
    const double dlnKc = sh * invT - m.dnu[k] * invT;
    sumC[k] = sc;
    dqdT[k] = Rf[k] * dlnkf - Rr[k] * (dlnkf - dlnKc) - sc * invT;
  }
  for (int e = tid; e < n * n; e += BS) A[(e / n) * lda + (e % n)] = 0.0;
  __syncthreads();
  // Row pass by wavefronts: when the reaction scratch (k_f, k_r and the rates
  // of progress, 4 I doubles, no longer needed) holds a D row and a column
  // accumulator for each wavefront, wavefront w takes rows w, w + 4, ...:
  // it gathers D_i. with LDS atomics (lanes over the row's reactions; one
  // wavefront owns the buffer, so the order of the adds is fixed), applies
  // the density chain rule and stores row i with lanes over the columns,
  // adding H_i D_i. to its column accumulator for the energy row.
  const int nw = BS / 64;
  if (4 * I >= 2 * N * nw) {
    const int lane = tid & 63, wv = tid >> 6;
    double *buf = c.p(c.L.kf) + (size_t)wv * 2 * N;
    double *col = buf + N;
    const bool ebal = c.energy == 1;
    for (int mm = lane; mm < N; mm += 64) col[mm] = 0.0;
    for (int i = wv; i < N; i += nw) {
      for (int mm = lane; mm < N; mm += 64) buf[mm] = 0.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double E = 0.0, dT = 0.0;
      for (int p = m.sp_ptr[i] + lane; p < m.sp_ptr[i + 1]; p += 64) {
        const int k = m.sp_rx[p];
        const double nu = m.sp_nu[p];
        for (int sl = 0; sl < 3; sl++) {
          const int ir = m.r_idx[3 * k + sl];
          if (ir >= 0) atomicAdd(&buf[ir], nu * dqdC[6 * k + sl]);
          const int ip = m.p_idx[3 * k + sl];
          if (ip >= 0) atomicAdd(&buf[ip], nu * dqdC[6 * k + 3 + sl]);
        }
        E += nu * sumC[k];
        dT += nu * dqdT[k];
      }
      E = wave_sum(E);
      dT = wave_sum(dT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const double yd = x[i] - Yin[i], Wi = m.W[i], Hi = kR * T * hRT[i];
      double *row = A + (int64_t)i * lda;
      for (int mm = lane; mm < N; mm += 64) {
        const double D = buf[mm];
        if (ebal) col[mm] += Hi * D;
        const double SW = S * m.W[mm];
        double v = -mdot / SW * yd - kV * Wi * (D * rho / m.W[mm] - E / SW);
        if (mm == i) v += mdot;
        row[mm] = v;
      }
      if (lane == 0) {
        Erow[i] = E;
        dwdT[i] = dT;
        if (c.energy) row[N] = -mdot * invT * yd - kV * Wi * dT;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    if (c.energy == 2) {  // prescribed temperature: the row V (T - T_in) / tau
      if (tid == 0) A[(int64_t)N * lda + N] = kV / c.tau;
      __syncthreads();
    } else if (c.energy) {
      double qin = 0.0, dqin = 0.0, tt = 0.0, hE = 0.0;
      for (int i = tid; i < N; i += BS) {
        const double H = kR * T * hRT[i];
        qin += Yin[i] * (H - Hin[i]) / m.W[i];
        dqin += Yin[i] * kR * cpR[i] / m.W[i];
        tt += kV * (kR * cpR[i] * wdot[i] + H * dwdT[i]);
        hE += H * Erow[i];
      }
      const double Qin = block_sum<BS>(qin, red);
      const double dQin = block_sum<BS>(dqin, red);
      const double TT = block_sum<BS>(tt, red);
      const double HE = block_sum<BS>(hE, red);
      const double *col0 = c.p(c.L.kf) + N;
      for (int mm = tid; mm < N; mm += BS) {
        double v = 0.0;
        for (int w = 0; w < nw; w++) v += col0[(size_t)w * 2 * N + mm];
        const double SW = S * m.W[mm];
        A[(int64_t)N * lda + mm] = -mdot * Qin / SW + kV * (v * rho / m.W[mm] - HE / SW);
      }
      if (tid == 0) A[(int64_t)N * lda + N] = -mdot * invT * Qin + mdot * dQin + TT;
      __syncthreads();
    }
    if (c.energy && m.soot) soot_jacobian<BS>(c, x, A, lda);
    return;
  }
  // gather D (into the species rows of A), E_i = sum_j D_ij C_j, dwdot_i/dT
  for (int i = tid; i < N; i += BS) {
    double E = 0.0, dT = 0.0;
    double *row = A + (int64_t)i * lda;
    for (int p = m.sp_ptr[i]; p < m.sp_ptr[i + 1]; p++) {
      const int k = m.sp_rx[p];
      const double nu = m.sp_nu[p];
      for (int sl = 0; sl < 3; sl++) {
        const int ir = m.r_idx[3 * k + sl];
        if (ir >= 0) row[ir] += nu * dqdC[6 * k + sl];
        const int ip = m.p_idx[3 * k + sl];
        if (ip >= 0) row[ip] += nu * dqdC[6 * k + 3 + sl];
      }
      E += nu * sumC[k];
      dT += nu * dqdT[k];
    }
    Erow[i] = E;
    dwdT[i] = dT;
  }
  __syncthreads();
  if (c.energy == 2) {  // prescribed temperature: the row V (T - T_in) / tau
    if (tid == 0) A[(int64_t)N * lda + N] = kV / c.tau;
    __syncthreads();
  } else if (c.energy) {
    // energy row: dF_T/dY_m = -mdot Q_in/(S W_m) + V sum_i H_i dwdot_i/dY_m
    double qin = 0.0, dqin = 0.0, tt = 0.0, hE = 0.0;
    for (int i = tid; i < N; i += BS) {
      const double H = kR * T * hRT[i];
      qin += Yin[i] * (H - Hin[i]) / m.W[i];
      dqin += Yin[i] * kR * cpR[i] / m.W[i];
      tt += kV * (kR * cpR[i] * wdot[i] + H * dwdT[i]);
      hE += H * Erow[i];
    }
    const double Qin = block_sum<BS>(qin, red);
    const double dQin = block_sum<BS>(dqin, red);
    const double TT = block_sum<BS>(tt, red);
    const double HE = block_sum<BS>(hE, red);
    for (int mm = tid; mm < N; mm += BS) {
      double v = 0.0;
      for (int i = 0; i < N; i++) v += kR * T * hRT[i] * A[(int64_t)i * lda + mm];
      const double SW = S * m.W[mm];
      A[(int64_t)N * lda + mm] = -mdot * Qin / SW + kV * (v * rho / m.W[mm] - HE / SW);
    }
    if (tid == 0) A[(int64_t)N * lda + N] = -mdot * invT * Qin + mdot * dQin + TT;
    __syncthreads();
  }
  for (int i = tid; i < N; i += BS) {
    double *row = A + (int64_t)i * lda;
    const double yd = x[i] - Yin[i], Wi = m.W[i], Ei = Erow[i];
    for (int mm = 0; mm < N; mm++) {
      const double SW = S * m.W[mm];
      double v = -mdot / SW * yd - kV * Wi * (row[mm] * rho / m.W[mm] - Ei / SW);
      if (mm == i) v += mdot;
      row[mm] = v;
    }
    if (c.energy) row[N] = -mdot * invT * yd - kV * Wi * dwdT[i];
  }
  __syncthreads();
  if (c.energy && m.soot) soot_jacobian<BS>(c, x, A, lda);
}

// ------------------------------------------------------------- dense LU

// In-place LU with partial pivoting of an n x n row-major matrix (leading
// dimension lda) by one workgroup.  Pivot = first row index of the largest
// |a_ik| at or below the diagonal; rows are swapped whole (LAPACK getrf
// convention for piv).  Returns 0 or k+1 for a zero pivot column.
template <int BS, typename T>
__device__ int lu_factor(T *A, int n, int lda, int *piv, double *red) {
  const int tid = threadIdx.x;
  int *ipiv_s = reinterpret_cast<int *>(red + BS);
  for (int k = 0; k < n; k++) {
    if (tid < 64) {
      double best = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += 64) {
        const double v = fabs((double)A[(int64_t)i * lda + k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) { ipiv_s[0] = bi; red[BS + 2] = best; }
    }
    __syncthreads();
    const int p = ipiv_s[0];
    const double amax = red[BS + 2];
    if (tid == 0) piv[k] = p;
    if (!(amax > 0.0)) {
      __syncthreads();
      return k + 1;
    }
    if (p != k) {
      for (int j = tid; j < n; j += BS) {
        const T t = A[(int64_t)k * lda + j];
        A[(int64_t)k * lda + j] = A[(int64_t)p * lda + j];
        A[(int64_t)p * lda + j] = t;
      }
      __syncthreads();
    }
    const T pivot = A[(int64_t)k * lda + k];
    for (int i = k + 1 + tid; i < n; i += BS) A[(int64_t)i * lda + k] /= pivot;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += BS) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      A[(int64_t)i * lda + j] -= A[(int64_t)i * lda + k] * A[(int64_t)k * lda + j];
    }
    __syncthreads();
  }
  return 0;
}

// Solve (P L U) z = b in place (b in double; factors of type T).
// Blocked right-looking LU with partial pivoting of a float matrix with up
// to 256 rows (kept in HBM for the large mechanisms), panel width 16.
//   panel:    the n - k0 by 16 panel is copied to LDS (pan, row stride 17);
//             per column a block argmax (first maximum), a row interchange
//             inside the panel and a rank-one update of the panel rows below
//             (measured faster here, two workgroups per CU, than factoring
//             the panel by one wavefront without block barriers);
//   swaps:    the panel's row interchanges applied to the other columns
//             (one column per thread);
//   U12:      L11^-1 A12 by forward substitution, one column per thread, L11
//             read from the panel in LDS;
//   A22:      A22 -= L21 U12 on the matrix cores, v_mfma_f32_16x16x4f32 per
//             16 x 16 tile and K step of 4; each wavefront takes every fourth
//             tile row and sweeps its tile columns four at a time.
// Operand layouts of the 16x16x4 instruction (lane l): A(l % 16, l / 16),
// B(l / 16, l % 16), D[v](4 (l / 16) + v, l % 16).  Same factor format as
// lu_factor (unit-lower L below the diagonal, LAPACK pivots).  BS must be
// 256.  red: LDS scratch of at least 24 doubles; pan: LDS scratch of at
// least 17 n floats.  Returns 0 or k+1.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Wavefront argmax for the panel pivot search: the largest v (v >= 0, -1 for
// rows not in the search) and the first lane index attaining it, for every
// lane; then a ballot of the lanes equal to the maximum.
__device__ __forceinline__ void wave_argmax(double v, int vi, double &best, int &bi) {
  const double m = wave_max(v);
  const unsigned long long hit = __ballot(v == m);
  best = m;
  bi = __builtin_amdgcn_readlane(vi, __builtin_ctzll(hit));
}

template <int BS>
__device__ __forceinline__ int lu_factor_mfma32(float *A, int n, int lda, int *piv, double *red, float *pan) {
  static_assert(BS == 256, "one panel row per thread");
  constexpr int PS = 17;  // panel row stride (floats)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double *wval = red + 16;                        // per-wavefront best |a|
  int *widx = reinterpret_cast<int *>(red + 20);  // per-wavefront best row
  for (int k0 = 0; k0 < n; k0 += 16) {
    const int kb = n - k0 < 16 ? n - k0 : 16;
    const int rows = n - k0;
    for (int e = tid; e < rows * 16; e += BS) {
      const int t = e >> 4, j = e & 15;
      pan[t * PS + j] = j < kb ? A[(int64_t)(k0 + t) * lda + k0 + j] : 0.f;
    }
    __syncthreads();
    for (int jj = 0; jj < kb; jj++) {
      const int k = k0 + jj;
      double v = (tid < rows && tid >= jj) ? fabs((double)pan[tid * PS + jj]) : -1.0;
      int vi = tid;
      wave_argmax(v, tid, v, vi);
      if (lane == 0) { wval[wv] = v; widx[wv] = vi; }
      __syncthreads();
      double best = wval[0];
      int bi = widx[0];
      for (int w = 1; w < BS / 64; w++)
        if (wval[w] > best || (wval[w] == best && widx[w] < bi)) { best = wval[w]; bi = widx[w]; }
      if (!(best > 0.0)) {
        __syncthreads();
        return k + 1;
      }
      if (tid == 0) piv[k] = k0 + bi;
      if (bi != jj && tid < 16) {
        const float t = pan[jj * PS + tid];
        pan[jj * PS + tid] = pan[bi * PS + tid];
        pan[bi * PS + tid] = t;
      }
      __syncthreads();
      if (tid < rows && tid > jj) {
        const float l = pan[tid * PS + jj] / pan[jj * PS + jj];
        pan[tid * PS + jj] = l;
        for (int j = jj + 1; j < kb; j++) pan[tid * PS + j] -= l * pan[jj * PS + j];
      }
      __syncthreads();
    }
    for (int e = tid; e < rows * 16; e += BS) {
      const int t = e >> 4, j = e & 15;
      if (j < kb) A[(int64_t)(k0 + t) * lda + k0 + j] = pan[t * PS + j];
    }
    // the panel's interchanges on the other columns, in order (n <= BS: at
    // most one column per thread)
    {
      const int c = tid;
      if (c < n && (c < k0 || c >= k0 + kb))
        for (int jj = 0; jj < kb; jj++) {
          const int pr = piv[k0 + jj];
          if (pr != k0 + jj) {
            float *x = A + (int64_t)(k0 + jj) * lda + c, *y = A + (int64_t)pr * lda + c;
            const float t = *x;
            *x = *y;
            *y = t;
          }
        }
    }
    __syncthreads();
    const int R0 = k0 + kb, m = n - R0;
    if (m <= 0) break;
    // U12 = L11^-1 A12 (one column per thread)
    if (R0 + tid < n) {
      const int c = R0 + tid;
      float u[16];
#pragma unroll
      for (int i = 0; i < 16; i++) u[i] = i < kb ? A[(int64_t)(k0 + i) * lda + c] : 0.f;
#pragma unroll
      for (int i = 1; i < 16; i++) {
        float acc = u[i];
#pragma unroll
        for (int q = 0; q < 16; q++)
          if (q < i) acc -= (i < kb ? pan[i * PS + q] : 0.f) * u[q];
        u[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < 16; i++)
        if (i < kb) A[(int64_t)(k0 + i) * lda + c] = u[i];
    }
    __syncthreads();
    // A22 -= L21 U12 on the matrix cores, four tile columns at a time
    const int nt = (m + 15) / 16;
    const int lr = lane & 15, lk = lane >> 4;
    for (int ti = wv; ti < nt; ti += BS / 64) {
      float aq[4];
      const int arow = R0 + 16 * ti + lr;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int k = 4 * q + lk;
        aq[q] = (arow < n && k < kb) ? -A[(int64_t)arow * lda + k0 + k] : 0.f;
      }
      const int crow = R0 + 16 * ti + 4 * lk;
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
            bq[t][q] = (cin && k < kb) ? A[(int64_t)(k0 + k) * lda + col] : 0.f;
          }
#pragma unroll
          for (int v = 0; v < 4; v++) acc[t][v] = (cin && crow + v < n) ? A[(int64_t)(crow + v) * lda + col] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
          for (int q = 0; q < 4; q++) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[q], bq[t][q], acc[t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int col = R0 + 16 * (tj0 + t) + lr;
          if ((tj0 + t) < nt && col < n) {
#pragma unroll
            for (int v = 0; v < 4; v++)
              if (crow + v < n) A[(int64_t)(crow + v) * lda + col] = acc[t][v];
          }
        }
      }
    }
    __syncthreads();
  }
  return 0;
}

// Blocked right-looking FP64 LU with partial pivoting for matrices kept in
// HBM (64 < n <= BS), panel width 16.  Same panel as lu_factor_mfma32 (copied
// to LDS, block argmax with the first-maximum rule, row interchange and
// rank-one update per column), then one column per thread for the panel's
// interchanges and U12 = L11^-1 A12 (forward substitution), then the trailing
// update A22 -= L21 U12 on the FP64 matrix cores in 16 x 16 tiles.  The
// trailing matrix is read and written once per panel.  pan: LDS scratch of at
// least 17 n doubles.  Returns 0 or k+1.
template <int BS>
__device__ __forceinline__ int lu_factor_blocked64(double *A, int n, int lda, int *piv, double *red, double *pan) {
  static_assert(BS == 256, "one panel row and one column per thread");
  constexpr int PS = 17;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double *wval = red + 16;
  int *widx = reinterpret_cast<int *>(red + 20);
  for (int k0 = 0; k0 < n; k0 += 16) {
    const int kb = n - k0 < 16 ? n - k0 : 16;
    const int rows = n - k0;
    for (int e = tid; e < rows * 16; e += BS) {
      const int t = e >> 4, j = e & 15;
      pan[t * PS + j] = j < kb ? A[(int64_t)(k0 + t) * lda + k0 + j] : 0.0;
    }
    __syncthreads();
    for (int jj = 0; jj < kb; jj++) {
      const int k = k0 + jj;
      double v = (tid < rows && tid >= jj) ? fabs(pan[tid * PS + jj]) : -1.0;
      int vi = tid;
      wave_argmax(v, tid, v, vi);
      if (lane == 0) { wval[wv] = v; widx[wv] = vi; }
      __syncthreads();
      double best = wval[0];
      int bi = widx[0];
      for (int w = 1; w < BS / 64; w++)
        if (wval[w] > best || (wval[w] == best && widx[w] < bi)) { best = wval[w]; bi = widx[w]; }
      if (!(best > 0.0)) {
        __syncthreads();
        return k + 1;
      }
      if (tid == 0) piv[k] = k0 + bi;
      if (bi != jj && tid < 16) {
        const double t = pan[jj * PS + tid];
        pan[jj * PS + tid] = pan[bi * PS + tid];
        pan[bi * PS + tid] = t;
      }
      __syncthreads();
      if (tid < rows && tid > jj) {
        const double l = pan[tid * PS + jj] / pan[jj * PS + jj];
        pan[tid * PS + jj] = l;
        for (int j = jj + 1; j < kb; j++) pan[tid * PS + j] -= l * pan[jj * PS + j];
      }
      __syncthreads();
    }
    for (int e = tid; e < rows * 16; e += BS) {
      const int t = e >> 4, j = e & 15;
      if (j < kb) A[(int64_t)(k0 + t) * lda + k0 + j] = pan[t * PS + j];
    }
    const int R0 = k0 + kb;
    const int c = tid;
    if (c < n && (c < k0 || c >= R0)) {
      int pr[16];
#pragma unroll
      for (int jj = 0; jj < 16; jj++) pr[jj] = jj < kb ? piv[k0 + jj] : k0 + jj;
#pragma unroll
      for (int jj = 0; jj < 16; jj++) {
        if (jj < kb && pr[jj] != k0 + jj) {
          double *x = A + (int64_t)(k0 + jj) * lda + c, *y = A + (int64_t)pr[jj] * lda + c;
          const double t = *x;
          *x = *y;
          *y = t;
        }
      }
      if (c >= R0) {
        double u[16];
#pragma unroll
        for (int i = 0; i < 16; i++) u[i] = i < kb ? A[(int64_t)(k0 + i) * lda + c] : 0.0;
#pragma unroll
        for (int i = 1; i < 16; i++) {
          double acc = u[i];
#pragma unroll
          for (int q = 0; q < 16; q++)
            if (q < i) acc -= (i < kb ? pan[i * PS + q] : 0.0) * u[q];
          u[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < 16; i++)
          if (i < kb) A[(int64_t)(k0 + i) * lda + c] = u[i];
      }
    }
    __syncthreads();
    const int m = n - R0;
    if (m <= 0) break;
    // A22 -= L21 U12 on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A lane l
    // -> (row l mod 16, k l / 16), B -> (k l / 16, col l mod 16), D register v
    // -> (row l / 16 + 4 v, col l mod 16)); L21 from the panel in LDS, U12 and
    // A22 from the matrix.  Each wavefront takes every fourth 16-row tile row
    // and sweeps its tile columns four at a time, with all their loads in flight.
    const int nt = (m + 15) / 16;
    const int lr = lane & 15, lk = lane >> 4;
    for (int ti = wv; ti < nt; ti += BS / 64) {
      double aq[4];
      const int arow = R0 + 16 * ti + lr;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int k = 4 * q + lk;
        aq[q] = (arow < n && k < kb) ? -pan[(arow - k0) * PS + k] : 0.0;
      }
      const int crow = R0 + 16 * ti + lk;
      for (int tj0 = 0; tj0 < nt; tj0 += 4) {
        double bq[4][4];
        v4d acc[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int col = R0 + 16 * (tj0 + t) + lr;
          const bool cin = (tj0 + t) < nt && col < n;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const int k = 4 * q + lk;
            bq[t][q] = (cin && k < kb) ? A[(int64_t)(k0 + k) * lda + col] : 0.0;
          }
#pragma unroll
          for (int v = 0; v < 4; v++)
            acc[t][v] = (cin && crow + 4 * v < n) ? A[(int64_t)(crow + 4 * v) * lda + col] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
          for (int q = 0; q < 4; q++) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[q], bq[t][q], acc[t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int col = R0 + 16 * (tj0 + t) + lr;
          if ((tj0 + t) < nt && col < n) {
#pragma unroll
            for (int v = 0; v < 4; v++)
              if (crow + 4 * v < n) A[(int64_t)(crow + 4 * v) * lda + col] = acc[t][v];
          }
        }
      }
    }
    __syncthreads();
  }
  return 0;
}

template <int BS, typename T>
__device__ void lu_solve(const T *A, int n, int lda, const int *piv, double *b) {
  // Column-oriented substitution taken 16 columns at a time: the block's own
  // 16 rows by the first wavefront (column by column, the finished element
  // passed by readlane), then every other row by all threads, each applying
  // the block's columns in order.  Every element receives the same updates in
  // the same order as one column at a time would give it, with two block
  // barriers per 16 columns instead of two per column.
  const int tid = threadIdx.x;
  if (tid == 0)
    for (int k = 0; k < n; k++) {
      const double t = b[k];
      b[k] = b[piv[k]];
      b[piv[k]] = t;
    }
  __syncthreads();
  for (int k0 = 0; k0 < n - 1; k0 += 16) {  // forward, unit lower
    const int k1 = k0 + 16 < n ? k0 + 16 : n;
    if (tid < 64) {
      const int i = k0 + tid;
      const bool mine = tid < 16 && i < k1;
      double zi = mine ? b[i] : 0.0;
      double r[16];  // this lane's row of the block, loaded up front
#pragma unroll
      for (int kk = 0; kk < 16; kk++) r[kk] = (mine && k0 + kk < k1) ? (double)A[(int64_t)i * lda + k0 + kk] : 0.0;
#pragma unroll
      for (int kk = 0; kk < 15; kk++) {
        if (k0 + kk < k1 - 1) {
          const double bk = lane_read(zi, kk);
          if (mine && tid > kk) zi -= r[kk] * bk;
        }
      }
      if (mine) b[i] = zi;
    }
    __syncthreads();
    for (int i = k1 + tid; i < n; i += BS) {
      double zi = b[i];
#pragma unroll
      for (int kk = 0; kk < 16; kk++)
        if (k0 + kk < k1) zi -= (double)A[(int64_t)i * lda + k0 + kk] * b[k0 + kk];
      b[i] = zi;
    }
    __syncthreads();
  }
  for (int k1 = n; k1 > 0; k1 -= 16) {  // back, upper
    const int k0 = k1 - 16 > 0 ? k1 - 16 : 0;
    if (tid < 64) {
      const int i = k0 + tid;
      const bool mine = tid < 16 && i < k1;
      double zi = mine ? b[i] : 0.0;
      double r[16];  // this lane's row of the block, loaded up front
#pragma unroll
      for (int kk = 0; kk < 16; kk++) r[kk] = (mine && k0 + kk < k1) ? (double)A[(int64_t)i * lda + k0 + kk] : 0.0;
#pragma unroll
      for (int kk = 15; kk >= 0; kk--) {
        if (k0 + kk < k1) {
          const double bk = lane_read(zi, kk) / lane_read(r[kk], kk);
          if (tid == kk) zi = bk;
          else if (mine && tid < kk) zi -= r[kk] * bk;
        }
      }
      if (mine) b[i] = zi;
    }
    __syncthreads();
    for (int i = tid; i < k0; i += BS) {
      double zi = b[i];
#pragma unroll
      for (int kk = 15; kk >= 0; kk--)
        if (k0 + kk < k1) zi -= (double)A[(int64_t)i * lda + k0 + kk] * b[k0 + kk];
      b[i] = zi;
    }
    __syncthreads();
  }
}

}  // namespace psr
