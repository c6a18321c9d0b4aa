// The per-reactor controller of the hybrid method (Section 3) as a round
// machine, plus the linear-algebra step of each round in FP64 or in mixed
// precision (FP32 factors + FP64 iterative refinement).
//
// A round is: one residual evaluation at the current evaluation point, a
// Jacobian + factorisation when the phase starts a new linearisation, one
// (possibly refined) solve, and the controller's decision.  Every thread of
// the workgroup runs the same scalar decisions on the same block-reduced
// values, so the controller state stays replicated without extra traffic.
//
// Phases:
//   NW_BASE   Newton iterate: F, J, LU, d = -J^-1 F, convergence test, then
//             the bound-limited step (undamped, lambda_min <= 0) or the
//             damping start.
//   NW_TRIAL  trial point x + lam d of the natural criterion, solved with
//             the same factors (lambda_min > 0 only).
//   TS1, TS2  the two stages of one ROS2 step of M dx/dt = -F(x).
//
// A gas-phase reactor whose first Newton attempt fails first tries the
// continuation in the residence time (ct_down / ct_walk below); the
// pseudo-transient steps start when that fails too.
#pragma once

#include "psr_device.hpp"

namespace psr {

template <int BS>
__device__ inline void vcopy(double *dst, const double *src, int n) {
  for (int i = threadIdx.x; i < n; i += BS) dst[i] = src[i];
  __syncthreads();
}

// Weighted max norm of a Newton step: max_k |v_k| / (atol_k + rtol |x_k|).
template <int BS>
__device__ inline double newton_norm(const Ctx &c, const Opts &o, const double *x, const double *v,
                                     double *red) {
  double r = 0.0;
  for (int k = threadIdx.x; k < c.n; k += BS) {
    const double w = (k < c.N ? o.atol_Y : (k == c.N ? o.atol_T : o.atol_lnM)) + o.rtol * fabs(x[k]);
    double t = fabs(v[k]) / w;
    if (t != t) t = __builtin_inf();
    r = fmax(r, t);
  }
  return block_max<BS>(r, red);
}

// out = x + lam d, Y projected onto Y >= 0, T onto [T_min, T_max]; soot
// ln M unbounded.
template <int BS>
__device__ inline void step_clamped(const Ctx &c, const Opts &o, const double *x, double lam,
                                    const double *d, double *out) {
  for (int i = threadIdx.x; i < c.n; i += BS) {
    double v = x[i] + lam * d[i];
    if (i < c.N) v = v > 0.0 ? v : 0.0;
    else if (i == c.N) v = v < o.T_min ? o.T_min : (v > o.T_max ? o.T_max : v);
    out[i] = v;
  }
  __syncthreads();
}

template <int BS>
__device__ inline int all_finite(const double *v, int n, double *red) {
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += BS) bad |= !isfinite(v[i]);
  return !block_or<BS>(bad, red);
}

template <int BS>
__device__ inline int matrix_finite(const double *A, int n, int lda, double *red) {
  int bad = 0;
  int e = threadIdx.x;
  for (; e + 3 * BS < n * n; e += 4 * BS) {  // four loads in flight
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int ee = e + u * BS;
      v[u] = A[(ee / n) * lda + (ee % n)];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) bad |= !isfinite(v[u]);
  }
  for (; e < n * n; e += BS) bad |= !isfinite(A[(e / n) * lda + (e % n)]);
  return !block_or<BS>(bad, red);
}

// ---------------------------------------------------------- linear algebra

// Power-of-two scales of A64 (exact): rs[i] puts row i's largest magnitude
// in [1/2, 1), then cs[j] does the same for column j of the row-scaled
// matrix.  The Jacobians of stiff mechanisms have rows whose magnitudes
// differ by tens of orders (gross reaction fluxes against the flow terms);
// every factorisation of the solve works on diag(rs) A diag(cs).
template <int BS>
__device__ void equilibration_scales(const Ctx &c, const double *A64, double *rs, double *cs) {
  const int n = c.n, lda = c.L.lda;
  // eight running maxima per thread keep eight loads in flight (a maximum is
  // exact, so the order does not change the result)
  for (int i = threadIdx.x; i < n; i += BS) {
    const double *row = A64 + (int64_t)i * lda;
    double m[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int j = 0;
    for (; j + 7 < n; j += 8)
#pragma unroll
      for (int u = 0; u < 8; u++) m[u] = fmax(m[u], fabs(row[j + u]));
    for (; j < n; j++) m[0] = fmax(m[0], fabs(row[j]));
    const double mx = fmax(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])), fmax(fmax(m[4], m[5]), fmax(m[6], m[7])));
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    rs[i] = ldexp(1.0, -e);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += BS) {
    double m[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 7 < n; i += 8)
#pragma unroll
      for (int u = 0; u < 8; u++) m[u] = fmax(m[u], fabs(A64[(int64_t)(i + u) * lda + j] * rs[i + u]));
    for (; i < n; i++) m[0] = fmax(m[0], fabs(A64[(int64_t)i * lda + j] * rs[i]));
    const double mx = fmax(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])), fmax(fmax(m[4], m[5]), fmax(m[6], m[7])));
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    cs[j] = ldexp(1.0, -e);
  }
  __syncthreads();
}

// Mixed precision: equilibrate A64 (scales above), round to float into A32
// and factor there; A64 stays unscaled for the FP64 refinement.  Returns the
// float LU's status.
template <int BS, bool BIG>
__device__ int factor_mixed(const Ctx &c, const double *A64, float *A32, int *piv, double *rs,
                            double *cs, double *red) {
  const int n = c.n, lda = c.L.lda;
  equilibration_scales<BS>(c, A64, rs, cs);
  // four elements per pass, their loads issued together
  int e = threadIdx.x;
  for (; e + 3 * BS < n * n; e += 4 * BS) {
    int64_t off[4];
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int ee = e + u * BS, i = ee / n, j = ee % n;
      off[u] = (int64_t)i * lda + j;
      v[u] = (float)(A64[off[u]] * rs[i] * cs[j]);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) A32[off[u]] = v[u];
  }
  for (; e < n * n; e += BS) {
    const int i = e / n, j = e % n;
    A32[(int64_t)i * lda + j] = (float)(A64[(int64_t)i * lda + j] * rs[i] * cs[j]);
  }
  __syncthreads();
  // large matrices: blocked matrix-core LU; its panel borrows the reaction
  // scratch in LDS (not in use between the Jacobian and the next residual)
  if (BIG && BS == 256 && n > 64 && n <= 256 && 12 * c.L.I * 2 >= 17 * n)
    return lu_factor_mfma32<256>(A32, n, lda, piv, red, reinterpret_cast<float *>(c.p(c.L.kf)));
  return lu_factor<BS, float>(A32, n, lda, piv, red);
}

// FP64 factorisation of the round's matrix, equilibrated in place (scales
// into rs, cs).  Large matrices (kept in HBM) use the blocked LU, whose
// panel borrows the reaction scratch in LDS (not in use between the
// Jacobian and the next residual).
template <int BS, bool BIG>
__device__ inline int factor64(const Ctx &c, double *A64, int *piv, double *red) {
  const int n = c.n, lda = c.L.lda;
  double *rs = c.p(c.L.rs), *cs = c.p(c.L.cs);
  equilibration_scales<BS>(c, A64, rs, cs);
  // four elements per pass, their loads issued together
  int e = threadIdx.x;
  for (; e + 3 * BS < n * n; e += 4 * BS) {
    int64_t off[4];
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int ee = e + u * BS, i = ee / n, j = ee % n;
      off[u] = (int64_t)i * lda + j;
      v[u] = A64[off[u]] * (rs[i] * cs[j]);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) A64[off[u]] = v[u];
  }
  for (; e < n * n; e += BS) {
    const int i = e / n, j = e % n;
    A64[(int64_t)i * lda + j] *= rs[i] * cs[j];
  }
  __syncthreads();
  if (BIG && BS == 256 && n > 64 && n <= 256 && 12 * c.L.I >= 17 * n)
    return lu_factor_blocked64<256>(A64, n, lda, piv, red, c.p(c.L.kf));
  return lu_factor<BS, double>(A64, n, lda, piv, red);
}

// z = A^-1 b with the float factors of the equilibrated matrix.
template <int BS>
__device__ inline void solve_scaled32(const Ctx &c, const float *A32, const int *piv, const double *rs,
                                      const double *cs, const double *b, double *z) {
  const int n = c.n;
  for (int i = threadIdx.x; i < n; i += BS) z[i] = rs[i] * b[i];
  __syncthreads();
  lu_solve<BS, float>(A32, n, c.L.lda, piv, z);
  for (int i = threadIdx.x; i < n; i += BS) z[i] *= cs[i];
  __syncthreads();
}

// Solve A z = b for the current round's matrix.  FP64: z = LU64 \ b.
// Mixed: float solve + FP64 iterative refinement against the unfactored
// FP64 matrix (r = b - A z in FP64); refinement stops when the correction
// is below tol of |z| in max norm; if the correction shrinks by less
// than half, or max_refine sweeps do not reach that, the call returns true
// (s.fb64 set): the caller refactors the matrix in FP64 for the rest of this
// linearisation and solves again.
template <int BS, bool MIXED, bool BIG>
__device__ bool solve_round(const Ctx &c, const Opts &o, RState &s, const double *b, double *z, double tol) {
  const int n = c.n, lda = c.L.lda;
  double *red = c.p(c.L.red);
  double *A64 = c.A64();
  int *piv = c.piv();
  if (!MIXED || s.fb64) {
    const double *rs = c.p(c.L.rs), *cs = c.p(c.L.cs);
    for (int i = threadIdx.x; i < n; i += BS) z[i] = rs[i] * b[i];
    __syncthreads();
    if (!s.sing) lu_solve<BS, double>(A64, n, lda, piv, z);
    for (int i = threadIdx.x; i < n; i += BS) z[i] *= cs[i];
    __syncthreads();
    return false;
  }
  const float *A32 = c.A32();
  const double *rs = c.p(c.L.rs), *cs = c.p(c.L.cs);
  double *r = c.p(c.L.rr), *bb = c.p(c.L.rb);
  vcopy<BS>(bb, b, n);
  solve_scaled32<BS>(c, A32, piv, rs, cs, bb, z);
  double prev = __builtin_inf();
  bool ok = false;
  for (int it = 0; it < o.max_refine; it++) {
    for (int i = threadIdx.x; i < n; i += BS) {
      double acc = bb[i];
      const double *row = A64 + (int64_t)i * lda;
      for (int j = 0; j < n; j++) acc -= row[j] * z[j];
      r[i] = acc;
    }
    __syncthreads();
    solve_scaled32<BS>(c, A32, piv, rs, cs, r, r);
    double dn = 0.0, zn = 0.0;
    for (int i = threadIdx.x; i < n; i += BS) {
      z[i] += r[i];
      dn = fmax(dn, fabs(r[i]));
      zn = fmax(zn, fabs(z[i]));
    }
    dn = block_max<BS>(dn, red);
    zn = block_max<BS>(zn, red);
    if (dn <= tol * zn) { ok = true; break; }
    if (!(dn <= 0.5 * prev)) break;
    prev = dn;
  }
  if (ok) return false;
  // FP64 fallback for this matrix
  s.fb64 = 1;
  s.n_fb64++;
  note_fallback(s);
  return true;
}

// ---------------------------------------------------------------- rounds

template <int BS>
__device__ inline void finish(RState &s, int status) {
  s.status = status;
  s.phase = PH_DONE;
}

// Start one ROS2 step from x (budget: two linear solves).
template <int BS>
__device__ inline void start_ts(const Ctx &c, const Opts &o, RState &s) {
  if (s.n_lin + 2 > o.max_lin) { finish<BS>(s, RS_MAXITER); return; }
  s.phase = PH_TS1;
  vcopy<BS>(c.p(c.L.xev), c.p(c.L.x), c.n);
}

// Start a steady Newton attempt from x at residence time tau_c (the
// residual and Jacobian of its rounds use tau_c).
template <int BS>
__device__ inline void start_attempt_at(const Ctx &c, const Opts &o, RState &s, double tau_c) {
  s.n_att++;
  s.nw_it = 0;
  s.tau_c = tau_c;
  vcopy<BS>(c.p(c.L.xnw), c.p(c.L.x), c.n);
  if (s.n_lin >= o.max_lin) { finish<BS>(s, RS_MAXITER); return; }
  s.phase = PH_NW_BASE;
  vcopy<BS>(c.p(c.L.xev), c.p(c.L.xnw), c.n);
}

template <int BS>
__device__ inline void start_attempt(const Ctx &c, const Opts &o, RState &s) {
  start_attempt_at<BS>(c, o, s, c.tau);
}

// Continuation in the residence time (gas-phase reactors whose first Newton
// attempt failed).  Down search: Newton from the initial guess (held in x)
// at tau / r^k, k = 1, 2, ... while tau / r^k >= ct_tau_min; once one
// converges, the walk raises tau from that root (x) by steps of at most a
// factor r, halving the step in ln tau after a failed attempt, until the
// reactor's own tau is reached or the step falls below ct_min_step.
template <int BS>
__device__ inline void ct_down(const Ctx &c, const Opts &o, RState &s) {
  s.ct_k++;
  const double ln = log(c.tau) - s.ct_k * log(o.ct_ratio);
  if (ln >= log(o.ct_tau_min)) {
    s.ct_ln = ln;
    start_attempt_at<BS>(c, o, s, exp(ln));
  } else {
    s.ct = CT_OFF;
    start_ts<BS>(c, o, s);
  }
}

template <int BS>
__device__ inline void ct_walk(const Ctx &c, const Opts &o, RState &s) {
  const double lt = log(c.tau);
  const bool last = s.ct_lc + s.ct_step >= lt;
  s.ct_ln = last ? lt : s.ct_lc + s.ct_step;
  start_attempt_at<BS>(c, o, s, last ? c.tau : exp(s.ct_ln));
}

// A Newton attempt has failed: the next continuation attempt, else ROS2
// pseudo-transient steps from x.
template <int BS>
__device__ inline void nw_failed(const Ctx &c, const Opts &o, RState &s) {
  if (s.ct == CT_FIRST) {
    s.ct = (o.ct_ratio > 1.0 && c.n == c.N + (c.energy ? 1 : 0)) ? CT_DOWN : CT_OFF;
    s.ct_k = 0;
  }
  if (s.ct == CT_DOWN) { ct_down<BS>(c, o, s); return; }
  if (s.ct == CT_WALK) {
    s.ct_step *= 0.5;
    if (s.ct_step >= o.ct_min_step) { ct_walk<BS>(c, o, s); return; }
    s.ct = CT_OFF;
  }
  start_ts<BS>(c, o, s);
}

// A Newton attempt has converged at tau_c, its root written to x: done at
// the reactor's own tau, else the next step of the continuation walk.
template <int BS>
__device__ inline void nw_converged(const Ctx &c, const Opts &o, RState &s, double *red) {
  if (s.ct == CT_DOWN || (s.ct == CT_WALK && s.tau_c != c.tau)) {
    const double lr = log(o.ct_ratio);
    s.ct_step = (s.ct == CT_DOWN) ? lr : (2.0 * s.ct_step < lr ? 2.0 * s.ct_step : lr);
    s.ct = CT_WALK;
    s.ct_lc = s.ct_ln;
    ct_walk<BS>(c, o, s);
    return;
  }
  finish<BS>(s, all_finite<BS>(c.p(c.L.x), c.n, red) ? RS_CONVERGED : RS_NONFINITE);
}

// Next damped trial point, or the attempt has failed.
template <int BS>
__device__ inline void try_trial(const Ctx &c, const Opts &o, RState &s) {
  if (s.lam >= o.lambda_min) {
    if (s.n_lin >= o.max_lin) { finish<BS>(s, RS_MAXITER); return; }
    step_clamped<BS>(c, o, c.p(c.L.xnw), s.lam, c.p(c.L.d), c.p(c.L.xev));
    s.phase = PH_NW_TRIAL;
  } else {
    nw_failed<BS>(c, o, s);
  }
}

// The Newton iterate xnw has moved: next iteration, or the attempt ends.
template <int BS>
__device__ inline void next_newton(const Ctx &c, const Opts &o, RState &s) {
  s.nw_it++;
  if (s.nw_it >= o.nw_max_it) { nw_failed<BS>(c, o, s); return; }
  if (s.n_lin >= o.max_lin) { finish<BS>(s, RS_MAXITER); return; }
  s.phase = PH_NW_BASE;
  vcopy<BS>(c.p(c.L.xev), c.p(c.L.xnw), c.n);
}

// A rejected ROS2 step: shrink h, or end (SINGULAR when the rejection was
// caused by a matrix without a nonzero pivot, else TS_FAILED).
template <int BS>
__device__ inline void reject_ts(const Ctx &c, const Opts &o, RState &s, bool bad, double err) {
  double fac = bad ? 0.25 : 0.9 / sqrt(err);
  s.h *= (fac < 0.2 ? 0.2 : fac);
  if (s.h < o.h_min) finish<BS>(s, s.sing ? RS_SINGULAR : RS_TS_FAILED);
  else start_ts<BS>(c, o, s);
}

// One round of the controller.
template <int BS, bool MIXED, bool BIG>
__device__ void round_step(Ctx &c, const Opts &o, RState &s) {
  const Layout &L = c.L;
  const int n = c.n, N = c.N, lda = L.lda;
  double *red = c.p(L.red);
  double *x = c.p(L.x), *xnw = c.p(L.xnw), *xev = c.p(L.xev), *d = c.p(L.d), *t = c.p(L.t);
  double *M = c.p(L.M), *G = c.p(L.G), *A64 = c.A64();
  int *piv = c.piv();
  const int ph = s.phase;
  const bool lin = (ph == PH_NW_BASE || ph == PH_TS1);
  const bool nw = (ph == PH_NW_BASE || ph == PH_NW_TRIAL);
  bool want64 = false;  // an FP64 factorisation of A64 is due

  // a Newton attempt of the continuation evaluates at its own residence time
  const double tau = c.tau;
  if (nw) c.tau = s.tau_c;
  const double sres = residual<BS>(c, xev, G, ph == PH_NW_BASE);
  if (lin) {
    jacobian<BS>(c, xev, A64, lda);
    if (ph == PH_TS1) {
      mass_diag<BS>(c, xev, M);
      for (int i = threadIdx.x; i < n; i += BS) A64[(int64_t)i * lda + i] += M[i] / (kGamma * s.h);
      __syncthreads();
    }
    s.n_jac++;
    if (MIXED && !s.fb64) s.stick_len = 0;  // the last linearisation went through in float
    s.fb64 = 0;
    s.fin = all_finite<BS>(G, n, red) && matrix_finite<BS>(A64, n, lda, red);
    s.sing = 0;
    if (s.fin) {
      if (MIXED && n > o.mixed_max_n) {  // above the float size limit: FP64 only
        s.fb64 = 1;
        want64 = true;
      } else if (MIXED && s.stick > 0) {  // recent fallback: FP64 directly
        s.stick--;
        s.fb64 = 1;
        s.n_fb64++;
        want64 = true;
      } else if (MIXED) {
        const int info = factor_mixed<BS, BIG>(c, A64, c.A32(), piv,
                                          c.p(L.rs), c.p(L.cs), red);
        if (info != 0) {
          s.fb64 = 1;
          s.n_fb64++;
          note_fallback(s);
          want64 = true;
        }
      } else {
        want64 = true;
      }
    }
  }
  c.tau = tau;
  // Every FP64 factorisation of the round (the linearisation's, and the
  // refactorisation after a float solve whose refinement stalls) goes
  // through the one call site at the top of this loop: one inlined copy of
  // the blocked LU keeps the kernel's register and scratch use down.
  bool skip = false, first = true;
  double *out = (ph == PH_NW_BASE || ph == PH_TS1) ? d : t;
  double tol = o.refine_tol;
  for (;;) {
    if (want64) {
      s.sing = factor64<BS, BIG>(c, A64, piv, red) != 0;
      want64 = false;
    }
    if (first) {
      first = false;
      skip = lin && (!s.fin || s.sing);
      if (skip) break;
      // right-hand side of this round, formed in place of the residual
      for (int i = threadIdx.x; i < n; i += BS) {
        double v;
        if (ph == PH_TS1) v = -G[i] / (kGamma * s.h);
        else if (ph == PH_TS2) v = (-G[i] - 2.0 * M[i] * d[i]) / (kGamma * s.h);
        else v = -G[i];
        G[i] = v;
      }
      __syncthreads();
    }
    if (solve_round<BS, MIXED, BIG>(c, o, s, G, out, tol)) {
      want64 = true;  // refactor in FP64, then solve again
      continue;
    }
    // a Newton step that would end the solve must rest on a tightly refined solve
    if (MIXED && ph == PH_NW_BASE && !s.sing && !s.fb64 && tol > kFinalRefine && sres <= o.ftol &&
        all_finite<BS>(out, n, red) && newton_norm<BS>(c, o, xnw, out, red) <= 1.0) {
      tol = kFinalRefine;
      continue;
    }
    break;
  }
  if (!skip) {
    if (MIXED && s.sing) {  // an FP64 refactorisation found the matrix singular
      if (ph == PH_NW_BASE) { nw_failed<BS>(c, o, s); return; }
      if (ph == PH_TS1) { s.n_lin += 2; reject_ts<BS>(c, o, s, true, 0.0); return; }
      for (int i = threadIdx.x; i < n; i += BS) out[i] = __builtin_nan("");
      __syncthreads();
    }
  }

  switch (ph) {
    case PH_NW_BASE: {
      if (skip) { nw_failed<BS>(c, o, s); return; }
      s.n_lin++;
      if (!all_finite<BS>(d, n, red)) { nw_failed<BS>(c, o, s); return; }
      const double nd = newton_norm<BS>(c, o, xnw, d, red);
      s.nd = nd;
      if (nd <= 1.0 && sres <= o.ftol) {
        s.sres = sres;
        step_clamped<BS>(c, o, xnw, 1.0, d, x);
        nw_converged<BS>(c, o, s, red);
        return;
      }
      // step length limited by the bounds: T inside [T_min, T_max], every
      // |d ln M_r| at most lnM_step
      double lam = 1.0;
      if (c.energy) {
        const double T = xnw[N], dT = d[N];
        if (dT > 0.0 && T + dT > o.T_max) lam = (o.T_max - T) / dT;
        if (dT < 0.0 && T + dT < o.T_min) lam = (T - o.T_min) / (-dT);
      }
      for (int r = N + 1; r < n; r++)  // same scalar decision on every thread
        if (fabs(d[r]) * lam > o.lnM_step) lam = o.lnM_step / fabs(d[r]);
      s.lam = lam;
      if (!(o.lambda_min > 0.0)) {  // undamped: take the bound-limited step
        step_clamped<BS>(c, o, xnw, lam, d, xnw);
        next_newton<BS>(c, o, s);
        return;
      }
      try_trial<BS>(c, o, s);
      return;
    }
    case PH_NW_TRIAL: {
      s.n_lin++;
      const double ndt = newton_norm<BS>(c, o, xnw, t, red);
      if (ndt < s.nd) {
        vcopy<BS>(xnw, xev, n);
        next_newton<BS>(c, o, s);
      } else {
        s.lam *= 0.5;
        try_trial<BS>(c, o, s);
      }
      return;
    }
    case PH_TS1: {
      if (skip) { s.n_lin += 2; reject_ts<BS>(c, o, s, true, 0.0); return; }
      s.n_lin++;
      for (int i = threadIdx.x; i < n; i += BS) {
        double v = x[i] + s.h * d[i];
        if (i == N) v = v < o.T_min ? o.T_min : (v > o.T_max ? o.T_max : v);
        xev[i] = v;
      }
      __syncthreads();
      s.phase = PH_TS2;
      return;
    }
    case PH_TS2: {
      s.n_lin++;
      const double h = s.h;
      double e2 = 0.0;
      int bad = 0;
      for (int i = threadIdx.x; i < n; i += BS) {
        const double xn = x[i] + 1.5 * h * d[i] + 0.5 * h * t[i];
        const double ax = fmax(fabs(x[i]), fabs(xn));
        // ln M_r: its change is a relative change of M_r already
        const double w = i > N ? o.ts_atol_lnM + o.ts_rtol
                               : (i < N ? o.ts_atol_Y : o.ts_atol_T) + o.ts_rtol * ax;
        const double e = 0.5 * h * (d[i] + t[i]) / w;
        e2 += e * e;
        bad |= !isfinite(xn);
        if (i < N) bad |= xn < -o.ts_neg_tol;
        else if (i == N) bad |= (xn < o.T_min || xn > o.T_max);
        xev[i] = xn;
      }
      const double err = sqrt(block_sum<BS>(e2, red) / n);
      const bool isbad = block_or<BS>(bad, red) || !isfinite(err);
      if (!isbad && err <= 1.0) {
        for (int i = threadIdx.x; i < n; i += BS) {
          const double v = xev[i];
          x[i] = (i < N && !(v > 0.0)) ? 0.0 : v;
        }
        __syncthreads();
        double fac = 0.9 / sqrt(err > 1e-10 ? err : 1e-10);
        s.h = h * (fac > 5.0 ? 5.0 : (fac < 0.2 ? 0.2 : fac));
        if (s.h > o.h_max * c.tau) s.h = o.h_max * c.tau;
        s.accepted++;
        s.n_ts++;
        if (s.accepted % o.nw_every == 0 && s.h >= o.nw_h_ratio * c.tau) start_attempt<BS>(c, o, s);
        else start_ts<BS>(c, o, s);
      } else {
        reject_ts<BS>(c, o, s, isbad, err);
      }
      return;
    }
    default:
      return;
  }
}

// Initial controller state for x0 (Y projected onto Y >= 0).
template <int BS>
__device__ inline void init_state(const Ctx &c, const Opts &o, RState &s) {
  s.phase = PH_NW_BASE;
  s.status = RS_RUNNING;
  s.n_lin = s.n_jac = s.n_ts = s.n_att = s.nw_it = s.accepted = 0;
  s.fb64 = s.n_fb64 = s.sing = s.stick = s.stick_len = 0;
  s.fin = 1;
  s.nd = s.lam = s.sres = 0.0;
  s.h = o.h0 * c.tau;
  s.ct = CT_FIRST;
  s.ct_k = 0;
  s.tau_c = c.tau;
  s.ct_lc = s.ct_ln = s.ct_step = 0.0;
  double *x = c.p(c.L.x);
  // inputs outside the domain of Eqs. 1-3: reported at once, x left as given
  const double *Yin = c.p(c.L.Yin);
  int bad = 0;
  for (int i = threadIdx.x; i < c.n; i += BS) bad |= !isfinite(x[i]) || (i < c.N && !isfinite(Yin[i]));
  bad = block_or<BS>(bad, c.p(c.L.red));
  if (bad || !(c.P > 0.0 && c.P < __builtin_inf()) || !(c.tau > 0.0 && c.tau < __builtin_inf()) ||
      !(c.Tin > 0.0 && c.Tin < __builtin_inf())) {
    finish<BS>(s, RS_NONFINITE);
    return;
  }
  for (int i = threadIdx.x; i < c.N; i += BS) x[i] = x[i] > 0.0 ? x[i] : 0.0;
  __syncthreads();
  start_attempt<BS>(c, o, s);
}

}  // namespace psr
