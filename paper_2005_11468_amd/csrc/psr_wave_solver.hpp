// The hybrid controller (Section 3) on the wavefront-per-reactor engine.
//
// Same round machine as psr_solver.hpp (same phases, same decisions, same
// linear-solve accounting), with every vector held one element per lane and
// the LU factors held in VGPRs across the rounds of one linearisation.
#pragma once

#include "psr_wave.hpp"

namespace psr {
namespace wave {

template <int NP, bool MIXED>
struct WState {
  double x, xnw, xev, d, t, M, rs, cs;  // lane vectors (lanes >= n hold 0)
  // LU factors of this linearisation in the form of lu_finish (lane k: pivot
  // row k, unit L and U, pinv = 1 / U_kk, perm = lane of pivot row k before
  // the permutation): FP64 factors, or in mixed mode the widened FP32
  // factors of the equilibrated matrix unless the linearisation fell back to
  // FP64 (s.fb64)
  double a[NP];
  int perm;
  double piv;
  RState s;
};

template <int NP>
__device__ __forceinline__ double newton_norm_w(const WCtx &c, const Opts &o, double xb, double v) {
  const int lane = lane_id();
  double r = 0.0;
  if (lane < c.n) {
    const double w = (lane < c.N ? o.atol_Y : o.atol_T) + o.rtol * fabs(xb);
    r = fabs(v) / w;
    if (r != r) r = __builtin_inf();
  }
  return wmax(r);
}

// x + lam d, Y projected onto Y >= 0, T onto [T_min, T_max].
__device__ __forceinline__ double clamp_step(const WCtx &c, const Opts &o, double x, double lam, double d) {
  const int lane = lane_id();
  if (lane >= c.n) return 0.0;
  double v = x + lam * d;
  if (lane < c.N) v = v > 0.0 ? v : 0.0;
  else v = v < o.T_min ? o.T_min : (v > o.T_max ? o.T_max : v);
  return v;
}

template <int NP, bool MIXED>
__device__ __forceinline__ void finish_w(WState<NP, MIXED> &r, int status) {
  r.s.status = status;
  r.s.phase = PH_DONE;
}

template <int NP, bool MIXED>
__device__ __forceinline__ void start_ts_w(const Opts &o, WState<NP, MIXED> &r) {
  if (r.s.n_lin + 2 > o.max_lin) { finish_w(r, RS_MAXITER); return; }
  r.s.phase = PH_TS1;
  r.xev = r.x;
}

template <int NP, bool MIXED>
__device__ __forceinline__ void start_attempt_w(const Opts &o, WState<NP, MIXED> &r, double tau_c) {
  r.s.n_att++;
  r.s.nw_it = 0;
  r.s.tau_c = tau_c;
  r.xnw = r.x;
  if (r.s.n_lin >= o.max_lin) { finish_w(r, RS_MAXITER); return; }
  r.s.phase = PH_NW_BASE;
  r.xev = r.xnw;
}

// Continuation in the residence time (see psr_solver.hpp): down search from
// the initial guess in x, then the walk back up from the last root in x.
template <int NP, bool MIXED>
__device__ __forceinline__ void ct_down_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r) {
  RState &s = r.s;
  s.ct_k++;
  const double ln = log(c.tau) - s.ct_k * log(o.ct_ratio);
  if (ln >= log(o.ct_tau_min)) {
    s.ct_ln = ln;
    start_attempt_w(o, r, exp(ln));
  } else {
    s.ct = CT_OFF;
    start_ts_w(o, r);
  }
}

template <int NP, bool MIXED>
__device__ __forceinline__ void ct_walk_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r) {
  RState &s = r.s;
  const double lt = log(c.tau);
  const bool last = s.ct_lc + s.ct_step >= lt;
  s.ct_ln = last ? lt : s.ct_lc + s.ct_step;
  start_attempt_w(o, r, last ? c.tau : exp(s.ct_ln));
}

template <int NP, bool MIXED>
__device__ __forceinline__ void nw_failed_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r) {
  RState &s = r.s;
  if (s.ct == CT_FIRST) {
    s.ct = (o.ct_ratio > 1.0 && c.n == c.N + (c.energy ? 1 : 0)) ? CT_DOWN : CT_OFF;
    s.ct_k = 0;
  }
  if (s.ct == CT_DOWN) { ct_down_w(c, o, r); return; }
  if (s.ct == CT_WALK) {
    s.ct_step *= 0.5;
    if (s.ct_step >= o.ct_min_step) { ct_walk_w(c, o, r); return; }
    s.ct = CT_OFF;
  }
  start_ts_w(o, r);
}

template <int NP, bool MIXED>
__device__ __forceinline__ void nw_converged_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r) {
  RState &s = r.s;
  if (s.ct == CT_DOWN || (s.ct == CT_WALK && s.tau_c != c.tau)) {
    const double lr = log(o.ct_ratio);
    s.ct_step = (s.ct == CT_DOWN) ? lr : (2.0 * s.ct_step < lr ? 2.0 * s.ct_step : lr);
    s.ct = CT_WALK;
    s.ct_lc = s.ct_ln;
    ct_walk_w(c, o, r);
    return;
  }
  finish_w(r, wany(lane_id() < c.n && !isfinite(r.x)) ? RS_NONFINITE : RS_CONVERGED);
}

template <int NP, bool MIXED>
__device__ __forceinline__ void try_trial_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r) {
  if (r.s.lam >= o.lambda_min) {
    if (r.s.n_lin >= o.max_lin) { finish_w(r, RS_MAXITER); return; }
    r.xev = clamp_step(c, o, r.xnw, r.s.lam, r.d);
    r.s.phase = PH_NW_TRIAL;
  } else {
    nw_failed_w(c, o, r);
  }
}

// The Newton iterate xnw has moved: next iteration, or the attempt ends.
template <int NP, bool MIXED>
__device__ __forceinline__ void next_newton_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r) {
  r.s.nw_it++;
  if (r.s.nw_it >= o.nw_max_it) { nw_failed_w(c, o, r); return; }
  if (r.s.n_lin >= o.max_lin) { finish_w(r, RS_MAXITER); return; }
  r.s.phase = PH_NW_BASE;
  r.xev = r.xnw;
}

template <int NP, bool MIXED>
__device__ __forceinline__ void reject_ts_w(const Opts &o, WState<NP, MIXED> &r, bool bad, double err) {
  const double fac = bad ? 0.25 : 0.9 / sqrt(err);
  r.s.h *= (fac < 0.2 ? 0.2 : fac);
  if (r.s.h < o.h_min) finish_w(r, r.s.sing ? RS_SINGULAR : RS_TS_FAILED);
  else start_ts_w(o, r);
}

// Power-of-two scales of the LDS rows (exact): r.rs puts lane i's row
// maximum in [1/2, 1), then r.cs (and A.cs[j]) does the same for column j of
// the row-scaled matrix.  The Jacobians of stiff mechanisms have rows whose
// magnitudes differ by tens of orders; every factorisation of the solve
// works on diag(rs) A diag(cs).
template <int NP, bool MIXED>
__device__ __forceinline__ void equilibrate_w(const WCtx &c, const WArea<NP> &A, WState<NP, MIXED> &r) {
  const int lane = lane_id(), n = c.n;
  const bool in = lane < n;
  const double *row = A.J + (in ? lane : 0) * A.ldj;
  double mx = 0.0;
  if (in) {
#pragma unroll 8
    for (int j = 0; j < n; j++) mx = fmax(mx, fabs(row[j]));
  }
  int e = 0;
  if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
  r.rs = in ? ldexp(1.0, -e) : 1.0;
  A.zs[lane] = r.rs;
  wsync();
  double cm = 0.0;
  if (in) {
#pragma unroll 8
    for (int i = 0; i < n; i++) cm = fmax(cm, fabs(A.J[i * A.ldj + lane]) * A.zs[i]);
  }
  e = 0;
  if (cm > 0.0 && isfinite(cm)) frexp(cm, &e);
  r.cs = in ? ldexp(1.0, -e) : 1.0;
  A.cs[lane] = r.cs;
  wsync();
}

// Factor the FP64 matrix held in the LDS rows (FP64 mode or mixed
// fallback), equilibrated as it is loaded into registers.
template <int NP, bool MIXED>
__device__ __forceinline__ int factor64(const WCtx &c, const WArea<NP> &A, WState<NP, MIXED> &r) {
  equilibrate_w<NP, MIXED>(c, A, r);
  const int lane = lane_id(), n = c.n;
  const bool in = lane < n;
  const double *row = A.J + (in ? lane : 0) * A.ldj;
#pragma unroll
  for (int j = 0; j < NP; j++) r.a[j] = (in && j < n) ? row[j] * r.rs * A.cs[j] : 0.0;
  wsync();
  int pos;
  double pk;
  const int info = lu_regs<NP, double>(r.a, n, pos, r.perm, pk);
  lu_finish<NP, double>(r.a, r.a, n, r.perm, pk, r.piv);
  return info;
}

// Mixed precision: equilibrate the LDS rows, round to float in registers,
// factor there.
template <int NP, bool MIXED>
__device__ __forceinline__ int factor32(const WCtx &c, const WArea<NP> &A, WState<NP, MIXED> &r) {
  equilibrate_w<NP, MIXED>(c, A, r);
  const int lane = lane_id(), n = c.n;
  const bool in = lane < n;
  const double *row = A.J + (in ? lane : 0) * A.ldj;
  float f[NP];
#pragma unroll
  for (int j = 0; j < NP; j++) {
    float v = 0.0f;
    if (j < n && in) v = (float)(row[j] * r.rs * A.cs[j]);
    f[j] = v;
  }
  wsync();
  float pf = 1.0f;
  int pos;
  const int info = lu_regs<NP, float>(f, n, pos, r.perm, pf);
  lu_finish<NP, float>(f, r.a, n, r.perm, pf, r.piv);
  return info;
}

// Solve with this round's factors.  Mixed: FP32 solve of the equilibrated
// system plus FP64 iterative refinement against the FP64 matrix in LDS; if a
// sweep does not halve the correction, or max_refine sweeps do not bring it
// below tol |z|, the matrix is refactored in FP64 for the rest of this
// linearisation.
template <int NP, bool MIXED>
__device__ __forceinline__ double solve_w(const WCtx &c, const WArea<NP> &A, const Opts &o, WState<NP, MIXED> &r,
                          double b, double tol) {
  const int lane = lane_id(), n = c.n;
  const bool in = lane < n;
  const double *row = A.J + (in ? lane : 0) * A.ldj;
  // One call site of the (unrolled) substitution: sweep 0 solves for z, the
  // refinement sweeps for corrections, and after an FP64 fallback the sweep
  // solves with the FP64 factors (of the same equilibrated matrix).
  bool fp64 = !MIXED || r.s.fb64;
  double z = 0.0, acc = b, prev = __builtin_inf();
  for (int it = 0;; it++) {
    const double rhs = r.rs * (in ? (fp64 ? b : acc) : 0.0);
    const double sol = lu_solve_w<NP>(r.a, n, r.perm, r.piv, rhs);
    if (fp64) return sol * r.cs;
    const double dz = sol * r.cs;
    z = (it == 0) ? dz : z + dz;
    bool fallback = false;
    if (it > 0) {
      const double dn = wmax(in ? fabs(dz) : 0.0), zn = wmax(in ? fabs(z) : 0.0);
      if (dn <= tol * zn) return z;
      fallback = !(dn <= 0.5 * prev) || it >= o.max_refine;
      prev = dn;
    } else if (o.max_refine <= 0) {
      fallback = true;
    }
    if (fallback) {
      r.s.fb64 = 1;
      r.s.n_fb64++;
      note_fallback(r.s);
      r.s.sing = factor64<NP, MIXED>(c, A, r) != 0;
      if (r.s.sing) return __builtin_nan("");
      fp64 = true;
      continue;
    }
    // FP64 residual of the refined solution against the FP64 matrix in LDS
    A.zs[lane] = in ? z : 0.0;
    wsync();
    acc = b;
    if (in) {
#pragma unroll 8
      for (int j = 0; j < n; j++) acc -= row[j] * A.zs[j];
    }
    wsync();
  }
}

// One round of the controller (see psr_solver.hpp for the phase semantics).
template <int NP, bool MIXED>
__device__ __forceinline__ void w_round(const WCtx &c, const WArea<NP> &A, const Opts &o, WState<NP, MIXED> &r) {
  RState &s = r.s;
  const int lane = lane_id(), n = c.n, N = c.N;
  const bool in = lane < n;
  const int ph = s.phase;
  const bool lin = (ph == PH_NW_BASE || ph == PH_TS1);
  Eval ev;
  double G = 0.0;
  // a Newton attempt of the continuation evaluates at its own residence time
  WCtx ce = c;
  if (ph == PH_NW_BASE || ph == PH_NW_TRIAL) ce.tau = s.tau_c;
  const double sres = w_residual<NP>(ce, A, r.xev, G, ev, ph == PH_NW_BASE);
  if (!in) G = 0.0;
  if (lin) {
    w_jacobian<NP>(ce, A, r.xev, ev);
    if (ph == PH_TS1) {
      const double cp = wsum(lane < N ? r.xev * kR * ev.cpR / c.t.W[lane] : 0.0);
      double M = 0.0;
      if (lane < N) M = ev.rho * kV;
      else if (lane == N && c.energy) M = ev.rho * kV * cp;
      r.M = M;
      if (in) A.J[lane * A.ldj + lane] += M / (kGamma * s.h);
      wsync();
    }
    s.n_jac++;
    if (MIXED && !s.fb64) s.stick_len = 0;  // the last linearisation went through in float
    s.fb64 = 0;
    bool bad = false;
    if (in) {
      bad = !isfinite(G);
      const double *row = A.J + lane * A.ldj;
#pragma unroll 8
      for (int j = 0; j < n; j++) bad |= !isfinite(row[j]);
    }
    s.fin = !wany(bad);
    s.sing = 0;
    if (s.fin) {
      if (MIXED) {
        // after a recent fallback the float attempt is skipped (one call
        // site of each factorisation either way)
        const bool big = c.n > o.mixed_max_n;  // above the float size limit: FP64 only
        const bool direct = !big && s.stick > 0;
        if (direct) s.stick--;
        if (big || direct || factor32<NP, MIXED>(c, A, r) != 0) {
          s.fb64 = 1;
          if (!big) s.n_fb64++;
          if (!big && !direct) note_fallback(s);
          s.sing = factor64<NP, MIXED>(c, A, r) != 0;
        }
      } else {
        s.sing = factor64<NP, MIXED>(c, A, r) != 0;
      }
    }
  }
  const bool skip = lin && (!s.fin || s.sing);
  if (!skip) {
    double rhs;
    if (ph == PH_TS1) rhs = -G / (kGamma * s.h);
    else if (ph == PH_TS2) rhs = (-G - 2.0 * r.M * r.d) / (kGamma * s.h);
    else rhs = -G;
    if (!in) rhs = 0.0;
    double out, tol = o.refine_tol;
    for (;;) {
      out = solve_w<NP, MIXED>(c, A, o, r, rhs, tol);
      if (!in) out = 0.0;
      // a Newton step that would end the solve must rest on a tightly refined solve
      if (MIXED && ph == PH_NW_BASE && !s.sing && !s.fb64 && tol > kFinalRefine && sres <= o.ftol &&
          !wany(in && !isfinite(out)) && newton_norm_w<NP>(c, o, r.xnw, out) <= 1.0) {
        tol = kFinalRefine;
        continue;
      }
      break;
    }
    if (MIXED && s.sing) {
      if (ph == PH_NW_BASE) { nw_failed_w(c, o, r); return; }
      if (ph == PH_TS1) { s.n_lin += 2; reject_ts_w(o, r, true, 0.0); return; }
      out = in ? __builtin_nan("") : 0.0;
    }
    if (ph == PH_NW_BASE || ph == PH_TS1) r.d = out;
    else r.t = out;
  }

  switch (ph) {
    case PH_NW_BASE: {
      if (skip) { nw_failed_w(c, o, r); return; }
      s.n_lin++;
      if (wany(in && !isfinite(r.d))) { nw_failed_w(c, o, r); return; }
      const double nd = newton_norm_w<NP>(c, o, r.xnw, r.d);
      s.nd = nd;
      if (nd <= 1.0 && sres <= o.ftol) {
        s.sres = sres;
        r.x = clamp_step(c, o, r.xnw, 1.0, r.d);
        nw_converged_w(c, o, r);
        return;
      }
      double lam = 1.0;
      if (c.energy) {
        const double T = bcast(r.xnw, N), dT = bcast(r.d, N);
        if (dT > 0.0 && T + dT > o.T_max) lam = (o.T_max - T) / dT;
        if (dT < 0.0 && T + dT < o.T_min) lam = (T - o.T_min) / (-dT);
      }
      s.lam = lam;
      if (!(o.lambda_min > 0.0)) {  // undamped: take the bound-limited step
        r.xnw = clamp_step(c, o, r.xnw, lam, r.d);
        next_newton_w(c, o, r);
        return;
      }
      try_trial_w(c, o, r);
      return;
    }
    case PH_NW_TRIAL: {
      s.n_lin++;
      const double ndt = newton_norm_w<NP>(c, o, r.xnw, r.t);
      if (ndt < s.nd) {
        r.xnw = r.xev;
        next_newton_w(c, o, r);
      } else {
        s.lam *= 0.5;
        try_trial_w(c, o, r);
      }
      return;
    }
    case PH_TS1: {
      if (skip) { s.n_lin += 2; reject_ts_w(o, r, true, 0.0); return; }
      s.n_lin++;
      double v = in ? r.x + s.h * r.d : 0.0;
      if (lane == N && c.energy) v = v < o.T_min ? o.T_min : (v > o.T_max ? o.T_max : v);
      r.xev = v;
      s.phase = PH_TS2;
      return;
    }
    case PH_TS2: {
      s.n_lin++;
      const double h = s.h;
      double e2 = 0.0, xn = 0.0;
      bool badl = false;
      if (in) {
        xn = r.x + 1.5 * h * r.d + 0.5 * h * r.t;
        const double ax = fmax(fabs(r.x), fabs(xn));
        const double w = (lane < N ? o.ts_atol_Y : o.ts_atol_T) + o.ts_rtol * ax;
        const double e = 0.5 * h * (r.d + r.t) / w;
        e2 = e * e;
        badl = !isfinite(xn);
        if (lane < N) badl |= xn < -o.ts_neg_tol;
        else badl |= (xn < o.T_min || xn > o.T_max);
      }
      const double err = sqrt(wsum(e2) / n);
      const bool bad = wany(badl) || !isfinite(err);
      if (!bad && err <= 1.0) {
        r.x = (in && lane < N && !(xn > 0.0)) ? 0.0 : xn;
        const double fac = 0.9 / sqrt(err > 1e-10 ? err : 1e-10);
        s.h = h * (fac > 5.0 ? 5.0 : (fac < 0.2 ? 0.2 : fac));
        if (s.h > o.h_max * c.tau) s.h = o.h_max * c.tau;
        s.accepted++;
        s.n_ts++;
        if (s.accepted % o.nw_every == 0 && s.h >= o.nw_h_ratio * c.tau) start_attempt_w(o, r, c.tau);
        else start_ts_w(o, r);
      } else {
        reject_ts_w(o, r, bad, err);
      }
      return;
    }
    default:
      return;
  }
}

// Reactor inputs for lane-distributed use; x0 in lane order.
template <int NP, bool MIXED>
__device__ __forceinline__ void init_w(const WCtx &c, const Opts &o, WState<NP, MIXED> &r, double x0) {
  const int lane = lane_id();
  r.x = (lane < c.n) ? ((lane < c.N && !(x0 > 0.0)) ? 0.0 : x0) : 0.0;
  r.xnw = r.xev = r.d = r.t = r.M = 0.0;
  r.rs = r.cs = 1.0;
  r.perm = 0;
  r.piv = 1.0;
  RState &s = r.s;
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
  // inputs outside the domain of Eqs. 1-3: reported at once, x left as given
  const bool bad_lane = (lane < c.N && !isfinite(c.Yin)) || (lane < c.n && !isfinite(x0));
  if (!(c.P > 0.0 && c.P < __builtin_inf()) || !(c.tau > 0.0 && c.tau < __builtin_inf()) ||
      !(c.Tin > 0.0 && c.Tin < __builtin_inf()) || wany(bad_lane)) {
    r.x = lane < c.n ? x0 : 0.0;
    finish_w(r, RS_NONFINITE);
    return;
  }
  start_attempt_w(o, r, c.tau);
}

__device__ __forceinline__ double inlet_enthalpy(const Tables &t, int i, double Tin) {
  const double *a = t.nasa + 7 * i;
  const double hRT = a[0] + Tin * (a[1] * 0.5 + Tin * (a[2] * kThird + Tin * (a[3] * 0.25 + Tin * a[4] * 0.2)))
                     + a[5] / Tin;
  return kR * Tin * hRT;
}

}  // namespace wave
}  // namespace psr
