/* Plain FP64 CPU oracle for the batched PSR steady-state solve.
 *
 * TEST INFRASTRUCTURE ONLY: the independent reference the GPU library is
 * checked against (see psr_oracle.h).  Single-threaded, no BLAS, no SIMD
 * intrinsics; every loop is written the way the equations read.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "psr_oracle.h"

#ifdef OM_TRACE
#include <stdio.h>
#define TRACE(...) fprintf(stderr, __VA_ARGS__)
#else
#define TRACE(...) ((void)0)
#endif

#define OM_R 8.314462618       /* J/(mol K), gas constant                        */
#define OM_PATM 101325.0       /* Pa, standard-state pressure of Eq. 8          */
#define OM_V 1.0               /* cm^3, reactor volume (cancels from the root)   */
#define OM_NA 6.02214076e23    /* 1/mol, Avogadro constant                       */
#define OM_KB 1.380649e-16     /* erg/K, Boltzmann constant (cgs)                */
#define OM_PI 3.14159265358979323846

/* Lagrange basis polynomial l of the nodes 0, 1, ..., m-1, at p. */
static double lagrange_basis(double p, int l, int m)
{
  double r = 1.0;
  for (int k = 0; k < m; k++)
    if (k != l) r *= (p - k) / (double)(l - k);
  return r;
}

/* Binomial coefficient C(n, k). */
static double binomial(int n, int k)
{
  double r = 1.0;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

/* ---- real instantiation ------------------------------------------------- */
#define REAL double
#define EXP_ exp
#define LOG_ log
#define RE_(z) (z)
#define FN(name) name##_r
#include "residual_body.inc"
#undef REAL
#undef EXP_
#undef LOG_
#undef RE_
#undef FN

/* ---- complex instantiation (complex-step derivative) --------------------- */
#define REAL double complex
#define EXP_ cexp
#define LOG_ clog
#define RE_(z) creal(z)
#define FN(name) name##_c
#include "residual_body.inc"
#undef REAL
#undef EXP_
#undef LOG_
#undef RE_
#undef FN

void om_prepare(om_mech *m)
{
  for (int i = 0; i < m->n_sp; i++) {
    double w = 0.0;
    for (int e = 0; e < m->n_el; e++) w += m->sp_el[i * m->n_el + e] * m->elem_w[e];
    m->W[i] = w;
  }
}

int om_n_unknowns(const om_mech *m, int energy)
{
  return m->n_sp + (energy ? 1 : 0) + (energy && m->soot ? 6 : 0);
}

double om_soot_ln_mu(const double *lnM, double p) { return soot_ln_mu_r(lnM, p); }

double om_soot_fxy(const double *lnM, int x, int y) { return soot_fxy_r(lnM, x, y); }

void om_soot_sources(const om_mech *m, double T, double CP, double CG, const double *lnM,
                     double *R, double *Wg, double *G, double *sinks)
{
  soot_sources_r(m, T, CP, CG, lnM, R, Wg, G, sinks);
}

void om_default_opts(om_opts *o)
{
  o->rtol = 1e-10;
  o->atol_Y = 1e-20;
  o->atol_T = 1e-12;
  o->ftol = 1e-10;
  o->lambda_min = 0.0;   /* <= 0: undamped Newton (bound-limited full steps) */
  o->T_min = 300.0;
  o->T_max = 4000.0;
  o->ts_rtol = 0.1;
  o->ts_atol_Y = 1e-6;
  o->ts_atol_T = 1e-3;
  o->ts_neg_tol = 1e-8;
  o->h0 = 1e-6;
  o->h_min = 1e-30;
  o->h_max = 1e6;
  o->nw_h_ratio = 0.0;
  o->nw_max_it = 30;
  o->nw_every = 10;
  o->max_lin = 1500;
  o->atol_lnM = 1e-10;
  o->ts_atol_lnM = 1e-3;
  o->lnM_step = 2.0;
  o->ct_ratio = 10.0;
  o->ct_tau_min = 1e-6;
  o->ct_min_step = 0.05;
}

void om_thermo(const om_mech *m, double T, double *cp_R, double *h_RT, double *s_R)
{
  thermo_r(m, T, cp_R, h_RT, s_R);
}

void om_rate_constants(const om_mech *m, double T, double *kf, double *Kc, double *kr)
{
  double *h = malloc(sizeof(double) * m->n_sp), *s = malloc(sizeof(double) * m->n_sp);
  thermo_r(m, T, NULL, h, s);
  rate_constants_r(m, T, h, s, kf, Kc, kr);
  free(h); free(s);
}

void om_production(const om_mech *m, double T, double P, const double *Y, double *C, double *q,
                   double *wdot)
{
  double *kf = malloc(sizeof(double) * m->n_rx), *kr = malloc(sizeof(double) * m->n_rx);
  om_rate_constants(m, T, kf, NULL, kr);
  production_r(m, T, P, Y, kf, kr, C, NULL, NULL, q, wdot);
  free(kf); free(kr);
}

void om_residual(const om_mech *m, const om_cond *c, const double *x, double *F)
{
  residual_r(m, c, x, F);
}

/* Scaled residual: each equation's residual divided by the sum of the
 * magnitudes of the terms it is made of (flow terms plus the gross forward
 * and reverse fluxes that enter it).  A value near 1 means the equation is
 * far from balanced; FP64 rounding alone gives ~1e-16 whatever the
 * stiffness, so a bound of 1e-10 is attainable for every reactor.          */
double om_scaled_residual(const om_mech *m, const om_cond *c, const double *x)
{
  const int N = m->n_sp, NR = m->n_rx;
  double *h = malloc(sizeof(double) * N), *s = malloc(sizeof(double) * N);
  double *hin = malloc(sizeof(double) * N);
  double *kf = malloc(sizeof(double) * NR), *kr = malloc(sizeof(double) * NR);
  double *Rf = malloc(sizeof(double) * NR), *Rr = malloc(sizeof(double) * NR);
  double *C = malloc(sizeof(double) * N), *wdot = malloc(sizeof(double) * N);
  const int n = om_n_unknowns(m, c->energy), soot = c->energy && m->soot;
  double *gross = calloc(N, sizeof(double)), *F = malloc(sizeof(double) * n);
  double R[6], Wg[6], G[6], sk[2] = {0.0, 0.0};
  int Ps = -1, Gs = -1;
  double T = c->energy ? x[N] : c->T_in;
  thermo_r(m, T, NULL, h, s);
  rate_constants_r(m, T, h, s, kf, NULL, kr);
  double rho = production_r(m, T, c->P, x, kf, kr, C, Rf, Rr, NULL, wdot);
  double mdot = rho * OM_V / c->tau;
  residual_r(m, c, x, F);
  if (soot) {
    Ps = m->soot->precursor; Gs = m->soot->growth;
    soot_sources_r(m, T, C[Ps], C[Gs], x + N + 1, R, Wg, G, sk);
  }
  for (int k = 0; k < NR; k++) {
    double g = fabs(Rf[k]) + fabs(Rr[k]);
    for (int sl = 0; sl < 3; sl++) {
      int i = m->r_idx[3 * k + sl];
      if (i >= 0) gross[i] += m->r_nu[3 * k + sl] * g;
      i = m->p_idx[3 * k + sl];
      if (i >= 0) gross[i] += m->p_nu[3 * k + sl] * g;
    }
  }
  double worst = 0.0;
  for (int i = 0; i < N; i++) {
    double den = mdot * (fabs(x[i]) + fabs(c->Y_in[i])) + OM_V * m->W[i] * gross[i];
    if (i == Ps) den += OM_V * m->W[i] * sk[0];
    if (i == Gs) den += OM_V * m->W[i] * sk[1];
    if (den > 0.0 && fabs(F[i]) / den > worst) worst = fabs(F[i]) / den;
    if (!(den >= 0.0) || F[i] != F[i]) worst = INFINITY;
  }
  if (c->energy == 2) {
    double den = OM_V * (fabs(T) + fabs(c->T_in)) / c->tau;
    if (fabs(F[N]) / den > worst) worst = fabs(F[N]) / den;
    if (F[N] != F[N]) worst = INFINITY;
  } else if (c->energy) {
    thermo_r(m, c->T_in, NULL, hin, NULL);
    double den = 0.0;
    for (int i = 0; i < N; i++) {
      double H = OM_R * T * h[i], Hin = OM_R * c->T_in * hin[i];
      den += mdot * fabs(c->Y_in[i] * (H - Hin) / m->W[i]) + OM_V * fabs(H) * gross[i];
    }
    if (soot) den += OM_V * OM_R * T * (fabs(h[Ps]) * sk[0] + fabs(h[Gs]) * sk[1]);
    if (den > 0.0 && fabs(F[N]) / den > worst) worst = fabs(F[N]) / den;
    if (F[N] != F[N]) worst = INFINITY;
  }
  /* moment rows: relative to outflow plus the magnitudes of the sources */
  for (int r = 0; soot && r < 6; r++) {
    double den = OM_V * (exp(x[N + 1 + r]) / c->tau + fabs(R[r]) + fabs(Wg[r]) + fabs(G[r]));
    double v = fabs(F[N + 1 + r]) / den;
    if (!(v <= worst)) worst = v; /* a NaN wins */
  }
  free(h); free(s); free(hin); free(kf); free(kr); free(Rf); free(Rr);
  free(C); free(wdot); free(gross); free(F);
  return worst;
}

/* d(k prod_s C_s^nu_s)/dC at slot s0 of one side of reaction k:
 * k * nu_s0 * C_s0^(nu_s0 - 1) * prod_{s != s0} C_s^nu_s.                  */
static double side_partial(double kconst, const int *idx, const int *nu, const double *C, int s0)
{
  double d = kconst * nu[s0] * ipow_r(C[idx[s0]], nu[s0] - 1);
  for (int s = 0; s < 3; s++)
    if (s != s0 && idx[s] >= 0) d *= ipow_r(C[idx[s]], nu[s]);
  return d;
}

/* Analytic Jacobian J[r*n + col] = dF_r / dx_col of the residual above.
 * Chain rule through rho(Y, T), C_j(Y, T), k_f(T), K_c(T):
 *   drho/dY_m = -rho/(S W_m),  drho/dT = -rho/T,  S = sum_j Y_j/W_j
 *   dC_j/dY_m = rho delta_jm / W_j - C_j/(S W_m),  dC_j/dT = -C_j/T
 *   d ln k_f/dT = beta/T + E/(R T^2)
 *   d ln K_c/dT = sum_i nu_i (H_i/RT)/T - (sum_i nu_i)/T   (van 't Hoff)
 *   d ln k_r/dT = d ln k_f/dT - d ln K_c/dT                                 */
void om_jacobian(const om_mech *m, const om_cond *c, const double *x, double *J)
{
  const int N = m->n_sp, NR = m->n_rx, n = om_n_unknowns(m, c->energy);
  for (size_t e = 0; e < (size_t)n * n; e++) J[e] = 0.0;
  double *cp = malloc(sizeof(double) * N), *h = malloc(sizeof(double) * N);
  double *s = malloc(sizeof(double) * N), *hin = malloc(sizeof(double) * N);
  double *kf = malloc(sizeof(double) * NR), *kr = malloc(sizeof(double) * NR);
  double *Rf = malloc(sizeof(double) * NR), *Rr = malloc(sizeof(double) * NR);
  double *C = malloc(sizeof(double) * N), *wdot = malloc(sizeof(double) * N);
  double *dwdY = calloc((size_t)N * N, sizeof(double)); /* dwdot_i/dY_m */
  double *dwdT = calloc(N, sizeof(double));             /* dwdot_i/dT   */
  double *dqdY = malloc(sizeof(double) * N);
  double T = c->energy ? x[N] : c->T_in;
  thermo_r(m, T, cp, h, s);
  rate_constants_r(m, T, h, s, kf, NULL, kr);
  double rho = production_r(m, T, c->P, x, kf, kr, C, Rf, Rr, NULL, wdot);
  double S = 0.0;
  for (int j = 0; j < N; j++) S += x[j] / m->W[j];
  double mdot = rho * OM_V / c->tau;

  for (int k = 0; k < NR; k++) {
    const int *ri = m->r_idx + 3 * k, *rn = m->r_nu + 3 * k;
    const int *pi = m->p_idx + 3 * k, *pn = m->p_nu + 3 * k;
    /* partial derivatives of q_k w.r.t. concentrations, at fixed T */
    double dqdC[6];
    int col[6];
    int nc = 0;
    for (int sl = 0; sl < 3; sl++) {
      if (ri[sl] >= 0) { col[nc] = ri[sl]; dqdC[nc] = side_partial(kf[k], ri, rn, C, sl); nc++; }
    }
    for (int sl = 0; sl < 3; sl++) {
      if (pi[sl] >= 0) { col[nc] = pi[sl]; dqdC[nc] = -side_partial(kr[k], pi, pn, C, sl); nc++; }
    }
    double sumC = 0.0; /* sum_j C_j dq_k/dC_j */
    for (int a = 0; a < nc; a++) sumC += C[col[a]] * dqdC[a];
    /* temperature derivative at fixed concentrations */
    double dlnkf = m->beta[k] / T + m->Ea[k] / (OM_R * T * T);
    double dlnKc = 0.0;
    int dnu = 0;
    for (int sl = 0; sl < 3; sl++) {
      if (pi[sl] >= 0) { dlnKc += pn[sl] * h[pi[sl]] / T; dnu += pn[sl]; }
      if (ri[sl] >= 0) { dlnKc -= rn[sl] * h[ri[sl]] / T; dnu -= rn[sl]; }
    }
    dlnKc -= dnu / T;
    double dlnkr = dlnkf - dlnKc;
    double dqdT = Rf[k] * dlnkf - Rr[k] * dlnkr - sumC / T;
    /* total derivative of q_k with respect to every Y_m */
    for (int mm = 0; mm < N; mm++) dqdY[mm] = -sumC / (S * m->W[mm]);
    for (int a = 0; a < nc; a++) dqdY[col[a]] += rho / m->W[col[a]] * dqdC[a];
    /* scatter into dwdot_i = sum_k nu_ik dq_k */
    for (int sl = 0; sl < 6; sl++) {
      int i = sl < 3 ? ri[sl] : pi[sl - 3];
      if (i < 0) continue;
      double nu = sl < 3 ? -rn[sl] : pn[sl - 3];
      for (int mm = 0; mm < N; mm++) dwdY[(size_t)i * N + mm] += nu * dqdY[mm];
      dwdT[i] += nu * dqdT;
    }
  }

  for (int i = 0; i < N; i++) {
    for (int mm = 0; mm < N; mm++) {
      double v = -mdot / (S * m->W[mm]) * (x[i] - c->Y_in[i])
                 - OM_V * m->W[i] * dwdY[(size_t)i * N + mm];
      if (i == mm) v += mdot;
      J[(size_t)i * n + mm] = v;
    }
    if (c->energy)
      J[(size_t)i * n + N] = -mdot / T * (x[i] - c->Y_in[i]) - OM_V * m->W[i] * dwdT[i];
  }
  if (c->energy == 2) {
    J[(size_t)N * n + N] = OM_V / c->tau;
  } else if (c->energy) {
    thermo_r(m, c->T_in, NULL, hin, NULL);
    double Qin = 0.0, dQin = 0.0;
    for (int i = 0; i < N; i++) {
      Qin += c->Y_in[i] * (OM_R * T * h[i] - OM_R * c->T_in * hin[i]) / m->W[i];
      dQin += c->Y_in[i] * OM_R * cp[i] / m->W[i];
    }
    for (int mm = 0; mm < N; mm++) {
      double v = -mdot / (S * m->W[mm]) * Qin;
      for (int i = 0; i < N; i++) v += OM_V * OM_R * T * h[i] * dwdY[(size_t)i * N + mm];
      J[(size_t)N * n + mm] = v;
    }
    double v = -mdot / T * Qin + mdot * dQin;
    for (int i = 0; i < N; i++) v += OM_V * (OM_R * cp[i] * wdot[i] + OM_R * T * h[i] * dwdT[i]);
    J[(size_t)N * n + N] = v;
  }
  /* soot block (precursor, growth, energy and moment rows; every column):
   * complex-step derivative of the soot terms alone, exact to rounding   */
  if (c->energy && m->soot) {
    double complex *xc = malloc(sizeof(double complex) * n), *Fc = malloc(sizeof(double complex) * n);
    for (int col = 0; col < n; col++) {
      double hstep = 1e-30 * (fabs(x[col]) > 1e-10 ? fabs(x[col]) : 1e-10);
      for (int j = 0; j < n; j++) xc[j] = x[j];
      xc[col] = x[col] + hstep * _Complex_I;
      soot_only_c(m, c, xc, Fc);
      for (int r = 0; r < n; r++) J[(size_t)r * n + col] += cimag(Fc[r]) / hstep;
    }
    free(xc); free(Fc);
  }
  free(cp); free(h); free(s); free(hin); free(kf); free(kr); free(Rf); free(Rr);
  free(C); free(wdot); free(dwdY); free(dwdT); free(dqdY);
}

/* Complex-step derivative (Squire & Trapp 1998) of the residual source
 * above: column m is Im F(x + i h e_m) / h.  No subtraction, so it is exact
 * to rounding for any h small enough; used only to pin om_jacobian.         */
void om_jacobian_complex_step(const om_mech *m, const om_cond *c, const double *x, double *J)
{
  const int n = om_n_unknowns(m, c->energy);
  double complex *xc = malloc(sizeof(double complex) * n), *Fc = malloc(sizeof(double complex) * n);
  for (int col = 0; col < n; col++) {
    double hstep = 1e-30 * (fabs(x[col]) > 1e-10 ? fabs(x[col]) : 1e-10);
    for (int j = 0; j < n; j++) xc[j] = x[j];
    xc[col] = x[col] + hstep * _Complex_I;
    residual_c(m, c, xc, Fc);
    for (int r = 0; r < n; r++) J[(size_t)r * n + col] = cimag(Fc[r]) / hstep;
  }
  free(xc); free(Fc);
}

/* Diagonal mass matrix of the transient form of Eqs. 2-3:
 * rho V for each species row, rho V cp_mix for the energy row (V for the
 * prescribed-temperature row, which relaxes T to T_in over tau), V M_r for
 * the ln M_r rows (d M_r/dt = M_r d ln M_r/dt).                             */
void om_mass_diag(const om_mech *m, const om_cond *c, const double *x, double *M)
{
  const int N = m->n_sp;
  double T = c->energy ? x[N] : c->T_in;
  double S = 0.0;
  for (int j = 0; j < N; j++) S += x[j] / m->W[j];
  double rho = c->P * 1.0e-6 / (OM_R * T * S);
  for (int i = 0; i < N; i++) M[i] = rho * OM_V;
  if (c->energy) {
    double *cp = malloc(sizeof(double) * N);
    thermo_r(m, T, cp, NULL, NULL);
    double cpmix = 0.0;
    for (int i = 0; i < N; i++) cpmix += x[i] * OM_R * cp[i] / m->W[i];
    M[N] = c->energy == 2 ? OM_V : rho * OM_V * cpmix;
    free(cp);
    if (m->soot)
      for (int r = 0; r < 6; r++) M[N + 1 + r] = OM_V * exp(x[N + 1 + r]);
  }
}

/* Soot outputs of one reactor from its moments (the quantities of the
 * Section 5 sweeps, Figs. 1-2): number density N = M_0 (cm^-3), volume
 * fraction f_v = M_1 m_C / rho_s (M_1 carbon atoms per cm^3 at mass m_C
 * each, soot density rho_s) and the diameter of a sphere of the mean
 * particle volume, d = (6 f_v / (pi N))^(1/3) (cm).  out = (f_v, N, d).   */
void om_soot_outputs(const om_mech *m, const double *lnM, double *out)
{
  const om_soot *sd = m->soot;
  const double mC = m->elem_w[sd->carbon] / OM_NA;
  const double N0 = exp(lnM[0]), fv = exp(lnM[1]) * mC / sd->soot_density;
  out[0] = fv;
  out[1] = N0;
  out[2] = cbrt(6.0 * fv / (OM_PI * N0));
}

/* Textbook LU with partial pivoting (Golub & Van Loan, Alg. 3.4.1), row
 * major, in place.  Pivot = first row index of the largest |a_ik| at or
 * below the diagonal; rows are swapped whole, so piv[] follows the LAPACK
 * getrf convention (row k was interchanged with row piv[k]).  Returns 0, or
 * k+1 if column k has no nonzero pivot.                                    */
int om_lu_factor(int n, double *a, int *piv)
{
  for (int k = 0; k < n; k++) {
    int p = k;
    double amax = fabs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; i++) {
      if (fabs(a[(size_t)i * n + k]) > amax) { amax = fabs(a[(size_t)i * n + k]); p = i; }
    }
    piv[k] = p;
    if (!(amax > 0.0)) return k + 1;
    if (p != k) {
      for (int j = 0; j < n; j++) {
        double t = a[(size_t)k * n + j];
        a[(size_t)k * n + j] = a[(size_t)p * n + j];
        a[(size_t)p * n + j] = t;
      }
    }
    for (int i = k + 1; i < n; i++) {
      a[(size_t)i * n + k] /= a[(size_t)k * n + k];
      for (int j = k + 1; j < n; j++) a[(size_t)i * n + j] -= a[(size_t)i * n + k] * a[(size_t)k * n + j];
    }
  }
  return 0;
}

/* Solve (P L U) z = b in place: apply the interchanges, then forward
 * substitution with unit-lower L and back substitution with U.             */
void om_lu_solve(int n, const double *lu, const int *piv, double *b)
{
  for (int k = 0; k < n; k++) {
    double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t;
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < i; j++) b[i] -= lu[(size_t)i * n + j] * b[j];
  for (int i = n - 1; i >= 0; i--) {
    for (int j = i + 1; j < n; j++) b[i] -= lu[(size_t)i * n + j] * b[j];
    b[i] /= lu[(size_t)i * n + i];
  }
}

/* Scale the rows, then the columns, of a by powers of two so that every
 * row and column has largest magnitude in [1/2, 1) (exact in binary
 * floating point), then factor the scaled matrix with om_lu_factor.  rs,
 * cs receive the scales.  The Jacobians of stiff mechanisms have rows whose
 * magnitudes differ by tens of orders (gross fluxes against the flow
 * terms); without this scaling the pivot order is set by those magnitudes
 * and the Newton steps of trace species lose every significant digit.    */
static int eq_factor(int n, double *a, int *piv, double *rs, double *cs)
{
  for (int i = 0; i < n; i++) {
    double mx = 0.0;
    int e = 0;
    for (int j = 0; j < n; j++)
      if (fabs(a[(size_t)i * n + j]) > mx) mx = fabs(a[(size_t)i * n + j]);
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    rs[i] = ldexp(1.0, -e);
  }
  for (int j = 0; j < n; j++) {
    double mx = 0.0;
    int e = 0;
    for (int i = 0; i < n; i++)
      if (fabs(a[(size_t)i * n + j] * rs[i]) > mx) mx = fabs(a[(size_t)i * n + j] * rs[i]);
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    cs[j] = ldexp(1.0, -e);
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) a[(size_t)i * n + j] *= rs[i] * cs[j];
  return om_lu_factor(n, a, piv);
}

/* Solve a z = b in place with the factors of eq_factor:
 * z = diag(cs) (R a C)^-1 diag(rs) b.                                       */
static void eq_solve(int n, const double *lu, const int *piv, const double *rs, const double *cs,
                     double *b)
{
  for (int i = 0; i < n; i++) b[i] *= rs[i];
  om_lu_solve(n, lu, piv, b);
  for (int i = 0; i < n; i++) b[i] *= cs[i];
}

/* ---- hybrid damped Newton / pseudo-transient driver (Section 3) -------- */

enum { NW_CONVERGED, NW_FAILED, NW_BUDGET };

static int all_finite(int n, const double *v)
{
  for (int i = 0; i < n; i++) if (!isfinite(v[i])) return 0;
  return 1;
}

/* x <- x + lam * d, then Y projected onto Y >= 0 and T onto [T_min, T_max];
 * ln M unbounded.                                                           */
static void step_clamped(const om_cond *c, const om_opts *o, int N, int n, const double *x,
                         double lam, const double *d, double *out)
{
  for (int i = N + 1; i < n; i++) out[i] = x[i] + lam * d[i];
  for (int i = 0; i < N; i++) {
    double v = x[i] + lam * d[i];
    out[i] = v > 0.0 ? v : 0.0;
  }
  if (c->energy) {
    double v = x[N] + lam * d[N];
    out[N] = v < o->T_min ? o->T_min : (v > o->T_max ? o->T_max : v);
  }
}

/* Largest lambda <= 1 keeping T + lambda dT inside [T_min, T_max] and every
 * soot unknown's change |lambda d ln M_r| at most lnM_step.                 */
static double bound_lambda(const om_cond *c, const om_opts *o, int N, int n, const double *x,
                           const double *d)
{
  double lam = 1.0;
  if (c->energy) {
    double T = x[N], dT = d[N];
    if (dT > 0.0 && T + dT > o->T_max) lam = (o->T_max - T) / dT;
    if (dT < 0.0 && T + dT < o->T_min) lam = (T - o->T_min) / (-dT);
  }
  for (int r = N + 1; r < n; r++)
    if (fabs(d[r]) * lam > o->lnM_step) lam = o->lnM_step / fabs(d[r]);
  return lam;
}

/* Weighted max norm of a Newton step: max_k |d_k| / (atol_k + rtol |x_k|). */
static double newton_norm(const om_opts *o, int N, int n, const double *x, const double *d)
{
  double r = 0.0;
  for (int k = 0; k < n; k++) {
    double w = (k < N ? o->atol_Y : (k == N ? o->atol_T : o->atol_lnM)) + o->rtol * fabs(x[k]);
    double t = fabs(d[k]) / w;
    if (!(t <= r)) r = t; /* a NaN wins */
  }
  return r;
}

/* Steady Newton attempt on F(x) = 0, started from x (not modified unless
 * it converges).  Each iteration: F(x), J(x), LU of the equilibrated J,
 * Newton step d = -J^-1 F.  Converged when the weighted step norm is <= 1
 * and the scaled residual is <= ftol; the result is then x + d.  Otherwise
 * the step length lambda starts at the bound limit (T inside [T_min,
 * T_max], |d ln M_r| <= lnM_step).  With lambda_min <= 0 that step is taken
 * as it is (mass fractions projected onto Y >= 0); with lambda_min > 0
 * lambda is halved until the trial point's step, solved with the same
 * factors, is smaller in the weighted norm than d (natural criterion), and
 * the attempt fails below lambda_min.  After nw_max_it iterations the
 * attempt has failed.  Every (residual, triangular solve) pair counts one
 * against the max_lin budget.                                               */
static int newton_attempt(const om_mech *m, const om_cond *c, const om_opts *o, double *xio,
                          om_stats *st)
{
  const int N = m->n_sp, n = om_n_unknowns(m, c->energy);
  double *x = malloc(sizeof(double) * n), *F = malloc(sizeof(double) * n);
  double *J = malloc(sizeof(double) * n * n), *d = malloc(sizeof(double) * n);
  double *dt = malloc(sizeof(double) * n), *xt = malloc(sizeof(double) * n);
  int *piv = malloc(sizeof(int) * n);
  double *rs = malloc(sizeof(double) * n), *cs = malloc(sizeof(double) * n);
  int result = NW_FAILED;
  memcpy(x, xio, sizeof(double) * n);
  for (int it = 0; it < o->nw_max_it; it++) {
    if (st->n_lin >= o->max_lin) { result = NW_BUDGET; break; }
    om_residual(m, c, x, F);
    om_jacobian(m, c, x, J);
    st->n_jac++;
    if (!all_finite(n, F) || !all_finite(n * n, J)) break;
    if (eq_factor(n, J, piv, rs, cs) != 0) break;
    for (int i = 0; i < n; i++) d[i] = -F[i];
    eq_solve(n, J, piv, rs, cs, d);
    st->n_lin++;
    if (!all_finite(n, d)) break;
    double nd = newton_norm(o, N, n, x, d);
    TRACE("NW it=%d nlin=%d nd=%.3e T=%.2f\n", it, st->n_lin, nd, c->energy ? x[N] : c->T_in);
    if (nd <= 1.0) {
      double sres = om_scaled_residual(m, c, x);
      if (sres <= o->ftol) {
        st->sres = sres;
        step_clamped(c, o, N, n, x, 1.0, d, xio);
        result = NW_CONVERGED;
        break;
      }
    }
    double lam = bound_lambda(c, o, N, n, x, d);
    if (!(o->lambda_min > 0.0)) {
      step_clamped(c, o, N, n, x, lam, d, xt);
      memcpy(x, xt, sizeof(double) * n);
      continue;
    }
    int accepted = 0;
    while (lam >= o->lambda_min) {
      if (st->n_lin >= o->max_lin) { result = NW_BUDGET; goto done; }
      step_clamped(c, o, N, n, x, lam, d, xt);
      om_residual(m, c, xt, dt);
      for (int i = 0; i < n; i++) dt[i] = -dt[i];
      eq_solve(n, J, piv, rs, cs, dt);
      st->n_lin++;
      if (newton_norm(o, N, n, x, dt) < nd) {
        memcpy(x, xt, sizeof(double) * n);
        accepted = 1;
        break;
      }
      lam *= 0.5;
    }
    if (!accepted) break;
  }
done:
  free(x); free(F); free(J); free(d); free(dt); free(xt); free(piv); free(rs); free(cs);
  return result;
}

enum { TS_ACCEPTED, TS_REJECTED, TS_SINGULAR, TS_BUDGET };

/* One pseudo-transient step of M dx/dt = -F(x) (M: the mass-matrix
 * diagonal frozen at x) with the two-stage L-stable Rosenbrock method ROS2
 * (Verwer, Spee, Blom & Hundsdorfer 1999), gamma = 1 + 1/sqrt(2):
 *   A = M/(gamma h) + J(x)
 *   A k1 = -F(x) / (gamma h)
 *   A k2 = (-F(x + h k1) - 2 M k1) / (gamma h)
 *   x_new = x + 3/2 h k1 + 1/2 h k2,   error estimate  h/2 (k1 + k2).
 * The matrix A is equilibrated before its LU, as in the Newton attempt.
 * Accepted when the RMS-weighted error is <= 1 (weights ts_atol + ts_rtol
 * max(|x|, |x_new|) for Y and T; ts_atol_lnM + ts_rtol for ln M_r, whose
 * changes are relative changes of M_r already), x_new is finite, T stays in [T_min, T_max] and no
 * mass fraction is below -ts_neg_tol; negative mass fractions are then set
 * to zero.  h is rescaled by 0.9/sqrt(err) within [0.2, 5] (0.25 after a
 * non-finite or out-of-bounds result).  Counts two linear solves.  Returns
 * TS_SINGULAR for a step rejected because A had no nonzero pivot.        */
static int ros2_step(const om_mech *m, const om_cond *c, const om_opts *o, double *x, double *h,
                     om_stats *st)
{
  const int N = m->n_sp, n = om_n_unknowns(m, c->energy);
  const double gam = 1.0 + 1.0 / sqrt(2.0);
  if (st->n_lin + 2 > o->max_lin) return TS_BUDGET;
  double *F = malloc(sizeof(double) * n), *A = malloc(sizeof(double) * n * n);
  double *M = malloc(sizeof(double) * n), *k1 = malloc(sizeof(double) * n);
  double *k2 = malloc(sizeof(double) * n), *x1 = malloc(sizeof(double) * n);
  double *xn = malloc(sizeof(double) * n);
  int *piv = malloc(sizeof(int) * n);
  double *rs = malloc(sizeof(double) * n), *cs = malloc(sizeof(double) * n);
  int result = TS_REJECTED, bad = 0;
  double hh = *h, err = INFINITY;

  om_residual(m, c, x, F);
  om_jacobian(m, c, x, A);
  om_mass_diag(m, c, x, M);
  st->n_jac++;
  for (int i = 0; i < n; i++) A[(size_t)i * n + i] += M[i] / (gam * hh);
  int sing = 0;
  if (!all_finite(n, F) || !all_finite(n * n, A)) {
    bad = 1;
  } else if (eq_factor(n, A, piv, rs, cs) != 0) {
    bad = 1;
    sing = 1;
  } else {
    for (int i = 0; i < n; i++) k1[i] = -F[i] / (gam * hh);
    eq_solve(n, A, piv, rs, cs, k1);
    for (int i = 0; i < n; i++) x1[i] = x[i] + hh * k1[i];
    if (c->energy) x1[N] = x1[N] < o->T_min ? o->T_min : (x1[N] > o->T_max ? o->T_max : x1[N]);
    om_residual(m, c, x1, F);
    for (int i = 0; i < n; i++) k2[i] = (-F[i] - 2.0 * M[i] * k1[i]) / (gam * hh);
    eq_solve(n, A, piv, rs, cs, k2);
    double s = 0.0;
    for (int i = 0; i < n; i++) {
      xn[i] = x[i] + 1.5 * hh * k1[i] + 0.5 * hh * k2[i];
      double ax = fabs(x[i]) > fabs(xn[i]) ? fabs(x[i]) : fabs(xn[i]);
      double w = i > N ? o->ts_atol_lnM + o->ts_rtol
                       : (i < N ? o->ts_atol_Y : o->ts_atol_T) + o->ts_rtol * ax;
      double e = 0.5 * hh * (k1[i] + k2[i]) / w;
      s += e * e;
    }
    err = sqrt(s / n);
    if (!all_finite(n, xn) || !isfinite(err)) bad = 1;
    if (c->energy && (xn[N] < o->T_min || xn[N] > o->T_max)) bad = 1;
    for (int i = 0; i < N; i++)
      if (xn[i] < -o->ts_neg_tol) bad = 1;
  }
  st->n_lin += 2;
  TRACE("ROS2 h/tau=%.3e err=%.3e bad=%d T=%.1f minY=%.3e\n", hh / c->tau, err, bad,
        c->energy ? xn[N] : c->T_in, xn[0]);
  if (!bad && err <= 1.0) {
    for (int i = 0; i < N; i++) x[i] = xn[i] > 0.0 ? xn[i] : 0.0;
    for (int i = N; i < n; i++) x[i] = xn[i];
    double fac = 0.9 / sqrt(err > 1e-10 ? err : 1e-10);
    *h = hh * (fac > 5.0 ? 5.0 : (fac < 0.2 ? 0.2 : fac));
    if (*h > o->h_max * c->tau) *h = o->h_max * c->tau;
    result = TS_ACCEPTED;
  } else {
    double fac = bad ? 0.25 : 0.9 / sqrt(err);
    *h = hh * (fac < 0.2 ? 0.2 : fac);
    if (sing) result = TS_SINGULAR;
  }
  free(F); free(A); free(M); free(k1); free(k2); free(x1); free(xn); free(piv); free(rs); free(cs);
  return result;
}

/* Continuation in the residence time for a gas-phase reactor whose Newton
 * attempt at its own tau failed: Newton attempts from the initial guess x0
 * at tau / r, tau / r^2, ... (r = ct_ratio, not below ct_tau_min seconds)
 * until one converges; from that root, the residence time is raised towards
 * tau in steps of at most a factor r, each step solved by a Newton attempt
 * started from the root before; a failed step is retried at half its length
 * in ln tau, and the walk stops once the step falls below ct_min_step.
 * Returns NW_CONVERGED with x the root at tau, NW_BUDGET, or NW_FAILED with
 * x the last root of the walk (x0 if no rung converged).                   */
static int tau_continuation(const om_mech *m, const om_cond *c, const om_opts *o, double *x,
                            om_stats *st)
{
  const int n = om_n_unknowns(m, c->energy);
  double *x0 = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
  memcpy(x0, x, sizeof(double) * n);
  om_cond cc = *c;
  const double lt = log(c->tau), lr = log(o->ct_ratio);
  double lc = 0.0;
  int found = 0, result = NW_FAILED;
  for (int k = 1; lt - k * lr >= log(o->ct_tau_min); k++) {
    cc.tau = exp(lt - k * lr);
    memcpy(y, x0, sizeof(double) * n);
    st->n_attempts++;
    int r = newton_attempt(m, &cc, o, y, st);
    if (r == NW_BUDGET) { result = NW_BUDGET; goto done; }
    if (r == NW_CONVERGED) { found = 1; lc = lt - k * lr; memcpy(x, y, sizeof(double) * n); break; }
  }
  if (!found) goto done;
  double step = lr;
  while (step >= o->ct_min_step) {
    const int last = lc + step >= lt;
    const double ln = last ? lt : lc + step;
    cc.tau = last ? c->tau : exp(ln);
    memcpy(y, x, sizeof(double) * n);
    st->n_attempts++;
    int r = newton_attempt(m, &cc, o, y, st);
    if (r == NW_BUDGET) { result = NW_BUDGET; break; }
    if (r == NW_CONVERGED) {
      memcpy(x, y, sizeof(double) * n);
      if (last) { result = NW_CONVERGED; break; }
      lc = ln;
      step = 2.0 * step < lr ? 2.0 * step : lr;
    } else {
      step *= 0.5;
    }
  }
done:
  free(x0); free(y);
  return result;
}

/* Hybrid solve (Section 3): a steady Newton attempt at the reactor's tau;
 * if it fails, a gas-phase reactor tries the continuation in tau above
 * (ct_ratio > 1); while Newton still fails, the estimate (the last root of
 * the continuation, else the initial guess) is conditioned by
 * pseudo-transient integration and Newton is tried again after every
 * nw_every accepted steps once the step size has grown to nw_h_ratio * tau.
 * Ends converged, with TS_FAILED when the step size falls below h_min
 * (seconds), or MAXITER when the linear-solve budget is spent.  x holds the
 * initial guess on entry, the result on exit.                              */
int om_solve(const om_mech *m, const om_cond *c, const om_opts *o, double *x, om_stats *st)
{
  const int N = m->n_sp, n = om_n_unknowns(m, c->energy);
  memset(st, 0, sizeof(*st));
  /* Eqs. 1-3 need a positive, finite pressure, residence time and inlet
   * temperature, and finite inlet and initial data; a reactor outside that
   * domain is reported as non-finite at once and its x is left as given.  */
  int bad = !(c->P > 0.0 && c->P < HUGE_VAL) || !(c->tau > 0.0 && c->tau < HUGE_VAL) ||
            !(c->T_in > 0.0 && c->T_in < HUGE_VAL);
  for (int i = 0; i < N; i++) bad |= !isfinite(c->Y_in[i]);
  for (int i = 0; i < n; i++) bad |= !isfinite(x[i]);
  if (bad) { st->status = OM_NONFINITE; return st->status; }
  for (int i = 0; i < N; i++) if (x[i] < 0.0) x[i] = 0.0;
  double h = o->h0 * c->tau;
  int attempt = 1, accepted = 0, first = 1;
  for (;;) {
    if (attempt) {
      st->n_attempts++;
      int r = newton_attempt(m, c, o, x, st);
      if (r == NW_CONVERGED) { st->status = OM_CONVERGED; break; }
      if (r == NW_BUDGET) { st->status = OM_MAXITER; break; }
      attempt = 0;
      if (first && o->ct_ratio > 1.0 && !(c->energy && m->soot)) {
        r = tau_continuation(m, c, o, x, st);
        if (r == NW_CONVERGED) { st->status = OM_CONVERGED; break; }
        if (r == NW_BUDGET) { st->status = OM_MAXITER; break; }
      }
      first = 0;
    }
    int r = ros2_step(m, c, o, x, &h, st);
    if (r == TS_BUDGET) { st->status = OM_MAXITER; break; }
    if (r == TS_ACCEPTED) {
      accepted++;
      st->n_ts++;
      if (accepted % o->nw_every == 0 && h >= o->nw_h_ratio * c->tau) attempt = 1;
    } else if (h < o->h_min) {
      st->status = r == TS_SINGULAR ? OM_SINGULAR : OM_TS_FAILED;
      break;
    }
  }
  if (st->status == OM_CONVERGED && !all_finite(n, x)) st->status = OM_NONFINITE;
  return st->status;
}

/* Pseudo-transient integration alone (no Newton attempt): max_steps
 * accepted steps, for checks that the time stepping reaches the same steady
 * state as Newton.                                                          */
int om_time_march_only(const om_mech *m, const om_cond *c, const om_opts *o, double *x,
                       int max_steps, om_stats *st)
{
  memset(st, 0, sizeof(*st));
  double h = o->h0 * c->tau;
  st->status = OM_CONVERGED;
  while (st->n_ts < max_steps) {
    int r = ros2_step(m, c, o, x, &h, st);
    if (r == TS_BUDGET) { st->status = OM_MAXITER; break; }
    if (r == TS_ACCEPTED) st->n_ts++;
    else if (h < o->h_min) { st->status = r == TS_SINGULAR ? OM_SINGULAR : OM_TS_FAILED; break; }
  }
  return st->status;
}
