/* Plain FP64 CPU oracle for the batched perfectly-stirred-reactor (PSR)
 * steady-state solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header or constant with the GPU library.
 *
 * What it computes (paper: Section 2, Eqs. 1-3; Section 3, Eqs. 4-9):
 *   - species thermodynamics from single-range NASA-7 polynomials (the S and
 *     H of Eq. 9),
 *   - forward rate constants (Eq. 6), equilibrium constants (Eqs. 8-9),
 *     reverse rate constants (Eq. 7), rates of progress (Eq. 5) and net
 *     molar production rates (Eq. 4),
 *   - the steady PSR residual from Eq. 2 (species) and Eq. 3 (energy),
 *   - its analytic Jacobian (the paper uses finite differences; the analytic
 *     form has the same root),
 *   - a textbook partial-pivoting LU factorisation and solve,
 *   - the hybrid damped-Newton / pseudo-transient solve of Section 3,
 *   - soot moments (MOMIC) coupled to the gas phase when om_mech.soot is set.
 *
 * Units: concentrations mol/cm^3, density g/cm^3, pressure Pa, energies
 * J/mol, A in (cm^3/mol)^(order-1)/s, V = 1 cm^3.
 */
#ifndef PSR_ORACLE_H
#define PSR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Soot particle population by the method of moments with interpolative
 * closure (MOMIC; the paper couples it to the gas phase for its sooting
 * reactor, Sections 1-2 and 6, citing Frenklach's method).  Unknowns
 * ln M_r, r = 0..5, with M_r = sum_i m_i^r N_i per cm^3 and m in carbon
 * atoms.  Nucleation from two molecules of a pure-carbon precursor P,
 * surface growth by a pure-carbon species G (n_C(G) atoms per step),
 * free-molecular coagulation.  Soot requires the energy equation.       */
typedef struct {
  int precursor, growth, carbon; /* species P, species G, element index of carbon */
  double A_nuc, beta_nuc, E_nuc;    /* k_n = A T^beta exp(-E/RT), cm^3/(mol s)   */
  double A_grow, beta_grow, E_grow; /* k_s per surface site, cm^3/(mol s)        */
  double site_density;              /* chi, sites per cm^2                       */
  double soot_density;              /* rho_s, g/cm^3                             */
  double coag_scale;                /* factor on the coagulation kernel (1 = Frenklach's) */
} om_soot;

typedef struct {
  int n_el, n_sp, n_rx;
  const double *elem_w;  /* [E] g/mol                               */
  const int *sp_el;      /* [N*E] atom counts                        */
  const double *nasa;    /* [N*7] a1..a7, single range               */
  const int *r_idx;      /* [I*3] reactant species, -1 = unused slot */
  const int *r_nu;       /* [I*3] reactant coefficients              */
  const int *p_idx;      /* [I*3] product species                    */
  const int *p_nu;       /* [I*3] product coefficients               */
  const double *A;       /* [I]                                      */
  const double *beta;    /* [I]                                      */
  const double *Ea;      /* [I] J/mol                                */
  const om_soot *soot;   /* NULL: gas phase only                     */
  double *W;             /* [N] work: species weights, filled by om_prepare */
} om_mech;

typedef struct {
  double P;          /* Pa                                  */
  double tau;        /* residence time, s                   */
  double T_in;       /* inlet temperature (isothermal: T)   */
  const double *Y_in;/* [N] inlet mass fractions            */
  int energy;        /* 0: isothermal, unknowns Y; 1: (Y, T) with the energy
                        balance; 2: (Y, T) with T prescribed (T = T_in)    */
} om_cond;

typedef struct {
  /* steady Newton attempt */
  double rtol, atol_Y, atol_T; /* step-norm weights w = atol + rtol |x|        */
  double ftol;                 /* scaled-residual bound for convergence        */
  double lambda_min;           /* smallest damping factor tried (<= 0: undamped) */
  double T_min, T_max;         /* temperature bounds, K                        */
  /* pseudo-transient (ROS2) conditioning */
  double ts_rtol, ts_atol_Y, ts_atol_T; /* local-error weights                 */
  double ts_neg_tol;           /* most negative mass fraction accepted         */
  double h0, h_max;            /* first and largest step, in units of tau      */
  double h_min;                /* smallest step before TS_FAILED, in seconds   */
  double nw_h_ratio;           /* retry Newton only once h >= nw_h_ratio tau   */
  int nw_max_it;               /* iterations per Newton attempt                */
  int nw_every;                /* accepted steps between Newton attempts       */
  int max_lin;                 /* total linear-solve budget                    */
  double atol_lnM;             /* step-norm weight offset of the ln M_r unknowns */
  double ts_atol_lnM;          /* local-error weight offset of the ln M_r unknowns */
  double lnM_step;             /* largest change of a ln M_r in one Newton step */
  /* continuation in tau (gas-phase reactors; off when ct_ratio <= 1)      */
  double ct_ratio;             /* largest factor between continuation rungs    */
  double ct_tau_min;           /* smallest residence time of a rung, s         */
  double ct_min_step;          /* smallest step in ln tau before giving up     */
} om_opts;

enum { OM_CONVERGED = 0, OM_MAXITER = 1, OM_TS_FAILED = 2, OM_NONFINITE = 3, OM_SINGULAR = 4 };

typedef struct {
  int status;
  int n_lin;      /* linear solves (residual + triangular solve pairs)      */
  int n_jac;      /* Jacobian evaluations + factorisations                  */
  int n_ts;       /* accepted pseudo-transient steps                        */
  int n_attempts; /* Newton attempts started                                */
  double sres;    /* scaled residual at the converged base point            */
} om_stats;

void om_prepare(om_mech *m);
void om_default_opts(om_opts *o);
int om_n_unknowns(const om_mech *m, int energy);

void om_thermo(const om_mech *m, double T, double *cp_R, double *h_RT, double *s_R);
void om_rate_constants(const om_mech *m, double T, double *kf, double *Kc, double *kr);
void om_production(const om_mech *m, double T, double P, const double *Y,
                   double *C, double *q, double *wdot);
void om_residual(const om_mech *m, const om_cond *c, const double *x, double *F);
double om_scaled_residual(const om_mech *m, const om_cond *c, const double *x);
void om_jacobian(const om_mech *m, const om_cond *c, const double *x, double *J);
void om_jacobian_complex_step(const om_mech *m, const om_cond *c, const double *x, double *J);
void om_mass_diag(const om_mech *m, const om_cond *c, const double *x, double *M);
/* (f_v, N, d) of a sooting reactor from its ln M_0..ln M_5 */
void om_soot_outputs(const om_mech *m, const double *lnM, double *out);

/* MOMIC pieces, exported for the tests.  lnM: [6] ln M_r.               */
double om_soot_ln_mu(const double *lnM, double p);
double om_soot_fxy(const double *lnM, int x, int y);
void om_soot_sources(const om_mech *m, double T, double CP, double CG, const double *lnM,
                     double *R, double *Wg, double *G, double *sinks);

int om_lu_factor(int n, double *a, int *piv);
void om_lu_solve(int n, const double *lu, const int *piv, double *b);

int om_solve(const om_mech *m, const om_cond *c, const om_opts *o, double *x, om_stats *st);
int om_time_march_only(const om_mech *m, const om_cond *c, const om_opts *o, double *x,
                       int max_steps, om_stats *st);

#ifdef __cplusplus
}
#endif
#endif
