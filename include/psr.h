/* psr.h - C ABI of the MI355X (gfx950) batched perfectly-stirred-reactor solver.
 *
 * The library solves, for many independent reactors at once, the steady
 * state of the PSR species and energy balances (paper: Section 2, Eqs. 1-3)
 * with mass-action kinetics (Section 3, Eqs. 4-9), by the hybrid Newton /
 * pseudo-transient method of Section 3.  All compute runs in hand-written
 * HIP kernels; this header uses plain C types only.
 *
 * Conventions
 *   - Every function returns psr_status; PSR_OK is 0.  Nothing throws across
 *     the ABI.  On a non-OK status psr_last_error() returns a message
 *     (thread-local, valid until the next call on that thread).
 *   - "device pointer" means memory allocated on the current HIP device
 *     (e.g. a torch tensor's data_ptr()); "host pointer" means CPU memory.
 *     The caller owns every array it passes; the library keeps no pointer to
 *     caller memory after a call returns, except that launches on `stream`
 *     may still be running after an asynchronous call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *   - Batch arrays use the structure-of-arrays layout [var][reactor]:
 *     element (i, b) of an [n][B] array is at index i*B + b.
 *   - Units: P in Pa, tau in s, T in K, mass fractions dimensionless,
 *     A in (cm^3/mol)^(order-1)/s, E in J/mol, NASA-7 coefficients for
 *     c_p/R, H/RT, S/R.  Concentrations are mol/cm^3; the reactor volume is
 *     1 cm^3 (it cancels from the steady state).
 */
#ifndef PSR_H
#define PSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSR_OK = 0,
  PSR_EINVAL = 1,       /* invalid argument or mechanism                    */
  PSR_ENOMEM = 2,       /* device allocation failed / workspace too small    */
  PSR_EDEVICE = 3,      /* a HIP call failed                                 */
  PSR_EUNSUPPORTED = 4  /* valid request outside what this library supports  */
} psr_status;

/* Per-reactor outcome written to psr_group.status. */
enum {
  PSR_R_CONVERGED = 0, /* root found: weighted Newton step <= 1 and scaled residual <= ftol */
  PSR_R_MAXITER = 1,   /* linear-solve budget spent                                         */
  PSR_R_TS_FAILED = 2, /* pseudo-transient step size fell below h_min                        */
  PSR_R_NONFINITE = 3, /* converged iterate not finite, or inputs outside the domain: P, tau or
                          T_in not positive and finite, or Y_in or the initial x not finite (x
                          is then left as given and no work is done for the reactor)          */
  PSR_R_SINGULAR = 4   /* pseudo-transient step size fell below h_min after a step rejected
                          because its matrix had no nonzero pivot                          */
};

enum { PSR_FP64 = 0, PSR_MIXED = 1 };        /* precision of the LU factorisation */
enum { PSR_PLAIN = 0, PSR_PERSISTENT = 1 };  /* scheduler                          */

typedef struct psr_mech *psr_mech_t; /* opaque; immutable after creation */

/* Soot particles coupled to the gas phase (the paper's sooting reactor,
 * Sections 1-2 and 6, modelled with Frenklach's method of moments with
 * interpolative closure, MOMIC).  Six extra unknowns per reactor, ln M_r for
 * r = 0..5, where M_r = sum_i m_i^r N_i per cm^3 with particle mass m in
 * carbon atoms; only for reactors with a temperature unknown (energy 1 or
 * 2).  Source terms:
 *   nucleation   I = k_n [P]^2 (mol/cm^3/s) from two molecules of the
 *                pure-carbon precursor P; nucleus of C = 2 n_C(P) atoms;
 *                R_r = N_A I C^r; P consumed at 2 I
 *   growth       by the pure-carbon species G, D = n_C(G) atoms per step:
 *                W_r = k_s [G] chi pi d^2 M_0 sum_{l<r} C(r,l) D^(r-l) mu_{l+2/3},
 *                d = (6 m_C/(pi rho_s))^(1/3); G consumed at W_1/(D N_A)
 *   coagulation  free-molecular, G_0 = -K_f M_0^2 f_00 / 2, G_1 = 0,
 *                G_r = K_f M_0^2 sum_{k=1}^{r-1} C(r,k) f_{k,r-k} / 2,
 *                K_f = 2.2 (3 m_C/(4 pi rho_s))^(1/6) (6 k_B T/rho_s)^(1/2) * coag_scale
 * with the reduced moments mu_p = M_p/M_0 of fractional order p from the
 * Lagrange interpolation of ln mu_l over l = 0..5 (p >= 0) or l = 0..2
 * (p < 0), and f_{x,y} the log-Lagrange interpolation at 1/2 of the
 * coagulation grid functions over l = 0..3.  Growth and coagulation are off
 * while M_0 < 1 per cm^3.  Soot has zero enthalpy.  Moment rows of the
 * residual: F_{M_r} = V (M_r/tau - R_r - W_r - G_r).                      */
typedef struct {
  int32_t precursor;      /* species index of P (carbon atoms only)          */
  int32_t growth;         /* species index of G (carbon atoms only)          */
  int32_t carbon;         /* element index of carbon                         */
  double A_nuc, beta_nuc, E_nuc;    /* k_n = A T^beta exp(-E/RT), cm^3/(mol s), J/mol */
  double A_grow, beta_grow, E_grow; /* k_s per surface site, same units      */
  double site_density;    /* chi, sites per cm^2                             */
  double soot_density;    /* rho_s, g/cm^3                                   */
  double coag_scale;      /* factor on the coagulation kernel (1 = Frenklach's) */
} psr_soot_desc;

/* Mechanism description (host pointers, copied at creation).
 * Reactions are elementary and reversible (Eqs. 4-7): up to three distinct
 * reactant species and three distinct product species, each with a positive
 * integer coefficient; index -1 marks an unused slot.                       */
typedef struct {
  int32_t n_elements, n_species, n_reactions;
  const double *elem_weight;     /* [E] g/mol                                  */
  const int32_t *species_elems;  /* [N][E] atom counts; W_i = sum_e a_ie W_e   */
  const double *nasa7;           /* [N][7] a1..a7, single range                */
  double t_low, t_high;          /* validity range of the polynomials, K       */
  const int32_t *reac_idx;       /* [I][3] reactant species or -1              */
  const int32_t *reac_nu;        /* [I][3] reactant coefficients (>= 1)        */
  const int32_t *prod_idx;       /* [I][3] product species or -1               */
  const int32_t *prod_nu;        /* [I][3] product coefficients (>= 1)         */
  const double *A;               /* [I] pre-exponential factor (Eq. 6)         */
  const double *beta;            /* [I] temperature exponent (Eq. 6)           */
  const double *Ea;              /* [I] activation energy, J/mol (Eq. 6)       */
  const psr_soot_desc *soot;     /* NULL: gas phase only                       */
} psr_mech_desc;

/* Validate and upload a mechanism to the current device.
 * Checks: counts positive, indices in range, coefficients >= 1, no species
 * on both sides of a reaction, every reaction balanced in every element,
 * positive species weights, t_low < t_high.  Errors: PSR_EINVAL (with the
 * offending reaction or species in psr_last_error), PSR_EDEVICE. */
psr_status psr_create_mechanism(const psr_mech_desc *desc, psr_mech_t *out);
psr_status psr_destroy_mechanism(psr_mech_t mech);

/* Number of unknowns per reactor: N (isothermal), N + 1 (energy 1 or 2) or
 * N + 7 (energy 1 or 2 with soot: Y, T, ln M_0..ln M_5).  Soot mechanisms
 * require a temperature unknown (the residual, Jacobian and solve calls
 * return PSR_EINVAL otherwise). */
int32_t psr_num_unknowns(psr_mech_t mech, int32_t energy);

/* Reactor conditions: device pointers, [B] or [N][B]. */
typedef struct {
  int64_t n_reactors;  /* B >= 1                                               */
  int32_t energy;      /* 0: isothermal at T = T_in, unknowns Y;
                          1: unknowns (Y, T), energy balance (Eq. 3);
                          2: unknowns (Y, T), reactor temperature prescribed: T = T_in
                             through the row F_T = V (T - T_in) / tau (the set-temperature
                             sooting reactors of the Section 5 sweeps; the root is the
                             isothermal root with T = T_in).  Mode 2 runs on the
                             workgroup engine. */
  const double *P;     /* [B] pressure, Pa                                     */
  const double *tau;   /* [B] residence time, s                                */
  const double *T_in;  /* [B] inlet temperature (isothermal: reactor T), K     */
  const double *Y_in;  /* [N][B] inlet mass fractions                          */
} psr_conditions;

/* Steady PSR residual F(x) (Eq. 2 and Eq. 3 multiplied by -rho V):
 *   F_i = mdot (Y_i - Y_in,i) - V W_i wdot_i,   mdot = rho V / tau
 *   F_T = mdot sum_i Y_in,i (h_i(T) - h_i(T_in)) + V sum_i H_i(T) wdot_i
 * with wdot from Eqs. 4-9.  x, F: device [n][B].  scaled: optional device
 * [B], each reactor's residual relative to the magnitudes of the terms that
 * make it up (max over equations).  Asynchronous on `stream`.             */
psr_status psr_residual(psr_mech_t mech, const psr_conditions *cond, const double *x, double *F,
                        double *scaled, void *stream);

/* Analytic Jacobian dF/dx of psr_residual at x.  J: device [B][n][n],
 * row-major per reactor (J[b*n*n + r*n + c] = dF_r/dx_c).  Asynchronous. */
psr_status psr_jacobian(psr_mech_t mech, const psr_conditions *cond, const double *x, double *J,
                        void *stream);

/* Finite-difference Jacobian, the route the paper takes (Section 1): n + 1
 * residual evaluations per reactor, column j = (F(x + h_j e_j) - F(x)) / h_j
 * with h_j = (x_j + d_j) - x_j, d_j = 2^-26 max(|x_j|, f_j), f_j = 1e-10 for
 * the species rows and 1 for the temperature and ln M_r rows.  x: device
 * [n][B]; J: device [B][n][n] as in psr_jacobian; work: device scratch of
 * 3 n B doubles owned by the caller (F(x), F of the perturbed state, the
 * perturbed state), contents undefined on return.  Asynchronous on
 * `stream`; errors as psr_residual, PSR_EINVAL for a null x, J or work. */
psr_status psr_jacobian_fd(psr_mech_t mech, const psr_conditions *cond, const double *x, double *J,
                           double *work, void *stream);

/* Soot outputs of a batch of sooting reactors (the quantities of the Section 5
 * sweeps, Figs. 1-2), from the moments of states x (device [n][B], n = N + 7):
 *   out[0][b] = f_v = M_1 m_C / rho_s       soot volume fraction
 *   out[1][b] = N   = M_0                   particle number density, cm^-3
 *   out[2][b] = d   = (6 f_v / (pi N))^(1/3) diameter of a sphere of the
 *                                            mean particle volume, cm
 * out: device [3][B], written by the call.  Asynchronous on `stream`.
 * Errors: PSR_EINVAL (null pointer, B < 1, mechanism without soot). */
psr_status psr_soot_outputs(psr_mech_t mech, int64_t n_reactors, const double *x, double *out, void *stream);

/* psr_jacobian_fd for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, with the 3 n B work doubles in a static device array of
 * 4 Mi doubles (32 MiB) that each device the library runs on holds until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or other
 * allocating routine); the first call on a device looks up that array's
 * address for the device.  Errors: those of psr_jacobian_fd, PSR_EINVAL for
 * a null x or J and when 3 n B exceeds 4194304 (nothing is launched then),
 * PSR_EDEVICE if the address lookup fails.  Every call on one device shares
 * that device's array and its contents are undefined after a call: calls
 * whose launches overlap on one device (two streams, two host threads) race
 * and give wrong Jacobians; serialise them. */
psr_status psr_jacobian_fd_noalloc(psr_mech_t mech, const psr_conditions *cond, const double *x, double *J,
                                   void *stream);

/* Batched LU with partial pivoting of B independent n x n row-major
 * matrices (device [B][n][n], overwritten by L\U with unit-lower L), pivots
 * device [B][n] (LAPACK convention: row k was swapped with row piv[k]),
 * info device [B] (0, or k+1 if column k had no nonzero pivot; the
 * factors and pivots from column k on are then unspecified).
 * precision PSR_FP64 factors in double; PSR_MIXED rounds each matrix to
 * float, factors in float and writes the float factors back as double.
 * Asynchronous.  For PSR_MIXED with 64 < n <= 256 and PSR_FP64 with
 * 64 < n <= 128 the factorisation works (one wavefront per matrix) in a
 * library-owned device buffer, one per (device, stream) pair, allocated
 * on the first such call and grown on demand (that call synchronises the
 * stream before freeing the smaller buffer); calls on one stream are ordered
 * and calls on different streams use different buffers, so concurrent calls
 * on different streams or host threads do not share scratch memory. */
psr_status psr_lu_factor_batch(int32_t n, int64_t batch, int32_t precision, double *A, int32_t *piv,
                               int32_t *info, void *stream);

/* Solve with the factors of psr_lu_factor_batch: b (device [B][n]) is
 * overwritten with the solution (interchanges in order, then forward and
 * back substitution; one wavefront per matrix).  Asynchronous.  n <= 256;
 * larger n returns PSR_EUNSUPPORTED, null pointers or n, B <= 0
 * PSR_EINVAL.                                                              */
psr_status psr_lu_solve_batch(int32_t n, int64_t batch, const double *LU, const int32_t *piv,
                              double *b, void *stream);

typedef struct {
  int32_t precision;  /* PSR_FP64 or PSR_MIXED                              */
  int32_t scheduler;  /* PSR_PLAIN or PSR_PERSISTENT                        */
  /* steady Newton attempt.  Every factorisation of the solve (Newton and
   * pseudo-transient, FP64 and FP32) works on the matrix scaled by powers of
   * two in its rows, then its columns, so that each has largest magnitude
   * in [1/2, 1). */
  double rtol, atol_Y, atol_T; /* step-norm weights w = atol + rtol |x|         */
  double ftol;                 /* scaled-residual bound for convergence         */
  double lambda_min;           /* 0 (default): every Newton step is taken at the
                                  length the bounds allow (T inside [T_min,
                                  T_max], |d ln M_r| <= lnM_step), mass
                                  fractions projected onto Y >= 0; > 0: that
                                  length is halved until the natural criterion
                                  holds, down to lambda_min                     */
  double T_min, T_max;         /* temperature bounds, K                         */
  /* pseudo-transient (ROS2) conditioning */
  double ts_rtol, ts_atol_Y, ts_atol_T; /* local-error weights                  */
  double ts_neg_tol;           /* most negative mass fraction accepted          */
  double h0, h_max;            /* first and largest step, in units of tau       */
  double h_min;                /* smallest step before TS_FAILED, s             */
  double nw_h_ratio;           /* retry Newton only once h >= nw_h_ratio * tau  */
  int32_t nw_max_it;           /* iterations per Newton attempt                 */
  int32_t nw_every;            /* accepted steps between Newton attempts        */
  int32_t max_lin;             /* per-reactor linear-solve budget               */
  /* mixed precision */
  int32_t max_refine;          /* refinement sweeps per solve before FP64 fallback */
  /* kernel engine: 0 automatic (wavefront engine when n <= 64 and the
   * mechanism fits its LDS, else one workgroup per reactor), 1 one workgroup
   * of 256 threads per reactor, 2 one wavefront per reactor (PSR_EUNSUPPORTED
   * if it does not fit). Results agree to rounding, not bitwise. */
  int32_t engine;
  /* plain scheduler: 1 replays the rounds between two host checks as one
   * captured HIP graph on a library stream (ordered after `stream`), 0
   * launches them one by one on `stream`.  Results are identical. */
  int32_t use_graph;
  /* mixed precision: refinement stops once the max-norm correction is below
   * refine_tol times the max norm of the solution (default 1e-6: enough to
   * steer the Newton and pseudo-transient iterations).  A Newton step that
   * passes the convergence tests is re-solved with refinement to 1e-10
   * before it is accepted, so the converged state does not depend on
   * refine_tol. */
  double refine_tol;
  /* soot: step-norm and local-error weight offsets of the ln M_r unknowns */
  double atol_lnM, ts_atol_lnM;
  /* launch shape, 0 = automatic (psr_autotune measures and picks these):
   * rpw: wavefront engine, reactors (one wavefront each) per workgroup that
   * share one LDS copy of the mechanism tables, 1, 2 or 4; when the asked
   * number does not fit the LDS the largest smaller one that fits is used.
   * grid_per_cu: persistent scheduler, resident workgroups per compute unit
   * (1..32), capped by what fits.  Results are bitwise independent of both;
   * they change only speed. */
  int32_t rpw;
  int32_t grid_per_cu;
  /* soot: largest change of a ln M_r in one Newton step (the step length is
   * cut so that every |lambda d ln M_r| <= lnM_step) */
  double lnM_step;
  /* continuation in the residence time (gas-phase reactors; off when
   * ct_ratio <= 1).  When a reactor's first Newton attempt fails, Newton
   * attempts from the initial guess at tau / ct_ratio^k, k = 1, 2, ... (not
   * below ct_tau_min seconds) until one converges; from that root tau is
   * raised back in steps of at most a factor ct_ratio, each solved by a
   * Newton attempt from the root before, a failed step retried at half its
   * length in ln tau until it falls below ct_min_step.  The pseudo-transient
   * steps start from the last root (else the initial guess) when this ends
   * short of the reactor's tau. */
  double ct_ratio, ct_tau_min, ct_min_step;
  /* persistent scheduler, order in which reactors are taken from the device
   * queue: 1 = longest residence time first (descending tau, ties by batch
   * index; a reactor's solve cost grows with tau, so the long solves start
   * first and the short ones fill the tail), groups of several mechanisms
   * taken largest n first; 0 = batch order.  The ordering reads tau back
   * to the host once per call.  Results are bitwise independent of it.
   * A persistent call with 2 to 4 groups, at most one of them on the
   * wavefront engine, and the automatic launch shape (engine, rpw and
   * grid_per_cu all 0) runs as ONE launch over one device queue: the
   * workgroup-engine groups' reactors first, then the wavefront-engine
   * group's, each workgroup switching to four independent wavefronts when it
   * reaches them.  Other multi-group persistent calls launch one kernel per
   * group, side by side.  Both give the same bits per reactor. */
  int32_t order;
  /* mixed precision: the largest system size n factored in FP32 first
   * (default 64, the wavefront engine's range).  Larger systems are factored
   * in FP64 directly: after equilibration their Jacobians (100 to 201
   * unknowns here) reach condition numbers near 1e13, 78-80 % of the float
   * attempts fall back to FP64, and the float attempt plus its refinement
   * costs more than it saves.  Such factorisations are not counted as
   * fallbacks in psr_solve_stats. */
  int32_t mixed_max_n;
} psr_solve_opts;

/* Fill opts with the defaults (FP64, plain scheduler, graph replay on,
 * automatic engine, tolerances above). */
void psr_default_opts(psr_solve_opts *opts);

/* One mechanism's reactors in a solve.  Device pointers. */
typedef struct {
  psr_mech_t mech;
  psr_conditions cond;
  double *x_inout;   /* [n][B] initial guess in, result out            */
  int32_t *status;   /* [B] PSR_R_* per reactor                         */
  int32_t *n_lin;    /* [B] linear solves used per reactor (may be NULL) */
} psr_group;

typedef struct {
  int64_t reactors, converged;
  int64_t lin_total, lin_max;   /* linear solves summed / worst reactor       */
  int64_t jac_total;            /* Jacobian evaluations + factorisations      */
  int64_t fp64_fallbacks;       /* mixed mode: matrices refactored in FP64    */
  int32_t rounds;               /* plain scheduler: host-driven rounds        */
  double kernel_ms;             /* device time of the solve, from HIP events  */
} psr_solve_stats;

/* Workspace (device bytes) psr_solve_batch needs for these groups/opts. */
size_t psr_workspace_bytes(const psr_group *groups, int32_t n_groups, const psr_solve_opts *opts);

/* Solve every reactor of every group.  workspace: device buffer of at
 * least psr_workspace_bytes() bytes (else PSR_ENOMEM).  Blocks until the
 * solve is complete on `stream`.  With the persistent scheduler and several
 * groups, each group runs in its own workspace region on its own library
 * stream (default priority, ordered after `stream` and joined back into it),
 * so the groups' launches overlap; otherwise groups run in turn.  A reactor
 * that does not converge is not an API error: its status says why.  stats
 * (host, optional) receives totals; kernel_ms spans the whole call. */
psr_status psr_solve_batch(const psr_group *groups, int32_t n_groups, const psr_solve_opts *opts,
                           void *workspace, size_t workspace_bytes, psr_solve_stats *stats,
                           void *stream);

/* Parameter a continuation sweep varies. */
enum { PSR_SWEEP_T_IN = 0, PSR_SWEEP_TAU = 1 };

/* Continuation sweep (paper Section 5: steady solutions followed along the
 * reactor temperature at a fixed residence time, and along the residence
 * time at a fixed temperature, each solution started from the one before).
 * group: one mechanism's B reactors, each the start of its own chain.  At
 * step k = 0..n_steps-1 the condition named by `param` (T_in, which for
 * isothermal reactors is the reactor temperature, or tau) is taken from
 * values + k*B (device, [n_steps][B] float64); the group's own pointer for
 * that condition is ignored and may be NULL.  group->x_inout holds the
 * initial guess of step 0 and, on return, the state the last step left;
 * every step starts from the state the step before left, whether or not
 * that reactor converged there (status_path says).  x_path (device
 * [n_steps][n][B], may be NULL) and status_path (device [n_steps][B], may
 * be NULL) receive each step's state and status; group->status and
 * group->n_lin hold the last step's.  workspace: at least
 * psr_workspace_bytes() of the group (the same at every step).  stats (host,
 * optional): reactors, converged, lin_total, jac_total, fp64_fallbacks,
 * rounds and kernel_ms summed over the steps, lin_max the largest.  Blocks
 * until the last step is complete on `stream`.  Errors: PSR_EINVAL for a
 * bad param, n_steps < 1 or a null `values`, else those of psr_solve_batch
 * (the sweep stops at the failing step). */
psr_status psr_sweep_batch(const psr_group *group, int32_t param, int32_t n_steps, const double *values,
                           const psr_solve_opts *opts, void *workspace, size_t workspace_bytes,
                           double *x_path, int32_t *status_path, psr_solve_stats *stats, void *stream);

/* Outcome of psr_autotune. */
typedef struct {
  int32_t engine, rpw, grid_per_cu; /* the chosen launch shape (as in opts)       */
  int32_t candidates;               /* shapes timed; 0 = taken from the cache     */
  double ms;                        /* sample solve time of the chosen shape      */
  double solves_per_s;              /* converged sample reactors per second       */
  double default_ms;                /* sample solve time of the automatic shape
                                       (0 when taken from the cache)              */
} psr_tune_result;

/* Launch-shape autotuner for the batch scheduling of the solve (the reactors
 * are independent, paper §1 and §4, so only speed depends on how they are
 * packed onto the GPU).  Solves the first `sample` reactors of every group
 * (1 <= sample; larger than a group's size means the whole group) under each
 * candidate shape -- engine (wavefront engine where it fits, or one
 * workgroup per reactor), rpw, and for the persistent scheduler grid_per_cu
 * -- one untimed run then the best of two timed ones, and writes the shape
 * with the most converged reactor-solves per second into opts->engine,
 * opts->rpw and opts->grid_per_cu (the other fields of opts are used as
 * given).  The caller's x_inout, status and n_lin are not touched: the
 * sample runs on copies.  cache_path (may be NULL): a text file of earlier
 * results, one line per key (device, compute units, each group's mechanism
 * sizes, energy flag and sample size, precision, scheduler); a hit is used
 * without timing, a miss is appended.  Allocates and frees its own device
 * buffers (not for use under stream capture); synchronises `stream`.
 * result (host, optional) receives the choice.  Errors: PSR_EINVAL for bad
 * arguments or an unreadable/unwritable cache file, PSR_EDEVICE for HIP
 * failures, any error of psr_solve_batch for a candidate that every shape
 * rejects. */
psr_status psr_autotune(const psr_group *groups, int32_t n_groups, psr_solve_opts *opts, int64_t sample,
                        const char *cache_path, psr_tune_result *result, void *stream);

/* Message for the last non-OK status on this thread ("" if none). */
const char *psr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
