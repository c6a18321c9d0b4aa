"""Python access to the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library; it reads the same seeded inputs (psr_inputs).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["psr_oracle.c"]
DEPENDS = ["psr_oracle.c", "psr_oracle.h", "residual_body.inc"]

STATUS = {0: "CONVERGED", 1: "MAXITER", 2: "TS_FAILED", 3: "NONFINITE", 4: "SINGULAR"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no vectorisation flags, no OpenMP)."""
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(os.path.join(HERE, f)) for f in DEPENDS)
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp,
           *[os.path.join(HERE, s) for s in SOURCES], "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Soot(C.Structure):
    _fields_ = [("precursor", C.c_int), ("growth", C.c_int), ("carbon", C.c_int),
                ("A_nuc", C.c_double), ("beta_nuc", C.c_double), ("E_nuc", C.c_double),
                ("A_grow", C.c_double), ("beta_grow", C.c_double), ("E_grow", C.c_double),
                ("site_density", C.c_double), ("soot_density", C.c_double),
                ("coag_scale", C.c_double)]


class _Mech(C.Structure):
    _fields_ = [("n_el", C.c_int), ("n_sp", C.c_int), ("n_rx", C.c_int),
                ("elem_w", C.POINTER(C.c_double)), ("sp_el", C.POINTER(C.c_int)),
                ("nasa", C.POINTER(C.c_double)),
                ("r_idx", C.POINTER(C.c_int)), ("r_nu", C.POINTER(C.c_int)),
                ("p_idx", C.POINTER(C.c_int)), ("p_nu", C.POINTER(C.c_int)),
                ("A", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("Ea", C.POINTER(C.c_double)), ("soot", C.POINTER(_Soot)),
                ("W", C.POINTER(C.c_double))]


class _Cond(C.Structure):
    _fields_ = [("P", C.c_double), ("tau", C.c_double), ("T_in", C.c_double),
                ("Y_in", C.POINTER(C.c_double)), ("energy", C.c_int)]


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("ftol", C.c_double), ("lambda_min", C.c_double),
                ("T_min", C.c_double), ("T_max", C.c_double),
                ("ts_rtol", C.c_double), ("ts_atol_Y", C.c_double), ("ts_atol_T", C.c_double),
                ("ts_neg_tol", C.c_double),
                ("h0", C.c_double), ("h_max", C.c_double), ("h_min", C.c_double),
                ("nw_h_ratio", C.c_double),
                ("nw_max_it", C.c_int), ("nw_every", C.c_int), ("max_lin", C.c_int),
                ("atol_lnM", C.c_double), ("ts_atol_lnM", C.c_double),
                ("lnM_step", C.c_double), ("ct_ratio", C.c_double),
                ("ct_tau_min", C.c_double), ("ct_min_step", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("n_lin", C.c_int), ("n_jac", C.c_int),
                ("n_ts", C.c_int), ("n_attempts", C.c_int), ("sres", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        mp, cp = C.POINTER(_Mech), C.POINTER(_Cond)
        L.om_prepare.argtypes = [mp]
        L.om_default_opts.argtypes = [C.POINTER(Opts)]
        L.om_thermo.argtypes = [mp, C.c_double, dp, dp, dp]
        L.om_rate_constants.argtypes = [mp, C.c_double, dp, dp, dp]
        L.om_production.argtypes = [mp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.om_residual.argtypes = [mp, cp, dp, dp]
        L.om_scaled_residual.argtypes = [mp, cp, dp]
        L.om_scaled_residual.restype = C.c_double
        L.om_jacobian.argtypes = [mp, cp, dp, dp]
        L.om_jacobian_complex_step.argtypes = [mp, cp, dp, dp]
        L.om_mass_diag.argtypes = [mp, cp, dp, dp]
        L.om_soot_ln_mu.argtypes = [dp, C.c_double]
        L.om_soot_ln_mu.restype = C.c_double
        L.om_soot_fxy.argtypes = [dp, C.c_int, C.c_int]
        L.om_soot_fxy.restype = C.c_double
        L.om_soot_sources.argtypes = [mp, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp, dp]
        L.om_soot_outputs.argtypes = [mp, dp, dp]
        L.om_lu_factor.argtypes = [C.c_int, dp, ip]
        L.om_lu_factor.restype = C.c_int
        L.om_lu_solve.argtypes = [C.c_int, dp, ip, dp]
        L.om_solve.argtypes = [mp, cp, C.POINTER(Opts), dp, C.POINTER(Stats)]
        L.om_time_march_only.argtypes = [mp, cp, C.POINTER(Opts), dp, C.c_int, C.POINTER(Stats)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def default_opts(**overrides) -> Opts:
    o = Opts()
    lib().om_default_opts(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class Mechanism:
    """Holds the mechanism arrays alive for the C struct that points at them."""

    def __init__(self, mech: dict):
        f64 = lambda k: np.ascontiguousarray(mech[k], dtype=np.float64)
        i32 = lambda k: np.ascontiguousarray(mech[k], dtype=np.int32)
        self._keep = dict(elem_w=f64("elem_weight"), sp_el=i32("species_elems"),
                          nasa=f64("nasa7"), r_idx=i32("reac_idx"), r_nu=i32("reac_nu"),
                          p_idx=i32("prod_idx"), p_nu=i32("prod_nu"), A=f64("A"),
                          beta=f64("beta"), Ea=f64("Ea"))
        self.n_sp = self._keep["sp_el"].shape[0]
        self.n_el = self._keep["sp_el"].shape[1]
        self.n_rx = self._keep["r_idx"].shape[0]
        self.W = np.zeros(self.n_sp)
        k = self._keep
        sd = mech.get("soot")
        self.soot = None if sd is None else _Soot(*(sd[name] for name, _ in _Soot._fields_))
        sp = C.pointer(self.soot) if self.soot is not None else C.POINTER(_Soot)()
        self.s = _Mech(self.n_el, self.n_sp, self.n_rx, _dp(k["elem_w"]), _ip(k["sp_el"]),
                       _dp(k["nasa"]), _ip(k["r_idx"]), _ip(k["r_nu"]), _ip(k["p_idx"]),
                       _ip(k["p_nu"]), _dp(k["A"]), _dp(k["beta"]), _dp(k["Ea"]), sp, _dp(self.W))
        lib().om_prepare(C.byref(self.s))

    # -- pointwise functions ------------------------------------------------
    def thermo(self, T):
        cp, h, s = (np.zeros(self.n_sp) for _ in range(3))
        lib().om_thermo(C.byref(self.s), float(T), _dp(cp), _dp(h), _dp(s))
        return cp, h, s

    def rate_constants(self, T):
        kf, Kc, kr = (np.zeros(self.n_rx) for _ in range(3))
        lib().om_rate_constants(C.byref(self.s), float(T), _dp(kf), _dp(Kc), _dp(kr))
        return kf, Kc, kr

    def production(self, T, P, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        Cc, wdot = np.zeros(self.n_sp), np.zeros(self.n_sp)
        q = np.zeros(self.n_rx)
        lib().om_production(C.byref(self.s), float(T), float(P), _dp(Y), _dp(Cc), _dp(q), _dp(wdot))
        return Cc, q, wdot

    def n_unknowns(self, energy):
        return self.n_sp + (1 if energy else 0) + (6 if energy and self.soot is not None else 0)

    # -- soot moments (MOMIC) -------------------------------------------------
    def soot_outputs(self, x):
        """(f_v, N, d) per reactor of states x [n][B] (or one state [n]) of a
        sooting mechanism with a T unknown: volume fraction, number density
        (cm^-3) and mean-volume sphere diameter (cm)."""
        x = np.asarray(x, dtype=np.float64)
        X = x.reshape(x.shape[0], -1)
        out = np.zeros((3, X.shape[1]))
        for b in range(X.shape[1]):
            lnM = np.ascontiguousarray(X[self.n_sp + 1:self.n_sp + 7, b])
            o = np.zeros(3)
            lib().om_soot_outputs(C.byref(self.s), _dp(lnM), _dp(o))
            out[:, b] = o
        return out if x.ndim == 2 else out[:, 0]

    def soot_sources(self, T, CP, CG, lnM):
        """(R, W, G, sinks): nucleation, growth and coagulation sources of the
        six moments, and the precursor / growth-species sinks (mol/cm^3/s)."""
        lnM = np.ascontiguousarray(lnM, dtype=np.float64)
        R, Wg, G, sk = np.zeros(6), np.zeros(6), np.zeros(6), np.zeros(2)
        lib().om_soot_sources(C.byref(self.s), float(T), float(CP), float(CG), _dp(lnM), _dp(R),
                              _dp(Wg), _dp(G), _dp(sk))
        return R, Wg, G, sk

    def _cond(self, P, tau, T_in, Y_in, energy):
        Y_in = np.ascontiguousarray(Y_in, dtype=np.float64)
        return _Cond(float(P), float(tau), float(T_in), _dp(Y_in), int(energy)), Y_in

    def residual(self, P, tau, T_in, Y_in, energy, x):
        c, keep = self._cond(P, tau, T_in, Y_in, energy)
        x = np.ascontiguousarray(x, dtype=np.float64)
        F = np.zeros(self.n_unknowns(energy))
        lib().om_residual(C.byref(self.s), C.byref(c), _dp(x), _dp(F))
        return F

    def scaled_residual(self, P, tau, T_in, Y_in, energy, x):
        c, keep = self._cond(P, tau, T_in, Y_in, energy)
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().om_scaled_residual(C.byref(self.s), C.byref(c), _dp(x))

    def jacobian(self, P, tau, T_in, Y_in, energy, x, complex_step=False):
        c, keep = self._cond(P, tau, T_in, Y_in, energy)
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = self.n_unknowns(energy)
        J = np.zeros((n, n))
        fn = lib().om_jacobian_complex_step if complex_step else lib().om_jacobian
        fn(C.byref(self.s), C.byref(c), _dp(x), _dp(J))
        return J

    def jacobian_fd(self, P, tau, T_in, Y_in, energy, x):
        """Forward-difference Jacobian, the paper's route (Section 1): column j
        is (F(x + h_j e_j) - F(x)) / h_j, n + 1 residual evaluations.  Step:
        h_j = (x_j + d_j) - x_j with d_j = 2^-26 max(|x_j|, f_j), f_j = 1e-10
        for species rows and 1 for the temperature and ln M_r rows."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = self.n_unknowns(energy)
        F0 = self.residual(P, tau, T_in, Y_in, energy, x)
        J = np.zeros((n, n))
        for j in range(n):
            floor = 1e-10 if j < self.n_sp else 1.0
            d = 2.0 ** -26 * max(abs(x[j]), floor)
            h = (x[j] + d) - x[j]
            xp = x.copy()
            xp[j] = x[j] + h
            J[:, j] = (self.residual(P, tau, T_in, Y_in, energy, xp) - F0) / h
        return J

    def mass_diag(self, P, tau, T_in, Y_in, energy, x):
        c, keep = self._cond(P, tau, T_in, Y_in, energy)
        x = np.ascontiguousarray(x, dtype=np.float64)
        M = np.zeros(self.n_unknowns(energy))
        lib().om_mass_diag(C.byref(self.s), C.byref(c), _dp(x), _dp(M))
        return M

    def solve(self, P, tau, T_in, Y_in, energy, x0, opts: Opts | None = None):
        c, keep = self._cond(P, tau, T_in, Y_in, energy)
        x = np.array(x0, dtype=np.float64, copy=True)
        st = Stats()
        lib().om_solve(C.byref(self.s), C.byref(c), C.byref(opts or default_opts()), _dp(x),
                       C.byref(st))
        return x, st

    def time_march(self, P, tau, T_in, Y_in, energy, x0, steps, opts: Opts | None = None):
        c, keep = self._cond(P, tau, T_in, Y_in, energy)
        x = np.array(x0, dtype=np.float64, copy=True)
        st = Stats()
        lib().om_time_march_only(C.byref(self.s), C.byref(c), C.byref(opts or default_opts()),
                                 _dp(x), int(steps), C.byref(st))
        return x, st


def soot_ln_mu(lnM, p):
    """ln mu_p by the interpolative closure (Lagrange in ln mu over the orders)."""
    lnM = np.ascontiguousarray(lnM, dtype=np.float64)
    return lib().om_soot_ln_mu(_dp(lnM), float(p))


def soot_fxy(lnM, x, y):
    """The coagulation grid-function interpolant f_{x,y}."""
    lnM = np.ascontiguousarray(lnM, dtype=np.float64)
    return lib().om_soot_fxy(_dp(lnM), int(x), int(y))


def lu_factor(a):
    a = np.array(a, dtype=np.float64, copy=True, order="C")
    n = a.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib().om_lu_factor(n, _dp(a), _ip(piv))
    return a, piv, info


def lu_solve(lu, piv, b):
    lu = np.ascontiguousarray(lu, dtype=np.float64)
    piv = np.ascontiguousarray(piv, dtype=np.int32)
    b = np.array(b, dtype=np.float64, copy=True)
    lib().om_lu_solve(lu.shape[0], _dp(lu), _ip(piv), _dp(b))
    return b


# -- batch driver ---------------------------------------------------------------

def _opts_dict(o: Opts | None):
    if o is None:
        return None
    return {name: getattr(o, name) for name, _ in Opts._fields_}


def _solve_chunk(args):
    mech, cond, x0, energy, idx, opts = args
    M = Mechanism(mech)
    o = default_opts(**opts) if opts else default_opts()
    n = x0.shape[0]
    xs = np.zeros((n, len(idx)))
    st = np.zeros((len(idx), 6))
    for j, b in enumerate(idx):
        x, s = M.solve(cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], energy,
                       x0[:, b], o)
        xs[:, j] = x
        st[j] = (s.status, s.n_lin, s.n_jac, s.n_ts, s.n_attempts, s.sres)
    return idx, xs, st


def solve_batch(mech: dict, cond: dict, x0: np.ndarray, energy: bool, *, idx=None,
                opts: Opts | None = None, processes: int = 1):
    """Solve the reactors `idx` (default: all) one at a time.

    With processes > 1 the reactors are dealt round-robin to that many
    worker processes, each running the single-threaded oracle.  Returns
    (x [n][len(idx)], stats dict of arrays).
    """
    build(force=False)
    B = x0.shape[1]
    idx = np.arange(B) if idx is None else np.asarray(idx)
    od = _opts_dict(opts)
    parts = [idx[p::processes] for p in range(max(1, processes))]
    parts = [p for p in parts if len(p)]
    pos = {int(b): j for j, b in enumerate(idx)}
    xs = np.zeros((x0.shape[0], len(idx)))
    st = np.zeros((len(idx), 6))
    jobs = [(mech, cond, x0, energy, p, od) for p in parts]
    if len(parts) == 1:
        results = [_solve_chunk(jobs[0])]
    else:
        with ProcessPoolExecutor(max_workers=len(parts)) as ex:
            results = list(ex.map(_solve_chunk, jobs))
    for p, xp, sp in results:
        cols = [pos[int(b)] for b in p]
        xs[:, cols] = xp
        st[cols] = sp
    stats = {"status": st[:, 0].astype(int), "n_lin": st[:, 1].astype(int),
             "n_jac": st[:, 2].astype(int), "n_ts": st[:, 3].astype(int),
             "n_attempts": st[:, 4].astype(int), "sres": st[:, 5]}
    return xs, stats


def sweep_batch(mech: dict, cond: dict, x0: np.ndarray, energy: bool, param: str,
                values: np.ndarray, *, opts: Opts | None = None, processes: int = 1):
    """Continuation sweep (paper Section 5: steady solutions followed along
    one condition, each started from the solution before).  At step k the
    condition `param` ("T_in" or "tau") of reactor b is values[k, b]; the
    initial guess of step k is the state step k-1 left (x0 at step 0).
    Returns (x [n_steps][n][B], status [n_steps][B])."""
    if param not in ("T_in", "tau"):
        raise ValueError(param)
    x = np.array(x0, dtype=np.float64, copy=True)
    xs, sts = [], []
    for row in np.asarray(values, dtype=np.float64):
        c = dict(cond)
        c[param] = np.ascontiguousarray(row)
        x, st = solve_batch(mech, c, x, energy, opts=opts, processes=processes)
        xs.append(x.copy())
        sts.append(st["status"])
    return np.stack(xs), np.stack(sts)
