"""Pins of the oracle's residual and hybrid solve against closed forms,
scalar reductions solved by bisection, conservation laws and an independent
Gibbs-energy minimisation (Section 2, Eqs. 1-3; Section 3, Eqs. 4-9)."""
import numpy as np
import pytest
from scipy.optimize import brentq, root

from tests import tiny_mechs as tm

R = 8.314462618
PATM = 101325.0


def _solve(m, tau, T, Yin, energy=False, x0=None):
    x0 = np.array(Yin if x0 is None else x0, float)
    x, st = m.solve(PATM, tau, T, np.asarray(Yin, float), energy, x0)
    assert st.status == 0, st.status
    return x, st


@pytest.mark.parametrize("tau", [1e-5, 3e-3, 0.2, 40.0])
def test_isomerisation_closed_form(oracle_mod, tau):
    # A <=> B, equal weights, isothermal: rho is constant and
    # Y_A* = (Y_A,in / tau + k_r) / (1/tau + k_f + k_r)
    A, da6, da7, T = 3.0e3, -1500.0, 0.7, 1500.0
    m = oracle_mod.Mechanism(tm.isomerisation(A=A, da6=da6, da7=da7))
    Kc = np.exp(da7 - da6 / T)
    kf, kr = A, A / Kc
    Yin = np.array([0.8, 0.2])
    x, st = _solve(m, tau, T, Yin)
    YA = (Yin[0] / tau + kr) / (1 / tau + kf + kr)
    np.testing.assert_allclose(x, [YA, 1 - YA], rtol=1e-13)
    assert st.sres <= 1e-10


def test_isomerisation_equilibrium_limit(oracle_mod):
    m = oracle_mod.Mechanism(tm.isomerisation())
    Kc = np.exp(0.7 + 1500.0 / 1500.0)
    x, _ = _solve(m, 1e7, 1500.0, [1.0, 0.0])
    np.testing.assert_allclose(x[0], 1 / (1 + Kc), rtol=1e-9)


def _rho(Y, W, T):
    return PATM * 1e-6 / (R * T * np.sum(Y / W))


@pytest.mark.parametrize("tau", [1e-6, 1e-3, 1.0])
def test_dimerisation_scalar_reduction(oracle_mod, tau):
    # 2A <=> A2, isothermal; Y_A2 = 1 - Y_A; scalar species-A balance
    #   (rho/tau)(Y_A - Y_A,in) = -2 W_A q,  q = k_f C_A^2 - k_r C_A2
    T = 1400.0
    mech = tm.dimerisation()
    m = oracle_mod.Mechanism(mech)
    W = m.W
    kf, Kc, kr = m.rate_constants(T)
    # the rate constants are pinned in test_oracle_thermo_rates; here the
    # reduction pins the residual, concentrations and the solver
    Yin = np.array([0.9, 0.1])

    def g(ya):
        Y = np.array([ya, 1 - ya])
        rho = _rho(Y, W, T)
        C = rho * Y / W
        q = kf[0] * C[0] ** 2 - kr[0] * C[1]
        return rho / tau * (ya - Yin[0]) + 2 * W[0] * q

    ya = brentq(g, 0.0, 1.0, xtol=1e-16, rtol=1e-15, maxiter=500)
    x, _ = _solve(m, tau, T, Yin)
    np.testing.assert_allclose(x, [ya, 1 - ya], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("tau", [1e-6, 1e-3, 1.0])
def test_association_scalar_reduction(oracle_mod, tau):
    # A + B <=> C; element balances fix Y_A, Y_B from Y_C; scalar C balance
    T = 1600.0
    m = oracle_mod.Mechanism(tm.association())
    W = m.W
    kf, _, kr = m.rate_constants(T)
    Yin = np.array([0.3, 0.2, 0.5])
    nC = Yin[0] / W[0] + Yin[2] / W[2]   # mol of C-element per gram
    nH = Yin[1] / W[1] + Yin[2] / W[2]

    def state(yc):
        return np.array([(nC - yc / W[2]) * W[0], (nH - yc / W[2]) * W[1], yc])

    def g(yc):
        Y = state(yc)
        rho = _rho(Y, W, T)
        C = rho * Y / W
        q = kf[0] * C[0] * C[1] - kr[0] * C[2]
        return rho / tau * (yc - Yin[2]) - W[2] * q

    ymax = min(nC, nH) * W[2]
    yc = brentq(g, 0.0, ymax, xtol=1e-17, rtol=1e-15, maxiter=500)
    x, _ = _solve(m, tau, T, Yin)
    np.testing.assert_allclose(x, state(yc), rtol=1e-11, atol=1e-15)


def _nu_matrix(mech):
    n_rx, n_sp = len(mech["A"]), mech["species_elems"].shape[0]
    nu = np.zeros((n_rx, n_sp))
    for k in range(n_rx):
        for s in range(3):
            if mech["reac_idx"][k, s] >= 0:
                nu[k, mech["reac_idx"][k, s]] -= mech["reac_nu"][k, s]
            if mech["prod_idx"][k, s] >= 0:
                nu[k, mech["prod_idx"][k, s]] += mech["prod_nu"][k, s]
    return nu


def _gibbs_equilibrium(m, a, T, Yin):
    """Element-potential solution of min G at fixed T, P = P_atm and element amounts.

    Mole fractions X_i = exp(-g_i + sum_e lambda_e a_ie) with g_i = H_i/RT - S_i/R,
    sum_i X_i = 1 and n_tot sum_i a_ie X_i = b_e.  Unknowns (lambda, ln n_tot),
    solved by Newton's method with a backtracking line search on |r|.
    """
    _, hRT, sR = m.thermo(T)
    g = hRT - sR
    b = a.T @ (Yin / m.W)
    E = a.shape[1]
    lam = np.linalg.lstsq(a, g - np.log(1.0 / len(g)), rcond=None)[0]
    u = np.r_[lam, np.log(np.sum(Yin / m.W))]

    def resid(u):
        X = np.exp(-g + a @ u[:E])
        n = np.exp(u[E])
        return np.r_[n * (a.T @ X) / b - 1.0, X.sum() - 1.0], X, n

    r, X, n = resid(u)
    for _ in range(200):
        Jm = np.zeros((E + 1, E + 1))
        Jm[:E, :E] = n * (a.T * X) @ a / b[:, None]
        Jm[:E, E] = n * (a.T @ X) / b
        Jm[E, :E] = X @ a
        step = np.linalg.solve(Jm, -r)
        t = 1.0
        while True:
            r2, X2, n2 = resid(u + t * step)
            if np.linalg.norm(r2) < np.linalg.norm(r) or t < 1e-8:
                break
            t *= 0.5
        u, r, X, n = u + t * step, r2, X2, n2
        if np.linalg.norm(r) < 1e-15:
            break
    assert np.linalg.norm(r) < 1e-13
    return n * X * m.W  # mass per gram of mixture = Y


def test_long_residence_time_reaches_gibbs_minimum(oracle_mod):
    """As tau grows the isothermal PSR tends to chemical equilibrium.

    Independent reference: the Gibbs-energy minimum at fixed T, P and element
    amounts (element potentials).  This pins the pressure factor of Eq. 8 and
    the signs of Eq. 9 against the mass-action residual.
    """
    mech = tm.small_network()
    m = oracle_mod.Mechanism(mech)
    a = mech["species_elems"].astype(float)
    nu = _nu_matrix(mech)
    assert np.linalg.matrix_rank(nu) == m.n_sp - np.linalg.matrix_rank(a)
    T = 1500.0
    Yin = np.array([0.2, 0.05, 0.25, 0.3, 0.2])
    Yeq = _gibbs_equilibrium(m, a, T, Yin)
    assert abs(Yeq.sum() - 1) < 1e-12
    errs = []
    for tau in (1e-1, 1e1, 1e3):
        x, _ = _solve(m, tau, T, Yin)
        errs.append(np.max(np.abs(x - Yeq) / Yeq))
    # the deviation from equilibrium falls like 1/tau
    assert errs[2] < 1e-6, errs
    assert 50 < errs[0] / errs[1] < 200 and 50 < errs[1] / errs[2] < 200, errs


def test_long_residence_time_detailed_balance(oracle_mod):
    mech = tm.small_network()
    m = oracle_mod.Mechanism(mech)
    nu = _nu_matrix(mech)
    T, Yin = 1500.0, np.array([0.2, 0.05, 0.25, 0.3, 0.2])
    _, Kc, _ = m.rate_constants(T)
    devs = []
    for tau in (1e-1, 1e1, 1e3):
        x, _ = _solve(m, tau, T, Yin)
        C, _, _ = m.production(T, PATM, x)
        devs.append(np.max(np.abs(nu @ np.log(C) - np.log(Kc))))
    assert devs[2] < 1e-5, devs
    assert 50 < devs[0] / devs[1] < 200 and 50 < devs[1] / devs[2] < 200, devs
