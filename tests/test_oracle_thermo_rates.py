"""Pins of the oracle's thermodynamics and rate constants (Eqs. 6-9).

Each check compares against a closed form or an identity that holds for any
coefficients, so a dropped term, a wrong sign or a wrong unit conversion in
the oracle fails at least one of them.
"""
import numpy as np
import pytest

from tests import tiny_mechs as tm

R = 8.314462618
PATM = 101325.0


@pytest.fixture(scope="module")
def net(oracle_mod):
    return oracle_mod.Mechanism(tm.small_network())


def test_nasa7_identities_by_finite_differences(net):
    # cp/R = d(H/R)/dT and (cp/R)/T = d(S/R)/dT for arbitrary a1..a7 (a4, a5 != 0)
    for T in (350.0, 900.0, 1700.0, 2600.0):
        h = 1e-5 * T
        cp, hRT, sR = net.thermo(T)
        _, hp, sp = net.thermo(T + h)
        _, hm, sm = net.thermo(T - h)
        dH = ((T + h) * hp - (T - h) * hm) / (2 * h)
        dS = (sp - sm) / (2 * h)
        np.testing.assert_allclose(dH, cp, rtol=1e-8)
        np.testing.assert_allclose(dS, cp / T, rtol=1e-8)


def test_constant_cp_thermo_closed_form(oracle_mod):
    m = oracle_mod.Mechanism(tm.isomerisation())
    for T in (400.0, 1500.0):
        cp, hRT, sR = m.thermo(T)
        np.testing.assert_allclose(cp, [3.5, 3.5], rtol=0, atol=0)
        np.testing.assert_allclose(hRT, [3.5, 3.5 - 1500.0 / T], rtol=1e-15)
        np.testing.assert_allclose(sR, [3.5 * np.log(T) + 5.0, 3.5 * np.log(T) + 5.7], rtol=1e-15)


def test_arrhenius_special_cases(oracle_mod):
    base = tm.small_network()
    base["beta"][:] = 0.0
    base["Ea"][:] = 0.0
    m = oracle_mod.Mechanism(base)
    kf, _, _ = m.rate_constants(1234.5)
    np.testing.assert_array_equal(kf, base["A"])          # beta = E = 0  ->  k_f = A exactly
    base["beta"][:] = 1.0
    m = oracle_mod.Mechanism(base)
    kf, _, _ = m.rate_constants(800.0)
    np.testing.assert_allclose(kf, base["A"] * 800.0, rtol=1e-14)
    base["beta"][:] = 0.0
    base["Ea"][:] = 1.0e5
    m = oracle_mod.Mechanism(base)
    k1, _, _ = m.rate_constants(1000.0)
    k2, _, _ = m.rate_constants(2000.0)
    # ln k linear in 1/T with slope -E/R
    np.testing.assert_allclose(np.log(k1 / k2), -1.0e5 / R * (1 / 1000.0 - 1 / 2000.0), rtol=1e-12)


def test_equilibrium_constant_without_mole_change(oracle_mod):
    # A <=> B between isomers: K_c = K_p = exp(da7 - da6/T), k_r = k_f / K_c
    m = oracle_mod.Mechanism(tm.isomerisation(A=3.0e3, da6=-1500.0, da7=0.7))
    for T in (500.0, 1500.0, 2500.0):
        kf, Kc, kr = m.rate_constants(T)
        assert kf[0] == 3.0e3
        np.testing.assert_allclose(Kc[0], np.exp(0.7 + 1500.0 / T), rtol=1e-14)
        np.testing.assert_allclose(kr[0], kf[0] / Kc[0], rtol=1e-15)


def test_equilibrium_constant_pressure_factor(oracle_mod):
    # 2 A <=> A2: one mole fewer, K_c = K_p (P_atm / R T in mol/cm^3)^(-1)
    mech = tm.dimerisation(a6_dimer=-3.0e4, a7_dimer=-2.0)
    m = oracle_mod.Mechanism(mech)
    for T in (700.0, 1800.0):
        _, Kc, _ = m.rate_constants(T)
        # constant cp: S/R = a1 ln T + a7, H/RT = a1 + a6/T
        dS = (3.5 * np.log(T) + 4.0) - 2 * (2.5 * np.log(T) + 8.0)
        dH = (3.5 - 3.0e4 / T) - 2 * 2.5
        Kp = np.exp(dS - dH)
        c_std = PATM / (R * T) * 1e-6
        np.testing.assert_allclose(Kc[0], Kp / c_std, rtol=1e-13)


def test_van_t_hoff(net):
    # d ln K_c / dT = sum_i nu_i H_i/(R T^2) - (sum_i nu_i)/T for every reaction
    mech = tm.small_network()
    nu = np.zeros((len(mech["A"]), 5))
    for k in range(len(mech["A"])):
        for s in range(3):
            if mech["reac_idx"][k, s] >= 0:
                nu[k, mech["reac_idx"][k, s]] -= mech["reac_nu"][k, s]
            if mech["prod_idx"][k, s] >= 0:
                nu[k, mech["prod_idx"][k, s]] += mech["prod_nu"][k, s]
    for T in (600.0, 1500.0, 2400.0):
        h = 1e-5 * T
        _, Kp_, _ = net.rate_constants(T + h)
        _, Km_, _ = net.rate_constants(T - h)
        dlnK = (np.log(Kp_) - np.log(Km_)) / (2 * h)
        _, hRT, _ = net.thermo(T)
        expect = nu @ hRT / T - nu.sum(axis=1) / T
        np.testing.assert_allclose(dlnK, expect, rtol=1e-7, atol=1e-12)


def test_production_conserves_elements_and_mass(oracle_mod):
    from psr_inputs import mechanism
    mech = mechanism("energy")
    m = oracle_mod.Mechanism(mech)
    a = mech["species_elems"].astype(float)
    rng = np.random.default_rng(3)
    for _ in range(5):
        Y = rng.dirichlet(np.full(m.n_sp, 0.3))
        T = rng.uniform(600, 2800)
        C, q, wdot = m.production(T, PATM, Y)
        gross = np.abs(a.T) @ np.abs(wdot) + 1e-300
        assert np.all(np.abs(a.T @ wdot) <= 1e-12 * gross)
        np.testing.assert_allclose(np.dot(m.W, wdot), 0.0, atol=1e-12 * np.abs(m.W * wdot).sum())
        # concentrations: C_j = rho Y_j / W_j with rho = P / (R T sum Y/W)
        rho = PATM * 1e-6 / (R * T * np.sum(Y / m.W))
        np.testing.assert_allclose(C, rho * Y / m.W, rtol=1e-14)


def test_rate_of_progress_signs(oracle_mod):
    # only reactants present -> every q_k >= 0 ; only products -> q_k <= 0
    m = oracle_mod.Mechanism(tm.association())
    _, q, _ = m.production(1500.0, PATM, np.array([0.5, 0.5, 0.0]))
    assert q[0] > 0
    _, q, _ = m.production(1500.0, PATM, np.array([0.0, 0.0, 1.0]))
    assert q[0] < 0
