"""Pins of the oracle's scaled residual (the "scaled residual <= 1e-10"
convergence test; reading: each equation's |F| over the sum of the
magnitudes of the terms it is made of) in limits where it has a closed form
that does not restate the general definition:

  * no reaction active (every A = 0): a species row is the flow balance
    alone, |Y - Y_in| / (|Y| + |Y_in|);
  * one reaction A <=> B and an unbounded residence time (the flow terms
    vanish against the reaction): the A row is |1 - Q/K| / (1 + Q/K) with
    Q = C_B / C_A and K = k_f / k_r;
  * no reaction, composition at the inlet, T above T_in: the energy row is
    the inflow enthalpy terms alone, all of one sign, so exactly 1;
  * a sooting reactor with every gas reaction off and an unbounded residence
    time: the precursor and growth-species rows are soot sinks alone, so
    |F| equals its own single term and the row's value is exactly 1 (a
    denominator without the soot sink would make it infinite).
A dropped or doubled term in any denominator moves one of these values."""
import numpy as np
import pytest

from tests import tiny_mechs as tm

PATM = 101325.0
R_GAS = 8.314462618


def _sres(m, tau, T, Yin, energy, x):
    return m.scaled_residual(PATM, tau, T, np.asarray(Yin, float), energy, np.asarray(x, float))


@pytest.mark.parametrize("Y", [[0.3, 0.7], [0.9, 0.1], [0.05, 0.95]])
def test_flow_only_rows_closed_form(oracle_mod, Y):
    mech = tm.isomerisation(A=0.0)
    m = oracle_mod.Mechanism(mech)
    Yin = np.array([0.8, 0.2])
    Y = np.array(Y)
    exact = np.max(np.abs(Y - Yin) / (np.abs(Y) + np.abs(Yin)))
    assert _sres(m, 1e-3, 1500.0, Yin, False, Y) == pytest.approx(exact, rel=1e-14)


@pytest.mark.parametrize("YA", [0.2, 0.5, 0.93])
def test_single_reaction_row_at_infinite_residence_time(oracle_mod, YA):
    A, da6, da7, T = 3.0e3, -1500.0, 0.7, 1500.0
    m = oracle_mod.Mechanism(tm.isomerisation(A=A, da6=da6, da7=da7))
    K = np.exp(da7 - da6 / T)  # k_f / k_r (equal weights: Q = Y_B / Y_A)
    Q = (1.0 - YA) / YA
    exact = abs(1.0 - Q / K) / (1.0 + Q / K)
    got = _sres(m, 1e30, T, [0.5, 0.5], False, [YA, 1.0 - YA])
    assert got == pytest.approx(exact, rel=1e-12)


def test_energy_row_flow_only(oracle_mod):
    """No reaction, composition at the inlet, T above T_in: the species rows
    vanish and the energy row is the inflow enthalpy terms alone, all of one
    sign (c_p > 0), so |F_T| equals the sum of their magnitudes: exactly 1."""
    m = oracle_mod.Mechanism(tm.isomerisation(A=0.0))
    Yin = np.array([0.35, 0.65])
    x = np.array([0.35, 0.65, 1900.0])
    assert _sres(m, 2e-3, 600.0, Yin, True, x) == pytest.approx(1.0, rel=1e-14)
    # at T = T_in every row vanishes
    assert _sres(m, 2e-3, 1900.0, Yin, True, x) == 0.0


def test_single_reaction_rows_with_energy_at_infinite_residence_time(oracle_mod):
    """With the energy equation the species rows keep their closed form, and
    the energy row (reaction enthalpy against the gross enthalpy flux) stays
    below them: |H_B - H_A| / (|H_A| + |H_B|) < 1."""
    A, da6, da7, T = 3.0e3, -1500.0, 0.7, 1500.0
    m = oracle_mod.Mechanism(tm.isomerisation(A=A, da6=da6, da7=da7))
    YA = 0.4
    K = np.exp(da7 - da6 / T)
    Q = (1.0 - YA) / YA
    reac = abs(1.0 - Q / K) / (1.0 + Q / K)
    x = np.array([YA, 1.0 - YA, T])
    assert _sres(m, 1e30, T, [0.5, 0.5], True, x) == pytest.approx(reac, rel=1e-12)


def test_soot_sink_rows_are_exactly_one(oracle_mod):
    from psr_inputs import mechanism
    mech = dict(mechanism("soot"))
    mech["A"] = np.zeros_like(mech["A"])  # every gas reaction off
    m = oracle_mod.Mechanism(mech)
    sd = mech["soot"]
    N = mech["species_elems"].shape[0]
    Y = np.full(N, 0.5 / (N - 2))
    Y[sd["precursor"]] = 0.2
    Y[sd["growth"]] = 0.3
    r = np.arange(6)
    lnM = np.log(1e10) + r * np.log(60.0) + r ** 2 * 0.3 ** 2 / 2
    x = np.concatenate([Y, [1700.0], lnM])
    Yin = Y.copy()
    # unbounded residence time: every flow term is negligible; the
    # precursor / growth rows are their soot sinks alone, and the other
    # species rows are exactly zero
    got = _sres(m, 1e30, 600.0, Yin, True, x)
    assert got == pytest.approx(1.0, rel=1e-12)
