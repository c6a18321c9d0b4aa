"""Invariants of the oracle's converged steady states on the synthetic
workloads: mass, elements, adiabatic enthalpy, residual, and agreement of
pure pseudo-transient integration with the hybrid solve."""
import numpy as np
import pytest

R = 8.314462618
PATM = 101325.0


@pytest.fixture(scope="module")
def energy_runs(oracle_mod):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 12)
    xs, st = oracle_mod.solve_batch(mech, cond, x0, energy)
    return mech, cond, xs, st


def test_all_converge_with_small_residual(energy_runs):
    _, _, _, st = energy_runs
    assert np.all(st["status"] == 0)
    assert np.all(st["sres"] <= 1e-10)


def test_mass_fractions_sum_to_one(energy_runs):
    mech, _, xs, _ = energy_runs
    N = mech["species_elems"].shape[0]
    assert np.max(np.abs(xs[:N].sum(axis=0) - 1.0)) <= 1e-13


def test_elements_conserved(energy_runs, oracle_mod):
    mech, cond, xs, _ = energy_runs
    m = oracle_mod.Mechanism(mech)
    a = mech["species_elems"].astype(float)
    N = m.n_sp
    out = a.T @ (xs[:N] / m.W[:, None])
    inn = a.T @ (cond["Y_in"] / m.W[:, None])
    np.testing.assert_allclose(out, inn, rtol=1e-12)


def test_adiabatic_enthalpy_balance(energy_runs, oracle_mod):
    # at the steady state of Eqs. 2-3 (adiabatic) h_mix(T*, Y*) = h_mix(T_in, Y_in)
    mech, cond, xs, _ = energy_runs
    m = oracle_mod.Mechanism(mech)
    N = m.n_sp
    for b in range(xs.shape[1]):
        T = xs[N, b]
        _, hRT, _ = m.thermo(T)
        _, hRT_in, _ = m.thermo(cond["T_in"][b])
        h_out = np.sum(xs[:N, b] * R * T * hRT / m.W)
        h_in = np.sum(cond["Y_in"][:, b] * R * cond["T_in"][b] * hRT_in / m.W)
        scale = np.sum(np.abs(xs[:N, b] * R * T * hRT / m.W))
        assert abs(h_out - h_in) <= 1e-12 * scale


def test_residual_vanishes_at_root(energy_runs, oracle_mod):
    mech, cond, xs, _ = energy_runs
    m = oracle_mod.Mechanism(mech)
    for b in range(3):
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], True)
        assert m.scaled_residual(*args, xs[:, b]) <= 1e-12


def test_time_stepping_alone_reaches_the_newton_root(energy_runs, oracle_mod):
    mech, cond, xs, _ = energy_runs
    m = oracle_mod.Mechanism(mech)
    N = m.n_sp
    from psr_inputs.conditions import initial_guess
    for b in range(3):
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], True)
        x0 = np.r_[cond["Y_in"][:, b], 2000.0]
        xt, st = m.time_march(*args, x0, 400)
        assert st.status == 0
        big = xs[:N, b] > 1e-12
        np.testing.assert_allclose(xt[:N][big], xs[:N, b][big], rtol=1e-9)
        np.testing.assert_allclose(xt[N], xs[N, b], rtol=1e-12)


def test_budget_exhaustion_reports_maxiter(oracle_mod):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 2)
    xs, st = oracle_mod.solve_batch(mech, cond, x0, energy, opts=oracle_mod.default_opts(max_lin=10))
    assert np.all(st["status"] == 1)
    assert np.all(st["n_lin"] <= 10)


def test_warm_start_converges_immediately(energy_runs, oracle_mod):
    # restarting from a converged root: the first Newton attempt converges
    mech, cond, xs, _ = energy_runs
    xs2, st2 = oracle_mod.solve_batch(mech, {k: v[..., :4] for k, v in cond.items()}, xs[:, :4], True)
    assert np.all(st2["status"] == 0)
    assert np.all(st2["n_lin"] <= 2)
    N = mech["species_elems"].shape[0]
    np.testing.assert_allclose(xs2[N], xs[N, :4], rtol=1e-13)
