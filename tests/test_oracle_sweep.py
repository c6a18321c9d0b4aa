"""Pins of the oracle's continuation sweep (paper Section 5: steady solutions
followed along the reactor temperature, then along the residence time, each
started from the solution before).  The pins do not rest on the oracle's own
solver: every converged step must (1) conserve each element between inlet
and reactor, which holds for any steady state because every reaction is
element balanced, (2) be the unique isothermal root at its own condition, so
a cold start from the inlet at that condition lands on it too, and (3) a
sweep of one step is the plain solve."""
import numpy as np
import pytest

from psr_inputs.configs import sweep_workload
from psr_inputs.mechanism import species_weights


def _element_flux(mech, Y):
    """sum_i a_ie Y_i / W_i per element and reactor (moles of element per gram)."""
    W = species_weights(mech)
    return mech["species_elems"].T.astype(float) @ (Y / W[:, None])


@pytest.mark.parametrize("param", ["T_in", "tau"])
def test_sweep_steps_are_element_balanced_roots(oracle_mod, param):
    mech, cond, x0, values = sweep_workload(param, 3)
    xs, st = oracle_mod.sweep_batch(mech, cond, x0, False, param, values, processes=3)
    assert xs.shape == (values.shape[0],) + x0.shape
    assert np.all(st == 0), st
    ein = _element_flux(mech, cond["Y_in"])
    for k in range(values.shape[0]):
        e = _element_flux(mech, xs[k])
        assert np.max(np.abs(e - ein) / np.abs(ein).max(axis=0)) < 1e-9, k
    # the swept condition really changes the root: no two steps agree
    d = np.abs(np.diff(xs, axis=0)).max(axis=(1, 2))
    assert np.all(d > 1e-6), d


@pytest.mark.parametrize("param", ["T_in", "tau"])
def test_sweep_matches_cold_starts(oracle_mod, param):
    mech, cond, x0, values = sweep_workload(param, 2)
    xs, st = oracle_mod.sweep_batch(mech, cond, x0, False, param, values, processes=2)
    n_sp = mech["species_elems"].shape[0]
    for k in range(0, values.shape[0], 3):
        c = dict(cond)
        c[param] = values[k].copy()
        xc, sc = oracle_mod.solve_batch(mech, c, x0, False, processes=2)
        ok = sc["status"] == 0
        assert ok.any()
        den = np.maximum(np.abs(xc[:n_sp]), 1e-20)
        err = (np.abs(xs[k][:n_sp] - xc[:n_sp]) / den)[:, ok]
        assert err.max() <= 1e-8, (k, err.max())


def test_one_step_sweep_is_the_plain_solve(oracle_mod):
    mech, cond, x0, values = sweep_workload("T_in", 2)
    xs, st = oracle_mod.sweep_batch(mech, cond, x0, False, "T_in", values[:1])
    c = dict(cond)
    c["T_in"] = values[0].copy()
    xp, sp = oracle_mod.solve_batch(mech, c, x0, False)
    assert np.array_equal(xs[0], xp) and np.array_equal(st[0], sp["status"])
