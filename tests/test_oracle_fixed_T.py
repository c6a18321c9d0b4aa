"""Pins of the oracle's prescribed-temperature mode (energy mode 2: T kept as
an unknown with the row F_T = V (T - T_in) / tau) used by the sooting sweeps
of Section 5, which set the reactor temperature: the species rows are the
isothermal reactor's (Eq. 2 at T = T_in), the roots are the isothermal
roots with T = T_in, and the analytic Jacobian matches the complex-step
derivative, with and without soot moments."""
import numpy as np
import pytest

FIXED_T = 2


def _state(mech, cond, b, T, rng):
    N = mech["species_elems"].shape[0]
    Y = cond["Y_in"][:, b] * rng.uniform(0.5, 1.5, N)
    return Y / Y.sum(), T


def test_species_rows_are_the_isothermal_rows(oracle_mod):
    from psr_inputs import workload
    mech, cond, _, _ = workload("energy", 4)
    M = oracle_mod.Mechanism(mech)
    rng = np.random.default_rng(5)
    for b in range(4):
        Y, _ = _state(mech, cond, b, 0, rng)
        Tin = 1400.0 + 100 * b
        args = (cond["P"][b], cond["tau"][b], Tin, cond["Y_in"][:, b])
        F0 = M.residual(*args, 0, Y)
        F2 = M.residual(*args, FIXED_T, np.append(Y, Tin))
        assert np.array_equal(F2[:-1], F0)
        assert F2[-1] == 0.0
        # away from T_in the temperature row is the relaxation term
        F3 = M.residual(*args, FIXED_T, np.append(Y, Tin + 10.0))
        assert F3[-1] == pytest.approx(10.0 / cond["tau"][b], rel=1e-15)
        assert M.scaled_residual(*args, FIXED_T, np.append(Y, Tin)) == M.scaled_residual(*args, 0, Y)
        Mm = M.mass_diag(*args, FIXED_T, np.append(Y, Tin))
        assert np.array_equal(Mm[:-1], M.mass_diag(*args, 0, Y)) and Mm[-1] == 1.0


@pytest.mark.parametrize("name", ["energy", "soot_sweep"])
def test_jacobian_matches_complex_step(oracle_mod, name):
    from psr_inputs import configs
    if name == "soot_sweep":
        mech, cond, x0, _ = configs.soot_sweep_workload("T_in", 3)
    else:
        mech, cond, x0, _ = configs.workload(name, 3)
        x0 = x0.copy()
        x0[-1] = cond["T_in"] + 900.0
    M = oracle_mod.Mechanism(mech)
    rng = np.random.default_rng(9)
    for b in range(3):
        x = x0[:, b].copy()
        N = mech["species_elems"].shape[0]
        x[:N] *= rng.uniform(0.5, 1.5, N)
        x[N] = 1600.0 + 50 * b
        args = (cond["P"][b], cond["tau"][b], 1700.0, cond["Y_in"][:, b])
        J = M.jacobian(*args, FIXED_T, x)
        Jc = M.jacobian(*args, FIXED_T, x, complex_step=True)
        scale = np.abs(Jc).max(axis=1, keepdims=True) + 1e-300
        assert np.max(np.abs(J - Jc) / scale) < 1e-10
        assert np.array_equal(J[N], np.eye(len(x))[N] * (1.0 / cond["tau"][b]))


def test_roots_are_the_isothermal_roots(oracle_mod):
    from psr_inputs import workload
    mech, cond, _, _ = workload("energy", 6)
    cond = dict(cond)
    cond["T_in"] = np.linspace(1500.0, 2000.0, 6)
    Y0 = cond["Y_in"].copy()
    x0 = np.concatenate([Y0, cond["T_in"][None, :]])
    xi, si = oracle_mod.solve_batch(mech, cond, Y0, 0)
    xf, sf = oracle_mod.solve_batch(mech, cond, x0, FIXED_T)
    ok = (si["status"] == 0) & (sf["status"] == 0)
    assert ok.sum() >= 5
    assert np.array_equal(xf[-1, ok], cond["T_in"][ok])
    d = np.abs(xf[:-1, ok] - xi[:, ok]) / np.maximum(np.abs(xi[:, ok]), 1e-20)
    assert d.max() < 1e-7
