"""Pins of the oracle's finite-difference Jacobian (the paper's Jacobian
route, Section 1) against the complex-step Jacobian, which is exact to
rounding and computed by other code: every element must agree to within
the forward difference's truncation (the change of the exact column over
the step, plus 1e-7 relative) and its rounding (64 eps S_r / h_j).  Gas-phase mechanisms only: with the soot moment rows the
interpolative closure's curvature exceeds this bound, so the soot case of
the finite-difference Jacobian is parity unpinned."""
import numpy as np
import pytest

from tests.fd_bound import fd_bound, fd_steps, shifted_columns, within


@pytest.mark.parametrize("name", ["isothermal", "energy"])
def test_fd_jacobian_matches_complex_step(oracle_mod, name):
    from psr_inputs import workload
    mech, cond, x0, energy = workload(name, 4)
    M = oracle_mod.Mechanism(mech)
    xs, st = oracle_mod.solve_batch(mech, cond, x0, energy, idx=np.arange(2))
    N = mech["species_elems"].shape[0]
    for b in range(2):
        a = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], energy)
        for x in (x0[:, b], xs[:, b]):
            Jf = M.jacobian_fd(*a, x)
            Jc = M.jacobian(*a, x, complex_step=True)
            F = M.residual(*a, x)
            h = fd_steps(x, N)
            Js = shifted_columns(lambda y: M.jacobian(*a, y, complex_step=True), x, h)
            bound = fd_bound(Jc, F, x, h, 1e-7, 64, Js)
            assert within(Jf - Jc, bound), (name, b)
            # the bound is tight where it matters: for most elements it is
            # below a thousandth of the row's largest entry
            tight = bound < 1e-3 * np.abs(Jc).max(axis=1, keepdims=True)
            assert tight.mean() > 0.8


def test_fd_pin_catches_a_swapped_column(oracle_mod):
    """A plausible slip (two columns exchanged) breaks the pin."""
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 1)
    M = oracle_mod.Mechanism(mech)
    a = (cond["P"][0], cond["tau"][0], cond["T_in"][0], cond["Y_in"][:, 0], energy)
    x = x0[:, 0]
    Jf = M.jacobian_fd(*a, x)
    Jc = M.jacobian(*a, x, complex_step=True)
    h = fd_steps(x, mech["species_elems"].shape[0])
    Js = shifted_columns(lambda y: M.jacobian(*a, y, complex_step=True), x, h)
    bound = fd_bound(Jc, M.residual(*a, x), x, h, 1e-7, 64, Js)
    n = Jf.shape[0]
    bad = Jf.copy()
    bad[:, [n - 1, 0]] = bad[:, [0, n - 1]]
    assert not within(bad - Jc, bound)
