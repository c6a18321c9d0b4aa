"""The oracle's reading of reactor inputs outside the domain of Eqs. 1-3
(Section 2: a steady PSR needs positive pressure, residence time and inlet
temperature, and finite inlet and initial data): such a reactor is reported
non-finite at once, without work, and its x is left as given."""
import numpy as np
import pytest


@pytest.mark.parametrize("what,val", [("tau", np.nan), ("tau", 0.0), ("tau", -1e-3), ("tau", np.inf),
                                      ("P", -1.0), ("P", np.nan), ("T_in", 0.0), ("Y_in", np.inf),
                                      ("x", np.nan), ("x", -np.inf)])
def test_reactor_outside_domain_is_flagged(oracle_mod, what, val):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 2)
    cond = {k: np.array(v, copy=True) for k, v in cond.items()}
    x0 = x0.copy()
    if what == "Y_in":
        cond["Y_in"][2, 1] = val
    elif what == "x":
        x0[-1, 1] = val
    else:
        cond[what][1] = val
    xo, so = oracle_mod.solve_batch(mech, cond, x0, energy)
    assert so["status"][1] == 3 and so["n_lin"][1] == 0
    assert np.array_equal(xo[:, 1], x0[:, 1], equal_nan=True)
    assert so["status"][0] == 0  # the neighbour is solved as usual
