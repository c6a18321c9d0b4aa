"""Host checks of the seeded input recipes (no solver arithmetic)."""
import numpy as np


def test_fod_recipe_gives_the_single_iteration_inlet():
    from psr_inputs import workload
    from psr_inputs.mechanism import species_weights
    mech, cond, x0, energy = workload("newton101", 7)
    assert not energy and mech["species_elems"].shape[0] == 101 and mech["A"].shape[0] == 542
    assert np.all(cond["T_in"] == 1800.0) and np.allclose(cond["tau"], 0.05, rtol=1e-14)
    Y = cond["Y_in"]
    assert np.all(Y == Y[:, :1]) and abs(Y[:, 0].sum() - 1.0) < 1e-15
    X = Y[:, 0] / species_weights(mech)
    X /= X.sum()
    np.testing.assert_allclose(X[[mech["fuel"], mech["oxidizer"], mech["diluent"]]], [0.15, 0.18, 0.67],
                               rtol=1e-13)
    assert np.count_nonzero(X) == 3
    np.testing.assert_array_equal(x0, Y)
