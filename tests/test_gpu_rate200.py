"""GPU parity of psr_residual (the rate/residual kernel with the scaled
residual) on the 200-species / 1200-reaction mechanism, whose per-reactor
working set takes the one-workgroup-per-reactor kernel, against the oracle
element by element; ragged batch of seeded states."""
import numpy as np
import pytest

from tests.gpu_util import cond_dev, dev

pytestmark = pytest.mark.gpu


def test_residual_200_species_matches_oracle(oracle_mod):
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    from psr_inputs import workload
    B = 29
    mech, cond, _, energy = workload("rate200", B)
    M = P.Mechanism(mech)
    O = oracle_mod.Mechanism(mech)
    N = M.n_species
    rng = np.random.default_rng(200)
    x = np.concatenate([rng.dirichlet(np.full(N, 0.4), B).T, rng.uniform(600, 2800, (1, B))], axis=0)
    sc = torch.empty(B, dtype=torch.float64, device="cuda:0")
    F = P.residual(M, cond_dev(cond), energy, dev(x), scaled=sc).cpu().numpy()
    sc = sc.cpu().numpy()
    for b in range(B):
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], energy, x[:, b])
        Fo = O.residual(*args)
        np.testing.assert_allclose(F[:, b], Fo, rtol=1e-10, atol=1e-12 * np.abs(Fo).max(), err_msg=f"b={b}")
        np.testing.assert_allclose(sc[b], O.scaled_residual(*args), rtol=1e-8, err_msg=f"b={b}")
