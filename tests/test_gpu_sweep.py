"""GPU parity of the continuation sweep (psr_sweep_batch, called through the
C ABI): the paper's Section 5 protocol -- temperature 1500 -> 2000 K at
tau = 5 ms and residence time 5 -> 95 ms at 1750 K, every step started from
the step before -- on isothermal reactors of the 53-species mechanism, each
reactor its own chain.  Every step's state is compared with the oracle's own
sweep element by element."""
import numpy as np
import pytest

from tests.gpu_util import cond_dev, dev, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-8, 1: 1e-7}  # PSR_FP64, PSR_MIXED
CHAINS = 48


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    return P


@pytest.fixture(scope="module")
def oracle_paths(oracle_mod):
    from psr_inputs.configs import sweep_workload
    out = {}
    for param in ("T_in", "tau"):
        mech, cond, x0, values = sweep_workload(param, CHAINS)
        xs, st = oracle_mod.sweep_batch(mech, cond, x0, False, param, values, processes=8)
        assert np.all(st == 0)
        out[param] = (mech, cond, x0, values, xs)
    return out


@pytest.mark.parametrize("precision,scheduler", [(0, 0), (1, 1)])
@pytest.mark.parametrize("param", ["T_in", "tau"])
def test_sweep_matches_oracle(P, oracle_paths, param, precision, scheduler):
    import torch
    mech, cond, x0, values, xo = oracle_paths[param]
    print(f"sweep {param} precision={precision} scheduler={scheduler} chains={CHAINS}", flush=True)
    M = P.Mechanism(mech)
    x = dev(x0)
    status = torch.full((CHAINS,), -1, dtype=torch.int32, device="cuda:0")
    g = dict(mech=M, cond=cond_dev(cond), energy=False, x=x, status=status)
    o = P.default_opts(precision=precision, scheduler=scheduler)
    st, xp, sp, _ = P.sweep_batch(g, param, dev(values), o)
    torch.cuda.synchronize()
    xp, sp = xp.cpu().numpy(), sp.cpu().numpy()
    assert np.all(sp == 0), sp
    assert st.reactors == CHAINS * values.shape[0] and st.converged == st.reactors
    n_sp = mech["species_elems"].shape[0]
    for k in range(values.shape[0]):
        err = rel_err(xp[k], xo[k], n_sp)
        assert err.max() <= TOL[precision], (k, err.max())
    # x_inout ends at the last step's state, status at the last step's
    assert np.array_equal(x.cpu().numpy(), xp[-1])
    assert np.array_equal(status.cpu().numpy(), sp[-1])


def test_one_step_sweep_equals_the_solve(P, oracle_paths):
    """A sweep of one step is the batched solve at that condition, bitwise."""
    import torch
    mech, cond, x0, values, _ = oracle_paths["T_in"]
    M = P.Mechanism(mech)
    o = P.default_opts()
    x1 = dev(x0)
    s1 = torch.full((CHAINS,), -1, dtype=torch.int32, device="cuda:0")
    _, xp, _, _ = P.sweep_batch(dict(mech=M, cond=cond_dev(cond), energy=False, x=x1, status=s1),
                                "T_in", dev(values[:1]), o)
    x2 = dev(x0)
    s2 = torch.full((CHAINS,), -1, dtype=torch.int32, device="cuda:0")
    c = dict(cond)
    c["T_in"] = values[0].copy()
    P.solve_batch([dict(mech=M, cond=cond_dev(c), energy=False, x=x2, status=s2)], o)
    torch.cuda.synchronize()
    assert torch.equal(xp[0], x2) and torch.equal(s1, s2)
