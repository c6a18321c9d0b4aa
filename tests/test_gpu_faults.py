"""Fault injection through the C ABI: reactors whose inputs lie outside the
domain of Eqs. 1-3 (a NaN residence time, an infinite inlet mass fraction, a
NaN initial value, a negative pressure, a zero residence time) are flagged
NONFINITE with their x left as given, and every other reactor of the same
batch is bitwise what a clean batch gives; a budget-limited solve resumed
from its returned state reaches the oracle's roots."""
import numpy as np
import pytest

from tests.gpu_util import parity, solve_gpu

pytestmark = pytest.mark.gpu

B = 48
BAD = {5: ("tau", np.nan), 9: ("Y_in", np.inf), 17: ("x", np.nan), 30: ("P", -1.0), 41: ("tau", 0.0)}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    return P


def _poison(cond, x0):
    cond = {k: np.array(v, copy=True) for k, v in cond.items()}
    x0 = x0.copy()
    for b, (what, val) in BAD.items():
        if what == "Y_in":
            cond["Y_in"][0, b] = val
        elif what == "x":
            x0[3, b] = val
        else:
            cond[what][b] = val
    return cond, x0


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheduler", [0, 1])
def test_bad_inputs_flagged_others_bitwise_unchanged(P, engine, precision, scheduler):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", B)
    M = P.Mechanism(mech)
    kw = dict(engine=engine, precision=precision, scheduler=scheduler)
    x, status, nlin, _ = solve_gpu(M, cond, x0, energy, **kw)
    bc, bx0 = _poison(cond, x0)
    print(f"faults engine={engine} precision={precision} scheduler={scheduler}", flush=True)
    xb, statusb, nlinb, st = solve_gpu(M, bc, bx0, energy, **kw)
    bad = np.zeros(B, bool)
    bad[list(BAD)] = True
    assert np.all(statusb[bad] == 3), statusb[bad]
    assert np.all(nlinb[bad] == 0)
    assert np.array_equal(xb[:, bad], bx0[:, bad], equal_nan=True)
    assert np.array_equal(xb[:, ~bad], x[:, ~bad])
    assert np.array_equal(statusb[~bad], status[~bad])
    assert np.array_equal(nlinb[~bad], nlin[~bad])
    assert st.converged == int(np.sum(statusb == 0))


def test_oracle_flags_the_same_reactors(oracle_mod):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", B)
    bc, bx0 = _poison(cond, x0)
    idx = np.array(sorted(BAD))
    xo, so = oracle_mod.solve_batch(mech, bc, bx0, energy, idx=idx)
    assert np.all(so["status"] == 3)
    assert np.array_equal(xo, bx0[:, idx], equal_nan=True)


@pytest.mark.parametrize("engine", [1, 2])
def test_budgeted_solve_resumes_to_the_oracle_roots(P, oracle_mod, engine):
    """A solve stopped by a small linear-solve budget (status MAXITER), then
    called again on its own output with the default budget (a warm start),
    ends at the roots the oracle finds from the original initial guess."""
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 32)
    M = P.Mechanism(mech)
    x1, s1, n1, _ = solve_gpu(M, cond, x0, energy, max_lin=6, engine=engine, scheduler=1)
    assert np.all(n1 <= 6) and np.sum(s1 == 1) >= 16
    x2, s2, _, _ = solve_gpu(M, cond, x1, energy, engine=engine, scheduler=1)
    xo, so = oracle_mod.solve_batch(mech, cond, x0, energy, processes=8)
    parity(oracle_mod, mech, cond, energy, x2, s2, xo, so, 1e-7, max_branch_frac=0.1,
           label=f"resume engine {engine}")
    assert np.all(s2[so["status"] == 0] == 0)
