"""GPU parity of the full batched solve against the oracle (called through
the C ABI): FP64 and mixed precision, plain and persistent schedulers."""
import numpy as np
import pytest

from tests import tiny_mechs as tm
from tests.gpu_util import rel_err, solve_gpu

pytestmark = pytest.mark.gpu

TOL = {0: 1e-8, 1: 1e-7}  # PSR_FP64, PSR_MIXED


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    return P


def _oracle(oracle_mod, mech, cond, x0, energy):
    xs, st = oracle_mod.solve_batch(mech, cond, x0, energy, processes=8)
    assert np.all(st["status"] == 0)
    return xs, st


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheduler", [0, 1])
def test_isothermal_workload(P, oracle_mod, precision, scheduler):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("isothermal")
    xo, _ = _oracle(oracle_mod, mech, cond, x0, energy)
    x, status, nlin, st = solve_gpu(P.Mechanism(mech), cond, x0, energy, precision=precision,
                                    scheduler=scheduler)
    assert np.all(status == 0)
    err = rel_err(x, xo, mech["species_elems"].shape[0])
    assert err.max() <= TOL[precision], err


@pytest.mark.parametrize("precision", [0, 1])
def test_energy_workload_sample(P, oracle_mod, precision):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 200)
    xo, so = _oracle(oracle_mod, mech, cond, x0, energy)
    M = P.Mechanism(mech)
    x, status, nlin, st = solve_gpu(M, cond, x0, energy, precision=precision,
                                    scheduler=P.PSR_PERSISTENT)
    assert np.all(status == 0)
    err = rel_err(x, xo, M.n_species)
    assert err.max() <= TOL[precision], (np.sort(err)[-5:], np.argsort(err)[-5:])


def test_schedulers_agree_bitwise(P):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 96)
    M = P.Mechanism(mech)
    a = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PLAIN)
    b = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PERSISTENT)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


def test_reactor_order_does_not_change_results(P):
    from psr_inputs import subset, workload
    mech, cond, x0, energy = workload("energy", 64)
    M = P.Mechanism(mech)
    perm = np.random.default_rng(1).permutation(64)
    c2, x2 = subset(cond, x0, perm)
    a = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PERSISTENT, precision=P.PSR_MIXED)
    b = solve_gpu(M, c2, x2, energy, scheduler=P.PSR_PERSISTENT, precision=P.PSR_MIXED)
    np.testing.assert_array_equal(a[0][:, perm], b[0])


@pytest.mark.parametrize("tau", [1e-5, 3e-3, 0.2, 40.0])
def test_isomerisation_closed_form_on_gpu(P, tau):
    A, da6, da7, T = 3.0e3, -1500.0, 0.7, 1500.0
    mech = tm.isomerisation(A=A, da6=da6, da7=da7)
    Kc = np.exp(da7 - da6 / T)
    kf, kr = A, A / Kc
    Yin = np.array([[0.8], [0.2]])
    cond = {"P": np.array([101325.0]), "tau": np.array([tau]), "T_in": np.array([T]), "Y_in": Yin}
    x, status, _, _ = solve_gpu(P.Mechanism(mech), cond, Yin.copy(), False)
    YA = (0.8 / tau + kr) / (1 / tau + kf + kr)
    assert status[0] == 0
    np.testing.assert_allclose(x[:, 0], [YA, 1 - YA], rtol=1e-13)


def test_warm_start_and_budget(P, oracle_mod):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 8)
    M = P.Mechanism(mech)
    x, status, nlin, _ = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PERSISTENT)
    x2, status2, nlin2, _ = solve_gpu(M, cond, x, energy, scheduler=P.PSR_PERSISTENT)
    assert np.all(status2 == 0) and np.all(nlin2 <= 2)
    x3, status3, nlin3, _ = solve_gpu(M, cond, x0, energy, max_lin=10)
    assert np.all(status3 == 1) and np.all(nlin3 <= 10)
