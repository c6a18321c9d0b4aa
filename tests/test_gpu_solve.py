"""GPU parity of the full batched solve against the oracle (called through
the C ABI): FP64 and mixed precision, plain and persistent schedulers."""
import numpy as np
import pytest

from tests import tiny_mechs as tm
from tests.gpu_util import parity, rel_err, solve_gpu

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


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheduler", [0, 1])
def test_isothermal_workload(P, oracle_mod, precision, scheduler, engine):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("isothermal")
    xo, _ = _oracle(oracle_mod, mech, cond, x0, energy)
    x, status, nlin, st = solve_gpu(P.Mechanism(mech), cond, x0, energy, precision=precision,
                                    scheduler=scheduler, engine=engine)
    assert np.all(status == 0)
    err = rel_err(x, xo, mech["species_elems"].shape[0])
    assert err.max() <= TOL[precision], err


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheduler", [0, 1])
def test_energy_workload_sample(P, oracle_mod, precision, scheduler, engine):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 200)
    xo, so = _oracle(oracle_mod, mech, cond, x0, energy)
    M = P.Mechanism(mech)
    x, status, nlin, st = solve_gpu(M, cond, x0, energy, precision=precision,
                                    scheduler=scheduler, engine=engine)
    assert np.all(status == 0)
    parity(oracle_mod, mech, cond, energy, x, status, xo, so, TOL[precision],
           label=f"energy p{precision} s{scheduler} e{engine}")


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_schedulers_agree_bitwise(P, engine, precision):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 96)
    M = P.Mechanism(mech)
    a = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PLAIN, engine=engine, precision=precision)
    b = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PERSISTENT, engine=engine, precision=precision)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager_launches(P, engine, precision):
    """The plain scheduler replays each check period (counter reset + four
    rounds) as a captured HIP graph; dozens of replays, with the host's reads
    of the active count and stream synchronisations between them, must give
    exactly what launching the same kernels one by one gives."""
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 80)
    M = P.Mechanism(mech)
    a = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PLAIN, engine=engine, precision=precision, use_graph=1)
    b = solve_gpu(M, cond, x0, energy, scheduler=P.PSR_PLAIN, engine=engine, precision=precision, use_graph=0)
    assert a[3].rounds == b[3].rounds and a[3].rounds >= 40
    for u, v in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(u, v)


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


@pytest.mark.parametrize("n_react", [1, 3, 5, 67])
def test_ragged_batches(P, oracle_mod, n_react):
    """Batch sizes that leave partly filled workgroups (4 reactors per workgroup)."""
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", n_react)
    xo, so = _oracle(oracle_mod, mech, cond, x0, energy)
    M = P.Mechanism(mech)
    for sched in (0, 1):
        x, status, _, _ = solve_gpu(M, cond, x0, energy, scheduler=sched, precision=1)
        assert np.all(status == 0)
        parity(oracle_mod, mech, cond, energy, x, status, xo, so, TOL[1], label=f"ragged {n_react}")


def test_tiny_mechanisms_on_wave_engine(P, oracle_mod):
    """n = 2 .. 6 unknowns (NP = 16 register rows), isothermal and with energy."""
    for mech, energy in ((tm.small_network(), False), (tm.small_network(), True),
                         (tm.association(), False)):
        n_sp = mech["species_elems"].shape[0]
        rng = np.random.default_rng(3)
        B = 9
        cond = {"P": np.full(B, 101325.0), "tau": np.exp(rng.uniform(np.log(1e-5), 0, B)),
                "T_in": rng.uniform(300, 900, B) if energy else np.full(B, 1400.0),
                "Y_in": rng.dirichlet(np.ones(n_sp), B).T.copy()}
        x0 = np.concatenate([cond["Y_in"], np.full((1, B), 1500.0)]) if energy else cond["Y_in"].copy()
        xo, so = oracle_mod.solve_batch(mech, cond, x0, energy)
        M = P.Mechanism(mech)
        for prec in (0, 1):
            x, status, _, _ = solve_gpu(M, cond, x0, energy, precision=prec, engine=2,
                                        scheduler=P.PSR_PERSISTENT)
            parity(oracle_mod, mech, cond, energy, x, status, xo, so, TOL[prec], label="tiny")


@pytest.mark.parametrize("scheduler", [0, 1])
def test_multi_group_stats_match_status_arrays(P, scheduler):
    """Two mechanisms in one call: the totals in psr_solve_stats equal the
    sums over the per-reactor status and linear-solve arrays of both groups
    (the plain scheduler runs the groups in turn on one workspace region)."""
    import torch
    from psr_inputs import workload
    from tests.gpu_util import cond_dev, dev
    gl = []
    for name, B in (("isothermal", 16), ("energy", 24)):
        mech, cond, x0, energy = workload(name, B)
        gl.append(dict(mech=P.Mechanism(mech), cond=cond_dev(cond), energy=energy, x=dev(x0),
                       status=torch.full((B,), -1, dtype=torch.int32, device="cuda:0"),
                       n_lin=torch.zeros((B,), dtype=torch.int32, device="cuda:0")))
    st, _ = P.solve_batch(gl, P.default_opts(scheduler=scheduler))
    torch.cuda.synchronize()
    status = np.concatenate([g["status"].cpu().numpy() for g in gl])
    nlin = np.concatenate([g["n_lin"].cpu().numpy() for g in gl])
    assert st.reactors == len(status)
    assert st.converged == int((status == 0).sum())
    assert st.lin_total == int(nlin.sum())
    assert st.lin_max == int(nlin.max())


@pytest.mark.parametrize("engine", [1, 2])
def test_queue_order_leaves_results_bitwise_unchanged(P, engine):
    """The persistent scheduler's longest-residence-time-first queue order
    changes only which reactor runs when: x, status and n_lin are bitwise
    those of batch order."""
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 96)
    M = P.Mechanism(mech)
    a = solve_gpu(M, cond, x0, energy, scheduler=1, engine=engine, precision=1, order=0)
    b = solve_gpu(M, cond, x0, energy, scheduler=1, engine=engine, precision=1, order=1)
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    assert a[3].converged == b[3].converged and a[3].lin_total == b[3].lin_total
