"""GPU parity on the sooting workload: 150 species / 900 reactions with six
soot moments (MOMIC) per reactor, n = 157 unknowns, workgroup engine with
the matrices in HBM.  Residual and Jacobian element by element at seeded
states; whole solves on a seeded sample against the oracle."""
import numpy as np
import pytest

from tests.gpu_util import cond_dev, dev, parity, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-8, 1: 1e-7}  # PSR_FP64, PSR_MIXED
# seeded sample of the 8192-reactor workload over its whole residence-time
# range (1 ms to 0.1 s)
SAMPLE = np.sort(np.random.default_rng(5).choice(8192, 16, replace=False))


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    return P


@pytest.fixture(scope="module")
def states():
    """Seeded soot states: random compositions and temperatures, lognormal
    moment sets from 1e6 to 1e11 particles per cm^3."""
    from psr_inputs import workload
    mech, cond, x0, _ = workload("soot", 24)
    N = mech["species_elems"].shape[0]
    rng = np.random.default_rng(31)
    x = x0.copy()
    r = np.arange(6)
    for b in range(x.shape[1]):
        x[:N, b] = rng.dirichlet(np.full(N, 0.3))
        x[N, b] = rng.uniform(1100, 2400)
        mg, s = rng.uniform(8, 400), rng.uniform(0.2, 1.0)
        x[N + 1:, b] = np.log(10 ** rng.uniform(6, 11)) + r * np.log(mg) + r ** 2 * s * s / 2
    x[N + 1:, 0] = np.log(0.5) + r * np.log(12.0)  # below one particle: growth, coagulation off
    return mech, cond, x


def test_soot_unknowns_and_isothermal_rejected(P, states):
    import torch
    mech, cond, x = states
    M = P.Mechanism(mech)
    N = mech["species_elems"].shape[0]
    assert M.n_unknowns(True) == N + 7 and M.n_unknowns(False) == N
    with pytest.raises(P.PSRError):
        P.residual(M, cond_dev(cond), False, dev(x[:N]))
    torch.cuda.synchronize()


def test_soot_residual_matches_oracle(P, oracle_mod, states):
    import torch
    mech, cond, x = states
    M = P.Mechanism(mech)
    O = oracle_mod.Mechanism(mech)
    B = x.shape[1]
    sc = torch.empty(B, dtype=torch.float64, device="cuda:0")
    F = P.residual(M, cond_dev(cond), True, dev(x), scaled=sc).cpu().numpy()
    sc = sc.cpu().numpy()
    N = O.n_sp
    for b in range(B):
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], True, x[:, b])
        Fo = O.residual(*args)
        gas = np.abs(Fo[:N + 1]).max()
        np.testing.assert_allclose(F[:N + 1, b], Fo[:N + 1], rtol=1e-10, atol=1e-12 * gas, err_msg=f"b={b}")
        # moment rows: each relative to its outflow term M_r / tau
        mr = np.exp(x[N + 1:, b]) / cond["tau"][b]
        assert np.all(np.abs(F[N + 1:, b] - Fo[N + 1:]) <= 1e-10 * (mr + np.abs(Fo[N + 1:]))), b
        np.testing.assert_allclose(sc[b], O.scaled_residual(*args), rtol=1e-8, err_msg=f"b={b}")


def test_soot_jacobian_matches_oracle(P, oracle_mod, states):
    mech, cond, x = states
    M = P.Mechanism(mech)
    O = oracle_mod.Mechanism(mech)
    B = 12
    c = {k: np.ascontiguousarray(v[..., :B]) for k, v in cond.items()}
    J = P.jacobian(M, cond_dev(c), True, dev(np.ascontiguousarray(x[:, :B]))).cpu().numpy()
    for b in range(B):
        Jo = O.jacobian(c["P"][b], c["tau"][b], c["T_in"][b], c["Y_in"][:, b], True, x[:, b])
        scale = np.abs(Jo).max(axis=1, keepdims=True)
        bad = np.abs(J[b] - Jo) > 1e-10 * np.abs(Jo) + 1e-12 * scale
        assert not bad.any(), (b, np.argwhere(bad)[:4])


@pytest.fixture(scope="module")
def sample(oracle_mod):
    from psr_inputs import subset, workload
    mech, cond, x0, _ = workload("soot")
    cond, x0 = subset(cond, x0, SAMPLE)
    print(f"oracle: soot B={len(SAMPLE)}", flush=True)
    xo, so = oracle_mod.solve_batch(mech, cond, x0, True, processes=8)
    return mech, cond, x0, xo, so


def _solve(P, mech, cond, x0, **opts):
    import torch
    M = P.Mechanism(mech)
    B = x0.shape[1]
    x = dev(x0)
    status = torch.full((B,), -1, dtype=torch.int32, device="cuda:0")
    nlin = torch.zeros((B,), dtype=torch.int32, device="cuda:0")
    st, _ = P.solve_batch([dict(mech=M, cond=cond_dev(cond), energy=True, x=x, status=status, n_lin=nlin)],
                          P.default_opts(**opts))
    torch.cuda.synchronize()
    return x.cpu().numpy(), status.cpu().numpy(), nlin.cpu().numpy(), st


@pytest.mark.parametrize("precision", [0, 1])
def test_soot_solve_matches_oracle(P, oracle_mod, sample, precision):
    """Oracle parity at the default budget (tests.gpu_util.parity): the
    oracle converges every sampled reactor, the GPU roots agree within the
    tolerance or are verified steady states, and no oracle root is missed."""
    mech, cond, x0, xo, so = sample
    x, status, nlin, st = _solve(P, mech, cond, x0, precision=precision, scheduler=P.PSR_PERSISTENT)
    assert np.all(so["status"] == 0), so["status"]
    parity(oracle_mod, mech, cond, True, x, status, xo, so, TOL[precision], label=f"soot p{precision}")


@pytest.mark.parametrize("precision", [0, 1])
def test_soot_schedulers_agree_bitwise(P, sample, precision):
    """Plain and persistent scheduling give identical results, also in mixed
    precision, where the controller state carried between rounds includes
    the FP64-fallback bookkeeping."""
    mech, cond, x0, _, _ = sample
    a = _solve(P, mech, cond, x0, precision=precision, scheduler=P.PSR_PERSISTENT)
    b = _solve(P, mech, cond, x0, precision=precision, scheduler=P.PSR_PLAIN)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0])
