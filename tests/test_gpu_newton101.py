"""GPU parity of one Newton iteration (residual, analytic Jacobian, FP64 LU
factorisation and solve) on the 101-species / 542-reaction stand-in for the
mechanism of the paper's single-iteration speed-up measurement (Section 6:
isothermal 1800 K, tau = 50 ms, fuel/oxidizer/diluent 0.15/0.18/0.67), called
through the C ABI and compared with the oracle element by element."""
import numpy as np
import pytest

from tests.gpu_util import cond_dev, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    import paper_2005_11468_amd as P
    return P


def _states(N, B, seed):
    rng = np.random.default_rng(seed)
    return rng.dirichlet(np.full(N, 0.4), B).T.copy()


def _newton_step_gpu(gpu, M, cond, x):
    """F, J and the Newton step d = -J^-1 F of every reactor on the GPU."""
    import torch
    cd = cond_dev(cond)
    xd = dev(x)
    F = gpu.residual(M, cd, False, xd)
    J = gpu.jacobian(M, cd, False, xd)
    LU, piv, info = gpu.lu_factor_batch(J.clone())
    rhs = (-F).t().contiguous()
    d = gpu.lu_solve_batch(LU, piv, rhs)
    torch.cuda.synchronize()
    return F.cpu().numpy(), J.cpu().numpy(), info.cpu().numpy(), d.cpu().numpy()


def _oracle_step(O, oracle_mod, cond, x, b):
    args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], False, x[:, b])
    Fo = O.residual(*args)
    Jo = O.jacobian(*args)
    lo, po, io = oracle_mod.lu_factor(Jo)
    assert io == 0
    do = oracle_mod.lu_solve(lo, po, -Fo)
    _check_step(Jo, Fo, do, -1)  # the oracle's own step meets the same bound
    return Fo, Jo, do


def _check_step(Jo, Fo, d, b):
    """The step solves the oracle's linear system to within the Jacobian's
    parity tolerance (normwise backward error).  These Jacobians have
    condition numbers of 1e18 and more (stiff kinetics at 1800 K, no
    equilibration), so the step's digits are not fixed by the system and an
    element-wise comparison with the oracle's own step would test rounding
    order, not correctness."""
    r = Jo @ d + Fo
    assert np.all(np.isfinite(d)), b
    assert np.abs(r).max() <= 1e-9 * (np.abs(Jo) @ np.abs(d) + np.abs(Fo)).max(), b


def test_newton_iteration_matches_oracle(gpu, oracle_mod):
    from psr_inputs import workload
    mech, cond, _, _ = workload("newton101", 37)  # ragged against every tile
    M = gpu.Mechanism(mech)
    O = oracle_mod.Mechanism(mech)
    N = M.n_species
    assert N == 101 and mech["A"].shape[0] == 542
    x = _states(N, 37, 101)
    F, J, info, d = _newton_step_gpu(gpu, M, cond, x)
    assert np.all(info == 0)
    for b in range(37):
        Fo, Jo, do = _oracle_step(O, oracle_mod, cond, x, b)
        np.testing.assert_allclose(F[:, b], Fo, rtol=1e-10, atol=1e-12 * np.abs(Fo).max(),
                                   err_msg=f"F b={b}")
        scale = np.abs(Jo).max(axis=1, keepdims=True)
        bad = np.abs(J[b] - Jo) > 1e-10 * np.abs(Jo) + 1e-13 * scale
        assert not bad.any(), (b, np.argwhere(bad)[:4])
        _check_step(Jo, Fo, d[b], b)


def test_newton_iteration_at_scale_sampled(gpu, oracle_mod):
    """100000 reactors at the measurement's inlet state (every reactor the
    same): all reactors give bitwise the same F, J and step, and sampled ones
    match the oracle."""
    from psr_inputs import workload
    B = 100_000
    mech, cond1, _, _ = workload("newton101", 1)  # every reactor of the workload is alike
    cond = {k: np.ascontiguousarray(np.repeat(v[..., :1], B, axis=-1)) for k, v in cond1.items()}
    x0 = cond["Y_in"].copy()
    assert x0.shape == (101, B) and cond["P"].shape == (B,)
    M = gpu.Mechanism(mech)
    O = oracle_mod.Mechanism(mech)
    F, J, info, d = _newton_step_gpu(gpu, M, cond, x0)
    assert np.all(info == 0)
    assert np.all(F == F[:, :1]) and np.all(d == d[:1])
    assert np.all(J[::997] == J[0])
    for b in (0, 4242, B - 1):
        Fo, Jo, do = _oracle_step(O, oracle_mod, cond, x0, b)
        np.testing.assert_allclose(F[:, b], Fo, rtol=1e-10, atol=1e-12 * np.abs(Fo).max())
        scale = np.abs(Jo).max(axis=1, keepdims=True)
        assert not (np.abs(J[b] - Jo) > 1e-10 * np.abs(Jo) + 1e-13 * scale).any()
        _check_step(Jo, Fo, d[b], b)
