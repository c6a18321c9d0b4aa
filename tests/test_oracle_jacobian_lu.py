"""Pins of the oracle's analytic Jacobian and LU factorisation."""
import numpy as np
import pytest
import scipy.linalg as sla

from tests import tiny_mechs as tm

PATM = 101325.0


def _close(A, B, rtol, row_atol):
    """|A - B| <= rtol |B| + row_atol * max_j |B_ij| elementwise, with a report."""
    scale = np.abs(B).max(axis=1, keepdims=True)
    bad = np.abs(A - B) > rtol * np.abs(B) + row_atol * scale
    assert not bad.any(), (np.argwhere(bad)[:5], (np.abs(A - B) / (np.abs(B) + 1e-300))[bad][:5])


def _states(m, energy, rng, count):
    for _ in range(count):
        Y = rng.dirichlet(np.full(m.n_sp, 0.5))
        x = np.r_[Y, rng.uniform(700, 2700)] if energy else Y
        yield x


@pytest.mark.parametrize("energy", [False, True])
def test_jacobian_matches_complex_step_small(oracle_mod, energy):
    m = oracle_mod.Mechanism(tm.small_network())
    rng = np.random.default_rng(11)
    Yin = np.array([0.1, 0.2, 0.3, 0.25, 0.15])
    for x in _states(m, energy, rng, 4):
        J = m.jacobian(PATM, 2e-3, 650.0, Yin, energy, x)
        Jc = m.jacobian(PATM, 2e-3, 650.0, Yin, energy, x, complex_step=True)
        _close(J, Jc, 1e-12, 1e-13)


@pytest.mark.parametrize("energy", [False, True])
def test_jacobian_matches_central_differences(oracle_mod, energy):
    m = oracle_mod.Mechanism(tm.small_network())
    rng = np.random.default_rng(12)
    Yin = np.array([0.1, 0.2, 0.3, 0.25, 0.15])
    for x in _states(m, energy, rng, 3):
        J = m.jacobian(PATM, 2e-3, 650.0, Yin, energy, x)
        Jfd = np.zeros_like(J)
        for k in range(len(x)):
            h = 1e-6 * max(abs(x[k]), 1e-3)
            xp, xm = x.copy(), x.copy()
            xp[k] += h
            xm[k] -= h
            Jfd[:, k] = (m.residual(PATM, 2e-3, 650.0, Yin, energy, xp)
                         - m.residual(PATM, 2e-3, 650.0, Yin, energy, xm)) / (2 * h)
        _close(Jfd, J, 1e-6, 1e-7)


def test_jacobian_matches_complex_step_generated(oracle_mod):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 4)
    m = oracle_mod.Mechanism(mech)
    rng = np.random.default_rng(13)
    for b in range(2):
        x = np.r_[rng.dirichlet(np.full(m.n_sp, 0.3)), rng.uniform(900, 2500)]
        args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], True, x)
        J = m.jacobian(*args)
        Jc = m.jacobian(*args, complex_step=True)
        _close(J, Jc, 1e-11, 1e-13)


@pytest.mark.parametrize("n", [1, 2, 7, 31, 54, 64])
def test_lu_matches_lapack(oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n))
    lu, piv, info = oracle_mod.lu_factor(A)
    assert info == 0
    lu_ref, piv_ref = sla.lu_factor(A)
    np.testing.assert_array_equal(piv, piv_ref)
    np.testing.assert_allclose(lu, lu_ref, rtol=1e-11, atol=1e-13)
    b = rng.standard_normal(n)
    z = oracle_mod.lu_solve(lu, piv, b)
    # backward error of the solve
    r = A @ z - b
    assert np.linalg.norm(r, np.inf) <= 10 * n * np.finfo(float).eps * (
        np.linalg.norm(A, np.inf) * np.linalg.norm(z, np.inf) + np.linalg.norm(b, np.inf))


def test_lu_on_psr_jacobian(oracle_mod):
    from psr_inputs import workload
    mech, cond, x0, energy = workload("energy", 2)
    m = oracle_mod.Mechanism(mech)
    x = np.r_[np.random.default_rng(5).dirichlet(np.full(m.n_sp, 0.5)), 1800.0]
    J = m.jacobian(cond["P"][0], cond["tau"][0], cond["T_in"][0], cond["Y_in"][:, 0], True, x)
    lu, piv, info = oracle_mod.lu_factor(J)
    lu_ref, piv_ref = sla.lu_factor(J)
    np.testing.assert_array_equal(piv, piv_ref)
    np.testing.assert_allclose(lu, lu_ref, rtol=1e-10, atol=1e-12 * np.abs(J).max())


def test_lu_reports_singular(oracle_mod):
    A = np.array([[1.0, 2.0], [2.0, 4.0]])
    _, _, info = oracle_mod.lu_factor(A)
    assert info == 2
    _, _, info = oracle_mod.lu_factor(np.zeros((3, 3)))
    assert info == 1
