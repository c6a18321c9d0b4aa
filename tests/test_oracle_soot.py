"""Pins of the oracle's soot-moment model (MOMIC) against closed forms.

The paper couples a soot population, by Frenklach's method of moments with
interpolative closure, to the gas phase of its sooting reactor (Sections
1-2 and 6) but prints no equations; the oracle follows the published method
(nucleation, surface growth, free-molecular coagulation, Lagrange closure
in ln mu).  What pins it:
  * a lognormal size distribution has ln mu_p exactly quadratic in p, so the
    interpolated (and extrapolated) fractional moments are exact;
  * a monodisperse population (mu_p = m^p) makes every coagulation grid
    function exact: f_{x,y} = 4 sqrt(2) m^(x+y+1/6), and the coagulation
    sources reduce to G_r / G_0 = -(2^r - 2) m^r (two particles of mass m
    merge into one of mass 2m); the growth sources to
    W_r / W_1 = ((m + D)^r - m^r) / D (D atoms added to a particle of mass m);
  * nucleation sources scale as C_min^r and [P]^2;
  * the species rows conserve mass with the soot: sum_i F_i =
    mdot (sum Y - 1) + V W_C (R_1 + W_1) / N_A at any state;
  * at a converged root: sum Y + Y_soot = 1, h_mix(T, Y) = h_mix(T_in, Y_in),
    and with growth and coagulation off M_r = tau R_r;
  * the Jacobian's soot block matches the complex-step derivative.
"""
import numpy as np
import pytest

NA = 6.02214076e23
R_GAS = 8.314462618


@pytest.fixture(scope="module")
def soot_mech():
    from psr_inputs import mechanism
    return mechanism("soot")


def _lognormal_lnM(M0, mg, sigma):
    r = np.arange(6)
    return np.log(M0) + r * np.log(mg) + r ** 2 * sigma ** 2 / 2


def _mono_lnM(M0, m):
    return np.log(M0) + np.arange(6) * np.log(m)


@pytest.mark.parametrize("p", [-0.5, -1.0 / 6, 1.0 / 6, 2.0 / 3, 2.5, 14.0 / 3, 5.5, 43.0 / 6])
def test_lognormal_closure_exact(oracle_mod, p):
    mg, sigma = 350.0, 0.9
    lnM = _lognormal_lnM(1e9, mg, sigma)
    exact = p * np.log(mg) + p ** 2 * sigma ** 2 / 2
    assert abs(oracle_mod.soot_ln_mu(lnM, p) - exact) <= 1e-12 * max(1.0, abs(exact))


@pytest.mark.parametrize("xy", [(0, 0), (1, 1), (1, 3), (2, 2), (3, 2), (4, 1)])
def test_monodisperse_coagulation_interpolant(oracle_mod, xy):
    m = 57.0
    f = oracle_mod.soot_fxy(_mono_lnM(3e10, m), *xy)
    exact = 4.0 * np.sqrt(2.0) * m ** (xy[0] + xy[1] + 1.0 / 6)
    assert f == pytest.approx(exact, rel=1e-12)


def test_monodisperse_sources(oracle_mod, soot_mech):
    O = oracle_mod.Mechanism(soot_mech)
    sd = soot_mech["soot"]
    D = soot_mech["species_elems"][sd["growth"], sd["carbon"]]
    Cmin = 2 * soot_mech["species_elems"][sd["precursor"], sd["carbon"]]
    m, M0, T, CP, CG = 40.0, 2e9, 1700.0, 3e-9, 2e-8
    R, W, G, sk = O.soot_sources(T, CP, CG, _mono_lnM(M0, m))
    # coagulation: G_1 = 0, G_r / G_0 = -(2^r - 2) m^r
    assert G[0] < 0 and G[1] == 0.0
    for r in range(2, 6):
        assert G[r] / G[0] == pytest.approx(-(2 ** r - 2) * m ** r, rel=1e-12)
    # growth: W_0 = 0, W_r / W_1 = ((m + D)^r - m^r) / D
    assert W[0] == 0.0 and W[1] > 0
    for r in range(2, 6):
        assert W[r] / W[1] == pytest.approx(((m + D) ** r - m ** r) / D, rel=1e-12)
    # nucleation: R_r / R_0 = C_min^r
    for r in range(1, 6):
        assert R[r] / R[0] == pytest.approx(float(Cmin) ** r, rel=1e-14)
    # gas sinks: 2 I of the precursor, W_1 / (D N_A) of the growth species
    assert sk[0] == pytest.approx(2 * R[0] / NA, rel=1e-14)
    assert sk[1] == pytest.approx(W[1] / (D * NA), rel=1e-14)
    # scalings: G ~ M_0^2 sqrt(T) at fixed m, W ~ [G], R ~ [P]^2
    R2, W2, G2, _ = O.soot_sources(4 * T, 2 * CP, 3 * CG, _mono_lnM(2 * M0, m))
    assert G2[0] / G[0] == pytest.approx(4.0 * 2.0, rel=1e-12)
    kn = lambda T_: sd["A_nuc"] * T_ ** sd["beta_nuc"] * np.exp(-sd["E_nuc"] / (R_GAS * T_))
    assert R2[0] / R[0] == pytest.approx(4.0 * kn(4 * T) / kn(T), rel=1e-12)


def test_growth_and_coagulation_off_below_one_particle(oracle_mod, soot_mech):
    O = oracle_mod.Mechanism(soot_mech)
    R, W, G, sk = O.soot_sources(1500.0, 1e-9, 1e-8, _mono_lnM(0.5, 12.0))
    assert np.all(W == 0.0) and np.all(G == 0.0) and R[0] > 0 and sk[1] == 0.0


def _soot_state(soot_mech, rng, B=1):
    from psr_inputs import workload
    mech, cond, x0, _ = workload("soot", 64)
    N = mech["species_elems"].shape[0]
    x = x0[:, :B].copy()
    for b in range(B):
        x[:N, b] = rng.dirichlet(np.full(N, 0.3))
        x[N, b] = rng.uniform(1100, 2400)
        x[N + 1:, b] = _lognormal_lnM(10 ** rng.uniform(6, 11), rng.uniform(8, 400), rng.uniform(0.2, 1.0))
    return mech, cond, x


def test_soot_jacobian_matches_complex_step(oracle_mod, soot_mech):
    mech, cond, x = _soot_state(soot_mech, np.random.default_rng(5))
    O = oracle_mod.Mechanism(mech)
    args = (cond["P"][0], cond["tau"][0], cond["T_in"][0], cond["Y_in"][:, 0], True, x[:, 0])
    J = O.jacobian(*args)
    Jc = O.jacobian(*args, complex_step=True)
    scale = np.abs(Jc).max(axis=1, keepdims=True)
    assert np.all(np.abs(J - Jc) <= 1e-12 * scale + 1e-300)


def test_species_rows_conserve_mass_with_soot(oracle_mod, soot_mech):
    mech, cond, x = _soot_state(soot_mech, np.random.default_rng(6), B=4)
    O = oracle_mod.Mechanism(mech)
    N = O.n_sp
    Wc = mech["elem_weight"][mech["soot"]["carbon"]]
    for b in range(4):
        P, tau, Tin, Yin = cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b]
        F = O.residual(P, tau, Tin, Yin, True, x[:, b])
        Y, T = x[:N, b], x[N, b]
        rho = P * 1e-6 / (R_GAS * T * np.sum(Y / O.W))
        mdot = rho / tau
        Cc, _, _ = O.production(T, P, Y)
        R, W, G, _ = O.soot_sources(T, Cc[mech["soot"]["precursor"]], Cc[mech["soot"]["growth"]],
                                    x[N + 1:, b])
        expect = mdot * (Y.sum() - 1.0) + Wc * (R[1] + W[1]) / NA
        scale = np.abs(F[:N]).sum()
        assert abs(F[:N].sum() - expect) <= 1e-12 * scale


def _converged(oracle_mod, mech, idx, **consts):
    from psr_inputs import workload
    m2 = dict(mech)
    m2["soot"] = dict(mech["soot"], **consts)
    O = oracle_mod.Mechanism(m2)
    _, cond, x0, _ = workload("soot", 64)
    b = idx
    args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b], True)
    x, st = O.solve(*args, x0[:, b])
    return O, m2, cond, b, x, st


@pytest.mark.parametrize("consts", [{}, {"A_grow": 0.0, "coag_scale": 0.0}])
def test_converged_root_invariants(oracle_mod, soot_mech, consts):
    """Reactor 3 of the sooting workload (tau 1.0 ms) converges."""
    O, m2, cond, b, x, st = _converged(oracle_mod, soot_mech, 3, **consts)
    assert st.status == 0
    N = O.n_sp
    P, tau, Tin, Yin = cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b]
    assert O.scaled_residual(P, tau, Tin, Yin, True, x) <= 1e-10
    Y, T, lnM = x[:N], x[N], x[N + 1:]
    Wc = m2["elem_weight"][m2["soot"]["carbon"]]
    rho = P * 1e-6 / (R_GAS * T * np.sum(Y / O.W))
    Ysoot = np.exp(lnM[1]) * Wc / (NA * rho)
    assert Y.sum() + Ysoot == pytest.approx(1.0, abs=1e-10)
    # adiabatic: mixture enthalpy of the gas at the root equals the inlet's
    hi = lambda T_: R_GAS * T_ * O.thermo(T_)[1] / O.W
    scale = np.sum(np.abs(Yin * hi(Tin)))
    assert abs(np.sum(Y * hi(T)) - np.sum(Yin * hi(Tin))) <= 1e-10 * scale
    if consts:
        Cc, _, _ = O.production(T, P, Y)
        R, W, G, _ = O.soot_sources(T, Cc[m2["soot"]["precursor"]], Cc[m2["soot"]["growth"]], lnM)
        assert np.allclose(np.exp(lnM), tau * R, rtol=1e-10)


def test_monodisperse_sources_absolute(oracle_mod, soot_mech):
    """Absolute source values at T = 1700 K for a monodisperse population
    (M_0 = 2e9 cm^-3, m = 40 carbon atoms) from the published formulas, the
    numbers worked out separately (double precision, constants: N_A =
    6.02214076e23 /mol, k_B = 1.380649e-16 erg/K, R = 8.314462618 J/mol/K,
    m_C = 12.011 g/mol / N_A, rho_s = 1.8 g/cm^3, chi = 2.3e15 /cm^2):
      K_f = 2.2 (3 m_C / (4 pi rho_s))^(1/6) (6 k_B T / rho_s)^(1/2)
          = 2.2884390353e-10 cm^3/s,
      G_0 = -(1/2) K_f M_0^2 f_00, f_00 = 4 sqrt(2) m^(1/6)
          = -4.78800208182e9 /(cm^3 s),
      W_1 = k_s [G] chi pi d_C^2 M_0 D m^(2/3), d_C = (6 m_C / (pi rho_s))^(1/3)
          = 2.7660012947e-8 cm, k_s = 1e9 exp(-4e4 / (R T)), [G] = 2e-8 mol/cm^3,
          D = 2: W_1 = 3.05271381607e11 /(cm^3 s),
      R_0 = N_A k_n [P]^2, k_n = 1e9 exp(-5e4 / (R T)), [P] = 3e-9 mol/cm^3:
          R_0 = 1.57655986748e14 /(cm^3 s).
    A wrong exponent, a missing pi or factor 2 in any prefactor fails."""
    O = oracle_mod.Mechanism(soot_mech)
    R, W, G, sk = O.soot_sources(1700.0, 3e-9, 2e-8, _mono_lnM(2e9, 40.0))
    assert G[0] == pytest.approx(-4.78800208182457e9, rel=1e-11)
    assert W[1] == pytest.approx(3.052713816068612e11, rel=1e-11)
    assert R[0] == pytest.approx(1.5765598674782403e14, rel=1e-11)


def test_soot_outputs_of_a_monodisperse_population(oracle_mod):
    """N spheres per cm^3 of diameter d: volume fraction N pi d^3 / 6 (a
    geometric identity, independent of the moment formulas), number density
    N and diameter d back; doubling N at fixed particle size doubles f_v and
    keeps d."""
    from psr_inputs import configs
    mech = configs.mechanism("soot")
    M = oracle_mod.Mechanism(mech)
    sd = mech["soot"]
    mC = mech["elem_weight"][sd["carbon"]] / 6.02214076e23
    for d_nm, N in ((10.0, 1e10), (1.0, 3e12), (80.0, 2e8)):
        d = d_nm * 1e-7
        m = sd["soot_density"] * np.pi * d ** 3 / 6.0 / mC  # carbon atoms per particle
        lnM = np.log(N) + np.arange(6) * np.log(m)
        x = np.concatenate([np.zeros(M.n_sp + 1), lnM])
        fv, n_out, d_out = M.soot_outputs(x)
        assert fv == pytest.approx(N * np.pi * d ** 3 / 6.0, rel=1e-12)
        assert n_out == pytest.approx(N, rel=1e-14)
        assert d_out == pytest.approx(d, rel=1e-12)
        x2 = x.copy()
        x2[M.n_sp + 1:] += np.log(2.0)
        fv2, n2, d2 = M.soot_outputs(x2)
        assert fv2 == pytest.approx(2 * fv, rel=1e-13) and d2 == pytest.approx(d, rel=1e-13)
