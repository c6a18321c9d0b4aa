"""Hand-written tiny mechanisms for closed-form and brute-force checks.

Every mechanism uses the same three elements as the synthetic generator
(C/H/O-like weights) and single-range NASA-7 coefficients chosen so the
quantity under test has a textbook closed form.
"""
from __future__ import annotations

import numpy as np

ELEM_W = np.array([12.011, 1.008, 15.999])


def mech(comps, nasa, reactions, A, beta=None, Ea=None):
    """Build a mechanism dict.  reactions: list of ({sp: nu}, {sp: nu})."""
    n_rx = len(reactions)
    r_idx = np.full((n_rx, 3), -1, np.int32)
    r_nu = np.zeros((n_rx, 3), np.int32)
    p_idx = np.full((n_rx, 3), -1, np.int32)
    p_nu = np.zeros((n_rx, 3), np.int32)
    for k, (reac, prod) in enumerate(reactions):
        for s, (i, nu) in enumerate(sorted(reac.items())):
            r_idx[k, s], r_nu[k, s] = i, nu
        for s, (i, nu) in enumerate(sorted(prod.items())):
            p_idx[k, s], p_nu[k, s] = i, nu
    return {
        "elem_weight": ELEM_W.copy(),
        "species_elems": np.array(comps, np.int32),
        "nasa7": np.array(nasa, np.float64),
        "t_low": 300.0, "t_high": 3000.0,
        "reac_idx": r_idx, "reac_nu": r_nu, "prod_idx": p_idx, "prod_nu": p_nu,
        "A": np.array(A, np.float64),
        "beta": np.zeros(n_rx) if beta is None else np.array(beta, np.float64),
        "Ea": np.zeros(n_rx) if Ea is None else np.array(Ea, np.float64),
    }


def const_cp(a1, a6, a7):
    """NASA-7 row of a constant-c_p species: c_p/R = a1, H/RT = a1 + a6/T, S/R = a1 ln T + a7."""
    return [a1, 0.0, 0.0, 0.0, 0.0, a6, a7]


def isomerisation(A=3.0e3, da6=-1500.0, da7=0.7):
    """A <=> B between two isomers (same composition, same weight).

    Identical a1..a5, so K_c = K_p = exp(da7 - da6/T) exactly (no pressure
    factor since the mole number does not change).
    """
    comps = [(1, 1, 0), (1, 1, 0)]
    nasa = [const_cp(3.5, 0.0, 5.0), const_cp(3.5, da6, 5.0 + da7)]
    return mech(comps, nasa, [({0: 1}, {1: 1})], [A])


def dimerisation(A=2.0e13, a6_dimer=-3.0e4, a7_dimer=-2.0):
    """2 A <=> A2 with A = (1,0,0) and A2 = (2,0,0)."""
    comps = [(1, 0, 0), (2, 0, 0)]
    nasa = [const_cp(2.5, 0.0, 8.0), const_cp(3.5, a6_dimer, 6.0 + a7_dimer)]
    return mech(comps, nasa, [({0: 2}, {1: 1})], [A])


def association(A=5.0e12):
    """A + B <=> C with A = (1,0,0), B = (0,1,0), C = (1,1,0)."""
    comps = [(1, 0, 0), (0, 1, 0), (1, 1, 0)]
    nasa = [const_cp(2.5, 0.0, 9.0), const_cp(2.5, 0.0, 7.0), const_cp(3.5, -2.0e4, 6.0)]
    return mech(comps, nasa, [({0: 1, 1: 1}, {2: 1})], [A])


def small_network():
    """Five species, six reactions with orders 1-3, polynomial c_p (a2..a5 != 0).

    Used for derivative checks where no closed form exists.
    """
    comps = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 1, 1)]
    rng = np.random.default_rng(7)
    nasa = []
    for c in comps:
        na = sum(c)
        nasa.append([2.5 + 0.5 * na, 3e-4 * na, -4e-8 * na, 2e-12 * na, 3e-17 * na,
                     -1.0e4 * (na - 1) + rng.uniform(-2e3, 2e3), 5.0 + 2.0 * na])
    reactions = [
        ({0: 1, 1: 1}, {2: 1}),          # C + H <=> CH
        ({2: 1, 3: 1}, {4: 1}),          # CH + O <=> CHO
        ({0: 1, 1: 1, 3: 1}, {4: 1}),    # C + H + O <=> CHO (third order)
        ({2: 2}, {0: 2, 1: 2}),          # 2 CH <=> 2 C + 2 H (fourth-order reverse)
        ({4: 2}, {2: 2, 3: 2}),          # 2 CHO <=> 2 CH + 2 O
    ]
    A = [4e12, 1e11, 3e15, 2e9, 6e12]
    beta = [0.5, -0.7, 0.0, 1.2, 0.3]
    Ea = [1.2e4, 4.0e4, 0.0, 1.5e5, 6.0e4]
    return mech(comps, nasa, reactions, A, beta, Ea)
