"""Seeded synthetic reaction mechanisms (input data only).

The paper's mechanisms (an ethylene/air set and a 101-species/542-reaction
set, Sections 5-6) are not available, so every workload runs on synthetic
mechanisms with the structure the paper describes: elementary reversible
reactions with mass-action rates (Eqs. 4-5), modified-Arrhenius forward rate
constants (Eq. 6) and reverse rates from equilibrium constants computed from
species thermodynamics (Eqs. 7-9).

This module only *draws* numbers.  It evaluates nothing the solver computes:
no thermodynamic function, rate, residual or derivative is evaluated here.
Positivity of the heat capacity polynomial is guaranteed by construction of
the coefficient signs (see ``_nasa7``), not by evaluating the polynomial.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* 3 elements with weights 12.011 / 1.008 / 15.999 (C/H/O-like).
* Species compositions a_i in {0..3}^3 minus the zero vector; distinct
  compositions first (in seeded random order), isomers once all 63 are used.
  Designated roles for the inlet mix: a fuel-like species (2,3,0), an
  oxidizer-like species (0,0,2), product-like species (1,0,2) and (0,2,1),
  and an inert diluent (an isomer of (1,0,1), weight ~28 like N2) that takes
  part in no reaction.  Optional soot roles: a pure-carbon precursor (3,0,0)
  and a C2 growth species (2,0,0).
* Reactions: the number of reactants and of products is drawn from {1,2,3}
  with probabilities (0.2, 0.6, 0.2); reactants uniformly with replacement;
  products uniformly among multisets of that size with exactly the same
  element sum; reactions with a species on both sides, and duplicates (in
  either direction), are rejected.  Every non-inert species is forced to be a
  reactant of at least one reaction.
  Each reaction is written in the direction in which the drawn formation
  enthalpy offsets decrease, so the drawn activation energy never has to
  cover an endothermic step and reverse rates (from K_c) stay physical.
* Arrhenius: ln A ~ U[ln 1e8, ln 1e14], beta ~ U[-1, 2], E ~ U[0, 2e5] J/mol.
* Thermo: single-range NASA-7 coefficients over [300, 3000] K (see _nasa7);
  formation enthalpy offsets = -1e5 J/mol per bond (atoms - 1) + U[-2e4, 2e4],
  +2.5e5 for the fuel and oxidizer, -2.5e5 for the product-like species;
  S/R near 1500 K = 14 + 3 * atoms + U[-2, 2].
"""
from __future__ import annotations

import numpy as np

ELEMENT_WEIGHTS = np.array([12.011, 1.008, 15.999], dtype=np.float64)
T_LOW, T_HIGH = 300.0, 3000.0
R_GAS = 8.314462618  # J/(mol K); used only to express drawn enthalpy offsets in kelvin

FUEL_COMP = (2, 3, 0)
OXID_COMP = (0, 0, 2)
PRODUCT_COMPS = ((1, 0, 2), (0, 2, 1))
DILUENT_COMP = (1, 0, 1)
PRECURSOR_COMP = (3, 0, 0)
GROWTH_COMP = (2, 0, 0)

# Enthalpy recipe (J/mol): a bond term makes larger molecules more stable than
# their fragments; the fuel/oxidizer pair sits high and the product-like
# species low, so that converting the inlet releases heat.
BOND_ENTHALPY = 1.0e5
NOISE_ENTHALPY = 2.0e4
FUEL_OX_OFFSET = 2.5e5
PRODUCT_OFFSET = -2.5e5
# Pure-carbon soot species (precursor, growth) are made more stable than the
# bond rule alone gives, so that they are present at the fuel-rich steady
# states where soot forms.
SOOT_OFFSET = -1.0e5
# Entropy recipe (dimensionless S/R near 1500 K): per-molecule + per-atom.
S_PER_MOLECULE = 14.0
S_PER_ATOM = 3.0
LN_T_REF = 7.313220387090301  # ln(1500): anchors the a1*lnT part of S/R near 1500 K


def _all_compositions():
    return [(c, h, o) for c in range(4) for h in range(4) for o in range(4)
            if (c, h, o) != (0, 0, 0)]


def _species_list(rng, n_species, soot):
    forced = [FUEL_COMP, OXID_COMP, *PRODUCT_COMPS]
    if soot:
        forced += [PRECURSOR_COMP, GROWTH_COMP]
    comps = list(forced)
    pool = [c for c in _all_compositions() if c not in comps]
    order = rng.permutation(len(pool))
    pool = [pool[i] for i in order]
    n_reactive = n_species - 1  # last species is the inert diluent
    while len(comps) < n_reactive:
        if pool:
            comps.append(pool.pop())
        else:  # all compositions used: draw isomers
            allc = _all_compositions()
            comps.append(allc[int(rng.integers(len(allc)))])
    comps = comps[:n_reactive]
    comps.append(DILUENT_COMP)
    return np.array(comps, dtype=np.int32)


def _nasa7(rng, comps, roles, heat_scale=1.0):
    """Single-range NASA-7 coefficients a1..a7 per species.

    c_p/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4 is positive on [300, 3000] K by
    construction: a1 >= 2.5, a4, a5 >= 0, and a2 + 3000 a3 >= 0 with a3 <= 0,
    so every term group is non-negative for 0 < T <= 3000.
    """
    n = comps.shape[0]
    na = comps.sum(axis=1).astype(np.float64)
    poly = na - 1.0
    a = np.zeros((n, 7))
    a[:, 0] = 2.5 + 0.5 * poly + rng.uniform(0.0, 0.5, n)
    a[:, 1] = poly * rng.uniform(2.0e-4, 6.0e-4, n)
    a[:, 2] = -poly * rng.uniform(0.0, 5.0e-8, n)
    a[:, 3] = poly * rng.uniform(0.0, 1.0e-12, n)
    a[:, 4] = poly * rng.uniform(0.0, 1.0e-16, n)
    h = -BOND_ENTHALPY * poly + rng.uniform(-NOISE_ENTHALPY, NOISE_ENTHALPY, n)
    for i in roles.get("fuel_ox", []):
        h[i] += heat_scale * FUEL_OX_OFFSET
    for i in roles.get("products", []):
        h[i] += heat_scale * PRODUCT_OFFSET
    for i in roles.get("soot", []):
        h[i] += SOOT_OFFSET
    a[:, 5] = h / R_GAS
    s_target = S_PER_MOLECULE + S_PER_ATOM * na + rng.uniform(-2.0, 2.0, n)
    a[:, 6] = s_target - a[:, 0] * LN_T_REF
    return a, h


def _multiset_table(n_reactive, comps, size):
    """All multisets of `size` species among 0..n_reactive-1, keyed by element sum."""
    idx = np.arange(n_reactive)
    if size == 1:
        ms = idx[:, None]
    elif size == 2:
        i, j = np.triu_indices(n_reactive)
        ms = np.stack([i, j], axis=1)
    else:
        i, j = np.triu_indices(n_reactive)
        pairs = np.stack([i, j], axis=1)
        rows = []
        for k in range(n_reactive):
            sel = pairs[pairs[:, 1] <= k]
            rows.append(np.concatenate([sel, np.full((len(sel), 1), k)], axis=1))
        ms = np.concatenate(rows, axis=0)
    csum = comps[ms].sum(axis=1)
    key = (csum[:, 0] * 100 + csum[:, 1] * 10 + csum[:, 2]).astype(np.int64)
    order = np.argsort(key, kind="stable")
    return ms[order].astype(np.int32), key[order]


def make_mechanism(n_species: int, n_reactions: int, seed: int, *, soot: bool = False,
                   heat_scale: float = 1.0) -> dict:
    """Draw an element-balanced reversible mechanism.

    Returns a dict of numpy arrays (see module docstring).  Reactant and
    product sides are stored as up to three (species index, coefficient)
    pairs; index -1 pads unused slots.
    """
    if n_species < 6:
        raise ValueError("need at least 6 species (roles + diluent)")
    rng = np.random.Generator(np.random.PCG64(seed))
    comps = _species_list(rng, n_species, soot)
    n_reactive = n_species - 1
    fuel = 0
    oxid = 1
    products = [2, 3]
    roles = {"fuel_ox": [fuel, oxid], "products": products}
    if soot:
        roles["soot"] = [4, 5]
    nasa, h_offset = _nasa7(rng, comps, roles, heat_scale)

    tables = {s: _multiset_table(n_reactive, comps, s) for s in (1, 2, 3)}
    p_count = np.array([0.2, 0.6, 0.2])
    seen = set()
    reactions = []
    force = list(rng.permutation(n_reactive))
    attempts = 0
    while len(reactions) < n_reactions:
        attempts += 1
        if attempts > 200000:
            raise RuntimeError("mechanism generation did not converge")
        nr = int(rng.choice(3, p=p_count)) + 1
        reac = list(rng.integers(0, n_reactive, nr))
        if force:
            reac[0] = force[-1]
        reac = tuple(sorted(int(r) for r in reac))
        csum = comps[list(reac)].sum(axis=0)
        key = int(csum[0] * 100 + csum[1] * 10 + csum[2])
        sizes = [int(rng.choice(3, p=p_count)) + 1]
        sizes += [s for s in (1, 2, 3) if s != sizes[0]]
        prod = None
        for np_ in sizes:
            ms, keys = tables[np_]
            lo, hi = np.searchsorted(keys, key, "left"), np.searchsorted(keys, key, "right")
            if hi <= lo:
                continue
            for _ in range(40):
                cand = tuple(int(v) for v in ms[int(rng.integers(lo, hi))])
                if set(cand) & set(reac):
                    continue
                if (reac, cand) in seen or (cand, reac) in seen:
                    continue
                prod = cand
                break
            if prod is not None:
                break
        if prod is None:
            continue
        # write the reaction in the direction in which the drawn formation
        # enthalpy offsets decrease, so the forward activation energy is not
        # asked to cover an endothermic step
        if sum(h_offset[list(prod)]) > sum(h_offset[list(reac)]):
            reac, prod = prod, reac
        seen.add((reac, prod))
        reactions.append((reac, prod))
        if force:
            force.pop()

    def pack(side_list):
        idx = np.full((n_reactions, 3), -1, dtype=np.int32)
        nu = np.zeros((n_reactions, 3), dtype=np.int32)
        for k, side in enumerate(side_list):
            uniq, cnt = np.unique(np.array(side), return_counts=True)
            idx[k, :len(uniq)] = uniq
            nu[k, :len(uniq)] = cnt
        return idx, nu

    reac_idx, reac_nu = pack([r for r, _ in reactions])
    prod_idx, prod_nu = pack([p for _, p in reactions])
    ln_a = rng.uniform(np.log(1e8), np.log(1e14), n_reactions)
    mech = {
        "elem_weight": ELEMENT_WEIGHTS.copy(),
        "species_elems": comps,
        "nasa7": nasa,
        "t_low": T_LOW,
        "t_high": T_HIGH,
        "reac_idx": reac_idx, "reac_nu": reac_nu,
        "prod_idx": prod_idx, "prod_nu": prod_nu,
        "A": np.exp(ln_a),
        "beta": rng.uniform(-1.0, 2.0, n_reactions),
        "Ea": rng.uniform(0.0, 2.0e5, n_reactions),
        "fuel": fuel, "oxidizer": oxid, "diluent": n_species - 1,
        "product_species": np.array(products, dtype=np.int32),
    }
    if soot:
        mech["precursor"] = 4
        mech["growth"] = 5
    return mech


def species_weights(mech: dict) -> np.ndarray:
    """W_i = sum_e a_ie W_e (g/mol): an input property, needed to turn mole into mass fractions."""
    return mech["species_elems"].astype(np.float64) @ mech["elem_weight"]
