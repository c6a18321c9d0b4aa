"""Seeded reactor conditions and initial guesses (input data only).

Each reactor of a batch gets a pressure P (Pa), a residence time tau (s), an
inlet temperature T_in (K) and inlet mass fractions Y_in.  Arrays come back
in the structure-of-arrays layout the solver reads: per-reactor scalars as
[B] vectors, species arrays as [N][B] (species-major, reactor index fastest).

Recipes (see also the workload table in psr_inputs.configs):

* "dirichlet": isothermal reactors, Y_in ~ Dirichlet(1) over all species,
  T fixed (given as T_in).
* "phi": fuel/oxidizer/diluent inlet, the diluent mole fraction is 0.67 (the
  paper's speed-up runs use 0.67 N2, Section 6), the rest split as
  X_F = 0.33 phi/(1+phi), X_O = 0.33/(1+phi) with phi ~ U[phi_lo, phi_hi],
  converted to mass fractions with the species weights.
* "fod": fixed fuel/oxidizer/diluent mole fractions 0.15/0.18/0.67 (the
  inlet of the paper's single-iteration speed-up runs, Section 6), T fixed
  (given as T_in); every reactor gets the same inlet.
"""
from __future__ import annotations

import numpy as np

from .mechanism import species_weights

P_ATM = 101325.0
M0_SOOT = 1e3  # initial soot number density, nuclei per cm^3


def make_conditions(mech: dict, n_reactors: int, seed: int, *, recipe: str,
                    tau_range=(1e-5, 1e-1), T_in=None, T_in_range=(300.0, 800.0),
                    phi_range=(0.5, 2.5), pressure=P_ATM) -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    n_sp = mech["species_elems"].shape[0]
    B = int(n_reactors)
    lt = rng.uniform(np.log(tau_range[0]), np.log(tau_range[1]), B)
    tau = np.exp(lt)
    if recipe == "dirichlet":
        Y = rng.dirichlet(np.ones(n_sp), B).T.copy()  # [N][B]
        Tin = np.full(B, float(T_in if T_in is not None else 1500.0))
    elif recipe == "phi":
        W = species_weights(mech)
        phi = rng.uniform(phi_range[0], phi_range[1], B)
        X = np.zeros((n_sp, B))
        X[mech["diluent"]] = 0.67
        X[mech["fuel"]] = 0.33 * phi / (1.0 + phi)
        X[mech["oxidizer"]] = 0.33 / (1.0 + phi)
        mass = X * W[:, None]
        Y = mass / mass.sum(axis=0, keepdims=True)
        Tin = rng.uniform(T_in_range[0], T_in_range[1], B)
    elif recipe == "fod":
        W = species_weights(mech)
        X = np.zeros(n_sp)
        X[mech["fuel"]], X[mech["oxidizer"]], X[mech["diluent"]] = 0.15, 0.18, 0.67
        y = X * W / (X * W).sum()
        Y = np.repeat(y[:, None], B, axis=1)
        Tin = np.full(B, float(T_in if T_in is not None else 1800.0))
    else:
        raise ValueError(f"unknown recipe {recipe!r}")
    return {
        "P": np.full(B, float(pressure)),
        "tau": tau,
        "T_in": Tin,
        "Y_in": np.ascontiguousarray(Y),
    }


def initial_guess(cond: dict, energy: bool, T0: float = 2000.0, soot_nucleus=None) -> np.ndarray:
    """x0 = (Y_in[, T0][, ln M_0..ln M_5]) in [n][B] layout; T0 = 2000 K aims
    at the ignited branch.  With soot (nucleus of `soot_nucleus` carbon
    atoms) the moments start as 1e3 nuclei per cm^3: ln M_r = ln 1e3 + r ln C."""
    Y = cond["Y_in"]
    if not energy:
        return Y.copy()
    B = Y.shape[1]
    rows = [Y, np.full((1, B), float(T0))]
    if soot_nucleus is not None:
        lnM = np.log(M0_SOOT) + np.arange(6) * np.log(float(soot_nucleus))
        rows.append(np.repeat(lnM[:, None], B, axis=1))
    return np.concatenate(rows, axis=0)
