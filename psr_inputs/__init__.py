"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds no solver arithmetic: it draws mechanisms, reactor conditions and
initial guesses, nothing else.
"""
from .conditions import initial_guess, make_conditions
from .configs import (SOOT_CONSTANTS, UNEVEN, WORKLOADS, mechanism, soot_nucleus_size, subset,
                      uneven_workload, workload)
from .mechanism import make_mechanism, species_weights

__all__ = ["make_mechanism", "species_weights", "make_conditions", "initial_guess",
           "WORKLOADS", "UNEVEN", "SOOT_CONSTANTS", "mechanism", "workload", "uneven_workload",
           "subset", "soot_nucleus_size"]
