"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds no solver arithmetic: it draws mechanisms, reactor conditions and
initial guesses, nothing else.
"""
from .conditions import initial_guess, make_conditions
from .configs import UNEVEN, WORKLOADS, mechanism, subset, uneven_workload, workload
from .mechanism import make_mechanism, species_weights

__all__ = ["make_mechanism", "species_weights", "make_conditions", "initial_guess",
           "WORKLOADS", "UNEVEN", "mechanism", "workload", "uneven_workload", "subset"]
