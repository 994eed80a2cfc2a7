"""Seeded synthetic inputs shared by the oracle tests, the HIP-path tests and the bench.

This package holds no arithmetic of the simulation method.  It draws random
circuit *structures* (gate symbols and the qubits they act on; each side maps
the symbols to matrices with its own gate table) and builds input states and
unitaries from their recipes: random right-canonical tensors and Haar
unitaries (``mps_inputs``), Bell-pair cluster unitaries (``degenerate``) and
exact paired states at the largest bond dimensions (``pairs``).
"""
from .circuits import (Gate, Circuit, random_structured, paper_random_structured, WORKLOADS, make_workload,
                       save_circuit, load_circuit)

__all__ = ["Gate", "Circuit", "random_structured", "paper_random_structured", "WORKLOADS", "make_workload",
           "save_circuit", "load_circuit"]
