"""Seeded synthetic inputs shared by the oracle tests, the HIP-path tests and the bench.

This package holds no arithmetic of the simulation method: it only draws random
circuit *structures* (gate symbols and the qubits they act on).  Each side maps
the symbols to matrices with its own gate table.
"""
from .circuits import (Gate, Circuit, random_structured, paper_random_structured, WORKLOADS, make_workload,
                       save_circuit, load_circuit)

__all__ = ["Gate", "Circuit", "random_structured", "paper_random_structured", "WORKLOADS", "make_workload",
           "save_circuit", "load_circuit"]
