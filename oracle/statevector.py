"""Brute-force statevector simulation (no truncation): the exact result the
MPS contraction must reproduce when nothing is discarded.  Big-endian: qubit 0
is the most significant bit of the amplitude index."""
from __future__ import annotations

import numpy as np

from . import gates as G


def apply_gate(psi: np.ndarray, n: int, u: np.ndarray, qubits) -> np.ndarray:
    """A gate on its qubits of the 2^n state (Sec. II.A), qubit 0 the most
    significant index bit, by a tensor contraction."""
    g = len(qubits)
    T = psi.reshape((2,) * n)
    T = np.tensordot(u.reshape((2,) * (2 * g)), T, axes=(list(range(g, 2 * g)), list(qubits)))
    T = np.moveaxis(T, list(range(g)), list(qubits))
    return T.reshape(-1)


def simulate(circuit) -> np.ndarray:
    """The circuit's exact state from |0...0> (Secs. II.A, IV.A), layer by
    layer."""
    n = circuit.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    for layer in circuit.layers:
        for g in layer:
            psi = apply_gate(psi, n, G.matrix(g.name), g.qubits)
    return psi
