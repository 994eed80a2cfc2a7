"""Stabilizer tableau (CHP update rules of Aaronson & Gottesman, PRA 70, 052328
(2004)) and bipartite entanglement from it (Fattal et al., quant-ph/0406168):
for a stabilizer state with generators g_1..g_n, the entropy of a region A in
bits is rank_GF(2)(generators restricted to A) - |A|.  Stabilizer states have
flat Schmidt spectra, sigma = 2^{-S/2} repeated 2^S times, so these integer
entropies pin the spectra of Clifford circuits exactly.

Only the stabilizer half of the tableau is kept (phases do not enter the
entropies).  Supported gates: H, S, X, Y, Z, CNOT, CZ, CY, SWAP.
"""
from __future__ import annotations

import numpy as np


class Tableau:
    def __init__(self, n: int):
        self.n = n
        # row i is the stabilizer Z_i of |0...0>: x = 0, z = e_i
        self.x = np.zeros((n, n), dtype=np.uint8)
        self.z = np.eye(n, dtype=np.uint8)

    def h(self, q):
        self.x[:, q], self.z[:, q] = self.z[:, q].copy(), self.x[:, q].copy()

    def s(self, q):
        self.z[:, q] ^= self.x[:, q]

    def cnot(self, c, t):
        self.x[:, t] ^= self.x[:, c]
        self.z[:, c] ^= self.z[:, t]

    def apply(self, name: str, qubits):
        if name == "H":
            self.h(qubits[0])
        elif name == "S":
            self.s(qubits[0])
        elif name in ("X", "Y", "Z", "I"):
            pass  # Paulis change only signs
        elif name == "CNOT":
            self.cnot(*qubits)
        elif name == "CZ":
            c, t = qubits
            self.h(t); self.cnot(c, t); self.h(t)
        elif name == "CY":
            c, t = qubits
            # CY = S_t CNOT S_t^dagger; S^dagger acts on the tableau like S^3
            self.s(t); self.s(t); self.s(t); self.cnot(c, t); self.s(t)
        elif name == "SWAP":
            a, b = qubits
            self.cnot(a, b); self.cnot(b, a); self.cnot(a, b)
        else:
            raise ValueError(f"not a Clifford gate: {name}")


def gf2_rank(rows: np.ndarray) -> int:
    """Rank over GF(2) of a 0/1 matrix, by elimination on Python-int bit rows."""
    ints = [int("".join(map(str, r)), 2) if r.size else 0 for r in rows.astype(np.uint8)]
    rank = 0
    ints = [v for v in ints if v]
    while ints:
        pivot = max(ints)
        top = pivot.bit_length() - 1
        ints = [v ^ pivot if (v >> top) & 1 else v for v in ints if v != pivot]
        ints = [v for v in ints if v]
        rank += 1
    return rank


def bond_entropies(tab: Tableau):
    """Entropy in bits across every bond b (region A = qubits 0..b)."""
    out = []
    for b in range(tab.n - 1):
        a = b + 1
        sub = np.concatenate([tab.x[:, :a], tab.z[:, :a]], axis=1)
        out.append(gf2_rank(sub) - a)
    return out


def circuit_entropies(circuit):
    """Bond entropies of a Clifford circuit's state from |0...0>, by the
    stabilizer tableau (the integer entropies that pin Clifford spectra)."""
    tab = Tableau(circuit.n)
    for layer in circuit.layers:
        for g in layer:
            tab.apply(g.name, g.qubits)
    return bond_entropies(tab)
