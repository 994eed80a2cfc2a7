"""Standard gate-by-gate TEBD, FP64 on the CPU: test infrastructure (an
oracle), not part of the product path.

Follows Sec. II.C: every gate of the circuit, layer by layer, is applied on
its own in three steps,
  1. orthogonalisation: QR decompositions move the orthogonality centre of the
     MPS to the gate's first site (tensors to its left left-isometric, to its
     right right-isometric; the norm is the Frobenius norm of the centre);
  2. contraction: the gate is applied to the two-site tensor of the centre and
     its right neighbour;
  3. truncated SVD: the two-site tensor is split back with the cutoff eta and
     the cap chi_max (Sec. II.B), the kept values renormalised, the kept weight
     f_i (Eq. f_i) recorded; the centre stays on the first site.
One-qubit gates act on their site.  A two-qubit gate on non-neighbouring
qubits is brought together by SWAP gates and the SWAPs are undone afterwards
(Sec. IV.A), each SWAP a gate like any other (with its own truncation).
F is estimated as prod f_i (Eq. approxF), accumulated as sum log f_i.

This keeps an explicit orthogonality centre (the paper's form), unlike the
Lambda-weighted right-canonical form of the cluster-TEBD oracle; without
truncation both are the exact state.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import gates as G
from .ctebd import truncation_rank


@dataclass
class CentredMPS:
    A: List[np.ndarray]          # site tensors (chi_{j-1}, 2, chi_j)
    centre: int = 0
    log_f: float = 0.0
    fs: List[float] = field(default_factory=list)

    @property
    def n(self) -> int:
        return len(self.A)

    def bond_dims(self) -> List[int]:
        return [t.shape[2] for t in self.A[:-1]]


def product_state(n: int) -> CentredMPS:
    """|0...0> with the orthogonality centre on site 0 (Secs. II.C, IV.A)."""
    A = []
    for _ in range(n):
        t = np.zeros((1, 2, 1), dtype=np.complex128)
        t[0, 0, 0] = 1.0
        A.append(t)
    return CentredMPS(A, 0)


def move_centre(psi: CentredMPS, i: int) -> None:
    """Step 1: QR sweeps until the orthogonality centre sits on site i."""
    while psi.centre < i:
        c = psi.centre
        t = psi.A[c]
        l, _, r = t.shape
        Q, R = np.linalg.qr(t.reshape(l * 2, r))
        psi.A[c] = Q.reshape(l, 2, Q.shape[1])
        psi.A[c + 1] = np.tensordot(R, psi.A[c + 1], axes=(1, 0))
        psi.centre = c + 1
    while psi.centre > i:
        c = psi.centre
        t = psi.A[c]
        l, _, r = t.shape
        # t = L Q' with Q' right-isometric: QR of the conjugate transpose
        Q, R = np.linalg.qr(t.reshape(l, 2 * r).conj().T)
        psi.A[c] = Q.conj().T.reshape(Q.shape[1], 2, r)
        psi.A[c - 1] = np.tensordot(psi.A[c - 1], R.conj().T, axes=(2, 0))
        psi.centre = c - 1


def apply_one_qubit(psi: CentredMPS, j: int, u: np.ndarray) -> None:
    """A one-qubit gate needs no SVD in TEBD (Sec. II.C)."""
    psi.A[j] = np.einsum("st,ltr->lsr", u, psi.A[j])


def apply_neighbour_gate(psi: CentredMPS, i: int, u: np.ndarray, chi_max: int, eps: float) -> None:
    """Steps 1-3 for a 4 x 4 gate on sites (i, i+1), big-endian: site i is the
    more significant qubit of u's index."""
    move_centre(psi, i)
    a, b = psi.A[i], psi.A[i + 1]
    l, r = a.shape[0], b.shape[2]
    theta = np.tensordot(a, b, axes=(2, 0)).reshape(l, 4, r)
    theta = np.einsum("st,ltr->lsr", u, theta).reshape(l * 2, 2 * r)
    U, sigma, Vh = np.linalg.svd(theta, full_matrices=False)
    k = truncation_rank(sigma, chi_max, eps)
    f = float(np.sum(sigma[:k] ** 2)) / float(np.sum(sigma ** 2))
    kept = sigma[:k] / np.linalg.norm(sigma[:k])
    psi.A[i] = (U[:, :k] * kept).reshape(l, 2, k)
    psi.A[i + 1] = Vh[:k].reshape(k, 2, r)
    psi.fs.append(f)
    psi.log_f += math.log(f)


def _permuted(u: np.ndarray, first_is_low: bool) -> np.ndarray:
    """u on (q0, q1) rewritten for (min, max) order."""
    if first_is_low:
        return u
    P = G.matrix("SWAP")
    return P @ u @ P


def apply_gate(psi: CentredMPS, gate, chi_max: int, eps: float) -> None:
    """One gate of the circuit by TEBD (Sec. II.C): one-qubit gates on their
    site, two-qubit gates on neighbours through steps 1-3, longer ones by
    SWAP chains (Sec. IV.A)."""
    u = G.matrix(gate.name)
    if len(gate.qubits) == 1:
        apply_one_qubit(psi, gate.qubits[0], u)
        return
    q0, q1 = gate.qubits
    lo, hi = min(q0, q1), max(q0, q1)
    v = _permuted(u, q0 < q1)
    swap = G.matrix("SWAP")
    # bring the far qubit next to the near one, apply, move it back
    for j in range(hi - 1, lo, -1):
        apply_neighbour_gate(psi, j, swap, chi_max, eps)
    apply_neighbour_gate(psi, lo, v, chi_max, eps)
    for j in range(lo + 1, hi):
        apply_neighbour_gate(psi, j, swap, chi_max, eps)


def run(circuit, chi_max: int, eps: float) -> CentredMPS:
    """Simulate the circuit from |0...0>, gate by gate, layer by layer."""
    psi = product_state(circuit.n)
    for layer in circuit.layers:
        for g in layer:
            apply_gate(psi, g, chi_max, eps)
    return psi


def amplitudes(psi: CentredMPS) -> np.ndarray:
    """The 2^n state of the MPS (Sec. II.B), for small n."""
    out = psi.A[0].reshape(2, -1)
    for t in psi.A[1:]:
        out = (out @ t.reshape(t.shape[0], -1)).reshape(-1, t.shape[2])
    return out.reshape(-1)
