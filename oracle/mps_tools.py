"""MPS read-outs used by the checks (definitions of Sec. II.B)."""
from __future__ import annotations

from typing import Sequence

import numpy as np


def amplitudes(B: Sequence[np.ndarray]) -> np.ndarray:
    """Full 2^n state vector of B_0 B_1 ... B_{n-1}, the MPS of Sec. II.B
    contracted over its bonds (small n only)."""
    psi = B[0].reshape(2, -1)
    for t in B[1:]:
        psi = (psi @ t.reshape(t.shape[0], -1)).reshape(-1, t.shape[2])
    return psi.reshape(-1)


def overlap(A: Sequence[np.ndarray], B: Sequence[np.ndarray]) -> complex:
    """<A|B> by a left-to-right transfer-matrix sweep, exact in FP64: the
    overlap in the exact fidelity of Sec. II.B."""
    E = np.ones((1, 1), dtype=np.complex128)
    for a, b in zip(A, B):
        # E[la, lb] -> sum_s a*[la, s, ra] E[la, lb] b[lb, s, rb]
        E = np.einsum("xy,xsa,ysb->ab", E, a.conj(), b, optimize=True)
    return complex(E[0, 0])


def infidelity(A: Sequence[np.ndarray], B: Sequence[np.ndarray]) -> float:
    """1 - |<A|B>|^2 / (<A|A><B|B>) (Eq. for the exact fidelity F)."""
    ab = overlap(A, B)
    aa = overlap(A, A).real
    bb = overlap(B, B).real
    return float(1.0 - abs(ab) ** 2 / (aa * bb))


def entropy_bits(lam: np.ndarray) -> float:
    """Von Neumann entanglement entropy in bits from normalised Schmidt values
    (S_b = -sum sigma^2 log2 sigma^2; chi_b grows as 2^{S_b})."""
    p = np.asarray(lam, dtype=np.float64) ** 2
    p = p[p > 0]
    p = p / p.sum()
    return float(-(p * np.log2(p)).sum())


def schmidt_from_state(psi: np.ndarray, n: int, cut: int) -> np.ndarray:
    """Schmidt values of a state vector across the cut after ``cut`` qubits
    (the singular values a bond of Sec. II.B holds)."""
    return np.linalg.svd(psi.reshape(2 ** cut, 2 ** (n - cut)), compute_uv=False)


def right_canonical_error(t: np.ndarray) -> float:
    """|| sum_{s,r} B B^dagger - 1 || for a site tensor (l, s, r): the
    right-canonical condition of the form the cluster step keeps (Sec. III.A)."""
    m = t.reshape(t.shape[0], -1)
    return float(np.abs(m @ m.conj().T - np.eye(t.shape[0])).max())
