"""Seeded random MPS inputs (right-canonical site tensors plus positive,
normalised bond weights) for step-level checks at chosen bond dimensions.

A site tensor B_j of shape (chi_{j-1}, 2, chi_j) is made right-canonical by
taking the first chi_{j-1} rows of a random unitary (QR of a complex Gaussian
matrix); bond weights are random decaying positive vectors with unit norm.
The weights are generic inputs, not the Schmidt values of the state.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def feasible_dims(n: int, chi: int) -> List[int]:
    return [min(chi, 2 ** min(b + 1, n - b - 1)) for b in range(n - 1)]


def random_mps(n: int, dims: Sequence[int], seed: int = 0, decay: float = 0.05
               ) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    rng = np.random.default_rng(np.random.SeedSequence([77, seed]))
    full = [1] + list(dims) + [1]
    B = []
    for j in range(n):
        cl, cr = full[j], full[j + 1]
        cols = 2 * cr
        assert cl <= cols, "bond dimensions must satisfy chi_{j-1} <= 2 chi_j"
        z = rng.standard_normal((cols, cl)) + 1j * rng.standard_normal((cols, cl))
        q, _ = np.linalg.qr(z)
        B.append(np.ascontiguousarray(q.T.reshape(cl, 2, cr)))
    lam = []
    for b in range(n - 1):
        w = np.exp(-decay * np.arange(dims[b])) * (1 + 0.5 * rng.random(dims[b]))
        w = np.sort(w)[::-1]
        lam.append(w / np.linalg.norm(w))
    # the first site carries the norm of the state
    B[0] = B[0] / np.linalg.norm(B[0])
    return B, lam


def haar_unitary(d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([78, seed]))
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))
