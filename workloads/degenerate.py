"""Seeded inputs whose truncation cuts through an exactly degenerate Schmidt
multiplet with a tie-invariant outcome (the truncation of Sec. II.B inside
the cluster split of Sec. III.A).  Input construction only: the cluster
unitary handed to both sides is built here from its recipe.

The state U |0...0> is k/2 Bell pairs (q, q + k/2) on a k-qubit cluster,
followed by Haar-random one-qubit gates on every qubit (local unitaries leave
every bond's spectrum unchanged).  Bond b (between qubits b and b + 1) is
crossed by S_b = min(b + 1, k - 1 - b) pairs, so its spectrum is flat,
2^{-S_b/2} with multiplicity 2^{S_b}; the middle bond k/2 - 1 holds 2^{k/2}
equal values.  With k/2 <= chi_max < 2^{k/2} only the middle bond is cut:
every bond right of it has rank <= chi_max and every bond left of it has
left dimension <= chi_max.  The kept vectors are then any chi_max-dimensional
subspace of the multiplet, yet the fidelity of the normalised result with the
exact state is exactly f = chi_max / 2^{k/2} (one truncation of a Schmidt
decomposition), the Schmidt values at and right of the cut are known in closed
form, and the Schmidt values left of the cut are those of the final state."""
import numpy as np

from .mps_inputs import haar_unitary

CASES = [(6, 4), (6, 7), (8, 8), (8, 13)]


def _local(k, mats):
    out = np.ones((1, 1), dtype=np.complex128)
    for m in mats:
        out = np.kron(out, m)
    return out


def cluster_unitary(k, seed):
    """2^k x 2^k: Hadamards on qubits 0..k/2-1, then CNOT(q -> q + k/2), then
    a Haar one-qubit gate on every qubit (qubit 0 the most significant bit)."""
    h = k // 2
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
    I2 = np.eye(2, dtype=np.complex128)
    had = _local(k, [H if q < h else I2 for q in range(k)])
    perm = np.zeros((2 ** k, 2 ** k), dtype=np.complex128)
    for b in range(2 ** k):
        c = b
        for q in range(h):
            if (b >> (k - 1 - q)) & 1:
                c ^= 1 << (k - 1 - (q + h))
        perm[c, b] = 1.0
    loc = _local(k, [haar_unitary(2, seed * 64 + q) for q in range(k)])
    return loc @ perm @ had


def crossing_pairs(k, b):
    return min(b + 1, k - 1 - b)
