"""The paired-qubit input states (workloads/pairs.py) against their
definition: the amplitudes of the product of pairs, the Schmidt values of the
statevector at every bond (Sec. II.B), right-canonical sites, and the bond
dimensions of the 24-qubit state used at chi_max = 2048."""
import numpy as np
import pytest

from oracle import mps_tools as MT
from workloads.pairs import pair_angles, paired_state


def _dense(n, pairs, thetas):
    psi = np.zeros(2 ** n, dtype=np.complex128)
    for bits in range(1 << len(pairs)):
        idx, amp = 0, 1.0
        for p, (lo, hi) in enumerate(pairs):
            x = (bits >> p) & 1
            amp *= np.cos(thetas[p]) if x == 0 else np.sin(thetas[p])
            if x:
                idx |= (1 << (n - 1 - lo)) | (1 << (n - 1 - hi))  # qubit 0 the most significant
        psi[idx] = amp
    return psi


@pytest.mark.parametrize("n,pairs,seed", [
    (9, [(0, 5), (1, 7), (3, 4), (6, 8)], 0),          # nested, crossing, adjacent; qubit 2 unpaired
    (10, [(q, q + 5) for q in range(5)], 1),             # every middle bond crossed by all pairs
    (7, [(2, 6)], 2),
])
def test_paired_state_is_the_exact_schmidt_form(n, pairs, seed):
    th = pair_angles(len(pairs), seed)
    B, lam = paired_state(n, pairs, th)
    psi = _dense(n, pairs, th)
    assert np.abs(MT.amplitudes(B) - psi).max() < 1e-14
    for b in range(n - 1):
        ref = MT.schmidt_from_state(psi, n, b + 1)
        assert lam[b].size == np.count_nonzero(ref > 1e-12)
        assert np.abs(lam[b] - ref[:lam[b].size]).max() < 1e-14
        assert np.all(np.diff(lam[b]) <= 0)
        assert abs(np.linalg.norm(lam[b]) - 1) < 1e-14
    for j in range(1, n):
        assert MT.right_canonical_error(B[j]) < 1e-14
    assert abs(np.linalg.norm(B[0]) - 1) < 1e-14


def test_largest_state_dimensions():
    """24 qubits, pairs (q, q + 13): bonds 10, 11 and 12 at 2048 (the bond
    cap of mps_create), bond 9 at 1024, counted from the pairs."""
    pairs = [(q, q + 13) for q in range(11)]
    crossing = [sum(lo <= b < hi for lo, hi in pairs) for b in range(23)]
    dims = [2 ** c for c in crossing]
    assert dims[9] == 1024 and dims[10] == dims[11] == dims[12] == 2048
    cap = [2 ** min(b + 1, 23 - b) for b in range(23)]
    assert all(d <= c for d, c in zip(dims, cap))
