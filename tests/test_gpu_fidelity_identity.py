"""The GPU path's fidelity estimate against the mathematics, not the oracle.

A cluster applied to a state held exactly truncates nested Schmidt
decompositions (each split of the right-to-left sweep cuts the state the
previous split left, Secs. II.B and III.A), so the product of its f_i is the
exact fidelity |<psi_exact|psi>|^2 of the normalised result.  The state is
an exact 14-qubit paired state (pairs (2, 11), (3, 12), (4, 13) with seeded
weights, bonds 4-8 of dimension 8; workloads/pairs.py) imported at
chi_max = 8; a 4-qubit Haar cluster on the unpaired qubits 5-8 raises the
middle bond's rank to 32, so the cap binds, and exp(delta log f) is compared
with the overlap against the statevector."""
import math

import numpy as np
import pytest

from oracle import mps_tools as MT
from oracle import statevector as SV
from workloads.mps_inputs import haar_unitary
from workloads.pairs import pair_angles, paired_state

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")

TOL = {"fp64": 1e-10, "fp32": 2e-6, "bf16x6": 2e-6}
N, PAIRS, CLUSTER = 14, [(2, 11), (3, 12), (4, 13)], [5, 6, 7, 8]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_cluster_estimate_is_the_exact_fidelity(prec, seed):
    B, lam = paired_state(N, PAIRS, pair_angles(len(PAIRS), seed))
    sv = MT.amplitudes(B)
    m = P.MPS(N, 8, 1e-12, k_max=4, precision=prec)
    m.import_state(B, lam)
    U = haar_unitary(16, seed=500 + seed)
    m.apply_cluster(CLUSTER, U)
    sv = SV.apply_gate(sv, N, U, CLUSTER)
    est = math.exp(m.fidelity()[1])
    amp = m.amplitudes()
    F = abs(np.vdot(sv, amp)) ** 2 / np.vdot(amp, amp).real
    print(f"{prec} seed {seed}: F_est {est:.12f}, exact {F:.12f}")
    assert est < 0.999  # the cap binds
    assert abs(F - est) < TOL[prec]
