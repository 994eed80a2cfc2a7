"""Truncation through an exactly degenerate Schmidt multiplet on the GPU
(Sec. II.B truncation inside the cluster split of Sec. III.A), through the C
ABI, against the oracle and the exact state.

Bell pairs across a k-qubit cluster with local Haar gates (inputs from
workloads.degenerate): chi_max cuts the middle bond through 2^{k/2} equal
Schmidt values and no other bond.  The GPU may keep any chi_max-dimensional
subspace of the multiplet (its eigen-solver's choice, not the oracle's); what
is unique is compared: the exact fidelity of the result (chi_max / 2^{k/2}),
the fidelity estimate, the bond dimensions, the Schmidt values at and right
of the cut; left of the cut the Schmidt values must be the final state's own,
and every site right-canonical."""
import math

import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import mps_tools as MT
from workloads.degenerate import CASES, cluster_unitary, crossing_pairs

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")

TOL = {"fp64": 1e-11, "fp32": 2e-6, "bf16x6": 2e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
@pytest.mark.parametrize("k,chi", CASES)
def test_cut_through_multiplet_vs_oracle(k, chi, prec):
    U = cluster_unitary(k, seed=k * 100 + chi)
    ref = CT.product_state(k)
    CT.apply_cluster(ref, 0, k, U, chi, 1e-12)
    assert any(r.degenerate_cut for r in ref.records)
    m = P.MPS(k, chi, 1e-12, k_max=k, precision=prec)
    m.apply_cluster(list(range(k)), U)
    h, mid, f = k // 2, k // 2 - 1, chi / 2 ** (k // 2)
    tol = TOL[prec]
    assert m.bond_dims() == ref.bond_dims()
    assert abs(math.exp(m.fidelity()[1]) - f) < tol
    amp = m.amplitudes()
    F = abs(np.vdot(U[:, 0], amp)) ** 2 / np.vdot(amp, amp).real
    assert abs(F - f) < tol, (F, f)
    for b in range(k - 1):
        lam = m.schmidt(b)
        if b >= mid:
            assert np.abs(lam - ref.lam[b]).max() < tol
        else:
            own = MT.schmidt_from_state(amp / np.linalg.norm(amp), k, b + 1)
            assert np.abs(lam - own[:lam.size]).max() < tol
    for j in range(1, k):
        assert MT.right_canonical_error(m.site(j)) < (1e-12 if prec == "fp64" else 1e-5)
    print(f"k {k} chi {chi} {prec}: F = {F:.12f} (exact {f}), pairs at the cut {crossing_pairs(k, mid)}")
    m.close()
