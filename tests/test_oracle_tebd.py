"""Pins of the standard-TEBD oracle (Sec. II.C, gate by gate with an explicit
orthogonality centre) and of the paper's circuit generator (Sec. IV.A)."""
import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import mps_tools as MT
from oracle import statevector as SV
from oracle import tebd as TB
from workloads import make_workload, paper_random_structured


@pytest.mark.parametrize("version,d_max,seed", [(1, 1, 0), (2, 1, 1), (2, 4, 2), (1, 8, 3)])
def test_tebd_exact_equals_statevector(version, d_max, seed):
    c = paper_random_structured(9, 8, version, d_max=d_max, seed=seed, workload_id=90)
    psi = TB.run(c, chi_max=512, eps=0.0)
    sv = SV.simulate(c)
    assert np.abs(TB.amplitudes(psi) - sv).max() < 1e-12
    assert abs(psi.log_f) < 1e-12
    # canonical form around the centre: isometries left and right, unit norm
    for j, t in enumerate(psi.A):
        if j < psi.centre:
            m = t.reshape(-1, t.shape[2])
            assert np.abs(m.conj().T @ m - np.eye(t.shape[2])).max() < 1e-12
        elif j > psi.centre:
            assert MT.right_canonical_error(t) < 1e-12
    assert abs(np.linalg.norm(psi.A[psi.centre]) - 1.0) < 1e-12


def test_single_truncation_fidelity_is_kept_weight():
    """With the centre on the gate, truncating one bond and renormalising gives
    an exact fidelity equal to the kept weight f (Sec. II.B)."""
    c = paper_random_structured(10, 10, 2, d_max=1, seed=7, workload_id=91)
    psi = TB.run(c, chi_max=1024, eps=0.0)
    exact = TB.amplitudes(psi)
    layer_gate = [g for g in c.layers[0] if len(g.qubits) == 2][0]
    ref = SV.apply_gate(exact, c.n, CT.G.matrix(layer_gate.name), list(layer_gate.qubits))
    lo = min(layer_gate.qubits)
    if abs(layer_gate.qubits[0] - layer_gate.qubits[1]) != 1:
        pytest.skip("the first two-qubit gate is not a neighbour gate")
    chi_here = psi.A[lo].shape[2]
    trunc = TB.CentredMPS([t.copy() for t in psi.A], psi.centre)
    TB.apply_gate(trunc, layer_gate, chi_max=max(1, chi_here // 2), eps=0.0)
    got = TB.amplitudes(trunc)
    F = abs(np.vdot(ref, got)) ** 2 / (np.vdot(ref, ref).real * np.vdot(got, got).real)
    assert trunc.fs[-1] < 1.0
    assert abs(F - trunc.fs[-1]) < 1e-12


def test_tebd_equals_cluster_tebd_with_one_gate_per_cluster():
    """Cluster-TEBD with k_max = 2 and one sub-layer per step is gate-by-gate
    TEBD: without truncation both oracles give the same state and the same
    number of SVDs (every two-qubit gate and every routing SWAP)."""
    c = paper_random_structured(10, 12, 2, d_max=3, seed=5, workload_id=92)
    a = TB.run(c, chi_max=1024, eps=0.0)
    b = CT.run(c, chi_max=1024, eps=0.0, k_max=2, l_max=1)
    assert MT.infidelity(a.A, b.psi.B) < 1e-13
    assert len(a.fs) == len(b.psi.records)


@pytest.mark.parametrize("seed", [8, 9])
def test_tebd_and_cluster_tebd_k2_agree_under_truncation(seed):
    """With truncation the two forms take the same SVD in exact arithmetic as
    long as the Lambda of the weighted form are the state's Schmidt values;
    after a truncation elsewhere they are only approximately so, which moves
    the result by a fraction of the discarded weight (measured: 5-15 % here).
    A wrong gate orientation or a dropped gate moves it by order one."""
    c = paper_random_structured(12, 30, 2, d_max=2, seed=seed, workload_id=93)
    a = TB.run(c, chi_max=12, eps=1e-12)
    b = CT.run(c, chi_max=12, eps=1e-12, k_max=2, l_max=1)
    assert len(a.fs) == len(b.psi.records)
    Fa, Fb = float(np.exp(a.log_f)), b.fidelity
    discarded = 1 - Fa
    assert 0.02 < discarded < 0.3
    assert abs(Fa - Fb) < 0.25 * discarded
    assert MT.infidelity(a.A, b.psi.B) < 0.25 * discarded


def test_paper_generator_structure():
    for version in (1, 2):
        c, _ = make_workload("paper_clifford_n40_l40" if version == 1 else "paper_nonclifford_n40_l40", seed=0)
        assert c.n == 40 and len(c.layers) == 40
        from workloads.circuits import PAPER_ONE_QUBIT, PAPER_TWO_QUBIT
        n2 = n1 = 0
        for layer in c.layers:
            used = [q for g in layer for q in g.qubits]
            assert sorted(used) == list(range(40))  # one gate per qubit per layer
            for g in layer:
                if len(g.qubits) == 2:
                    assert g.name in PAPER_TWO_QUBIT[version] and abs(g.qubits[0] - g.qubits[1]) == 1
                    n2 += 1
                else:
                    assert g.name in PAPER_ONE_QUBIT[version]
                    n1 += 1
        # a qubit draws a two-qubit gate with p = 0.5 when a neighbour is free:
        # about half of the qubits end up in two-qubit gates
        assert 0.4 < 2 * n2 / (2 * n2 + n1) < 0.7
    # version 2: half of each set non-Clifford
    c2, _ = make_workload("paper_nonclifford_n40_l40", seed=1)
    names = [g.name for layer in c2.layers for g in layer]
    nc = sum(n in ("T", "P3PI4", "X4", "SQRTW", "CH", "CS", "CT", "SQRTSWAP") for n in names)
    assert 0.4 < nc / len(names) < 0.6
