"""Pins of the FP64 cluster-TEBD oracle against things other than itself:
brute-force statevectors, exact Schmidt values, the single-truncation closed
form of the fidelity, canonical-form invariants, and stabilizer-tableau
entropies of Clifford circuits."""
import math

import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import gates as G
from oracle import mps_tools as MT
from oracle import planner as PL
from oracle import stabilizer as ST
from oracle import statevector as SV
from workloads import Circuit, Gate, make_workload, random_structured


def haar(d, rng):
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def dense_circuit(n, layers, d_max, seed):
    # every qubit active each layer: denser entanglement than the workloads
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(layers):
        order = rng.permutation(n)
        used = set()
        L = []
        for a in order:
            a = int(a)
            if a in used:
                continue
            b = a + int(rng.integers(1, d_max + 1)) * (1 if rng.random() < 0.5 else -1)
            if 0 <= b < n and b not in used:
                used |= {a, b}
                L.append(Gate(str(rng.choice(["CNOT", "CZ", "SQRTSWAP", "CT"])), (a, b)))
            else:
                used.add(a)
                L.append(Gate(str(rng.choice(["H", "T", "X4", "SQRTW"])), (a,)))
        out.append(L)
    return Circuit(n, out)


def test_truncation_rule():
    s = np.array([0.8, 0.5, 0.3, 1e-13, 0.0])
    assert CT.truncation_rank(s, 10, 1e-12) == 3      # cutoff on normalised values
    assert CT.truncation_rank(s, 2, 1e-12) == 2       # then the cap
    assert CT.truncation_rank(np.array([1e-20, 1e-21]), 4, 0.5) == 1   # at least one
    assert CT.truncation_rank(s * 1e-6, 10, 1e-12) == 3  # scale free


@pytest.mark.parametrize("seed,k_max", [(0, 2), (1, 3), (2, 4), (3, 6)])
def test_exact_vs_statevector_dense(seed, k_max):
    c = dense_circuit(10, 8, 4, seed)
    res = CT.run(c, chi_max=1 << 10, eps=0.0, k_max=k_max)
    sv = SV.simulate(c)
    amp = MT.amplitudes(res.psi.B)
    assert np.abs(amp - sv).max() < 1e-12
    assert abs(res.fidelity - 1.0) < 1e-12
    # Lambda_b are the exact Schmidt values of the state at every bond
    for b, lam in enumerate(res.psi.lam):
        ref = MT.schmidt_from_state(sv, c.n, b + 1)
        ref = ref[ref > 1e-12]
        assert lam.size >= ref.size
        assert np.abs(np.sort(lam)[::-1][: ref.size] - ref).max() < 1e-10
    # every site but B_0 is right-canonical
    for t in res.psi.B[1:]:
        assert MT.right_canonical_error(t) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_exact_workload_vs_statevector(seed):
    c, p = make_workload("exact_n12_l10", seed=seed)
    res = CT.run(c, **p)
    sv = SV.simulate(c)
    assert np.abs(MT.amplitudes(res.psi.B) - sv).max() < 1e-12
    assert res.cluster_updates > 0


def test_random_cluster_unitaries_vs_statevector():
    rng = np.random.default_rng(7)
    n = 9
    psi = CT.product_state(n)
    sv = np.zeros(2 ** n, complex); sv[0] = 1
    for a, k in [(0, 3), (2, 4), (5, 4), (1, 6), (3, 2), (0, 9), (4, 5)]:
        U = haar(2 ** k, rng)
        CT.apply_cluster(psi, a, k, U, chi_max=1 << 9, eps=0.0)
        sv = SV.apply_gate(sv, n, U, list(range(a, a + k)))
    assert np.abs(MT.amplitudes(psi.B) - sv).max() < 1e-12


def test_single_truncation_closed_form():
    """One truncated SVD of a canonical state: exact fidelity = f (Eq. f_i)."""
    rng = np.random.default_rng(3)
    n = 6
    psi = CT.product_state(n)
    CT.apply_cluster(psi, 0, 6, haar(64, rng), chi_max=64, eps=0.0)
    assert psi.bond_dims() == [2, 4, 8, 4, 2]
    U = haar(4, rng)
    exact = SV.apply_gate(MT.amplitudes(psi.B), n, U, [2, 3])
    trunc = psi.copy(); trunc.records = []
    CT.apply_cluster(trunc, 2, 2, U, chi_max=3, eps=0.0)
    assert len(trunc.records) == 1 and trunc.records[0].rank == 3
    f = trunc.records[0].f
    assert f < 0.999
    amp = MT.amplitudes(trunc.B)
    F = abs(np.vdot(exact, amp)) ** 2 / (np.vdot(amp, amp).real * np.vdot(exact, exact).real)
    assert abs(F - f) < 1e-12
    assert abs(math.exp(trunc.log_f) - f) < 1e-14
    # after renormalisation the state has unit norm
    assert abs(np.vdot(amp, amp).real - 1.0) < 1e-12
    # the kept Schmidt values equal the exact ones at that bond, renormalised
    ref = MT.schmidt_from_state(exact, n, 3)[:3]
    assert np.abs(trunc.lam[2] - ref / np.linalg.norm(ref)).max() < 1e-12


def test_identity_and_bell_ghz():
    psi = CT.product_state(4)
    CT.apply_cluster(psi, 1, 2, np.eye(4, dtype=complex), 8, 1e-12)
    assert psi.bond_dims() == [1, 1, 1]
    assert abs(MT.amplitudes(psi.B)[0] - 1) < 1e-15
    bell = G.CNOT @ np.kron(G.H, G.I2)
    CT.apply_cluster(psi, 0, 2, bell, 8, 1e-12)
    assert np.allclose(psi.lam[0], [2 ** -0.5] * 2, atol=1e-15)
    # GHZ on 4 qubits: every bond has two equal Schmidt values
    psi = CT.product_state(4)
    c = Circuit(4, [[Gate("H", (0,))], [Gate("CNOT", (0, 1))], [Gate("CNOT", (1, 2))], [Gate("CNOT", (2, 3))]])
    res = CT.run(c, chi_max=8, eps=1e-12, k_max=2)
    for lam in res.psi.lam:
        assert np.allclose(lam, [2 ** -0.5] * 2, atol=1e-14)


def test_product_state_keeps_chi_one():
    c = Circuit(6, [[Gate("H", (q,)) for q in range(6)], [Gate("T", (q,)) for q in range(6)],
                    [Gate("CZ", (0, 1)), Gate("CZ", (2, 3))], [Gate("CZ", (0, 1)), Gate("CZ", (2, 3))]])
    res = CT.run(c, chi_max=8, eps=1e-12, k_max=4)
    assert res.psi.bond_dims() == [1] * 5


def test_tableau_vs_statevector_entropies():
    for seed in range(3):
        c = random_structured(10, 12, 9, ("H", "S", "CNOT"), 0.0, seed=seed, workload_id=21)
        S_tab = ST.circuit_entropies(c)
        sv = SV.simulate(c)
        S_sv = [MT.entropy_bits(MT.schmidt_from_state(sv, 10, b + 1)) for b in range(9)]
        assert np.allclose(S_tab, S_sv, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_clifford_workload_entropies(seed):
    c, p = make_workload("clifford_n100_l20", seed=seed)
    S_tab = ST.circuit_entropies(c)
    assert max(S_tab) <= 8    # chi_max = 256 is never reached: no truncation
    res = CT.run(c, **p)
    assert abs(res.fidelity - 1.0) < 1e-12
    for b, lam in enumerate(res.psi.lam):
        assert lam.size == 2 ** S_tab[b]
        # flat spectrum of a stabilizer state
        assert np.abs(lam - 2.0 ** (-S_tab[b] / 2)).max() < 1e-10


def test_truncating_run_fidelity_estimate():
    """Several truncations: prod f tracks the exact fidelity (Eq. approxF) and
    never exceeds one."""
    c = dense_circuit(12, 10, 3, seed=4)
    exact = SV.simulate(c)
    for chi in (2, 4):
        res = CT.run(c, chi_max=chi, eps=1e-12, k_max=4)
        amp = MT.amplitudes(res.psi.B)
        F = abs(np.vdot(exact, amp)) ** 2 / np.vdot(amp, amp).real
        assert 0.3 < res.fidelity < 0.95
        assert abs(F - res.fidelity) < 0.05 * (1 - res.fidelity)
