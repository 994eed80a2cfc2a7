"""Pins of the oracle's planner: the worked example of Fig. 6 (Sec. III.A), the
size formula (Eq. size), the caps, and exactness of the SWAP routing."""
import json
import os

import numpy as np
import pytest

from oracle import planner as PL
from oracle import statevector as SV
from workloads import Circuit, Gate, random_structured


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig6_worked_example.json")


def fig6():
    with open(GOLDEN) as f:
        g = json.load(f)
    layers = [[Gate(name, tuple(q)) for name, q in L] for L in g["layers"]]
    return g, layers


def test_fig6_worked_example():
    g, layers = fig6()
    subs = PL.legalize(layers, k_max=8)
    assert len(subs) == len(layers)
    bond = [False] * 7
    PL.mark_bonds(bond, subs[0]); PL.mark_bonds(bond, subs[1])
    assert PL.clusters_of(bond) == [tuple(c) for c in g["clusters_after_layer_2"]]
    # the third layer's gate on (5, 6) joins the last two clusters
    PL.mark_bonds(bond, subs[2])
    assert PL.clusters_of(bond) == [tuple(c) for c in g["clusters_after_layer_3"]]
    # Eq. size for the cluster on 4..7 (bonds marked, chi = 1): 2^{q_n - q_1 + 2}
    e = g["size_exponent_of_cluster_4_to_7"]
    assert PL.cluster_fits(4, 4, [1] * 7, k_max=8, q_max=e)
    assert not PL.cluster_fits(4, 4, [1] * 7, k_max=8, q_max=e - 1)
    # with Q_max = 5 the step ends after layer 4 (layer 5 would make six qubits)
    end, cl = PL.plan_step(subs, 0, 8, [1] * 7, k_max=8, q_max=g["q_max"], l_max=1 << 30)
    assert end == g["step_end_layer"]
    assert cl == [tuple(c) for c in g["step_clusters"]]


def test_size_uses_outer_bonds():
    chi = [2, 4, 8, 4, 2]
    # cluster on sites 1..3: chi_l = chi[0] = 2, chi_r = chi[3] = 4, size = 2^3 * 8 = 2^6
    assert PL.cluster_fits(1, 3, chi, k_max=8, q_max=6)
    assert not PL.cluster_fits(1, 3, chi, k_max=8, q_max=5)
    # edges have a trivial outer bond
    assert PL.cluster_fits(0, 2, chi, k_max=8, q_max=2 + 3)   # chi_r = chi[1] = 4 -> 2^2*4
    assert not PL.cluster_fits(0, 2, chi, k_max=8, q_max=3)
    assert not PL.cluster_fits(0, 3, chi, k_max=2, q_max=99)


def test_l_max_and_single_layer_fallback():
    layers = [[Gate("CNOT", (0, 1))]] * 5
    subs = PL.legalize(layers, 4)
    end, _ = PL.plan_step(subs, 0, 4, [1] * 3, 4, 99, l_max=2)
    assert end == 2
    # a first sub-layer that breaks Q_max is contracted on its own
    end, cl = PL.plan_step(subs, 0, 4, [1] * 3, 4, q_max=1, l_max=99)
    assert end == 1 and cl == [(0, 2)]


def test_legalized_subs_are_disjoint_and_capped():
    c = random_structured(40, 6, 10, ("H", "S", "CNOT"), 0.2, seed=3, workload_id=9)
    for k_max in (2, 3, 5):
        for sub in PL.legalize(c.layers, k_max):
            ivs = sorted((min(g.qubits), max(g.qubits)) for g in sub if len(g.qubits) > 1)
            for (a0, b0), (a1, b1) in zip(ivs, ivs[1:]):
                assert b0 < a1
            assert all(b - a + 1 <= k_max for a, b in ivs)
            qs = [q for g in sub for q in g.qubits]
            assert len(qs) == len(set(qs))


@pytest.mark.parametrize("k_max", [2, 3, 4])
def test_routing_is_exact(k_max):
    c = random_structured(9, 6, 8, ("H", "S", "CNOT", "T"), 0.0, seed=11, workload_id=8)
    subs = PL.legalize(c.layers, k_max)
    routed = Circuit(c.n, subs)
    assert any(g.name == "SWAP" for s in subs for g in s) or k_max >= 9
    a = SV.simulate(c)
    b = SV.simulate(routed)
    assert np.abs(a - b).max() < 1e-13


def test_step_gates_partition():
    c = random_structured(30, 8, 5, ("H", "S", "CNOT"), 0.3, seed=5, workload_id=7)
    subs = PL.legalize(c.layers, 4)
    start = 0
    total = sum(len(s) for s in subs)
    seen = 0
    while start < len(subs):
        end, cl = PL.plan_step(subs, start, 30, [1] * 29, 4, 99, 1 << 30)
        pc, ps = PL.step_gates(subs, start, end, cl, 30)
        seen += sum(map(len, pc)) + sum(map(len, ps))
        for (a, k), gl in zip(cl, pc):
            assert 2 <= k <= 4
            assert all(a <= q < a + k for g in gl for q in g.qubits)
        start = end
    assert seen == total
