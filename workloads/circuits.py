"""Random-structured circuit generator (structure only, no gate arithmetic).

The paper's benchmark circuits (Sec. IV.A) are random-structured: in every layer
each qubit receives a random one- or two-qubit gate, the initial state is the
all-|0> product state, and a layer holds gates on disjoint qubits (Sec. II.A).
The circuits used here keep that structure with the following seeded recipe:

  per layer
    1. choose floor(n/2) active qubits uniformly without replacement;
    2. visit the active qubits in random order; an unpaired qubit ``a`` draws a
       distance d ~ U{1..d_max} and a direction +-1 and pairs with ``a +- d`` if
       that qubit is active and unpaired (at most 8 draws, else ``a`` stays alone);
    3. every pair draws a symbol uniformly from ``symbols``: ``CNOT`` becomes a
       CNOT with the first-drawn qubit as control, a one-qubit symbol is applied
       to both qubits of the pair;
    4. with T density rho_T > 0, every qubit still without a gate in this layer
       receives a T gate with probability min(1, rho_T * n / #eligible), so the
       expected number of T gates per qubit-layer is rho_T while every qubit
       keeps at most one gate per layer.

The generator is a numpy PCG64 stream seeded with (workload id, seed).
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np


@dataclass(frozen=True)
class Gate:
    """A gate symbol and the qubits it acts on, in the order of its matrix
    (for CNOT: (control, target))."""
    name: str
    qubits: Tuple[int, ...]


@dataclass
class Circuit:
    n: int
    layers: List[List[Gate]]
    meta: Dict = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return sum(len(l) for l in self.layers)


ONE_QUBIT = ("H", "S", "T", "X", "Y", "Z")


def _rng(workload_id: int, seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload_id, seed])))


def random_structured(n: int, n_layers: int, d_max: int, symbols: Sequence[str],
                      rho_t: float = 0.0, seed: int = 0, workload_id: int = 0) -> Circuit:
    rng = _rng(workload_id, seed)
    layers: List[List[Gate]] = []
    for _ in range(n_layers):
        active = rng.choice(n, size=n // 2, replace=False)
        is_active = np.zeros(n, dtype=bool)
        is_active[active] = True
        paired = np.zeros(n, dtype=bool)
        pairs: List[Tuple[int, int]] = []
        for a in rng.permutation(active):
            a = int(a)
            if paired[a]:
                continue
            for _try in range(8):
                d = int(rng.integers(1, d_max + 1))
                b = a + d if rng.random() < 0.5 else a - d
                if 0 <= b < n and is_active[b] and not paired[b]:
                    pairs.append((a, b))
                    paired[a] = paired[b] = True
                    break
        gates: List[Gate] = []
        used = np.zeros(n, dtype=bool)
        for a, b in pairs:
            sym = symbols[int(rng.integers(0, len(symbols)))]
            if sym == "CNOT":
                gates.append(Gate("CNOT", (a, b)))
            else:
                gates.append(Gate(sym, (a,)))
                gates.append(Gate(sym, (b,)))
            used[a] = used[b] = True
        if rho_t > 0.0:
            eligible = np.flatnonzero(~used)
            if eligible.size:
                p = min(1.0, rho_t * n / eligible.size)
                draws = rng.random(eligible.size)
                for q in eligible[draws < p]:
                    gates.append(Gate("T", (int(q),)))
        gates.sort(key=lambda g: (min(g.qubits), g.qubits))
        layers.append(gates)
    return Circuit(n=n, layers=layers,
                   meta=dict(d_max=d_max, symbols=list(symbols), rho_t=rho_t,
                             seed=seed, workload_id=workload_id))


# The paper's own random-structured circuits (Sec. IV.A): in every layer each
# qubit receives either a single-qubit or a two-qubit gate with probability
# p = 0.5, gates drawn uniformly from the version's sets; version 1 is
# Clifford, version 2 adds four non-Clifford gates to each set (half of each
# set is then non-Clifford).
PAPER_ONE_QUBIT = {1: ("H", "X", "Y", "Z"), 2: ("H", "X", "Y", "Z", "T", "P3PI4", "X4", "SQRTW")}
PAPER_TWO_QUBIT = {1: ("CNOT", "CY", "CZ", "SWAP"), 2: ("CNOT", "CY", "CZ", "SWAP", "CH", "CS", "CT", "SQRTSWAP")}


def paper_random_structured(n: int, n_layers: int, version: int, p_two: float = 0.5, d_max: int = 1,
                            seed: int = 0, workload_id: int = 0) -> Circuit:
    """Per layer, the qubits are visited in a random order; a qubit still free
    in this layer draws a two-qubit gate with probability p_two (else a
    single-qubit gate); a two-qubit gate takes as second qubit a free qubit at
    distance 1..d_max drawn uniformly (the first drawn qubit is the control of
    a controlled gate); with no free qubit in reach the qubit gets a
    single-qubit gate.  Every qubit thus carries exactly one gate per layer."""
    rng = _rng(workload_id, seed)
    ones, twos = PAPER_ONE_QUBIT[version], PAPER_TWO_QUBIT[version]
    layers: List[List[Gate]] = []
    for _ in range(n_layers):
        free = np.ones(n, dtype=bool)
        gates: List[Gate] = []
        for a in rng.permutation(n):
            a = int(a)
            if not free[a]:
                continue
            free[a] = False
            if rng.random() < p_two:
                cand = [b for d in range(1, d_max + 1) for b in (a - d, a + d) if 0 <= b < n and free[b]]
                if cand:
                    b = int(cand[int(rng.integers(0, len(cand)))])
                    free[b] = False
                    gates.append(Gate(twos[int(rng.integers(0, len(twos)))], (a, b)))
                    continue
            gates.append(Gate(ones[int(rng.integers(0, len(ones)))], (a,)))
        gates.sort(key=lambda g: (min(g.qubits), g.qubits))
        layers.append(gates)
    return Circuit(n=n, layers=layers, meta=dict(generator="paper", version=version, p_two=p_two, d_max=d_max,
                                                 seed=seed, workload_id=workload_id))


# Named workloads: the circuit recipe plus the truncation / clustering parameters
# (cap chi_max, cutoff eps, largest cluster k_max) each one is simulated with.
WORKLOADS = {
    "exact_n12_l10": dict(wid=1, n=12, layers=10, d_max=11, symbols=("H", "S", "CNOT", "T"),
                          rho_t=0.0, k_max=3, chi_max=64, eps=1e-12),
    "clifford_n100_l20": dict(wid=2, n=100, layers=20, d_max=10, symbols=("H", "S", "CNOT"),
                              rho_t=0.0, k_max=5, chi_max=256, eps=1e-12),
    "batched_n1000_l100": dict(wid=3, n=1000, layers=100, d_max=10, symbols=("H", "S", "CNOT"),
                               rho_t=0.1, k_max=8, chi_max=128, eps=1e-12),
    "chi1024_n200_l50": dict(wid=4, n=200, layers=50, d_max=10, symbols=("H", "S", "CNOT"),
                             rho_t=0.2, k_max=6, chi_max=1024, eps=1e-10),
    "learned_n500_l60": dict(wid=5, n=500, layers=60, d_max=10, symbols=("H", "S", "CNOT"),
                             rho_t=0.15, k_max=6, chi_max=512, eps=1e-10),
    # the paper's generator (Sec. IV.A): Clifford and non-Clifford versions,
    # nearest-neighbour two-qubit gates, 40 qubits and 40 layers (the size at
    # which the paper reports its largest cluster-TEBD speed-ups)
    "paper_clifford_n40_l40": dict(wid=6, n=40, layers=40, version=1, d_max=1, k_max=6, chi_max=1024, eps=1e-12),
    "paper_nonclifford_n40_l40": dict(wid=7, n=40, layers=40, version=2, d_max=1, k_max=6, chi_max=1024,
                                      eps=1e-12),
    # deeper and wider: entanglement reaches the cap (the regime of the paper's
    # 100-layer Clifford and 80-layer non-Clifford comparisons)
    "paper_clifford_n100_l100": dict(wid=8, n=100, layers=100, version=1, d_max=1, k_max=6, chi_max=1024,
                                     eps=1e-12),
    "paper_nonclifford_n100_l80": dict(wid=9, n=100, layers=80, version=2, d_max=1, k_max=6, chi_max=1024,
                                       eps=1e-12),
    # the smallest of the paper's DMRG benchmark sizes (60 qubits, 60 layers, non-Clifford)
    "paper_nonclifford_n60_l60": dict(wid=10, n=60, layers=60, version=2, d_max=1, k_max=6, chi_max=1024,
                                      eps=1e-12),
}


def make_workload(name: str, seed: int = 0, n: int | None = None, layers: int | None = None) -> Tuple[Circuit, Dict]:
    """Circuit and simulation parameters of a named workload (optionally shrunk
    in n or depth for quick tests; the recipe is unchanged)."""
    w = dict(WORKLOADS[name])
    nn = w["n"] if n is None else n
    ll = w["layers"] if layers is None else layers
    if "version" in w:
        c = paper_random_structured(nn, ll, w["version"], 0.5, min(w["d_max"], nn - 1), seed, w["wid"])
    else:
        c = random_structured(nn, ll, min(w["d_max"], nn - 1), w["symbols"], w["rho_t"], seed, w["wid"])
    c.meta["workload"] = name
    params = dict(k_max=w["k_max"], chi_max=w["chi_max"], eps=w["eps"])
    return c, params


def save_circuit(c: Circuit, path: str) -> None:
    with open(path, "w") as f:
        json.dump({"n": c.n, "meta": c.meta,
                   "layers": [[[g.name, list(g.qubits)] for g in l] for l in c.layers]}, f)


def load_circuit(path: str) -> Circuit:
    with open(path) as f:
        d = json.load(f)
    return Circuit(n=d["n"], meta=d.get("meta", {}),
                   layers=[[Gate(name, tuple(q)) for name, q in l] for l in d["layers"]])
