"""Cluster-TEBD planner of the oracle (Sec. III.A, Fig. 6 worked example).

The paper's iteration keeps a boolean array over the n-1 bonds; a gate on qubits
i..i+n-1 marks bonds i..i+n-2; after each layer the entanglement clusters are
the maximal runs of marked bonds; the circuit is contracted up to the last layer
for which every cluster obeys log2(size) <= Q_max (size = 2^k chi_left chi_right,
Eqs. size and cond_cTEBD) and the number of layers obeys L <= L_max (Eq.
cond2_cTEBD).  Readings where the paper is silent:

  * a gate on non-adjacent qubits (a, b) marks every bond a..b-1, so its cluster
    is the whole span and counts the idle qubits inside it;
  * a cluster may in addition hold at most k_max qubits;
  * gates whose span exceeds k_max are routed with chains of adjacent SWAPs
    (Sec. IV.A: long-range gates are brought next to each other by SWAPs and
    moved back afterwards), each SWAP in a layer of its own;
  * gates of one layer act on disjoint qubits and commute, so a layer is split
    into sub-layers whose gate spans are pairwise disjoint; sub-layers are the
    unit the planner advances by (and the unit L_max counts);
  * if even the first sub-layer of a step breaks a cap it is contracted anyway;
  * the size test uses exact integers: 2^k * chi_l * chi_r <= 2^Q_max.

Bonds are 0-based: bond b joins sites b and b+1; chi_{-1} = chi_{n-1} = 1.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

from workloads.circuits import Gate


def _span(g: Gate) -> Tuple[int, int]:
    return min(g.qubits), max(g.qubits)


def _route(g: Gate, k_max: int) -> List[Gate]:
    """SWAP chain that brings the far qubit of ``g`` to distance k_max-1 from
    the near one, the gate itself, then the chain undone."""
    lo, hi = _span(g)
    p = lo + k_max - 1
    down = [Gate("SWAP", (j, j + 1)) for j in range(hi - 1, p - 1, -1)]
    moved = Gate(g.name, tuple(p if q == hi else q for q in g.qubits))
    return down + [moved] + down[::-1]


def _disjoint(iv: Tuple[int, int], ivs: Sequence[Tuple[int, int]]) -> bool:
    return all(iv[1] < a or iv[0] > b for a, b in ivs)


def legalize_layer(gates: Sequence[Gate], k_max: int) -> List[List[Gate]]:
    """One layer (Sec. II.A) as sub-layers of pairwise disjoint spans, gates
    wider than k_max routed by SWAP chains (Sec. IV.A)."""
    ones = [g for g in gates if len(g.qubits) == 1]
    multi = sorted((g for g in gates if len(g.qubits) > 1), key=lambda g: (_span(g), g.qubits))
    short = [g for g in multi if _span(g)[1] - _span(g)[0] + 1 <= k_max]
    far = [g for g in multi if _span(g)[1] - _span(g)[0] + 1 > k_max]

    subs: List[List[Gate]] = [list(ones)]
    ivs: List[List[Tuple[int, int]]] = [[]]
    for g in short:
        iv = _span(g)
        for i in range(len(subs)):
            if _disjoint(iv, ivs[i]):
                subs[i].append(g)
                ivs[i].append(iv)
                break
        else:
            subs.append([g])
            ivs.append([iv])

    groups: List[List[List[Gate]]] = []
    givs: List[List[Tuple[int, int]]] = []
    for g in far:
        iv = _span(g)
        ops = _route(g, k_max)
        for i in range(len(groups)):
            if _disjoint(iv, givs[i]):
                groups[i].append(ops)
                givs[i].append(iv)
                break
        else:
            groups.append([ops])
            givs.append([iv])
    for units in groups:
        depth = max(len(u) for u in units)
        for t in range(depth):
            subs.append([u[t] for u in units if t < len(u)])
    return [s for s in subs if s]


def legalize(layers: Sequence[Sequence[Gate]], k_max: int) -> List[List[Gate]]:
    """Every layer of a circuit through legalize_layer, in order."""
    out: List[List[Gate]] = []
    for layer in layers:
        out.extend(legalize_layer(layer, k_max))
    return out


def mark_bonds(bond: List[bool], gates: Sequence[Gate]) -> None:
    """The bond array of Sec. III.A: a multi-qubit gate marks every bond its
    span crosses."""
    for g in gates:
        if len(g.qubits) > 1:
            lo, hi = _span(g)
            for b in range(lo, hi):
                bond[b] = True


def clusters_of(bond: Sequence[bool]) -> List[Tuple[int, int]]:
    """Maximal runs of marked bonds as (first site a, number of sites k)."""
    out = []
    b, nb = 0, len(bond)
    while b < nb:
        if bond[b]:
            e = b
            while e + 1 < nb and bond[e + 1]:
                e += 1
            out.append((b, e - b + 2))
            b = e + 1
        else:
            b += 1
    return out


def cluster_fits(a: int, k: int, chi: Sequence[int], k_max: int, q_max: int) -> bool:
    """k <= k_max and size = 2^k chi_l chi_r <= 2^Q_max (Eqs. size and
    cond_cTEBD), in exact integers."""
    n_bonds = len(chi)
    chi_l = chi[a - 1] if a > 0 else 1
    chi_r = chi[a + k - 1] if a + k - 1 < n_bonds else 1
    return k <= k_max and (chi_l * chi_r) << k <= (1 << q_max)


def plan_step(subs: Sequence[Sequence[Gate]], start: int, n: int, chi: Sequence[int],
              k_max: int, q_max: int, l_max: int) -> Tuple[int, List[Tuple[int, int]]]:
    """Last sub-layer index (exclusive) of the step starting at ``start`` and the
    clusters of that step (Sec. III.A, Eqs. size, cond_cTEBD, cond2_cTEBD)."""
    bond = [False] * (n - 1)
    end = start
    while end < len(subs) and end - start < l_max:
        trial = list(bond)
        mark_bonds(trial, subs[end])
        if all(cluster_fits(a, k, chi, k_max, q_max) for a, k in clusters_of(trial)):
            bond = trial
            end += 1
        else:
            break
    if end == start:
        bond = [False] * (n - 1)
        mark_bonds(bond, subs[start])
        end = start + 1
    return end, clusters_of(bond)


def default_q_max(k_max: int, chi_max: int) -> int:
    """Q_max that never binds when every bond is at most chi_max."""
    return k_max + 2 * max(0, (chi_max - 1).bit_length())


def step_gates(subs: Sequence[Sequence[Gate]], start: int, end: int,
               clusters: Sequence[Tuple[int, int]], n: int):
    """Gates of each cluster (in circuit order) and the one-qubit gates of the
    sites that belong to no cluster."""
    owner = [-1] * n
    for ci, (a, k) in enumerate(clusters):
        for q in range(a, a + k):
            owner[q] = ci
    per_cluster: List[List[Gate]] = [[] for _ in clusters]
    per_site: List[List[Gate]] = [[] for _ in range(n)]
    for s in range(start, end):
        for g in subs[s]:
            c = owner[g.qubits[0]]
            if c >= 0:
                per_cluster[c].append(g)
            else:
                assert len(g.qubits) == 1
                per_site[g.qubits[0]].append(g)
    return per_cluster, per_site
