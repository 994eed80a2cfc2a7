"""Seeded paired-qubit states at the largest bond dimensions: an exact MPS in
the form the cluster step keeps (right-canonical sites, Lambda_b the Schmidt
values of bond b, descending; Secs. II.B, III.A), written down in closed form
so that no SVD is needed to build it.  Input construction only.

Pair p joins qubits (a_p, b_p) in the state cos t_p |00> + sin t_p |11>; the
other qubits are |0>.  Bond b is crossed by the pairs with a_p <= b < b_p; its
Schmidt vectors are labelled by the bits x of those pairs and its Schmidt
values are prod_p w_p(x_p) with w_p = (cos t_p, sin t_p).  In that basis the
sites are copy tensors: at a left end a_p the right bond gains the bit x_p = s
with weight w_p(s); at a right end b_p the bit leaves the bond and s = x_p;
an unpaired qubit passes the bond through with s = 0.  Every such tensor is
right-canonical (each left index has one outgoing entry of weight 1, or two
of squared weights summing to 1) and the product of the weights along any
configuration is the amplitude.  Each bond's basis is then sorted by
descending Schmidt value (ties by label)."""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def pair_angles(npairs: int, seed: int) -> np.ndarray:
    """Angles in [0.35, 0.65] * pi/2: no pair is close to a product or to a
    maximally entangled pair, and products of distinct subsets of the
    weights are generically distinct."""
    rng = np.random.default_rng(np.random.SeedSequence([79, seed]))
    return (0.35 + 0.3 * rng.random(npairs)) * (np.pi / 2)


def _crossing(pairs: Sequence[Tuple[int, int]], b: int) -> List[int]:
    return [p for p, (lo, hi) in enumerate(pairs) if lo <= b < hi]


def paired_state(n: int, pairs: Sequence[Tuple[int, int]], thetas: Sequence[float]
                 ) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """(B, lam): B[j] of shape (chi_{j-1}, 2, chi_j), complex128; lam[b] the
    Schmidt values of bond b, descending."""
    used = [q for pr in pairs for q in pr]
    assert len(used) == len(set(used)) and all(0 <= q < n for q in used)
    assert all(lo < hi for lo, hi in pairs) and len(thetas) == len(pairs)
    w = np.array([[np.cos(t), np.sin(t)] for t in thetas])
    role = {}
    for p, (lo, hi) in enumerate(pairs):
        role[lo] = ("left", p)
        role[hi] = ("right", p)
    plist = [_crossing(pairs, b) for b in range(n - 1)]
    # Schmidt values by label, and the order that sorts them descending
    lam, new_of = [], []
    for b in range(n - 1):
        x = np.arange(1 << len(plist[b]))
        val = np.ones(x.size)
        for i, p in enumerate(plist[b]):
            val *= w[p][(x >> i) & 1]
        order = np.lexsort((x, -val))     # descending value, then label
        inv = np.empty_like(order)
        inv[order] = np.arange(order.size)
        lam.append(val[order])
        new_of.append(inv)
    B = []
    for j in range(n):
        L = plist[j - 1] if j > 0 else []
        R = plist[j] if j < n - 1 else []
        xl = np.arange(1 << len(L))
        bits = {p: (xl >> i) & 1 for i, p in enumerate(L)}
        kind, pp = role.get(j, ("none", -1))
        T = np.zeros((xl.size, 2, 1 << len(R)), dtype=np.complex128)
        for s in (0, 1):
            if kind == "left":
                bits_r = dict(bits)
                bits_r[pp] = np.full(xl.size, s)
                amp = np.full(xl.size, w[pp][s])
                ok = np.ones(xl.size, bool)
            elif kind == "right":
                bits_r = {p: v for p, v in bits.items() if p != pp}
                ok = bits[pp] == s
                amp = np.ones(xl.size)
            else:
                bits_r = bits
                ok = np.full(xl.size, s == 0)
                amp = np.ones(xl.size)
            xr = np.zeros(xl.size, dtype=np.int64)
            for i, p in enumerate(R):
                xr |= bits_r[p].astype(np.int64) << i
            T[xl[ok], s, xr[ok]] = amp[ok]
        # relabel both bonds in descending Schmidt order
        li = new_of[j - 1] if j > 0 else np.zeros(1, dtype=np.int64)
        ri = new_of[j] if j < n - 1 else np.zeros(1, dtype=np.int64)
        S = np.zeros_like(T)
        S[np.ix_(li, [0, 1], ri)] = T
        B.append(S)
    return B, lam
