"""Pins of the oracle's truncation through an exactly degenerate multiplet
(Sec. II.B, Sec. III.A): Bell pairs across a cluster, cut at the middle bond
by chi_max (inputs from workloads.degenerate).  Whatever subspace of the
multiplet is kept, one truncation of a Schmidt decomposition leaves the
exact fidelity f = chi_max / 2^{k/2}; the cut is flagged degenerate; the
Schmidt values at and right of the cut are flat; left of the cut they are the
final state's own."""
import math

import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import mps_tools as MT
from workloads.degenerate import CASES, cluster_unitary, crossing_pairs


@pytest.mark.parametrize("k,chi", CASES)
def test_cut_through_multiplet(k, chi):
    U = cluster_unitary(k, seed=k * 100 + chi)
    psi = CT.product_state(k)
    CT.apply_cluster(psi, 0, k, U, chi, 1e-12)
    h = k // 2
    f = chi / 2 ** h
    mid = h - 1
    # records: only the middle bond truncates, and it is flagged
    for r in psi.records:
        if r.bond == mid:
            assert r.rank == chi and r.full == 2 ** h and r.degenerate_cut
            assert abs(r.f - f) < 1e-13
        else:
            assert r.rank == r.full == 2 ** crossing_pairs(k, r.bond) and not r.degenerate_cut
    assert abs(math.exp(psi.log_f) - f) < 1e-13
    # the exact fidelity of the result: the closed form of one truncation
    amp = MT.amplitudes(psi.B)
    exact = U[:, 0]
    F = abs(np.vdot(exact, amp)) ** 2 / np.vdot(amp, amp).real
    assert abs(F - f) < 1e-12
    # Schmidt values: flat at and right of the cut, the final state's own left of it
    for b in range(k - 1):
        lam = psi.lam[b]
        if b >= mid:
            r = chi if b == mid else 2 ** crossing_pairs(k, b)
            assert np.abs(lam - 1 / math.sqrt(r)).max() < 1e-13
        else:
            ref = MT.schmidt_from_state(amp / np.linalg.norm(amp), k, b + 1)
            assert np.abs(lam - ref[:lam.size]).max() < 1e-12
    for j in range(1, k):
        assert MT.right_canonical_error(psi.B[j]) < 1e-13


def test_inputs_are_flat_at_every_bond():
    """The recipe itself: the exact state's spectra are 2^{-S_b/2}, S_b pairs."""
    for k, chi in CASES:
        psi = cluster_unitary(k, seed=k * 100 + chi)[:, 0]
        for b in range(k - 1):
            s = MT.schmidt_from_state(psi, k, b + 1)
            S = crossing_pairs(k, b)
            assert np.abs(s[:2 ** S] - 2 ** (-S / 2)).max() < 1e-13
            assert s[2 ** S:].max(initial=0.0) < 1e-13
