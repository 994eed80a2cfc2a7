"""Property-based pins of the oracle (hypothesis): random small circuits,
caps and gate sets, each property fixed by the definition it follows rather
than by the oracle itself.

* Without truncation the cluster-TEBD oracle (Secs. II.B, III.A) is exact:
  its amplitudes are the statevector's, every f_i is 1, sites 1..n-1 are
  right-canonical on the support of the Schmidt values left of them (at
  eta = 0 exact zeros are kept, and a row behind a zero weight carries no
  amplitude) and Lambda_b holds the statevector's Schmidt values at bond b,
  for any k_max, Q_max and L_max (the caps change the steps, not the
  state).  With a cutoff of 1e-10 the exact zeros are dropped and every
  site is right-canonical.
* With truncation: the caps hold, F_est = prod f_i as recorded, the Schmidt
  values stay normalised and descending; a run whose only truncation is one
  split has exact fidelity |<psi|psi_exact>|^2 = f of that split (one cut of
  a Schmidt decomposition).  (Right-canonical form and the norm hold only up
  to the discarded weight once a cluster's leftmost site absorbs a
  truncation, so they are not asserted here.)
* One cluster applied to an exact state: its splits truncate nested
  Schmidt decompositions (each split cuts the state the previous one left),
  so the exact fidelity is the product of its f_i.  Between clusters of one
  step Eq. approxF is an approximation: a weighted GHZ state
  a|0000> + b|1111> cut to one value at bonds 0 and 2 by two clusters has
  F_est = a^4 while the exact fidelity is a^2.
* The gate-by-gate TEBD oracle (Sec. II.C) without truncation is exact too.
* The grouping of the DMRG variant (Eqs. cond_group1 / cond_group2)
  partitions the chain into consecutive groups, each a single site or within
  Q_max.
"""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import ctebd as CT
from oracle import dmrg as DM
from oracle import mps_tools as MT
from oracle import statevector as SV
from oracle import tebd as TB
from workloads import Circuit, Gate
from workloads.mps_inputs import haar_unitary

ONE = ["H", "S", "T", "X", "Y", "Z", "X4", "SQRTW", "P3PI4"]
TWO = ["CNOT", "CY", "CZ", "SWAP", "SQRTSWAP"]


@st.composite
def circuits(draw, n_max=8):
    n = draw(st.integers(2, n_max))
    nl = draw(st.integers(1, 5))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    layers = []
    for _ in range(nl):
        free = list(rng.permutation(n))
        layer = []
        while free:
            q = int(free.pop())
            if free and rng.random() < 0.55:
                # a partner at any distance (long-range gates are routed)
                r = int(free.pop(int(rng.integers(len(free)))))
                layer.append(Gate(TWO[int(rng.integers(len(TWO)))], (q, r)))
            elif rng.random() < 0.8:
                layer.append(Gate(ONE[int(rng.integers(len(ONE)))], (q,)))
        layers.append(layer)
    return Circuit(n, layers)


SETTINGS = settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])


def _rc_error_on_support(B, lam_left):
    """max |(B B^H)[i, i'] - delta| over the rows i, i' with lam_left > 0."""
    M = B.reshape(B.shape[0], -1)
    on = np.nonzero(lam_left > 1e-12)[0]
    M = M[on]
    return float(np.abs(M @ M.conj().T - np.eye(on.size)).max()) if on.size else 0.0


@SETTINGS
@given(circuits(), st.integers(2, 6), st.sampled_from([None, 0, 1, 3]), st.sampled_from([1 << 30, 1, 2]))
def test_untruncated_cluster_tebd_is_exact(c, k_max, q_extra, l_max):
    q_max = None if q_extra is None else k_max + q_extra  # None: never binds
    ref = CT.run(c, chi_max=1 << 20, eps=0.0, k_max=k_max, q_max=q_max, l_max=l_max)
    sv = SV.simulate(c)
    assert np.abs(MT.amplitudes(ref.psi.B) - sv).max() < 1e-12
    assert abs(ref.psi.log_f) < 1e-12
    assert all(abs(r.f - 1) < 1e-12 for r in ref.psi.records)
    for j in range(1, c.n):
        assert _rc_error_on_support(ref.psi.B[j], ref.psi.lam[j - 1]) < 1e-12
    for b in range(c.n - 1):
        exact = MT.schmidt_from_state(sv, c.n, b + 1)
        lam = ref.psi.lam[b]
        assert np.abs(lam - exact[:lam.size]).max() < 1e-10
        assert np.all(exact[lam.size:] < 1e-7)  # only numerically zero values left out
    # exact zeros dropped by a cutoff: the same state, every site right-canonical
    cut = CT.run(c, chi_max=1 << 20, eps=1e-10, k_max=k_max, q_max=q_max, l_max=l_max)
    assert np.abs(MT.amplitudes(cut.psi.B) - sv).max() < 1e-9
    for j in range(1, c.n):
        assert MT.right_canonical_error(cut.psi.B[j]) < 1e-12


@SETTINGS
@given(circuits(n_max=7), st.integers(2, 5), st.integers(1, 3))
def test_truncated_run_keeps_the_form_and_its_bookkeeping(c, k_max, chi_max):
    ref = CT.run(c, chi_max=chi_max, eps=1e-12, k_max=k_max)
    psi = ref.psi
    assert max(psi.bond_dims()) <= chi_max
    assert abs(psi.log_f - sum(math.log(r.f) for r in psi.records)) < 1e-12
    amp = MT.amplitudes(psi.B)
    for b in range(c.n - 1):
        assert abs(np.linalg.norm(psi.lam[b]) - 1) < 1e-12
        assert np.all(np.diff(psi.lam[b]) <= 1e-15)
    cut = [r for r in psi.records if r.rank < r.full and r.f < 1 - 1e-12]
    if len(cut) == 1 and len(ref.steps) == 1:
        # one step, one truncating split: the exact fidelity is that f
        sv = SV.simulate(c)
        F = abs(np.vdot(sv, amp)) ** 2 / np.vdot(amp, amp).real
        assert abs(F - cut[0].f) < 1e-10


@SETTINGS
@given(circuits(n_max=7))
def test_untruncated_gate_by_gate_tebd_is_exact(c):
    psi = TB.run(c, chi_max=1 << 20, eps=0.0)
    assert np.abs(TB.amplitudes(psi) - SV.simulate(c)).max() < 1e-12


@settings(max_examples=300, deadline=None, derandomize=True)
@given(st.integers(2, 24), st.data())
def test_dmrg_grouping_partitions_within_the_caps(n, data):
    chit = [data.draw(st.sampled_from([1, 2, 4, 8, 16, 32, 64])) for _ in range(n - 1)]
    q_max = data.draw(st.integers(1, 24))
    groups = DM.group_sites(chit, n, q_max)
    assert groups[0][0] == 0 and groups[-1][1] == n - 1
    assert all(groups[i][1] + 1 == groups[i + 1][0] for i in range(len(groups) - 1))
    for a, b in groups:
        assert a <= b
        chi_l = chit[a - 1] if a > 0 else 1
        chi_r = chit[b] if b < n - 1 else 1
        N = b - a + 1
        assert N == 1 or N + math.log2(chi_l) + math.log2(chi_r) <= q_max
    # a chain that fits whole is one group
    if n <= q_max:
        assert groups == [(0, n - 1)]


@SETTINGS
@given(circuits(), st.data())
def test_one_cluster_fidelity_is_the_product_of_its_f(c, data):
    prep = CT.run(c, chi_max=1 << 20, eps=1e-12, k_max=4)
    psi = prep.psi.copy()
    k = data.draw(st.integers(2, min(5, c.n)))
    a = data.draw(st.integers(0, c.n - k))
    chi_max = data.draw(st.integers(1, 4))
    U = haar_unitary(2 ** k, seed=data.draw(st.integers(0, 10 ** 6)))
    lf0 = psi.log_f
    CT.apply_cluster(psi, a, k, U, chi_max, 1e-12)
    exact = SV.apply_gate(SV.simulate(c), c.n, U, list(range(a, a + k)))
    amp = MT.amplitudes(psi.B)
    F = abs(np.vdot(exact, amp)) ** 2 / np.vdot(amp, amp).real
    assert abs(F - math.exp(psi.log_f - lf0)) < 1e-10


def test_estimate_between_clusters_is_an_approximation():
    a, b = math.cos(0.4), math.sin(0.4)
    n = 4
    B = [np.zeros((1, 2, 2), complex), np.zeros((2, 2, 2), complex), np.zeros((2, 2, 2), complex),
         np.zeros((2, 2, 1), complex)]
    B[0][0, 0, 0], B[0][0, 1, 1] = a, b
    for s in (0, 1):
        B[1][s, s, s] = B[2][s, s, s] = 1.0
        B[3][s, s, 0] = 1.0
    lam = [np.array([a, b]) for _ in range(n - 1)]
    psi = CT.MPS(B, lam)
    exact = MT.amplitudes(psi.B)
    assert abs(exact[0] - a) < 1e-15 and abs(exact[-1] - b) < 1e-15
    for start in (0, 2):  # two clusters of one step, order-free
        CT.apply_cluster(psi, start, 2, np.eye(4), 1, 0.0)
    assert [round(r.f, 15) for r in psi.records] == [round(a * a, 15)] * 2
    amp = MT.amplitudes(psi.B)
    F = abs(np.vdot(exact, amp)) ** 2 / np.vdot(amp, amp).real
    assert abs(F - a ** 2) < 1e-14
    assert abs(math.exp(psi.log_f) - a ** 4) < 1e-14
