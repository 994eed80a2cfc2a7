"""Pins of the adaptive-grouping DMRG oracle (Sec. III.B): the virtual MPS of
Eq. chi_est, the recursive bipartition of Eqs. cond_group1 / cond_group2,
exactness without a cap, monotone update fidelities, and the fidelity of the
fitted state against its definition."""
import math

import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import dmrg as DM
from oracle import mps_tools as MT
from oracle import statevector as SV
from workloads import Gate, paper_random_structured


def test_virtual_bond_dimensions_worked_example():
    # 6 qubits: gates (0,1), (1,2) twice, (2,5) crossing bonds 2,3,4, (3,4)
    layers = [[Gate("CNOT", (0, 1)), Gate("CZ", (2, 5))], [Gate("CNOT", (1, 2)), Gate("CY", (3, 4))],
              [Gate("SWAP", (1, 2))]]
    E = DM.entangling_counts(layers, 6)
    assert E == [1, 2, 1, 2, 1]
    chi = [1, 2, 4, 2, 1]
    # min(2^E chi, chi_max, 2^min(b+1, n-b-1)) with chi_max = 8
    assert DM.virtual_bond_dims(E, chi, 8, 6) == [2, 4, 8, 4, 2]
    assert DM.virtual_bond_dims(E, chi, 3, 6) == [2, 3, 3, 3, 2]


def test_bipartition_respects_the_caps_and_cuts_at_minima():
    chit = [2, 8, 16, 4, 32, 32, 2, 8, 4]
    n = 10
    for q_max in (4, 6, 8, 12):
        groups = DM.group_sites(chit, n, q_max)
        # a partition of the chain into consecutive groups
        assert groups[0][0] == 0 and groups[-1][1] == n - 1
        assert all(groups[i][1] + 1 == groups[i + 1][0] for i in range(len(groups) - 1))
        for a, b in groups:
            chi_l = chit[a - 1] if a > 0 else 1
            chi_r = chit[b] if b < n - 1 else 1
            N = b - a + 1
            assert N == 1 or N + math.log2(chi_l) + math.log2(chi_r) <= q_max
    # the first cut of the whole chain is at the smallest virtual bond (2, at
    # bond 0 or 6: the more balanced one, bond 6)
    assert DM.group_sites(chit, n, 9)[0] == (0, 6)
    # a chain that fits is one group
    assert DM.group_sites(chit, n, 40) == [(0, n - 1)]


@pytest.mark.parametrize("l_max,q_max,seed", [(3, 6, 0), (5, 8, 1), (12, 30, 2)])
def test_uncapped_dmrg_is_exact(l_max, q_max, seed):
    c = paper_random_structured(10, 12, 2, d_max=3, seed=seed, workload_id=98)
    psi, recs = DM.run(c, l_max=l_max, chi_max_dmrg=1 << 20, chi_max_svd=1 << 20, eps=0.0, q_max=q_max, sweeps=1)
    sv = SV.simulate(c)
    assert np.abs(MT.amplitudes(psi.B) - sv).max() < 1e-12
    assert abs(psi.log_f) < 1e-12
    for r in recs:
        assert abs(r.f_dmrg - 1) < 1e-12
    # the output is in the cluster-TEBD form: right-canonical sites, Lambda =
    # the state's Schmidt values
    for j in range(1, c.n):
        assert MT.right_canonical_error(psi.B[j]) < 1e-12
    for b in range(c.n - 1):
        ref = MT.schmidt_from_state(sv, c.n, b + 1)
        lam = psi.lam[b]
        assert np.abs(lam - ref[:lam.size]).max() < 1e-12


def test_capped_dmrg_fidelities():
    c = paper_random_structured(10, 18, 2, d_max=3, seed=3, workload_id=97)
    psi0 = CT.product_state(10)
    out, rec = DM.dmrg_step(psi0, c.layers, chi_max_dmrg=4, chi_max_svd=1024, eps=0.0, q_max=6, sweeps=2)
    # every update maximises the overlap given the rest, so f never decreases
    assert np.all(np.diff(rec.f_updates) >= -1e-13)
    assert rec.f_updates[-1] > rec.f_updates[0] + 1e-4  # the sweeps improve on the compression
    # f of the last update is |<M|U psi>|^2 by definition: the output state
    # (no truncation in the decomposition) against the exact statevector
    sv = SV.simulate(c)
    amp = MT.amplitudes(out.B)
    F = abs(np.vdot(sv, amp)) ** 2 / (np.vdot(amp, amp).real * np.vdot(sv, sv).real)
    assert abs(F - rec.f_dmrg) < 1e-12
    assert abs(math.exp(out.log_f) - rec.f_dmrg) < 1e-12
    # every group cut holds at most its virtual dimension
    dims = out.bond_dims()
    for (a, b) in rec.groups[:-1]:
        assert dims[b] <= rec.chi_virtual[b]


def test_compression_alone_reports_its_fidelity():
    """With no sweep the fit is the compression at the group cuts; its f is
    the weight the compressed state keeps, |<M|U psi>|^2 by definition."""
    c = paper_random_structured(10, 18, 2, d_max=3, seed=4, workload_id=97)
    out, rec = DM.dmrg_step(CT.product_state(10), c.layers, chi_max_dmrg=2, chi_max_svd=1024, eps=0.0,
                            q_max=5, sweeps=0)
    sv = SV.simulate(c)
    amp = MT.amplitudes(out.B)
    F = abs(np.vdot(sv, amp)) ** 2 / (np.vdot(amp, amp).real * np.vdot(sv, sv).real)
    assert rec.f_dmrg < 0.9
    assert abs(F - rec.f_dmrg) < 1e-12
