"""The adaptive-grouping DMRG step (Sec. III.B) through the C ABI against the
FP64 DMRG oracle and the statevector.

Both sides take the same grouping (Eq. chi_est, Eqs. cond_group1/2), start
from the evolved state compressed at the group cuts and run the same sweeps;
they orthonormalise in different gauges (polar factors on the GPU, QR in the
oracle), which leaves the physical state unchanged.  The cutoff is set above
the GPU's FP64 floor (4 * 2^-26.5) so that both keep the same values."""
import math

import numpy as np
import pytest

from oracle import dmrg as DM
from oracle import mps_tools as MT
from oracle import statevector as SV
from workloads import Circuit, Gate, paper_random_structured

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")


def _gpu_dmrg(c, l_max, chi_dmrg, chi_svd, eps, q_max, sweeps):
    m = P.MPS(c.n, chi_svd, eps, k_max=4, precision="fp64")
    fs = []
    for t0 in range(0, len(c.layers), l_max):
        seg = [[(g.qubits, P.GATES[g.name]) for g in layer] for layer in c.layers[t0:t0 + l_max]]
        fs.append(m.dmrg_step(seg, chi_dmrg, q_max, sweeps))
    return m, fs


@pytest.mark.parametrize("l_max,q_max,seed", [(3, 6, 0), (5, 8, 1), (12, 30, 2)])
def test_uncapped_dmrg_exact(l_max, q_max, seed):
    c = paper_random_structured(10, 12, 2, d_max=3, seed=seed, workload_id=98)
    m, fs = _gpu_dmrg(c, l_max, 1 << 20, 1024, 1e-7, q_max, 1)
    sv = SV.simulate(c)
    amp = m.amplitudes()
    assert np.abs(amp - sv).max() < 1e-10
    assert all(abs(f - 1) < 1e-10 for f in fs)
    assert abs(m.fidelity()[1]) < 1e-10


@pytest.mark.parametrize("chi_dmrg,q_max,sweeps,seed", [(4, 6, 2, 3), (2, 5, 1, 4), (8, 7, 3, 5), (2, 5, 0, 4)])
def test_capped_dmrg_vs_oracle(chi_dmrg, q_max, sweeps, seed):
    c = paper_random_structured(10, 18, 2, d_max=3, seed=seed, workload_id=97)
    l_max = 6
    m, fs = _gpu_dmrg(c, l_max, chi_dmrg, 1024, 1e-7, q_max, sweeps)
    ref, recs = DM.run(c, l_max=l_max, chi_max_dmrg=chi_dmrg, chi_max_svd=1024, eps=1e-7, q_max=q_max,
                       sweeps=sweeps)
    for f, r in zip(fs, recs):
        assert abs(f - r.f_dmrg) < 1e-10, (f, r.f_dmrg)
    assert min(fs) < 0.999  # the caps bind
    assert abs(m.fidelity()[1] - ref.log_f) < 1e-9
    assert m.bond_dims() == ref.bond_dims()
    assert MT.infidelity(m.sites(), ref.B) < 1e-10
    # against the exact state: the estimate and the true fidelity
    sv = SV.simulate(c)
    amp = m.amplitudes()
    F = abs(np.vdot(sv, amp)) ** 2 / np.vdot(amp, amp).real
    print(f"DMRG chi~ <= {chi_dmrg}, Q_max {q_max}, {sweeps} sweeps: F = {F:.6f}, estimate {math.exp(ref.log_f):.6f}")


def test_dmrg_rejects_mixed_precision_handles():
    m = P.MPS(6, 8, 1e-10, precision="fp32")
    with pytest.raises(P.CtebdError) as e:
        m.dmrg_step([[((0, 1), P.GATES["CNOT"])]], 4, 6, 1)
    assert e.value.status == -6


def _run_both(c, l_max, chi_dmrg, q_max, sweeps):
    m, fs = _gpu_dmrg(c, l_max, chi_dmrg, 1024, 1e-7, q_max, sweeps)
    ref, recs = DM.run(c, l_max=l_max, chi_max_dmrg=chi_dmrg, chi_max_svd=1024, eps=1e-7, q_max=q_max,
                       sweeps=sweeps)
    return m, fs, ref, recs


def test_dmrg_two_qubits():
    """n = 2: one bond, the grouping is one group (or two single sites)."""
    c = Circuit(2, [[Gate("H", (0,)), Gate("X4", (1,))], [Gate("CNOT", (0, 1))], [Gate("T", (0,))],
                    [Gate("SQRTSWAP", (0, 1))]])
    for q_max in (1, 2, 4):
        m, fs, ref, recs = _run_both(c, 2, 4, q_max, 2)
        assert np.abs(m.amplitudes() - SV.simulate(c)).max() < 1e-12
        assert all(abs(f - 1) < 1e-12 for f in fs)
        groups = [(0, 0), (1, 1)] if q_max == 1 else [(0, 1)]
        assert all(r.groups == groups for r in recs)


def test_dmrg_segment_without_entangling_gates():
    """E(b) = 0 on every bond: chi~ = chi, the fit is exact whatever the
    grouping, and the entangled input state is carried through unchanged
    up to the one-qubit gates."""
    base = paper_random_structured(8, 4, 2, d_max=2, seed=7, workload_id=96)
    ones = [[Gate(g, (q,)) for q, g in zip(range(8), ["H", "T", "X", "Y", "Z", "P3PI4", "X4", "SQRTW"])]] * 3
    c = Circuit(8, base.layers + ones)
    m, fs = _gpu_dmrg(c, 4, 1 << 20, 1024, 1e-7, 6, 1)
    assert np.abs(m.amplitudes() - SV.simulate(c)).max() < 1e-10
    assert abs(fs[-1] - 1) < 1e-10


@pytest.mark.parametrize("chi_dmrg,q_max", [(1, 6), (2, 3)])
def test_dmrg_degenerate_caps_vs_oracle(chi_dmrg, q_max):
    """chi~ = 1 (the fit is a product state across the group cuts) and
    Q_max = 3 (groups of one to three qubits): each step's fit fidelity and
    the final state against the oracle; the caps bind in one step each."""
    c = paper_random_structured(8, 9, 2, d_max=1, seed=0, workload_id=96)
    m, fs, ref, recs = _run_both(c, 3, chi_dmrg, q_max, 2)
    for f, r in zip(fs, recs):
        assert abs(f - r.f_dmrg) < 1e-10, (f, r.f_dmrg)
    assert min(fs) < 0.99
    assert abs(m.fidelity()[1] - ref.log_f) < 1e-9
    assert m.bond_dims() == ref.bond_dims()
    assert MT.infidelity(m.sites(), ref.B) < 1e-10
