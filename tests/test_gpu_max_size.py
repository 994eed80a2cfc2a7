"""The largest sizes the library accepts.

The largest cluster, k = 12 (Sec. III.A): a 4096 x 4096 unitary on a
12-qubit chain through mps_apply_cluster (its unitarity checked on the
matrix cores) and a 12-qubit cluster planned from circuit layers with
k_max = 12 (its unitary built from the gates in 64 KiB of LDS per column),
both against the statevector; non-unitary matrices rejected on either side of
the size at which the check moves to the GPU.

The largest bond cap, chi_max = 2048 (mps_create's limit), so that a split's
Gram matrix is 2c = 4096 wide (the automatic eigen-solver choice is block
Jacobi above 2048) and the selection sorts 4096 eigenvalues.

Input: 24 qubits in the exact Schmidt form of eleven entangled pairs
(q, q + 13) with distinct weights (workloads/pairs.py), so bonds 10, 11 and
12 hold 2048 Schmidt values each.  One k = 3 cluster on qubits 10, 11, 12 (a
Haar unitary) is applied by the GPU and by the oracle (LAPACK SVDs, Secs.
II.B and III.A).  Its first split is a full-rank 4096 x 4096 problem whose cap
binds (2048 of 4096 values kept, a clean gap at the cut); its second is
4096 wide with exact rank 1854, the rest being zeros that each side resolves
to its own floor.  Compared: the fidelity sum, the Schmidt values (all of
bond 11, the resolved ones of bond 10), the bond dimensions and the state."""
import functools

import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import mps_tools as MT
from oracle import statevector as SV
from workloads import paper_random_structured
from workloads.mps_inputs import haar_unitary
from workloads.pairs import pair_angles, paired_state

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")

N, CHI, EPS = 24, 2048, 1e-10
PAIRS = [(q, q + 13) for q in range(11)]
A, K = 10, 3
INF_TOL = {"fp64": 1e-11, "fp32": 1e-6, "bf16x6": 1e-6}
# the GPU keeps normalised values above max(eta, 4 u) (u = 2^-26.5 for FP64,
# 2^-24 with FP32 contractions); values below the Gram route's resolution at
# 2c = 4096, sqrt(64 u sqrt(4096)), may be kept by one side only
RESOLVED = {"fp64": (64 * 2.0 ** -53 * 4096 ** 0.5) ** 0.5, "fp32": 1.01 * 4 * 2.0 ** -24,
            "bf16x6": 1.01 * 4 * 2.0 ** -24}


@pytest.fixture(scope="module")
def case():
    B, lam = paired_state(N, PAIRS, pair_angles(len(PAIRS), seed=0))
    U = haar_unitary(2 ** K, seed=21)
    ref = CT.MPS([b.copy() for b in B], [l.copy() for l in lam])
    CT.apply_cluster(ref, A, K, U, CHI, EPS)
    return B, lam, U, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_chi2048_cluster_vs_oracle(case, prec):
    B, lam, U, ref = case
    assert [l.size for l in lam][A - 1:A + K] == [1024, 2048, 2048, 2048]
    r1, r2 = ref.records
    assert (r1.full, r1.rank, r1.degenerate_cut) == (4096, CHI, False)  # the cap binds, no tie at the cut
    assert r1.f < 0.99
    assert r2.rank == 1854 and r2.f > 1 - 1e-12
    m = P.MPS(N, CHI, EPS, k_max=4, precision=prec)
    m.import_state(B, lam)
    m.apply_cluster(list(range(A, A + K)), U)
    F, lf = m.fidelity()
    print(f"chi_max 2048 {prec}: log f {lf:.12f} (oracle {ref.log_f:.12f}), bond 10 {m.bond_dims()[A]}")
    assert abs(lf - ref.log_f) < (1e-10 if prec == "fp64" else 1e-6)
    dims = m.bond_dims()
    ref_dims = ref.bond_dims()
    assert dims[:A] == ref_dims[:A] and dims[A + 1:] == ref_dims[A + 1:]
    assert dims[A + 1] == CHI
    vtol = 1e-9 if prec == "fp64" else 1e-5
    got, exp = m.schmidt(A + 1), ref.lam[A + 1]
    assert np.abs(got - exp).max() < vtol
    # bond 10: the exact rank, plus at most values below the resolution
    got, exp = m.schmidt(A), ref.lam[A]
    assert got.size >= exp.size
    assert np.abs(got[:exp.size] - exp).max() < vtol
    assert got.size == exp.size or got[exp.size:].max() < RESOLVED[prec]
    inf = MT.infidelity(m.sites(), ref.B)
    print(f"  infidelity vs oracle {inf:.3e}")
    assert inf < INF_TOL[prec]


# ---- the largest cluster, k = 12
AMP_TOL = {"fp64": 1e-11, "fp32": 5e-6, "bf16x6": 5e-6}


@functools.lru_cache(maxsize=None)
def _haar(dim, seed):
    return haar_unitary(dim, seed=seed)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_k12_cluster_unitary_vs_statevector(prec):
    n = 12
    U = _haar(2 ** n, 31)
    m = P.MPS(n, 64, 0.0, k_max=12, precision=prec)
    m.apply_cluster(list(range(n)), U)
    sv = U[:, 0]  # U |0...0>
    assert np.abs(m.amplitudes() - sv).max() < AMP_TOL[prec]
    assert m.bond_dims() == [2 ** min(b + 1, n - b - 1) for b in range(n - 1)]
    assert abs(m.fidelity()[1]) < 1e-12


@pytest.mark.parametrize("k", [8, 9, 12])
def test_non_unitary_cluster_rejected(k):
    """2^k = 256 is checked on the host, 512 and 4096 on the GPU.  A Haar
    unitary scaled by 1 + 1e-9 (||U^H U - 1||_max = 2e-9) and one with an
    entry changed by 1e-7 are rejected and leave the state as it was; scaled
    by 1 + 1e-12 it passes."""
    n = 12
    m = P.MPS(n, 64, 0.0, k_max=12, precision="fp64")
    m.apply_cluster([0, 1], _haar(4, 5))
    before = m.amplitudes()
    U = _haar(2 ** k, 40 + k)
    bumped = U.copy()
    bumped[3, 2 ** k - 2] += 1e-7
    for bad in (U * (1 + 1e-9), bumped):
        with pytest.raises(P.CtebdError) as e:
            m.apply_cluster(list(range(k)), bad)
        assert e.value.status == -4  # MPS_ENOTUNITARY
        assert np.array_equal(m.amplitudes(), before)
    m.apply_cluster(list(range(k)), U * (1 + 1e-12))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_k12_cluster_from_layers_vs_statevector(prec):
    """Eight nearest-neighbour layers of the paper's generator on 12 qubits
    with k_max = 12 and no other cap: the planner makes the whole chain one
    cluster, whose 4096 x 4096 unitary is built on the GPU from the gates."""
    c = paper_random_structured(12, 8, 2, d_max=1, seed=5, workload_id=95)
    layers = [[(g.qubits, P.GATES[g.name]) for g in layer] for layer in c.layers]
    assert P.plan(c.n, 12, layers, [1] * (c.n - 1)) == (8, [(0, 12)], 8)
    m = P.MPS(c.n, 64, 0.0, k_max=12, precision=prec)
    P.run_circuit(m, c.layers)
    assert m.stats()["cluster_updates"] == 1
    assert np.abs(m.amplitudes() - SV.simulate(c)).max() < AMP_TOL[prec]
