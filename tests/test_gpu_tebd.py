"""Standard gate-by-gate TEBD (Sec. II.C) on the library's kernels, and both
algorithms on the paper's own random-structured circuits (Sec. IV.A).

Gate-by-gate TEBD is the cluster-TEBD machinery with clusters of at most two
qubits and one sub-layer per step (k_max = 2, l_max = 1): every two-qubit
gate, and every SWAP that brings a distant pair together, is applied on its
own and followed by one truncated SVD.  Checked against the Lambda-weighted
oracle with the same caps (the same arithmetic), against the statevector
where nothing is truncated, and against the orthogonality-centre TEBD oracle
(the paper's form) at the bar its pins fix."""
import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import mps_tools as MT
from oracle import statevector as SV
from oracle import tebd as TB
from workloads import make_workload, paper_random_structured

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")

INF_TOL = {"fp64": 1e-11, "fp32": 1e-6}


def _tebd_gpu(c, chi, eps, prec, batch="wave"):
    m = P.MPS(c.n, chi, eps, k_max=2, l_max=1, precision=prec, batch=batch)
    P.run_circuit(m, c.layers)
    return m


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("version,d_max", [(1, 1), (2, 1), (2, 3)])
def test_tebd_exact_vs_statevector(prec, version, d_max):
    c = paper_random_structured(10, 16, version, d_max=d_max, seed=version + d_max, workload_id=95)
    m = _tebd_gpu(c, 1024, 0.0, prec)
    sv = SV.simulate(c)
    assert np.abs(m.amplitudes() - sv).max() < (1e-11 if prec == "fp64" else 5e-6)
    assert abs(m.fidelity()[0] - 1.0) < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tebd_truncating_vs_oracles(prec):
    c = paper_random_structured(12, 30, 2, d_max=2, seed=9, workload_id=93)
    chi, eps = 12, 1e-12
    m = _tebd_gpu(c, chi, eps, prec)
    ref = CT.run(c, chi_max=chi, eps=eps, k_max=2, l_max=1)
    if prec == "fp64":
        assert m.bond_dims() == ref.psi.bond_dims()
    assert abs(m.fidelity()[1] - ref.psi.log_f) < (1e-10 if prec == "fp64" else 1e-6)
    assert MT.infidelity(m.sites(), ref.psi.B) < INF_TOL[prec]
    assert m.stats()["svds"] == len(ref.psi.records)
    # the orthogonality-centre form: the same up to a fraction of the discarded weight
    qr = TB.run(c, chi_max=chi, eps=eps)
    discarded = 1 - float(np.exp(qr.log_f))
    assert discarded > 0.02
    assert MT.infidelity(m.sites(), qr.A) < 0.25 * discarded


@pytest.mark.parametrize("name", ["paper_clifford_n40_l40", "paper_nonclifford_n40_l40"])
def test_cluster_tebd_on_paper_circuits_vs_oracle(name):
    """Cluster-TEBD on the paper's circuits, shrunk to 10 layers so that the
    oracle finishes in seconds, FP32 against the FP64 oracle."""
    c, p = make_workload(name, seed=0, layers=10)
    m = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision="fp32", batch="wave")
    P.run_circuit(m, c.layers)
    ref = CT.run(c, **p)
    assert MT.infidelity(m.sites(), ref.psi.B) < 1e-6
    assert abs(m.fidelity()[1] - ref.psi.log_f) < 1e-6
