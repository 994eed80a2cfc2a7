"""The wavefront executor (MPS_BATCH_WAVE: the clusters of several steps as a
dependency graph, one split level per round) against the step executor
(MPS_BATCH_STEP): every cluster runs the same kernels on the same inputs, so
site tensors, Schmidt values and bond dimensions agree bit for bit; only the
sum of log f is added up in another order."""
import numpy as np
import pytest

from workloads import make_workload

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")


def _queued(c, p, prec, batch, eig="auto"):
    m = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision=prec, batch=batch, eig=eig)
    for layer in c.layers:
        m.queue_layer([(g.qubits, P.GATES[g.name]) for g in layer])
    return m


def _same(a, b, n, stats=True):
    assert a.bond_dims() == b.bond_dims()
    for j in range(n):
        assert np.array_equal(a.site(j), b.site(j)), j
    for bnd in range(n - 1):
        assert np.array_equal(a.schmidt(bnd), b.schmidt(bnd)), bnd
    la, lb = a.fidelity()[1], b.fidelity()[1]
    assert abs(la - lb) <= 1e-13 * max(1.0, abs(la))
    if stats:
        sa, sb = a.stats(), b.stats()
        for key in ("steps", "cluster_updates", "svds", "site_updates"):
            assert sa[key] == sb[key], key


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name,n,layers,chi", [("batched_n1000_l100", 200, 14, 32), ("learned_n500_l60", 120, 16, 64),
                                              ("clifford_n100_l20", 100, 20, 256)])
def test_wave_equals_step_executor(name, n, layers, chi, prec):
    c, p = make_workload(name, seed=3, n=n, layers=layers)
    p = dict(p, chi_max=chi)
    a = _queued(c, p, prec, "step")
    while a.step()[1]:
        pass
    b = _queued(c, p, prec, "wave")
    clusters, rem = b.run_steps(10 ** 6)
    assert rem == 0 and clusters == a.stats()["cluster_updates"]
    _same(a, b, c.n)


def test_wave_with_forced_jacobi_and_run_layer():
    c, p = make_workload("batched_n1000_l100", seed=4, n=80, layers=12)
    p = dict(p, chi_max=24)
    a = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision="fp32", batch="step", eig="jacobi")
    P.run_circuit(a, c.layers)
    b = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision="fp32", batch="wave", eig="jacobi")
    P.run_circuit(b, c.layers)  # mps_run_layer hands the complete steps to the executor, then mps_flush
    _same(a, b, c.n)


def test_wave_window_at_chi1024():
    """Twenty steps of the chi_max = 1024 workload from a state whose bonds
    reach the cap: several 2048 x 2048 tridiagonal solves per round."""
    c, p = make_workload("chi1024_n200_l50", seed=0)
    a = _queued(c, p, "fp32", "step")
    while True:
        d = np.array(a.bond_dims())
        if (d >= p["chi_max"]).mean() >= 0.2:
            break
        a.step()
    b = a.clone(batch="wave")
    before = a.stats()["cluster_updates"]
    for _ in range(20):
        a.step()
    clusters, _ = b.run_steps(20)
    assert clusters == a.stats()["cluster_updates"] - before
    assert b.stats()["steps"] == 20
    assert max(b.bond_dims()) == p["chi_max"]
    _same(a, b, c.n, stats=False)
