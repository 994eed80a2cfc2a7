"""Checkpoint / resume and option changes through the C ABI (mps_save,
mps_load, mps_set_options): a run that is saved after some steps, loaded into
a fresh handle and continued must equal the uninterrupted run bit for bit
(sites, Schmidt values, bond dimensions, sum log f, counters)."""
import numpy as np
import pytest

from workloads import make_workload

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")


def _start(c, p, prec):
    m = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision=prec, batch="step")
    for layer in c.layers:
        m.queue_layer([(g.qubits, P.GATES[g.name]) for g in layer])
    return m


def _finish(m):
    while True:
        _, rem = m.step()
        if rem == 0:
            return m


def _assert_identical(a, b, n):
    assert a.bond_dims() == b.bond_dims()
    for j in range(n):
        assert np.array_equal(a.site(j), b.site(j)), j
    for bnd in range(n - 1):
        assert np.array_equal(a.schmidt(bnd), b.schmidt(bnd)), bnd
    assert a.fidelity() == b.fidelity()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_save_load_resumes_bit_for_bit(tmp_path, prec):
    # non-Clifford (T density 0.1), truncating at chi_max = 16
    c, p = make_workload("batched_n1000_l100", seed=2, n=60, layers=14)
    p = dict(p, chi_max=16)
    ref = _finish(_start(c, p, prec))
    a = _start(c, p, prec)
    for _ in range(6):
        a.step()
    path = str(tmp_path / "state.ctebd")
    a.save(path)
    b = P.MPS.load(path)
    assert b.n == c.n and b.options()["precision"] == prec
    assert b.stats() == a.stats()
    _assert_identical(a, b, c.n)
    del a
    _finish(b)
    _assert_identical(ref, b, c.n)
    assert b.stats() == ref.stats()
    assert ref.fidelity()[0] < 1.0  # the run truncated


def test_set_options_precision_matches_clone():
    c, p = make_workload("batched_n1000_l100", seed=5, n=40, layers=10)
    p = dict(p, chi_max=32)
    a = _start(c, p, "fp32")
    for _ in range(4):
        a.step()
    b = a.clone(precision="fp64")
    a.set_options(precision="fp64")
    assert a.options()["precision"] == "fp64"
    _finish(a)
    _finish(b)
    _assert_identical(a, b, c.n)


def test_set_options_k_max_flushes_buffered_layers_first():
    c, p = make_workload("clifford_n100_l20", seed=1, n=30, layers=6)
    a = _start(c, p, "fp64")
    a.set_options(k_max=3)
    # every buffered layer was contracted with the old k_max
    _, rem = a.step()
    assert rem == 0
    ref = _finish(_start(c, p, "fp64"))
    _assert_identical(a, ref, c.n)
    assert a.options()["k_max"] == 3


def test_set_options_rejects_invalid_and_keeps_state():
    m = P.MPS(8, 8, 1e-12, k_max=3, precision="fp64")
    m.apply_cluster([2, 3], P.GATES["CNOT"] @ np.kron(P.GATES["H"], np.eye(2)))
    before = m.amplitudes()
    with pytest.raises(P.CtebdError) as e:
        m.set_options(k_max=99)
    assert e.value.status == -1
    assert np.array_equal(m.amplitudes(), before)
    assert m.options()["k_max"] == 3
