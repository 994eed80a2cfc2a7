"""Kernel timing through the C ABI: burst timing re-launches the column update
and the HEMV of the tridiagonal reduction on their own inputs, which must
leave every result bit-identical to an untimed run."""
import numpy as np
import pytest

from workloads import Circuit, Gate

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")


def _run(c, p, timing):
    m = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision="fp32", batch="step", eig="tridiag")
    if timing:
        m.set_timing(True)
        m.set_burst_timing("trd_hemv", 1, 2)
        m.set_burst_timing("trd_col", 2, 3)
    P.run_circuit(m, c.layers)
    return m


def _entangling_circuit(n, layers, seed):
    """Layers of two-qubit gates at distance 1..3 on random pairs (bonds grow fast)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(layers):
        used, L = set(), []
        for a in rng.permutation(n):
            a = int(a)
            b = a + int(rng.integers(1, 4))
            if a in used or b >= n or b in used:
                continue
            used |= {a, b}
            L.append(Gate(str(rng.choice(["CNOT", "CZ", "SQRTSWAP", "CT"])), (a, b)))
        L += [Gate("H", (q,)) for q in range(n) if q not in used]
        out.append(L)
    return Circuit(n, out)


def test_burst_timing_leaves_results_unchanged():
    c = _entangling_circuit(16, 20, seed=3)
    p = dict(k_max=4, chi_max=96, eps=1e-12)
    m0 = _run(c, p, False)
    m1 = _run(c, p, True)
    assert m0.bond_dims() == m1.bond_dims()
    assert max(m0.bond_dims()) == 96  # capped: Gram matrices of up to 192, six 32-column panels
    for j in range(c.n):
        assert np.array_equal(m0.site(j), m1.site(j))
    assert m0.fidelity() == m1.fidelity()
    kt, disp = m1.kernel_times(), m1.kernel_dispatches()
    # every HEMV launch is a burst of 3; every other column update a burst of 4
    assert kt["trd_hemv"][1] > 0 and disp["trd_hemv"] == 3 * kt["trd_hemv"][1]
    n_col = kt["trd_col"][1]
    assert n_col > 0 and 4 * n_col + (n_col - 1) <= disp["trd_col"] <= 4 * n_col + n_col
    assert kt["trd_hemv"][3] > 0 and kt["trd_hemv"][0] > 0


def test_burst_timing_rejects_other_classes():
    m = P.MPS(8, 8, 1e-12, k_max=3, precision="fp32")
    with pytest.raises(P.CtebdError):
        m.set_burst_timing("gram", 1, 1)
    with pytest.raises(P.CtebdError):
        m.set_burst_timing("trd_hemv", 0, 1)
    with pytest.raises(P.CtebdError):
        m.set_burst_timing("trd_hemv", 1, 65)
    m.set_burst_timing(None)
