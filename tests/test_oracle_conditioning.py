"""Conditioning of the oracle (the truncation of Sec. II.B inside the cluster
steps of Sec. III.A): the same run with every gate multiplied by its own
random unitary exp(i 1e-9 H) (seeded, |H| = 1).  The exact states differ by
about the number of gates times 1e-9.  Without a cut through a degenerate
multiplet the truncated results differ by as little, also where the caps
truncate real weight: end-to-end parity is well posed there.  A flagged
degenerate cut keeps an arbitrary basis of the multiplet, so the states may
differ at order one, while the tie-invariant fidelity estimate does not:
there parity is asserted only on tie-invariant quantities."""
import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import gates as G
from oracle import mps_tools as MT
from workloads import make_workload


def _perturbed_lookup(seed, scale=1e-9):
    rng = np.random.default_rng(seed)
    plain = G.matrix

    def matrix(name):
        u = plain(name)
        d = u.shape[0]
        h = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        h = (h + h.conj().T) / 2
        h /= np.linalg.norm(h, 2)
        w, v = np.linalg.eigh(h)
        return u @ (v * np.exp(1j * scale * w)) @ v.conj().T

    return matrix


# (workload structure, n, layers, chi_max): the workloads' own caps, and
# chi_max = 4 so that the caps truncate real weight
CASES = [("batched_n1000_l100", 60, 12, None), ("learned_n500_l60", 40, 10, None),
         ("batched_n1000_l100", 24, 16, 4), ("learned_n500_l60", 24, 16, 4), ("chi1024_n200_l50", 24, 16, 4)]


@pytest.mark.parametrize("name,n,layers,chi", CASES)
def test_oracle_under_gate_perturbation(monkeypatch, name, n, layers, chi):
    c, p = make_workload(name, seed=0, n=n, layers=layers)
    chi_max, k_max = chi or p["chi_max"], min(p["k_max"], 6)
    ref = CT.run(c, chi_max, p["eps"], k_max)
    monkeypatch.setattr(G, "matrix", _perturbed_lookup(seed=n * 1000 + layers))
    per = CT.run(c, chi_max, p["eps"], k_max)
    deg = sum(1 for r in ref.psi.records if r.degenerate_cut)
    inf = MT.infidelity(ref.psi.B, per.psi.B)
    print(f"{name} n={n} layers={layers} chi_max={chi_max}: log F {ref.psi.log_f:.3e}, degenerate cuts {deg}, "
          f"oracle vs perturbed oracle infidelity {inf:.2e}")
    assert abs(ref.psi.log_f - per.psi.log_f) < 1e-8
    if deg == 0:
        assert inf < 1e-9
