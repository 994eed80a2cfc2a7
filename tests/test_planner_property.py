"""The library's host planner (mps_plan, C++) against the oracle's planner
(Sec. III.A: bond array, clusters as runs of marked bonds, Eqs. size,
cond_cTEBD and cond2_cTEBD, SWAP routing) on many random small circuits,
caps and bond dimensions: the legalised sub-layer count, every step's end
and its clusters must be identical.  Also the planner's rejection of gates
that mps_run_layer rejects.  Host code only: no GPU needed."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import planner as PL
from workloads import Gate


def _ffi():
    from paper_2502_19289_amd import ffi
    return ffi


@st.composite
def planner_cases(draw):
    n = draw(st.integers(2, 14))
    k_max = draw(st.integers(2, 8))
    q_max = draw(st.sampled_from([0, 0, k_max, k_max + 2, k_max + 6, 12]))
    l_max = draw(st.sampled_from([0, 0, 1, 2, 3]))
    nl = draw(st.integers(1, 6))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    layers = []
    for _ in range(nl):
        free = list(rng.permutation(n))
        layer = []
        while free:
            q = int(free.pop())
            if free and rng.random() < 0.5:
                # a partner at any distance (long-range gates are routed)
                r = int(free.pop(int(rng.integers(len(free)))))
                layer.append(Gate("CNOT", (q, r)))
            elif rng.random() < 0.7:
                layer.append(Gate("H", (q,)))
        layers.append(layer)
    chi = [int(min(2 ** rng.integers(0, 6), 2 ** min(b + 1, n - b - 1))) for b in range(n - 1)]
    return n, k_max, q_max, l_max, layers, chi


def _abi_layers(layers):
    from paper_2502_19289_amd.gates import GATES
    return [[(g.qubits, GATES[g.name]) for g in l] for l in layers]


@settings(max_examples=300, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(planner_cases())
def test_planner_matches_oracle_on_random_cases(case):
    ffi = _ffi()
    n, k_max, q_max, l_max, layers, chi = case
    subs = PL.legalize(layers, k_max)
    qm = q_max if q_max > 0 else 62
    lm = l_max if l_max > 0 else 1 << 30
    abi = _abi_layers(layers)
    start = 0
    if not subs:
        e_c, cl_c, nsub = ffi.plan(n, k_max, abi, chi, start=0, q_max=q_max, l_max=l_max)
        assert (e_c, cl_c, nsub) == (0, [], 0)
        return
    while start < len(subs):
        e_o, cl_o = PL.plan_step(subs, start, n, chi, k_max, qm, lm)
        e_c, cl_c, nsub = ffi.plan(n, k_max, abi, chi, start=start, q_max=q_max, l_max=l_max)
        assert nsub == len(subs)
        assert e_c == e_o and cl_c == [tuple(x) for x in cl_o], (start, e_o, cl_o, e_c, cl_c)
        assert all(k <= k_max for _, k in cl_c)
        start = e_o


@pytest.mark.parametrize("gates,why", [
    ([((0, 9), None)], "out of range"),
    ([((0, 1), None), ((1,), None)], "disjoint"),
    ([((-1,), None)], "out of range"),
])
def test_planner_rejects_what_run_layer_rejects(gates, why):
    ffi = _ffi()
    from paper_2502_19289_amd.gates import GATES
    layer = [(q, GATES["CNOT"] if len(q) == 2 else GATES["H"]) for q, _ in gates]
    with pytest.raises(ffi.CtebdError) as e:
        ffi.plan(8, 4, [layer], [1] * 7)
    assert e.value.status == ffi.MPS_EINVAL
    assert why in str(e.value)
