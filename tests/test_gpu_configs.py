"""Per-workload parity with the FP64 oracle through the C ABI.

* The batched workload (1000 qubits, clusters of 2..8 qubits, chi_max = 128)
  and the learned-sketch workload (500 qubits, chi_max = 512), both shrunk in
  depth so that the oracle finishes in seconds, run end to end on the GPU and
  in the oracle from the same circuit file: infidelity of the final states
  (transfer-matrix overlap), fidelity estimates and bond dimensions.
* One saturated step of the chi_max = 1024 workload (200 qubits, 50 layers,
  k <= 6): the GPU state is evolved until a quarter of the bonds hold 1024
  Schmidt values, then a step whose clusters put at least two 2048 x 2048
  Gram matrices into one tridiagonal launch is taken by the FP64, FP32 and
  BF16X6 paths from the same state and by the oracle's cluster update
  (LAPACK SVDs) from the exported site tensors; per cluster the discarded
  weight, the Schmidt values of the inner bonds and the state of the cluster
  (Lambda-weighted block, the environments being shared) are compared.

The infidelity bars are those of the target: 1e-6 for the mixed-precision
paths, 1e-11 for the FP64 path.
"""
import math

import numpy as np
import pytest

from oracle import ctebd as CT
from oracle import mps_tools as MT
from oracle import planner as PL
from workloads import make_workload

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")

INF_TOL = {"fp64": 1e-11, "fp32": 1e-6, "bf16x6": 1e-6}
# the GPU path keeps normalised values above max(eta, 4 u) with u = 2^-26.5
# (FP64 Gram resolution) or 2^-24 (FP32 / BF16X6 contractions); the oracle
# keeps everything above eta
KEPT_FLOOR = {"fp64": 4 * 2.0 ** -26.5, "fp32": 4 * 2.0 ** -24, "bf16x6": 4 * 2.0 ** -24}
# largest normalised value that one side may keep and the other not: the kept
# floor, or for FP64 the Gram route's resolution at 2c = 2048, sqrt(64 u sqrt(2048))
RESOLVED = {"fp64": max(1.01 * KEPT_FLOOR["fp64"], (64 * 2.0 ** -53 * 2048 ** 0.5) ** 0.5),
            "fp32": 1.01 * KEPT_FLOOR["fp32"], "bf16x6": 1.01 * KEPT_FLOOR["bf16x6"]}


def _run_gpu(c, p, prec, batch="step"):
    m = P.MPS(c.n, p["chi_max"], p["eps"], k_max=p["k_max"], precision=prec, batch=batch)
    P.run_circuit(m, c.layers)
    return m


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,layers", [("batched_n1000_l100", 10), ("learned_n500_l60", 10)])
def test_workload_end_to_end_vs_oracle(name, layers, prec):
    c, p = make_workload(name, seed=0, layers=layers)
    ref = CT.run(c, **p)
    assert max(k for (_, _, cl) in ref.steps for (_, k) in cl) == p["k_max"]  # the largest clusters occur
    m = _run_gpu(c, p, prec)
    inf = MT.infidelity(m.sites(), ref.psi.B)
    print(f"{name} {layers} layers {prec}: infidelity vs oracle {inf:.3e}, max chi {max(m.bond_dims())}")
    assert inf < INF_TOL[prec]
    F, lf = m.fidelity()
    assert abs(lf - ref.psi.log_f) < (1e-10 if prec == "fp64" else 1e-6)
    if prec == "fp64":
        assert m.bond_dims() == ref.psi.bond_dims()


# ---- one saturated step of the chi_max = 1024 workload
def _split_bounds(a, k, chi, chi_max):
    """2c of every split of a cluster (bounds before the step's truncations)."""
    n_b = len(chi)
    chi_l = chi[a - 1] if a > 0 else 1
    c = chi[a + k - 1] if a + k - 1 < n_b else 1
    out = []
    for m in range(k - 1, 0, -1):
        rows = chi_l << m
        out.append(2 * c)
        c = min(chi_max, rows, 2 * c)
    return out


def _oracle_cost(a, k, chi, chi_max):
    chi_l = chi[a - 1] if a > 0 else 1
    return sum((chi_l << (k - 1 - t)) * n2 * n2 for t, n2 in enumerate(_split_bounds(a, k, chi, chi_max)))


def _segment(lam_l, B):
    """Lambda-weighted block of a cluster as a (chi_l 2^k) x chi_r matrix."""
    th = lam_l[:, None] * B[0].reshape(B[0].shape[0], -1)
    for t in B[1:]:
        th = th.reshape(-1, t.shape[0]) @ t.reshape(t.shape[0], -1)
    return th.reshape(-1, B[-1].shape[2])


@pytest.fixture(scope="module")
def saturated_step():
    c, p = make_workload("chi1024_n200_l50", seed=0)
    chi_max = p["chi_max"]
    m = P.MPS(c.n, chi_max, p["eps"], k_max=p["k_max"], precision="fp32", batch="step")
    for layer in c.layers:
        m.queue_layer([(g.qubits, P.GATES[g.name]) for g in layer])
    subs = PL.legalize(c.layers, p["k_max"])
    q_max = PL.default_q_max(p["k_max"], chi_max)
    start = 0
    while True:
        d = np.array(m.bond_dims())
        if (d >= chi_max).mean() >= 0.25:
            break
        _, rem = m.step()
        start = len(subs) - rem
        assert rem > 0
    # the next step with >= 2 Gram matrices of 2048 at one split level and an
    # oracle cost the CPU takes in seconds
    for _ in range(120):
        chi = m.bond_dims()
        end, clusters = PL.plan_step(subs, start, c.n, chi, p["k_max"], q_max, 1 << 30)
        levels = {}
        for a, k in clusters:
            for t, n2 in enumerate(_split_bounds(a, k, chi, chi_max)):
                if n2 == 2 * chi_max:
                    levels[t] = levels.get(t, 0) + 1
        cost = sum(_oracle_cost(a, k, chi, chi_max) for a, k in clusters)
        if levels and max(levels.values()) >= 2 and cost <= 1.5e11:
            break
        _, rem = m.step()
        start = end
        assert rem > 0
    else:
        pytest.fail("no step with two 2048-wide splits in one level found")
    per_cluster, _ = PL.step_gates(subs, start, end, clusters, c.n)
    print(f"saturated step: clusters {clusters}, 2048-wide splits per level {levels}, oracle cost {cost:.2e}")
    inputs = []
    for ci, (a, k) in enumerate(clusters):
        B = [m.site(j) for j in range(a, a + k)]
        lam = [m.schmidt(b) for b in range(a - 1, a + k - 1) if b >= 0]
        lam_l = m.schmidt(a - 1) if a > 0 else np.ones(1)
        inputs.append((a, k, B, lam_l, lam, CT.cluster_unitary(a, k, per_cluster[ci])))
    # oracle: each cluster's update on its exported block (the clusters of a
    # step are independent)
    expected = []
    for a, k, B, lam_l, _, U in inputs:
        psi = CT.MPS([np.ones((1, 2, B[0].shape[0]))] + [b.copy() for b in B],
                     [lam_l.copy()] + [np.ones(b.shape[2]) for b in B[:-1]])
        CT.apply_cluster(psi, 1, k, U, chi_max, p["eps"])
        expected.append(dict(B=psi.B[1:], lam=psi.lam[1:], log_f=psi.log_f, recs=list(psi.records),
                             seg=_segment(lam_l, psi.B[1:])))
    yield m, clusters, inputs, expected, chi_max
    m.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_saturated_chi1024_step_vs_oracle(saturated_step, prec):
    m, clusters, inputs, expected, chi_max = saturated_step
    g = m.clone(precision=prec)
    lf0 = g.fidelity()[1]
    g.step()
    assert abs((g.fidelity()[1] - lf0) - sum(e["log_f"] for e in expected)) < (1e-10 if prec == "fp64" else 1e-6)
    worst, worst_lam = 0.0, 0.0
    for (a, k, B, lam_l, _, _), e in zip(inputs, expected):
        gotB = [g.site(j) for j in range(a, a + k)]
        for t in range(k - 1):
            got = g.schmidt(a + t)
            exp = e["lam"][t]
            r = min(got.size, exp.size)
            # the Gram route computes lambda = sigma^2 to about u lambda_1, so a
            # small sigma carries an error of order u / sigma (sigma_1 <= 1)
            tol = (1e-9 if prec == "fp64" else 1e-5) + 32 * 2.0 ** -52 / exp[:r]
            dev = np.abs(got[:r] - exp[:r])
            worst_lam = max(worst_lam, float((dev / tol).max()))
            assert (dev < tol).all(), (a, k, t, float(dev.max()), float(exp[np.argmax(dev / tol)]))
            if got.size != exp.size:
                # only values near the path's kept floor may be kept by one side
                # alone: the oracle keeps everything above eta, the GPU drops
                # values below its floor and, at the Gram route's resolution
                # (eigenvalue noise of order sqrt(n) u lambda_1), may keep noise
                # directions just above it
                extra = exp[r:] if exp.size > r else got[r:]
                assert extra.max() < RESOLVED[prec], (a, k, t, got.size, exp.size, float(extra.max()))
        if any(rec.degenerate_cut for rec in e["recs"]):
            continue  # a cut through a multiplet: the kept vectors are not unique
        seg = _segment(lam_l, gotB)
        ov = np.vdot(seg, e["seg"])
        inf = 1.0 - abs(ov) ** 2 / (np.vdot(seg, seg).real * np.vdot(e["seg"], e["seg"]).real)
        worst = max(worst, inf)
    print(f"{prec}: worst cluster infidelity {worst:.3e} over {len(clusters)} clusters, "
          f"largest Schmidt-value deviation {worst_lam:.3f} of its bar")
    assert worst < INF_TOL[prec]
    g.close()
