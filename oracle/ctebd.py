"""FP64 cluster-TEBD on the CPU: the oracle the HIP path is checked against.

State (Sec. II.B; inversion-free TEBD form of M. B. Hastings, J. Math. Phys. 50,
095207 (2009)): right-canonical site tensors B_j of shape (chi_{j-1}, 2, chi_j)
and, on every bond b (between sites b and b+1), the normalised Schmidt values
Lambda_b.  The physical state is the contraction B_0 B_1 ... B_{n-1}; the
initial state is |0...0> (Sec. IV.A), i.e. B_j = e_0 with shape (1, 2, 1).

One step (Sec. III.A): plan the clusters, then for every cluster on sites
a..a+k-1 (the clusters of a step are independent and are processed in order):
  1. U_c  = product of the cluster's gates, later gates to the left;
  2. Theta = B_a B_{a+1} ... B_{a+k-1}  (chi_l x 2^k x chi_r);
  3. Theta' = U_c Theta on the physical index;
  4. split right to left by k-1 truncated SVDs (Fig. firstMPS, Sec. II.B): for
     m = k-1..1, X is Theta' projected so far, reshaped (chi_l 2^m) x (2 c);
     the SVD is taken of D X with D = diag(Lambda_{a-1}) (x) 1; keep r values
     (cutoff eta on the normalised values, then the cap chi_max, r >= 1); the
     per-SVD fidelity f = sum of kept sigma^2 / sum of all sigma^2 (Eq. f_i);
     B_{a+m} = first r rows of V^dagger; Lambda_{a+m-1} = sigma[:r]/||sigma[:r]||;
     X <- X V[:, :r] (unweighted);
  5. B_a = X / sqrt(prod f) so the cluster's weighted norm is one again.
Sites outside every cluster get the product of their one-qubit gates.  The
fidelity estimate is F = prod f_i (Eq. approxF), accumulated as sum log f_i.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import gates as G
from . import planner as PL


@dataclass
class SvdRecord:
    step: int
    bond: int
    rank: int
    full: int
    f: float
    degenerate_cut: bool


@dataclass
class MPS:
    B: List[np.ndarray]
    lam: List[np.ndarray]
    log_f: float = 0.0
    records: List[SvdRecord] = field(default_factory=list)

    @property
    def n(self) -> int:
        return len(self.B)

    def bond_dims(self) -> List[int]:
        return [b.shape[2] for b in self.B[:-1]]

    def copy(self) -> "MPS":
        return MPS([b.copy() for b in self.B], [l.copy() for l in self.lam], self.log_f, list(self.records))


def product_state(n: int) -> MPS:
    """|0...0> as an MPS with all bonds of dimension one (Secs. II.A, IV.A)."""
    B = []
    for _ in range(n):
        t = np.zeros((1, 2, 1), dtype=np.complex128)
        t[0, 0, 0] = 1.0
        B.append(t)
    return MPS(B, [np.ones(1) for _ in range(n - 1)])


def apply_gate_to_columns(M: np.ndarray, k: int, u: np.ndarray, pos: Sequence[int]) -> np.ndarray:
    """Left-multiply a 2^k x c matrix by gate u acting on local qubits ``pos``
    (big-endian: local qubit 0 is the most significant bit); a gate acts on
    its qubits' indices of the state tensor (Sec. II.A)."""
    c = M.shape[1]
    g = len(pos)
    T = M.reshape((2,) * k + (c,))
    U = u.reshape((2,) * (2 * g))
    T = np.tensordot(U, T, axes=(list(range(g, 2 * g)), list(pos)))
    # tensordot puts the gate's output axes first; move them back in place
    rest = [ax for ax in range(k) if ax not in pos]
    order = [0] * k
    for i, p in enumerate(pos):
        order[p] = i
    for j, p in enumerate(rest):
        order[p] = g + j
    T = np.transpose(T, order + [k])
    return T.reshape(2 ** k, c)


def cluster_unitary(a: int, k: int, gates: Sequence) -> np.ndarray:
    """U_c: the ordered product of the cluster's gates embedded on its k qubits
    (Sec. III.A: the gates of a cluster over the step's layers are contracted
    into one tensor before it meets the MPS)."""
    U = np.eye(2 ** k, dtype=np.complex128)
    for g in gates:
        U = apply_gate_to_columns(U, k, G.matrix(g.name), [q - a for q in g.qubits])
    return U


def truncation_rank(sigma: np.ndarray, chi_max: int, eps: float) -> int:
    """Number of singular values kept (Sec. II.B): values below the cutoff eta
    are discarded (compared on the normalised spectrum), then at most chi_max
    are kept, and at least one."""
    s = sigma / np.linalg.norm(sigma)
    r = int(np.count_nonzero(s >= eps))
    return max(1, min(chi_max, r))


def apply_cluster(psi: MPS, a: int, k: int, U: np.ndarray, chi_max: int, eps: float,
                  step: int = 0) -> None:
    """Steps 2-5 of the module docstring for one cluster, in place: contract
    and apply U_c, then split right to left by truncated SVDs with eta and
    chi_max (Sec. III.A with the truncation of Sec. II.B), recording each
    f_i (Eq. f_i) and adding log f_i to the fidelity sum (Eq. approxF)."""
    theta = psi.B[a]
    for j in range(1, k):
        theta = np.tensordot(theta, psi.B[a + j], axes=([theta.ndim - 1], [0]))
    chi_l, chi_r = theta.shape[0], theta.shape[-1]
    theta = theta.reshape(chi_l, 2 ** k, chi_r)
    theta = np.einsum("st,ltr->lsr", U, theta)
    lam_l = psi.lam[a - 1] if a > 0 else np.ones(1)
    X = theta.reshape(chi_l * 2 ** (k - 1), 2 * chi_r)
    c = chi_r
    log_f = 0.0
    for m in range(k - 1, 0, -1):
        rows = chi_l * 2 ** m
        W = (lam_l[:, None] * X.reshape(chi_l, -1)).reshape(rows, 2 * c)
        _, sigma, Vh = np.linalg.svd(W, full_matrices=False)
        r = truncation_rank(sigma, chi_max, eps)
        tot = float(np.sum(sigma ** 2))
        f = float(np.sum(sigma[:r] ** 2)) / tot
        degenerate = r < sigma.size and (sigma[r - 1] - sigma[r]) < 1e-8 * sigma[0]
        psi.records.append(SvdRecord(step, a + m - 1, r, sigma.size, f, bool(degenerate)))
        psi.B[a + m] = Vh[:r].reshape(r, 2, c)
        kept = sigma[:r]
        psi.lam[a + m - 1] = kept / np.linalg.norm(kept)
        X = (X @ Vh[:r].conj().T).reshape(rows // 2, 2 * r)
        c = r
        log_f += math.log(f)
    psi.B[a] = X.reshape(chi_l, 2, c) / math.sqrt(math.exp(log_f))
    psi.log_f += log_f


def apply_one_qubit(psi: MPS, j: int, u: np.ndarray) -> None:
    """A one-qubit gate on a site outside every cluster of the step (Sec.
    III.A: no bond grows, no SVD)."""
    psi.B[j] = np.einsum("st,ltr->lsr", u, psi.B[j])


@dataclass
class RunResult:
    psi: MPS
    steps: List[Tuple[int, int, List[Tuple[int, int]]]]
    cluster_updates: int

    @property
    def fidelity(self) -> float:
        """F_est = prod f_i (Eq. approxF)."""
        return math.exp(self.psi.log_f)


def run_step(psi: MPS, subs, start: int, chi_max: int, eps: float, k_max: int,
             q_max: int, l_max: int, step: int):
    """One cluster-TEBD iteration (Sec. III.A) from sub-layer ``start``."""
    n = psi.n
    end, clusters = PL.plan_step(subs, start, n, psi.bond_dims(), k_max, q_max, l_max)
    per_cluster, per_site = PL.step_gates(subs, start, end, clusters, n)
    for (a, k), gl in zip(clusters, per_cluster):
        apply_cluster(psi, a, k, cluster_unitary(a, k, gl), chi_max, eps, step)
    for j in range(n):
        if per_site[j]:
            u = np.eye(2, dtype=np.complex128)
            for g in per_site[j]:
                u = G.matrix(g.name) @ u
            apply_one_qubit(psi, j, u)
    return end, clusters


def run(circuit, chi_max: int, eps: float, k_max: int, q_max: Optional[int] = None,
        l_max: int = 1 << 30, psi: Optional[MPS] = None, max_steps: Optional[int] = None) -> RunResult:
    """Simulate ``circuit`` from |0...0> (or ``psi``) with cluster-TEBD: the
    iteration of Sec. III.A, one step after another until every layer is
    contracted."""
    if q_max is None:
        q_max = PL.default_q_max(k_max, chi_max)
    subs = PL.legalize(circuit.layers, k_max)
    psi = product_state(circuit.n) if psi is None else psi
    start, step, steps, updates = 0, 0, [], 0
    while start < len(subs) and (max_steps is None or step < max_steps):
        end, clusters = run_step(psi, subs, start, chi_max, eps, k_max, q_max, l_max, step)
        steps.append((start, end, clusters))
        updates += len(clusters)
        start, step = end, step + 1
    return RunResult(psi, steps, updates)
