"""Adaptive-grouping DMRG for circuits, FP64 on the CPU: test infrastructure
(an oracle), not part of the product path.

Follows Sec. III.B of the paper (with the DMRG iteration of Sec. II.C):
  * Eq. chi_est: per bond b, the two-qubit gates of the segment crossing it,
    E(b), give the virtual bond dimension
        chi~_b = min(2^E(b) chi_b, chi_max^DMRG, 2^min(b+1, n-b-1))
    (0-based bond b between sites b and b+1 of n);
  * Eqs. cond_group1 / cond_group2: the virtual MPS is cut recursively in two;
    a part of N sites between cuts of virtual dimensions chi~_L, chi~_R is a
    group when N + log2 chi~_L + log2 chi~_R <= Q_max (an open end counts
    chi~ = 1), else it is cut again;
  * DMRG: a grouped MPS M (one site per group, bond dimensions chi~ at the
    group cuts) is fitted to the evolved state U |psi> (U = the segment's
    layers) by updates of one group tau at a time, M^[tau] = F / sqrt(f_tau)
    with F the network of U |psi> contracted with M^dagger on every other group
    (M orthonormal around tau) and f_tau = ||F||^2 the fidelity after the
    update; a pass over the groups is a sweep;
  * the fitted M is decomposed back into one tensor per qubit by SVDs with
    chi_max^SVD and the cutoff eta (Sec. II.B), their kept weights recorded.

Readings where the paper is silent:
  * cut choice: the 1-D chain is cut at the bond of smallest virtual
    dimension (the minimum cut of the chain graph), ties going to the most
    balanced cut, then to the leftmost;
  * the network F is contracted by first forming U |psi> exactly as an MPS
    (the cluster-TEBD oracle without truncation) and then contracting it with
    M: the same tensor as any other contraction order;
  * the initial M is not random: it is U |psi> compressed at the group cuts by
    a left-to-right sweep of truncated SVDs (deterministic, so that two
    implementations can be compared); the sweeps then improve it;
  * a sweep goes right to left over the groups and then left to right, so
    it ends with the centre on the last group, from where the decomposition
    runs right to left (right-canonical qubit tensors with exact Schmidt
    values on every bond, the form the cluster-TEBD state uses);
  * the step's fidelity is f of the last update times the kept weights of the
    decomposition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

from . import ctebd as CT
from . import planner as PL


def entangling_counts(layers, n: int) -> List[int]:
    """E(b): two-qubit gates of the segment whose span crosses bond b."""
    E = [0] * (n - 1)
    for layer in layers:
        for g in layer:
            if len(g.qubits) > 1:
                lo, hi = min(g.qubits), max(g.qubits)
                for b in range(lo, hi):
                    E[b] += 1
    return E


def virtual_bond_dims(E: Sequence[int], chi: Sequence[int], chi_max_dmrg: int, n: int) -> List[int]:
    """Eq. chi_est."""
    out = []
    for b in range(n - 1):
        cap = 1 << min(b + 1, n - b - 1, 60)
        out.append(int(min((1 << min(E[b], 60)) * chi[b], chi_max_dmrg, cap)))
    return out


def group_sites(chit: Sequence[int], n: int, q_max: int) -> List[Tuple[int, int]]:
    """Eqs. cond_group1 / cond_group2 by recursive bipartition; groups as
    (first site, last site), left to right."""
    def fits(lo, hi, chi_l, chi_r):
        return (chi_l * chi_r) << (hi - lo + 1) <= (1 << q_max)

    def rec(lo, hi, chi_l, chi_r):
        if lo == hi or fits(lo, hi, chi_l, chi_r):
            return [(lo, hi)]
        best = None
        for b in range(lo, hi):
            key = (chit[b], abs((b - lo + 1) - (hi - b)), b)
            if best is None or key < best[0]:
                best = (key, b)
        k = best[1]
        return rec(lo, k, chi_l, chit[k]) + rec(k + 1, hi, chit[k], chi_r)

    return rec(0, n - 1, 1, 1)


def _merge(sites: Sequence[np.ndarray]) -> np.ndarray:
    """Contract consecutive qubit tensors into one grouped tensor (l, 2^d, r)."""
    t = sites[0]
    for s in sites[1:]:
        t = np.tensordot(t, s, axes=(t.ndim - 1, 0))
    return t.reshape(t.shape[0], -1, t.shape[-1])


@dataclass
class DmrgRecord:
    groups: List[Tuple[int, int]]
    chi_virtual: List[int]
    f_updates: List[float] = field(default_factory=list)  # f_tau after every update, in order
    f_dmrg: float = 1.0
    f_svd: List[float] = field(default_factory=list)


def exact_target(psi: CT.MPS, layers, k_max: int) -> CT.MPS:
    """U |psi> without truncation (the cluster-TEBD oracle, no cap, eta = 0)."""
    out = psi.copy()
    circ = type("C", (), {})()
    circ.n, circ.layers = psi.n, list(layers)
    res = CT.run(circ, chi_max=1 << 30, eps=0.0, k_max=k_max, psi=out)
    return res.psi


def dmrg_step(psi: CT.MPS, layers, chi_max_dmrg: int, chi_max_svd: int, eps: float, q_max: int,
              sweeps: int = 2, k_max: int = 4) -> Tuple[CT.MPS, DmrgRecord]:
    n = psi.n
    E = entangling_counts(layers, n)
    chit = virtual_bond_dims(E, psi.bond_dims(), chi_max_dmrg, n)
    groups = group_sites(chit, n, q_max)
    rec = DmrgRecord(groups, chit)
    T = exact_target(psi, layers, k_max)
    g = len(groups)
    Tg = [_merge(T.B[a:b + 1]) for a, b in groups]
    norm_T = math.sqrt(abs(_overlap_grouped(Tg, Tg)))
    Tg[0] = Tg[0] / norm_T
    cut = [chit[b] for (_, b) in groups[:-1]]  # virtual dimension at each group cut
    # initial M: left-to-right truncated-SVD compression at the group cuts
    M: List[np.ndarray] = []
    C = Tg[0]
    for tau in range(g - 1):
        l, d, r = C.shape
        U, s, Vh = np.linalg.svd(C.reshape(l * d, r), full_matrices=False)
        # directions below 1e-10 of the largest singular value carry no weight
        # (1e-20) and would make the compressed sites rank-deficient
        k = max(1, min(cut[tau], int(np.count_nonzero(s > 1e-10 * s[0]))))
        M.append(U[:, :k].reshape(l, d, k))
        C = np.tensordot(s[:k, None] * Vh[:k], Tg[tau + 1], axes=(1, 0))
    M.append(C / np.linalg.norm(C))
    C = M[-1] * np.linalg.norm(C)
    # environments: L[t] = <M_0..M_{t-1} | T_0..T_{t-1}>, R[t] = <M_t..| T_t..>
    def left_env(t):
        Lm = np.ones((1, 1), dtype=np.complex128)
        for j in range(t):
            Lm = np.einsum("xy,xsa,ysb->ab", Lm, M[j].conj(), Tg[j])
        return Lm

    def right_env(t):
        Rm = np.ones((1, 1), dtype=np.complex128)
        for j in range(g - 1, t - 1, -1):
            Rm = np.einsum("asx,bsy,xy->ab", M[j].conj(), Tg[j], Rm)
        return Rm

    def update(tau):
        F = np.einsum("xa,asb,yb->xsy", left_env(tau), Tg[tau], right_env(tau + 1))
        f = float(np.vdot(F, F).real)
        rec.f_updates.append(f)
        return F / math.sqrt(f), f

    # fidelity of the compression itself: the weight its centre kept
    f = float(np.vdot(C, C).real)
    rec.f_updates.append(f)
    for _ in range(sweeps):
        for tau in range(g - 1, -1, -1):  # right to left: right-orthonormalise after the update
            Mt, f = update(tau)
            if tau > 0:
                l, d, r = Mt.shape
                Q, R = np.linalg.qr(Mt.reshape(l, d * r).conj().T)
                M[tau] = Q.conj().T.reshape(Q.shape[1], d, r)
                M[tau - 1] = np.tensordot(M[tau - 1], R.conj().T, axes=(2, 0))
            else:
                M[tau] = Mt
        for tau in range(g):  # left to right: left-orthonormalise after the update
            Mt, f = update(tau)
            if tau < g - 1:
                l, d, r = Mt.shape
                Q, R = np.linalg.qr(Mt.reshape(l * d, r))
                M[tau] = Q.reshape(l, d, Q.shape[1])
                M[tau + 1] = np.tensordot(R, M[tau + 1], axes=(1, 0))
            else:
                M[tau] = Mt
    rec.f_dmrg = f
    # decomposition right to left into qubit tensors: M is left-orthonormal up
    # to its centre (the last group), so every split sees an orthonormal left
    # environment and gives the Schmidt values of its bond
    out = CT.MPS([None] * n, [None] * (n - 1), psi.log_f)
    log_f = math.log(f)
    X = np.ones((1, 1), dtype=np.complex128)
    for tau in range(g - 1, -1, -1):
        a, b = groups[tau]
        t = np.tensordot(M[tau], X, axes=(2, 0))
        l, D, r = t.shape
        cur = t.reshape(l * D // 2, 2 * r)
        right = r
        for q in range(b, a - 1, -1):
            if q == 0:
                out.B[0] = cur.reshape(1, 2, right) / np.linalg.norm(cur)
                break
            U, sv, Vh = np.linalg.svd(cur, full_matrices=False)
            kk = CT.truncation_rank(sv, chi_max_svd, eps)
            fq = float(np.sum(sv[:kk] ** 2) / np.sum(sv ** 2))
            rec.f_svd.append(fq)
            log_f += math.log(fq)
            out.B[q] = Vh[:kk].reshape(kk, 2, right)
            out.lam[q - 1] = sv[:kk] / np.linalg.norm(sv[:kk])
            rest = U[:, :kk] * sv[:kk]
            if q > a:
                cur = rest.reshape(-1, 2 * kk)
                right = kk
            else:
                X = rest
    out.log_f = psi.log_f + log_f
    return out, rec


def _overlap_grouped(A: Sequence[np.ndarray], B: Sequence[np.ndarray]) -> complex:
    E = np.ones((1, 1), dtype=np.complex128)
    for a, b in zip(A, B):
        E = np.einsum("xy,xsa,ysb->ab", E, a.conj(), b)
    return complex(E[0, 0])


def run(circuit, l_max: int, chi_max_dmrg: int, chi_max_svd: int, eps: float, q_max: int, sweeps: int = 2,
        k_max: int = 4):
    """The circuit from |0...0>, one DMRG step per l_max layers."""
    psi = CT.product_state(circuit.n)
    records = []
    for t0 in range(0, len(circuit.layers), l_max):
        psi, rec = dmrg_step(psi, circuit.layers[t0:t0 + l_max], chi_max_dmrg, chi_max_svd, eps, q_max, sweeps,
                             k_max)
        records.append(rec)
    return psi, records
