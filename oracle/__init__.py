"""Plain FP64 CPU oracle for the cluster-TEBD hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything here; only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.  It shares no code with
the HIP path: the one module both sides read is the seeded circuit-structure
generator in ``workloads``.

Contents (each function cites the passage of arXiv:2502.19289 it follows):
  gates        gate matrices of App. A plus H, S, T (one table of its own)
  planner      bond-array clustering, caps, SWAP routing (Sec. III.A)
  ctebd        the cluster-TEBD iteration in FP64 with LAPACK SVDs (Secs. II.B, III.A)
  statevector  brute-force 2^n simulation (pins exact contraction)
  stabilizer   CHP tableau + GF(2)-rank entanglement entropies (pins Clifford spectra)
  mps_tools    amplitudes, overlaps, entropies of an MPS (Sec. II.B definitions)
  tebd         gate-by-gate TEBD with an orthogonality centre (Sec. II.C)
  dmrg         adaptive-grouping DMRG: virtual bond dimensions, bipartition,
               fitting sweeps, decomposition (Sec. III.B)
  sketch       randomized range finder and the kept-rank MLP (the learned
               sketch, not in the paper); the range finder, the network's
               forward pass, its gradients and the optimiser are pinned, the
               trained weights are not (parity unpinned: they come from data)
"""
