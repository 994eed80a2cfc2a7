// Host planner of the cluster-TEBD iteration (arXiv:2502.19289, Sec. III.A).
//
// The iteration keeps one flag per bond; a gate spanning qubits lo..hi flags
// bonds lo..hi-1; after every (sub-)layer the entanglement clusters are the
// maximal runs of flagged bonds.  The step covers the longest prefix of
// sub-layers for which every cluster holds at most k_max qubits and fits
// 2^k chi_l chi_r <= 2^q_max (Eqs. size / cond_cTEBD; chi_l, chi_r are the bonds
// just outside the cluster) with at most l_max sub-layers (Eq. cond2_cTEBD).
// A first sub-layer that already breaks a cap is contracted on its own.
//
// Before planning, each circuit layer is legalised: gates of span > k_max are
// replaced by a chain of adjacent SWAPs that brings the far qubit to distance
// k_max-1, the gate, and the chain undone (Sec. IV.A routes long-range gates with
// SWAPs); the remaining gates are packed first-fit into sub-layers whose spans
// are pairwise disjoint (gates of one layer commute, so this is exact).
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

namespace ctebd {

using cplx = std::complex<double>;

struct HostGate {
  int nq = 1;
  int q[2] = {0, 0};
  cplx u[16];
  int lo() const { return nq == 1 ? q[0] : (q[0] < q[1] ? q[0] : q[1]); }
  int hi() const { return nq == 1 ? q[0] : (q[0] < q[1] ? q[1] : q[0]); }
};

using SubLayer = std::vector<HostGate>;

struct Cluster {
  int a;  // first site
  int k;  // number of sites
};

// Legalises one circuit layer into sub-layers (appended to out).
void legalize_layer(const std::vector<HostGate>& layer, int k_max, std::vector<SubLayer>& out);

// Plans one step from sub-layer `start`; returns the end index (exclusive) and
// fills `clusters`.  chi has n-1 entries.
int plan_step(const std::vector<SubLayer>& subs, int start, int n, const std::vector<int>& chi,
              int k_max, int q_max, int l_max, std::vector<Cluster>& clusters);

bool cluster_fits(int a, int k, const std::vector<int>& chi, int k_max, int q_max);

int default_q_max(int k_max, int chi_max);

HostGate make_swap(int a, int b);

}  // namespace ctebd
