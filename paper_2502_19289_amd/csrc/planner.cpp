#include "planner.hpp"

#include <algorithm>

namespace ctebd {

HostGate make_swap(int a, int b) {
  HostGate g;
  g.nq = 2;
  g.q[0] = a;
  g.q[1] = b;
  for (auto& x : g.u) x = 0.0;
  g.u[0] = g.u[6] = g.u[9] = g.u[15] = 1.0;  // |00>,|01>->|10>,|10>->|01>,|11>
  return g;
}

namespace {

struct Span {
  int lo, hi;
};

bool overlaps_any(const Span& s, const std::vector<Span>& v) {
  for (const auto& t : v)
    if (!(s.hi < t.lo || s.lo > t.hi)) return true;
  return false;
}

bool span_less(const HostGate& x, const HostGate& y) {
  if (x.lo() != y.lo()) return x.lo() < y.lo();
  if (x.hi() != y.hi()) return x.hi() < y.hi();
  if (x.q[0] != y.q[0]) return x.q[0] < y.q[0];
  return x.q[1] < y.q[1];
}

// SWAP chain bringing the far qubit of g to lo+k_max-1, g itself, chain undone.
std::vector<HostGate> route(const HostGate& g, int k_max) {
  const int lo = g.lo(), hi = g.hi(), p = lo + k_max - 1;
  std::vector<HostGate> down;
  for (int j = hi - 1; j >= p; --j) down.push_back(make_swap(j, j + 1));
  HostGate moved = g;
  for (int i = 0; i < g.nq; ++i)
    if (moved.q[i] == hi) moved.q[i] = p;
  std::vector<HostGate> ops = down;
  ops.push_back(moved);
  for (auto it = down.rbegin(); it != down.rend(); ++it) ops.push_back(*it);
  return ops;
}

}  // namespace

void legalize_layer(const std::vector<HostGate>& layer, int k_max, std::vector<SubLayer>& out) {
  std::vector<SubLayer> subs(1);
  std::vector<std::vector<Span>> spans(1);
  std::vector<HostGate> multi;
  for (const auto& g : layer) {
    if (g.nq == 1)
      subs[0].push_back(g);
    else
      multi.push_back(g);
  }
  std::stable_sort(multi.begin(), multi.end(), span_less);
  std::vector<HostGate> far;
  for (const auto& g : multi) {
    if (g.hi() - g.lo() + 1 > k_max) {
      far.push_back(g);
      continue;
    }
    Span s{g.lo(), g.hi()};
    size_t i = 0;
    for (; i < subs.size(); ++i)
      if (!overlaps_any(s, spans[i])) break;
    if (i == subs.size()) {
      subs.emplace_back();
      spans.emplace_back();
    }
    subs[i].push_back(g);
    spans[i].push_back(s);
  }
  // routed gates: units with disjoint spans share sub-layers position by position
  std::vector<std::vector<std::vector<HostGate>>> groups;
  std::vector<std::vector<Span>> gspans;
  for (const auto& g : far) {
    Span s{g.lo(), g.hi()};
    size_t i = 0;
    for (; i < groups.size(); ++i)
      if (!overlaps_any(s, gspans[i])) break;
    if (i == groups.size()) {
      groups.emplace_back();
      gspans.emplace_back();
    }
    groups[i].push_back(route(g, k_max));
    gspans[i].push_back(s);
  }
  for (const auto& units : groups) {
    size_t depth = 0;
    for (const auto& u : units) depth = std::max(depth, u.size());
    for (size_t t = 0; t < depth; ++t) {
      SubLayer sl;
      for (const auto& u : units)
        if (t < u.size()) sl.push_back(u[t]);
      subs.push_back(sl);
    }
  }
  for (auto& s : subs)
    if (!s.empty()) out.push_back(std::move(s));
}

bool cluster_fits(int a, int k, const std::vector<int>& chi, int k_max, int q_max) {
  if (k > k_max) return false;
  const int nb = (int)chi.size();
  const uint64_t cl = a > 0 ? (uint64_t)chi[a - 1] : 1u;
  const uint64_t cr = (a + k - 1 < nb) ? (uint64_t)chi[a + k - 1] : 1u;
  if (q_max >= 62) return true;
  // 2^k * cl * cr <= 2^q_max without overflow: compare in log space exactly
  const unsigned __int128 size = ((unsigned __int128)cl * cr) << k;
  return size <= ((unsigned __int128)1 << q_max);
}

static void runs(const std::vector<char>& bond, std::vector<Cluster>& out) {
  out.clear();
  const int nb = (int)bond.size();
  for (int b = 0; b < nb;) {
    if (!bond[b]) {
      ++b;
      continue;
    }
    int e = b;
    while (e + 1 < nb && bond[e + 1]) ++e;
    out.push_back({b, e - b + 2});
    b = e + 1;
  }
}

static void mark(std::vector<char>& bond, const SubLayer& sl) {
  for (const auto& g : sl)
    if (g.nq > 1)
      for (int b = g.lo(); b < g.hi(); ++b) bond[b] = 1;
}

int plan_step(const std::vector<SubLayer>& subs, int start, int n, const std::vector<int>& chi,
              int k_max, int q_max, int l_max, std::vector<Cluster>& clusters) {
  std::vector<char> bond(n - 1, 0), trial;
  std::vector<Cluster> cl;
  int end = start;
  while (end < (int)subs.size() && end - start < l_max) {
    trial = bond;
    mark(trial, subs[end]);
    runs(trial, cl);
    bool ok = true;
    for (const auto& c : cl)
      if (!cluster_fits(c.a, c.k, chi, k_max, q_max)) {
        ok = false;
        break;
      }
    if (!ok) break;
    bond.swap(trial);
    ++end;
  }
  if (end == start) {
    std::fill(bond.begin(), bond.end(), 0);
    mark(bond, subs[start]);
    end = start + 1;
  }
  runs(bond, clusters);
  return end;
}

int default_q_max(int k_max, int chi_max) {
  int bits = 0;
  while ((1 << bits) < chi_max) ++bits;
  return k_max + 2 * bits;
}

}  // namespace ctebd
