// Handle state and step executor of the cluster-TEBD library.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <complex>
#include <cstring>
#include <cstdint>
#include <string>
#include <map>
#include <vector>

#include "../../include/cluster_tebd.h"
#include "kernels.hpp"
#include "planner.hpp"

namespace ctebd {

// Bump allocator over one device allocation; reset at every step.  Grows (by
// reallocation, only between steps) when a step needs more than it holds.
struct DeviceArena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  hipError_t reserve(size_t bytes);
  void reset() { used = 0; }
  void* take(size_t bytes) {
    const size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    return base + off;
  }
  void release();
};

// Device blocks for the workspaces of the wavefront executor's tasks, which
// live for several rounds: a freed block goes to a free list and serves a
// later request that fits in it and needs at least half of it (sizes are
// rounded up to 2 MiB multiples).  Blocks return to the runtime only with the
// handle.
struct BlockPool {
  std::multimap<size_t, char*> free_blocks;  // capacity -> block
  std::vector<std::pair<char*, size_t>> all;
  hipError_t get(size_t bytes, char** out, size_t* cap);
  void put(char* p, size_t cap) { free_blocks.emplace(cap, p); }
  void release();
};

// Host-side blob of descriptors uploaded once per step (pinned host staging).
struct DescBlob {
  std::vector<char> host;
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  char* dev = nullptr;
  size_t dev_cap = 0;
  size_t add(const void* p, size_t bytes) {
    const size_t off = (host.size() + 15) & ~size_t(15);
    host.resize(off + bytes);
    memcpy(host.data() + off, p, bytes);
    return off;
  }
  template <typename T>
  size_t add_vec(const std::vector<T>& v) {
    return add(v.data(), v.size() * sizeof(T));
  }
  hipError_t prepare();  // sizes the pinned and device buffers to the blob
  hipError_t upload(hipStream_t s);
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(dev + off);
  }
  template <typename T>
  T* host_at(size_t off) {
    return reinterpret_cast<T*>(host.data() + off);
  }
  void release();
};

// A cluster to contract and split: sites a..a+k-1 and either the gates that
// make its unitary or an explicit unitary.
struct Job {
  int a = 0, k = 0;
  std::vector<HostGate> gates;
  std::vector<std::complex<double>> U;  // explicit 2^k x 2^k, row-major (if non-empty)
};

struct KernelTimer {
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<int64_t> launches;
  std::vector<double> flop;  // algorithmic real flops per class (8 per complex MAC)
  std::vector<double> bytes; // algorithmic HBM bytes per class (bandwidth-bound classes)
  std::vector<int64_t> dispatches;  // kernel dispatches per class, repeats of a burst included
  // Burst-timed classes (see mps_set_burst_timing): class -> (stride, reps);
  // every stride-th launch is followed by reps re-launches inside one pair of
  // events.  burst_seen counts the launches of each class.
  std::map<int, std::pair<int, int>> burst;
  std::vector<int64_t> burst_seen;
  struct Pending {
    int cls;
    hipEvent_t a, b;
    int div;  // launches between the events
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int cls_of(const char* name);
};

}  // namespace ctebd

struct mps_ctx {
  int n = 0, chi_max = 1;
  double eps = 0.0;
  mps_options opt{};
  ctebd::Prec prec = ctebd::Prec::FP32;
  size_t esz = 8;  // bytes per complex entry of the site tensors
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<int> cap;             // bond capacity (n-1)
  std::vector<int> chi;             // host mirror of bond dimensions (n-1)
  std::vector<void*> site;          // per-site device tensors
  std::vector<double*> lam;         // per-bond Schmidt values (device)
  char* state_mem = nullptr;        // one allocation holding sites and lambdas
  int* d_chi = nullptr;             // device bond dimensions (n-1)
  unsigned long long* d_work = nullptr;  // eig_update complex-MAC counter
  double* d_logf = nullptr;         // device sum log f
  double* d_ones = nullptr;         // weights of a left edge (all ones)
  int ones_len = 0;
  ctebd::DeviceArena arena;
  ctebd::BlockPool pool;            // task workspaces of the wavefront executor
  ctebd::DescBlob blob;
  int* h_flags = nullptr;           // pinned: eigen convergence flags
  std::vector<ctebd::SubLayer> pending;
  mps_stats stats{};
  std::string err;
  bool timing = false;
  ctebd::KernelTimer timer;
  int q_max_eff = 0, l_max_eff = 0;
  double eps_eff = 0.0;
  // learned sketch: attached network (device parameters) and the log of
  // (features, log2 kept rank) of every truncated SVD since the last read
  const float* mlp_params = nullptr;
  std::vector<float> log_x, log_t;
  // spectrum tail of each bond's last split (features of its next splits):
  // discarded weight and smallest kept / largest singular value
  std::vector<float> prev_dw, prev_tail;
  // DMRG: the handle that holds each step's evolved segment, kept between
  // steps (same stream; owned, destroyed with this handle; never cloned)
  mps_ctx* dmrg_scratch = nullptr;
  // the tridiagonal solver's descriptors of the problems it actually solves
  // (host copy kept until the next solve, which first synchronises; device
  // copy read by the kernels)
  std::vector<ctebd::HtdDesc> htd_host;
  ctebd::HtdDesc* htd_dev = nullptr;
  size_t htd_dev_cap = 0;
  uint64_t sketch_seed = 0x9E3779B97F4A7C15ull;
  uint32_t sketch_stream = 0;
};

struct mlp_ctx {
  float* P = nullptr;      // parameters (device)
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* g = nullptr;      // gradient
  int t = 0;               // Adam step count
  hipStream_t stream = nullptr;
  std::string err;
};

namespace ctebd {
constexpr int N_FEAT = 12;
}
