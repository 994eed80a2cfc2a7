// Host side of the cluster-TEBD library: handle state, the step executor that
// queues the kernels of one iteration (arXiv:2502.19289, Sec. III.A), and the
// C ABI declared in include/cluster_tebd.h.
//
// One step = the clusters chosen by the planner plus the one-qubit gates of the
// sites outside them.  Every cluster goes through
//   unitary build -> merge chain -> unitary application -> (k-1) x split,
//   split = Gram (FP64) -> block-Jacobi eigen (FP64) -> select -> gather -> project,
//   finalize (B_a = X / sqrt(prod f)).
// With MPS_BATCH_STEP all clusters of the step share each launch (the kernels
// are grouped: one workgroup per output tile of any cluster); with
// MPS_BATCH_NONE every cluster gets its own launches.  Ranks chosen by a
// truncation are written to device memory and read there by the later kernels
// of the same step, so a step needs one host synchronisation at its end (plus
// one per Jacobi sweep to stop converged solves).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <iterator>
#include <mutex>
#include <tuple>
#include <unordered_map>

#include "engine.hpp"

using namespace ctebd;

namespace ctebd {

hipError_t DeviceArena::reserve(size_t bytes) {
  if (bytes <= cap) return hipSuccess;
  const size_t want = std::max(bytes, cap * 3 / 2);
  if (base) (void)hipFree(base);
  base = nullptr;
  cap = 0;
  hipError_t e = hipMalloc(&base, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    base = nullptr;
    return e;
  }
  cap = want;
  return hipSuccess;
}

void DeviceArena::release() {
  if (base) (void)hipFree(base);
  base = nullptr;
  cap = used = 0;
}

hipError_t DescBlob::prepare() {
  const size_t bytes = std::max<size_t>(host.size(), 16);
  if (bytes > pinned_cap) {
    if (pinned) (void)hipHostFree(pinned);
    pinned_cap = std::max(bytes, pinned_cap * 2);
    hipError_t e = hipHostMalloc(&pinned, pinned_cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      pinned = nullptr;
      pinned_cap = 0;
      return e;
    }
  }
  if (bytes > dev_cap) {
    if (dev) (void)hipFree(dev);
    dev_cap = std::max(bytes, dev_cap * 2);
    hipError_t e = hipMalloc(&dev, dev_cap);
    if (e != hipSuccess) {
      dev = nullptr;
      dev_cap = 0;
      return e;
    }
  }
  return hipSuccess;
}

hipError_t DescBlob::upload(hipStream_t s) {
  const size_t bytes = host.size();
  if (bytes == 0) return hipSuccess;
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  memcpy(pinned, host.data(), bytes);
  return hipMemcpyAsync(dev, pinned, bytes, hipMemcpyHostToDevice, s);
}

void DescBlob::release() {
  if (pinned) (void)hipHostFree(pinned);
  if (dev) (void)hipFree(dev);
  pinned = dev = nullptr;
  pinned_cap = dev_cap = 0;
  host.clear();
}

hipError_t BlockPool::get(size_t bytes, char** out, size_t* cap) {
  const size_t want = (bytes + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
  auto it = free_blocks.lower_bound(want);
  if (it != free_blocks.end() && it->first <= 2 * want) {
    *out = it->second;
    *cap = it->first;
    free_blocks.erase(it);
    return hipSuccess;
  }
  char* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  all.push_back({p, want});
  *out = p;
  *cap = want;
  return hipSuccess;
}

void BlockPool::release() {
  for (auto& b : all) (void)hipFree(b.first);
  all.clear();
  free_blocks.clear();
}

int KernelTimer::cls_of(const char* name) {
  for (size_t i = 0; i < names.size(); ++i)
    if (names[i] == name) return (int)i;
  names.push_back(name);
  ms.push_back(0.0);
  launches.push_back(0);
  flop.push_back(0.0);
  bytes.push_back(0.0);
  dispatches.push_back(0);
  return (int)names.size() - 1;
}

}  // namespace ctebd

namespace {

struct Fail {
  mps_status st;
};

#define HIP_OK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);              \
      throw Fail{e_ == hipErrorOutOfMemory ? MPS_ENOMEM : MPS_EDEVICE};          \
    }                                                                            \
  } while (0)

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Size and timing traces on stderr (CTEBD_EIG_TRACE, CTEBD_HTD_TRACE,
// CTEBD_SKETCH_TRACE) synchronise the stream; they exist only in builds with
// -DCTEBD_DEBUG_TRACE.
#ifdef CTEBD_DEBUG_TRACE
constexpr bool kDebugTrace = true;
#else
constexpr bool kDebugTrace = false;
#endif

[[noreturn]] void fail(mps_ctx* ctx, mps_status st, const char* msg) {
  ctx->err = msg;
  throw Fail{st};
}

// --------------------------------------------------------------- timing --
// Times the launches of its scope for kernel class `name` with events on the
// handle's stream; `div` is the number of launches the scope holds when the
// class time is to be counted per launch (a burst).
struct Timed {
  mps_ctx* ctx;
  int cls;
  int div;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(mps_ctx* c, const char* name, int launches = 1) : ctx(c), cls(-1), div(launches) {
    if (!ctx->timing) return;
    cls = ctx->timer.cls_of(name);
    auto take = [&]() {
      hipEvent_t e;
      if (!ctx->timer.pool.empty()) {
        e = ctx->timer.pool.back();
        ctx->timer.pool.pop_back();
      } else {
        (void)hipEventCreate(&e);
      }
      return e;
    };
    a = take();
    b = take();
    (void)hipEventRecord(a, ctx->stream);
  }
  ~Timed() {
    if (cls < 0) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->timer.pending.push_back({cls, a, b, div});
  }
};

// One launch (`go`) of a kernel that is idempotent on its inputs: running it
// again reads nothing it writes, so a re-launch reproduces the same outputs.
// Under burst timing of class `name` (stride, reps) every stride-th launch is
// followed by reps re-launches and one pair of events spans them all
// (separate events around every launch add the latency of two marker packets
// to each measurement); the other launches of the class are not timed.
// Returns whether the launch is counted in the class statistics.
template <class F>
bool timed_repeatable(mps_ctx* ctx, const char* name, F go) {
  if (!ctx->timing) {
    HIP_OK(go());
    return false;
  }
  KernelTimer& t = ctx->timer;
  const int cls = t.cls_of(name);
  const auto it = t.burst.find(cls);
  if (it == t.burst.end()) {
    Timed tm(ctx, name);
    HIP_OK(go());
    return true;
  }
  if (t.burst_seen.size() < t.names.size()) t.burst_seen.resize(t.names.size(), 0);
  if (t.burst_seen[cls]++ % it->second.first != 0) {
    HIP_OK(go());
    t.dispatches[cls] += 1;
    return false;
  }
  const int reps = it->second.second;
  Timed tm(ctx, name, 1 + reps);
  for (int r = 0; r <= reps; ++r) HIP_OK(go());
  return true;
}

void collect_timing(mps_ctx* ctx) {
  for (auto& p : ctx->timer.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->timer.ms[p.cls] += ms / p.div;
      ctx->timer.launches[p.cls] += 1;
      ctx->timer.dispatches[p.cls] += p.div;
    }
    ctx->timer.pool.push_back(p.a);
    ctx->timer.pool.push_back(p.b);
  }
  ctx->timer.pending.clear();
}

// ------------------------------------------------------ job bookkeeping --
struct Level {
  int m;        // split index: site a+m is split off
  int rows;     // chi_l 2^m
  int c_bound;  // bound of c (bond right of site a+m)
  int r_bound;  // bound of the kept rank
  int ksplit;
};

struct JobRun {
  const Job* job;
  int a, k, chi_l, chi_r;
  std::vector<int> mid;  // bonds a..a+k-2 before the step
  int64_t theta;
  std::vector<Level> lv;
  int ld;
  void* U64 = nullptr;
  void* Uw = nullptr;
  void* buf[2] = {nullptr, nullptr};
  void* Vr = nullptr;
  double2 *G = nullptr, *V = nullptr, *part = nullptr;
  void* J = nullptr;
  int *pair_rot = nullptr, *flags = nullptr, *perm = nullptr;
  double *scale = nullptr, *logf = nullptr, *rec = nullptr;
  int cur = 0;
  int flag_index = 0;
  bool htd = false;  // some level uses the tridiagonal solver: hw holds its buffers
  HtdDesc hw{};
};

int bond_dim(const mps_ctx* ctx, int b) { return (b < 0 || b >= ctx->n - 1) ? 1 : ctx->chi[b]; }

Dim fixed(int v) { return Dim{v, nullptr}; }

// Dim of c (the bond right of site a+m) at level t
Dim c_dim(mps_ctx* ctx, const JobRun& j, int t, int mult) {
  if (t == 0) return fixed(mult * j.chi_r);
  return Dim{mult, ctx->d_chi + (j.a + j.lv[t].m)};
}

// Eigen-solver of a split level: the tridiagonal route wherever it applies
// (2c <= HTD_MAX) unless Jacobi is asked for.  "auto" takes it at every size:
// measured on the chi_max = 1024 workload, even the small splits finish
// sooner there (their launches are shared with the large ones).
bool level_htd(const mps_ctx* ctx, const Level& lv) {
  const int n = 2 * lv.c_bound;
  if (n > HTD_MAX) return false;
  return ctx->opt.eig_method != MPS_EIG_JACOBI;
}

bool job_htd(const mps_ctx* ctx, const JobRun& j) {
  for (const auto& L : j.lv)
    if (level_htd(ctx, L)) return true;
  return false;
}


void plan_job(mps_ctx* ctx, const Job& job, JobRun& j) {
  j.job = &job;
  j.a = job.a;
  j.k = job.k;
  j.chi_l = bond_dim(ctx, job.a - 1);
  j.chi_r = bond_dim(ctx, job.a + job.k - 1);
  j.mid.clear();
  for (int b = job.a; b < job.a + job.k - 1; ++b) j.mid.push_back(ctx->chi[b]);
  // largest tensor of the merge chain: Theta_j = (chi_l 2^{j+1}) x chi_{a+j}
  j.theta = (int64_t)j.chi_l * ((int64_t)1 << job.k) * j.chi_r;
  for (int q = 1; q < job.k - 1; ++q)
    j.theta = std::max(j.theta, (int64_t)j.chi_l * ((int64_t)2 << q) * j.mid[q]);
  j.lv.clear();
  int c = j.chi_r, cmax = c;
  for (int m = job.k - 1; m >= 1; --m) {
    Level L;
    L.m = m;
    L.rows = j.chi_l << m;
    L.c_bound = c;
    L.r_bound = std::min(ctx->chi_max, std::min(L.rows, 2 * c));
    L.r_bound = std::min(L.r_bound, ctx->cap[job.a + m - 1]);
    const int T = ceil_div(2 * c, 64);
    const int tiles = T * (T + 1) / 2;
    int ks = std::max(1, 256 / std::max(1, tiles));
    ks = std::min(ks, std::max(1, L.rows / 256));
    ks = std::min(ks, 16);
    L.ksplit = ks;
    cmax = std::max(cmax, c);
    c = L.r_bound;
    j.lv.push_back(L);
  }
  j.ld = ((2 * cmax + 63) / 64) * 64;
}

size_t job_bytes(const mps_ctx* ctx, const JobRun& j) {
  const size_t dimU = (size_t)1 << (2 * j.k);
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  add(dimU * sizeof(double2));
  if (ctx->prec != Prec::FP64) add(dimU * ctx->esz);
  add(j.theta * ctx->esz);
  add(j.theta * ctx->esz);
  const size_t ld = j.ld;
  add(ld * ld * sizeof(double2));  // G
  add(ld * ld * sizeof(double2));  // V
  add(ld * 64 * sizeof(double2));  // J
  int ks = 1;
  size_t vr = 0;
  for (const auto& L : j.lv) {
    ks = std::max(ks, L.ksplit);
    vr = std::max(vr, (size_t)2 * L.c_bound * L.r_bound);
  }
  if (ks > 1) add((size_t)ks * ld * ld * sizeof(double2));
  add(vr * ctx->esz);
  add(ld / JP * sizeof(int) + 16);
  add(ld * sizeof(int));
  add(sizeof(double));
  add(4 * j.k * sizeof(double));
  if (job_htd(ctx, j)) {
    HtdDesc tmp{};
    htd_layout(ld, tmp, [&](size_t x) -> void* {
      add(x);
      return nullptr;
    });
  }
  return b;
}

void assign_job(mps_ctx* ctx, JobRun& j, DeviceArena& A) {
  const size_t dimU = (size_t)1 << (2 * j.k);
  j.U64 = A.take(dimU * sizeof(double2));
  j.Uw = (ctx->prec == Prec::FP64) ? j.U64 : A.take(dimU * ctx->esz);
  j.buf[0] = A.take(j.theta * ctx->esz);
  j.buf[1] = A.take(j.theta * ctx->esz);
  const size_t ld = j.ld;
  j.G = (double2*)A.take(ld * ld * sizeof(double2));
  j.V = (double2*)A.take(ld * ld * sizeof(double2));
  j.J = A.take(ld * 64 * sizeof(double2));
  int ks = 1;
  size_t vr = 0;
  for (const auto& L : j.lv) {
    ks = std::max(ks, L.ksplit);
    vr = std::max(vr, (size_t)2 * L.c_bound * L.r_bound);
  }
  j.part = ks > 1 ? (double2*)A.take((size_t)ks * ld * ld * sizeof(double2)) : nullptr;
  j.Vr = A.take(vr * ctx->esz);
  j.pair_rot = (int*)A.take(ld / JP * sizeof(int) + 16);
  j.perm = (int*)A.take(ld * sizeof(int));
  j.scale = (double*)A.take(sizeof(double));
  j.rec = (double*)A.take(4 * j.k * sizeof(double));
  j.htd = job_htd(ctx, j);
  if (j.htd) htd_layout(ld, j.hw, [&](size_t x) { return A.take(x); });
}

// Algorithmic flops per kernel class, once the sizes are final on the host:
// merge and unitary products as written (account_merge), and per split level
// (account_level, after that level's truncation is back) the Hermitian half of
// the Gram matrix and the projection.
void account_merge(mps_ctx* ctx, const JobRun& r) {
  double merge = 0;
  for (int j = 1; j < r.k; ++j) {
    const double M = (double)r.chi_l * (1 << j), K = r.mid[j - 1];
    const double N = 2.0 * ((j == r.k - 1) ? r.chi_r : r.mid[j]);
    merge += M * N * K;
  }
  const double apply = (double)(1 << r.k) * (1 << r.k) * r.chi_l * r.chi_r;
  ctx->timer.flop[ctx->timer.cls_of("merge")] += 8.0 * merge;
  ctx->timer.flop[ctx->timer.cls_of("apply")] += 8.0 * apply;
}

void account_level(mps_ctx* ctx, const JobRun& r, int t) {
  const int m = r.lv[t].m;
  const double c = (t == 0) ? r.chi_r : ctx->chi[r.a + m];
  const double rr = ctx->chi[r.a + m - 1];
  const double n2 = 2.0 * c, rows = r.lv[t].rows;
  ctx->timer.flop[ctx->timer.cls_of("gram")] += 8.0 * n2 * (n2 + 1) / 2 * rows;
  ctx->timer.flop[ctx->timer.cls_of("project")] += 8.0 * rows * n2 * rr;
}

// All of a finished step's, plus the rotation tiles eig_update counted on the device.
void account_flops(mps_ctx* ctx, const std::vector<JobRun>& runs, double eig_cmac, double pair_flops) {
  for (const auto& r : runs) {
    account_merge(ctx, r);
    for (size_t t = 0; t < r.lv.size(); ++t) account_level(ctx, r, (int)t);
  }
  ctx->timer.flop[ctx->timer.cls_of("eig_update")] += 8.0 * eig_cmac;
  ctx->timer.flop[ctx->timer.cls_of("eig_pairs")] += pair_flops;
}

// ------------------------------------------------------------ executor --
// Runs the given clusters (all in the same launches) plus the one-qubit site
// updates; ends with the host synchronisation of the step.
// ------------------------------------------------------- learned sketch --
// Features of every split of a job (12 per level, see mps_svd_log).
bool non_clifford_phase(const HostGate& g) {
  if (g.nq != 1 || std::abs(g.u[1]) > 1e-12 || std::abs(g.u[2]) > 1e-12) return false;
  const cplx ph = g.u[3] / g.u[0];
  const double a = std::arg(ph) / (M_PI / 2);
  return std::abs(a - std::round(a)) > 1e-9;
}

void job_features(const mps_ctx* ctx, const JobRun& r, const Job& job, int nsub, std::vector<float>& out) {
  int n2q = 0, nt = 0;
  for (const auto& g : job.gates) {
    if (g.nq == 2) ++n2q;
    if (non_clifford_phase(g)) ++nt;
  }
  for (const auto& L : r.lv) {
    const int b = r.a + L.m - 1;
    int cross = 0;
    for (const auto& g : job.gates)
      if (g.nq == 2 && g.lo() <= b && b < g.hi()) ++cross;
    const float f[N_FEAT] = {(float)r.k, std::log2((float)r.chi_l), std::log2((float)r.chi_r),
                             (float)L.m / (float)r.k, std::log10(std::max(ctx->prev_dw[b], 1e-30f)),
                             std::log2(2.f * L.c_bound), (float)cross, (float)n2q, (float)nt, (float)nsub,
                             std::log2((float)ctx->chi[b]), std::log10(std::max(ctx->prev_tail[b], 1e-30f))};
    out.insert(out.end(), f, f + N_FEAT);
  }
}

// Spectrum tail of the splits of a finished cluster (records: f, smallest
// kept / largest singular value, discarded weight, degenerate-cut flag per
// level) into the per-bond history the features read.
void record_tails(mps_ctx* ctx, const JobRun& r, const double* rec) {
  for (size_t t = 0; t < r.lv.size(); ++t) {
    const int b = r.a + r.lv[t].m - 1;
    ctx->prev_tail[b] = (float)rec[4 * t + 1];
    ctx->prev_dw[b] = (float)rec[4 * t + 2];
  }
}

// Workspace of one sketched split (n = 2c bound, s = sketch size).
struct SkRun {
  int job = 0, t = 0, s = 0, ld_s = 0, ld_y = 0, nb = 2;
  double2 *Omega, *Probe, *Y, *Q, *Vs, *R1, *R2, *C8, *Bq, *Gy, *Uy, *Hw, *Wh;
  void *Ja, *Jb;
  int *pr_a, *pr_b, *flags_a, *flags_b, *use;
  double *scale_a, *scale_b, *lam, *est;
};

size_t sk_bytes(int n, const SkRun& k) {
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  const size_t pan = (size_t)n * k.ld_s * sizeof(double2);
  for (int i = 0; i < 7; ++i) add(pan);  // Omega, Probe, Y, Q, Vs, R1, R2
  add((size_t)k.ld_y * k.ld_s * sizeof(double2) * 2);  // C8, Bq
  for (int i = 0; i < 4; ++i) add((size_t)k.ld_y * k.ld_y * sizeof(double2));
  add((size_t)k.ld_y * 64 * sizeof(double2) * 2);
  add((size_t)k.ld_y / JP * sizeof(int) * 2 + 32);
  add(k.ld_y * sizeof(double) + 64);
  return b;
}

void sk_assign(DeviceArena& A, SkRun& k, int n, int* flags, double* scales) {
  const size_t pan = (size_t)n * k.ld_s * sizeof(double2);
  double2** pans[7] = {&k.Omega, &k.Probe, &k.Y, &k.Q, &k.Vs, &k.R1, &k.R2};
  for (auto p : pans) *p = (double2*)A.take(pan);
  k.C8 = (double2*)A.take((size_t)k.ld_y * k.ld_s * sizeof(double2));
  k.Bq = (double2*)A.take((size_t)k.ld_y * k.ld_s * sizeof(double2));
  double2** sq[4] = {&k.Gy, &k.Uy, &k.Hw, &k.Wh};
  for (auto p : sq) *p = (double2*)A.take((size_t)k.ld_y * k.ld_y * sizeof(double2));
  k.Ja = A.take((size_t)k.ld_y * 64 * sizeof(double2));
  k.Jb = A.take((size_t)k.ld_y * 64 * sizeof(double2));
  k.pr_a = (int*)A.take((size_t)k.ld_y / JP * sizeof(int) + 16);
  k.pr_b = (int*)A.take((size_t)k.ld_y / JP * sizeof(int) + 16);
  k.lam = (double*)A.take(k.ld_y * sizeof(double));
  k.est = (double*)A.take(2 * sizeof(double));
  k.flags_a = flags;
  k.flags_b = flags + 4;
  k.use = flags + 8;
  k.scale_a = scales;
  k.scale_b = scales + 1;
}

GemmDesc gemm64(const void* A, const void* B, void* C, Dim M, Dim N, Dim K, Dim lda, Dim ldb, Dim ldc, int mb,
                int nbnd) {
  GemmDesc d{};
  d.A = A;
  d.B = B;
  d.C = C;
  d.M = M;
  d.N = N;
  d.K = K;
  d.lda = lda;
  d.ldb = ldb;
  d.ldc = ldc;
  d.batch = 1;
  d.tm = ceil_div(mb, 64);
  d.tn = ceil_div(nbnd, 64);
  d.ksplit = 1;
  d.alpha = 1.0;
  return d;
}

// Runs a group of FP64/FP32 block-Jacobi solves to convergence (host checks
// the convergence flags after every sweep).  flags_dev/h_flags hold `stride`
// ints per problem at the indices given.
void solve_eig(mps_ctx* ctx, EigDesc* de, const std::vector<EigDesc>& host, const int* b_pair,
               const int* b_upd, int n_pair, int n_upd, const int* flags_dev, int nflag_ints,
               const std::vector<int>& flag_at, bool sketch = false) {
  hipStream_t s = ctx->stream;
  const int np = (int)host.size();
  if (!np) return;
  // Sizes set by earlier splits of this step live in d_chi: read them so that
  // a sweep runs the rounds of the largest actual size, not of its bound.
  std::vector<int> chi_now(ctx->n - 1);
  HIP_OK(hipMemcpyAsync(chi_now.data(), ctx->d_chi, chi_now.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  int nb_all = 2;
  for (const auto& e : host) {
    const ptrdiff_t at = e.n.ptr ? e.n.ptr - ctx->d_chi : -1;
    const bool in_chi = at >= 0 && at < (ptrdiff_t)chi_now.size();
    const int n = !e.n.ptr ? e.n.mult : (in_chi ? e.n.mult * chi_now[at] : e.nb_max * JB);
    int nb = std::max(2, ceil_div(n, JB));
    nb += nb & 1;
    nb_all = std::max(nb_all, std::min(nb, e.nb_max));
  }
  const bool trace = kDebugTrace && std::getenv("CTEBD_EIG_TRACE") != nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  int sweeps = 0;
  for (int sw = 0; sw < 30; ++sw) {
    ++sweeps;
    for (int round = 0; round < nb_all - 1; ++round) {
      {
        Timed tm(ctx, sketch ? "sketch_eig" : "eig_pairs");
        HIP_OK(launch_eig_pairs(de, b_pair, np, n_pair, round, s));
      }
      {
        Timed tm(ctx, sketch ? "sketch_eig" : "eig_update");
        HIP_OK(launch_eig_update(de, b_upd, np, n_upd, round, s));
      }
    }
    HIP_OK(launch_eig_sweep_end(de, np, s));
    ctx->stats.jacobi_sweeps += 1;
    HIP_OK(hipMemcpyAsync(ctx->h_flags, flags_dev, (size_t)nflag_ints * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    bool all = true;
    for (int q : flag_at)
      if (!ctx->h_flags[q]) all = false;
    if (all) break;
  }
  if (trace) {
    std::string sizes;
    for (const auto& e : host) {
      int v = 1;
      if (e.n.ptr) HIP_OK(hipMemcpy(&v, e.n.ptr, sizeof(int), hipMemcpyDeviceToHost));
      sizes += " " + std::to_string(e.n.mult * v) + "/" + std::to_string(e.nb_max * JB);
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "eig np=%d rounds=%d sweeps=%d ms=%.2f n/bound:%s\n", np,
                 nb_all - 1, sweeps, ms, sizes.c_str());
  }
}

// Tridiagonal divide-and-conquer solves of one split level.  The sizes set
// by earlier splits of the step are read back first: the host needs them for
// the launch grids and passes them to every kernel by value (2 launches per
// column and 1 per panel of the reduction, 7 per merge level, 3 per block of
// reflectors).  Groups of more than HTD_GROUP problems run in chunks.
void solve_htd_chunk(mps_ctx* ctx, const HtdDesc* dd, const HtdSizes& sz, const HtdArgs& ha) {
  hipStream_t s = ctx->stream;
  const int np = sz.np;
  int nmax = 0;
  for (int p = 0; p < np; ++p) nmax = std::max(nmax, sz.n[p]);
  auto total = [&](auto f) {
    int t = 0;
    for (int p = 0; p < np; ++p) t += f(sz.n[p]);
    return t;
  };
  auto total_c = [&](auto f) {
    int t = 0;
    for (int p = 0; p < np; ++p) t += f(sz.n[p], sz.nc[p]);
    return t;
  };
  const bool timing = ctx->timing;
  const int c_hemv = timing ? ctx->timer.cls_of("trd_hemv") : -1;
  const int c_her2k = timing ? ctx->timer.cls_of("trd_her2k") : -1;
  const int c_bt = timing ? ctx->timer.cls_of("bt") : -1;
  const int c_col = timing ? ctx->timer.cls_of("trd_col") : -1;
  const int c_tail = timing ? ctx->timer.cls_of("trd_tail") : -1;
  const int c_dc = timing ? ctx->timer.cls_of("dc") : -1;
  const bool trace = kDebugTrace && std::getenv("CTEBD_HTD_TRACE") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!trace) return;
    const double host = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    HIP_OK(hipStreamSynchronize(s));
    const double all = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "htd np=%d nmax=%d %s: host enqueue %.2f ms, done %.2f ms\n", np, nmax, what, host, all);
    t0 = std::chrono::steady_clock::now();
  };
  if (trace) {
    std::fprintf(stderr, "htd sizes:");
    for (int p = 0; p < np; ++p) std::fprintf(stderr, " %d", sz.n[p]);
    std::fprintf(stderr, "\n");
  }
  lap("start");
  int kmain = 0;  // the blocked kernels run the columns below htd_tail_start(n)
  for (int p = 0; p < np; ++p) kmain = std::max(kmain, htd_tail_start(sz.n[p]));
  for (int p0 = 0; p0 < kmain; p0 += HTD_NB) {
    for (int j = 0; j < HTD_NB; ++j) {
      const int k = p0 + j;
      auto most = [&](auto f) {
        int t = 0;
        for (int p = 0; p < np; ++p) t = std::max(t, f(sz.n[p]));
        return t;
      };
      const int nb_col = most([k](int n) { return htd_col_blocks(n, k); });
      const bool col_counted = timed_repeatable(ctx, "trd_col", [&] { return launch_trd_col(ha, k, nb_col, s); });
      if (col_counted)  // algorithmic traffic of the column update: the column, the panel rows of V and W
                        // written so far and y, once each
        for (int p = 0; p < np; ++p) {
          const double m = sz.n[p] - k - 1;
          if (m <= 0 || k >= htd_tail_start(sz.n[p])) continue;
          ctx->timer.bytes[c_col] += 16.0 * m * (2.0 + 2.0 * j);
          ctx->timer.flop[c_col] += 8.0 * 2.0 * j * m;
        }
      const int nb_hemv = most([k](int n) { return htd_hemv_blocks(n, k); });
      const bool counted = timed_repeatable(ctx, "trd_hemv", [&] { return launch_trd_hemv(ha, k, nb_hemv, s); });
      if (counted)  // algorithmic traffic of the HEMV: one triangle of the trailing block, the rows of
                    // the j panel columns of V and W and the vector x, each read once
        for (int p = 0; p < np; ++p) {
          const double m = sz.n[p] - k - 1;
          if (m <= 0 || k >= htd_tail_start(sz.n[p])) continue;
          ctx->timer.bytes[c_hemv] += 16.0 * m * (m + 1) / 2 + 16.0 * m * (2.0 * j + 1.0);
          ctx->timer.flop[c_hemv] += 8.0 * m * m;
        }
    }
    {
      Timed tm(ctx, "trd_her2k");
      HIP_OK(launch_trd_her2k(dd, sz, p0, total([p0](int n) { return htd_her2k_blocks(n, p0); }), s));
    }
    if (timing)  // rank-2 HTD_NB update of the trailing block (Hermitian: count one triangle)
      for (int p = 0; p < np; ++p) {
        const double nbp = std::min(HTD_NB, sz.n[p] - 1 - p0);
        if (nbp <= 0 || p0 >= htd_tail_start(sz.n[p])) continue;
        const double mt = sz.n[p] - p0 - nbp;
        ctx->timer.flop[c_her2k] += 8.0 * 2.0 * nbp * mt * (mt + 1) / 2;
      }
  }
  {
    Timed tm(ctx, "trd_tail");
    HIP_OK(launch_trd_tail(dd, sz, s));
  }
  if (timing)  // unblocked tail: a Hermitian rank-2 update and a HEMV of the trailing block per column
    for (int p = 0; p < np; ++p)
      for (int k = htd_tail_start(sz.n[p]); k < sz.n[p] - 1; ++k) {
        const double mt = sz.n[p] - k - 1;
        ctx->timer.flop[c_tail] += 8.0 * 3.0 * mt * mt;
      }
  lap("reduction");
  {
    Timed tm(ctx, "dc");
    HIP_OK(launch_trd_finish(dd, sz, s));
    HIP_OK(launch_dc_init(dd, sz, total([](int n) { return n; }), s));
  }
  int Lmax = 0;
  while ((1 << Lmax) < nmax) ++Lmax;
  for (int L = 1; L <= Lmax; ++L) {
    Timed tm(ctx, "dc");
    const int nodes = total([L](int n) { return htd_nodes(n, L); });
    const int rows = total([](int n) { return htd_rows(n); });
    const int waves = total([](int n) { return htd_waves(n); });
    HIP_OK(launch_dc_prep(dd, sz, L, nodes, s));
    HIP_OK(launch_dc_rot(dd, sz, L, rows, s));
    for (int stage = 1; stage < 4; ++stage) HIP_OK(launch_dc_wave(stage, dd, sz, L, waves, s));
    HIP_OK(launch_dc_place(dd, sz, L, total([L](int n) { return htd_place_blocks(n, L); }), s));
    HIP_OK(launch_dc_gemm(dd, sz, L, total([L](int n) { return htd_gemm_tiles(n, L); }), s));
    if (timing)  // merge products of the real eigenvector blocks: two (h x h) by (h x s) per node, h = s / 2
      for (int p = 0; p < np; ++p)
        for (int a = 0; a < sz.n[p]; a += 1 << L) {
          const double sn = std::min(1 << L, sz.n[p] - a), h = sn / 2;
          ctx->timer.flop[c_dc] += 2.0 * 2.0 * h * h * sn;
        }
  }
  lap("divide and conquer");
  {
    Timed tm(ctx, "bt");
    HIP_OK(launch_bt_init(dd, sz, Lmax, total([](int n) { return htd_tiles64(n); }), s));
    HIP_OK(launch_bt_larft(dd, sz, total([](int n) { return htd_nblk(n); }), s));
  }
  int nbmax = 0;
  for (int p = 0; p < np; ++p) nbmax = std::max(nbmax, htd_nblk(sz.n[p]));
  for (int b = nbmax - 1; b >= 0; --b) {
    Timed tm(ctx, "bt");
    HIP_OK(launch_bt_wpart(dd, sz, b, total_c([b](int n, int c) { return htd_wpart_blocks(n, c, b); }), s));
    HIP_OK(launch_bt_wred(dd, sz, b, total_c([b](int n, int c) { return htd_wred_blocks(n, c, b); }), s));
    HIP_OK(launch_bt_update(dd, sz, b, total_c([b](int n, int c) { return htd_update_blocks(n, c, b); }), s));
    if (timing)  // two products of (rows x BT_NB) by (BT_NB x nc) complex
      for (int p = 0; p < np; ++p)
        if (b < htd_nblk(sz.n[p])) {
          const double rows = htd_bt_rows(sz.n[p], b), nb = std::min(BT_NB, sz.n[p] - 1 - BT_NB * b);
          ctx->timer.flop[c_bt] += 2.0 * 8.0 * rows * nb * sz.nc[p];
        }
  }
  lap("back-transformation");
}

// The buffers a kernel derives with htd_view are the ones the host laid out.
bool htd_view_matches(const HtdArgs& a, int q, const HtdDesc& h) {
  const HtdDesc g = htd_view(a, q);
  return g.d == h.d && g.e == h.e && g.tau == h.tau && g.PV == h.PV && g.PW == h.PW && g.Y == h.Y &&
         g.xb == h.xb && g.kpart == h.kpart && g.part == h.part && g.A == h.A && g.ld == h.ld &&
         g.skip == h.skip;
}

void solve_htd(mps_ctx* ctx, const HtdDesc* dd_all, const std::vector<HtdDesc>& host_all) {
  hipStream_t s = ctx->stream;
  if (host_all.empty()) return;
  std::vector<int> chi_now(std::max(0, ctx->n - 1));
  if (!chi_now.empty())
    HIP_OK(hipMemcpyAsync(chi_now.data(), ctx->d_chi, chi_now.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  // problems whose learned sketch was accepted need no exact solve: leave them
  // out of the launches (their kernels would return at once, but every column
  // would still cost two launches)
  std::vector<int> skip(host_all.size(), 0);
  for (size_t q = 0; q < host_all.size(); ++q)
    if (host_all[q].skip) HIP_OK(hipMemcpyAsync(&skip[q], host_all[q].skip, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // The problems solved here, in order, with no skip flag: every kernel of
  // the solver would otherwise read the flag from memory before its data
  // (one more dependent round trip per launch), and the host has already
  // decided.  When any problem carries a flag the descriptors are copied to
  // a device array of the handle (which also makes the chunks consecutive);
  // flagless descriptors (single solves, DMRG, the no-allocation entry
  // point) are used where they are.
  bool flagged = false;
  for (const auto& h : host_all) flagged = flagged || h.skip != nullptr;
  std::vector<HtdDesc>& host = ctx->htd_host;
  host.clear();
  for (size_t q = 0; q < host_all.size(); ++q)
    if (!skip[q]) {
      host.push_back(host_all[q]);
      host.back().skip = nullptr;
    }
  const int np = (int)host.size();
  if (np == 0) return;
  const HtdDesc* base = dd_all;
  if (flagged) {
    if ((size_t)np > ctx->htd_dev_cap) {  // the stream is idle here (synchronised above)
      if (ctx->htd_dev) HIP_OK(hipFree(ctx->htd_dev));
      ctx->htd_dev = nullptr;
      ctx->htd_dev_cap = 0;
      HIP_OK(hipMalloc(&ctx->htd_dev, (size_t)np * 2 * sizeof(HtdDesc)));
      ctx->htd_dev_cap = (size_t)np * 2;
    }
    HIP_OK(hipMemcpyAsync(ctx->htd_dev, host.data(), (size_t)np * sizeof(HtdDesc), hipMemcpyHostToDevice, s));
    base = ctx->htd_dev;
  }
  for (int c0 = 0; c0 < np; c0 += HTD_GROUP) {
    HtdSizes sz{};
    HtdArgs ha{};
    sz.np = std::min(HTD_GROUP, np - c0);
    const HtdDesc* dd = base + c0;
    for (int q = 0; q < sz.np; ++q) {
      const Dim& dm = host[c0 + q].n;
      const ptrdiff_t at = dm.ptr ? dm.ptr - ctx->d_chi : -1;
      if (dm.ptr && (at < 0 || at >= (ptrdiff_t)chi_now.size())) fail(ctx, MPS_EINVAL, "tridiagonal solve: size pointer");
      const int n = dm.ptr ? dm.mult * chi_now[at] : dm.mult;
      if (n < 1 || n > HTD_MAX) fail(ctx, MPS_EINVAL, "tridiagonal solve: size out of range");
      sz.n[q] = n;
      sz.nc[q] = std::min(n, host[c0 + q].rcap);
      const HtdDesc& h = host[c0 + q];
      ha.pr[q] = HtdProb{h.A, (char*)h.d, nullptr, n, h.ld};
      if (!htd_view_matches(ha, q, h)) fail(ctx, MPS_EINVAL, "tridiagonal solve: workspace layout");
    }
    ha.np = sz.np;
    solve_htd_chunk(ctx, dd, sz, ha);
  }
}

struct LevelDescs {
  std::vector<int> jobs;
  std::vector<GemmDesc> gram, proj;
  std::vector<GramReduceDesc> red;
  std::vector<EigDesc> eig;    // block-Jacobi solves (FP64)
  std::vector<int> eig_jobs;
  std::vector<HtdDesc> htd;   // tridiagonal solves
  std::vector<EigDesc> eig_h;  // their trace / flag initialisation
  size_t o_htd = 0, o_eig_h = 0;
  std::vector<SelectDesc> sel;
  std::vector<GatherDesc> gat;
  size_t o_gram, b_gram, o_proj, b_proj, o_red, b_red, o_sel, o_gat, b_gat;
  size_t o_eig = 0, b_pair = 0, b_upd = 0;
  int n_pair = 0, n_upd = 0;
  int n_gram, n_proj, n_red, n_gat;
  int nb_max_all;
};

int upload_gemms(DescBlob& B, const std::vector<GemmDesc>& v, size_t& off, size_t& boff) {
  std::vector<int> base{0};
  for (const auto& d : v) base.push_back(base.back() + gemm_tiles(d));
  off = B.add_vec(v);
  boff = B.add_vec(base);
  return base.back();
}

// Serialises the descriptors of one level into the step's blob.
void upload_level(DescBlob& B, LevelDescs& L) {
  L.n_gram = upload_gemms(B, L.gram, L.o_gram, L.b_gram);
  L.n_proj = upload_gemms(B, L.proj, L.o_proj, L.b_proj);
  L.n_red = 0;
  if (!L.red.empty()) {
    std::vector<int> base{0};
    for (const auto& g : L.red) base.push_back(base.back() + g.tiles);
    L.o_red = B.add_vec(L.red);
    L.b_red = B.add_vec(base);
    L.n_red = base.back();
  }
  if (!L.eig.empty()) {
    std::vector<int> pb{0}, ub{0};
    for (const auto& e : L.eig) {
      pb.push_back(pb.back() + e.nb_max / 2);
      ub.push_back(ub.back() + 2 * (e.nb_max / 2) * (e.nb_max / 2));
    }
    L.o_eig = B.add_vec(L.eig);
    L.b_pair = B.add_vec(pb);
    L.b_upd = B.add_vec(ub);
    L.n_pair = pb.back();
    L.n_upd = ub.back();
  }
  if (!L.htd.empty()) {
    L.o_htd = B.add_vec(L.htd);
    L.o_eig_h = B.add_vec(L.eig_h);
  }
  L.o_sel = B.add_vec(L.sel);
  std::vector<int> gb{0};
  for (const auto& g : L.gat) gb.push_back(gb.back() + g.tiles);
  L.o_gat = B.add_vec(L.gat);
  L.b_gat = B.add_vec(gb);
  L.n_gat = gb.back();
}

// Launches of one split level: Gram matrices, eigen-solver initialisation,
// `between` (the learned-sketch launches of the level, if any), the exact
// solves, selection, gather and projection.  flags holds the convergence
// flags of the level's jobs, 4 ints per job index, nflag_ints in all.
template <class F>
void launch_level(mps_ctx* ctx, DescBlob& B, LevelDescs& L, int* flags, int nflag_ints, F between) {
  hipStream_t s = ctx->stream;
  const Prec P = ctx->prec;
  const int np = (int)L.jobs.size();
  {
    Timed tm(ctx, "gram");
    HIP_OK(launch_gram(P == Prec::FP64 ? Prec::FP64 : Prec::FP32, B.at<GemmDesc>(L.o_gram),
                       B.at<int>(L.b_gram), np, L.n_gram, s));
  }
  if (L.n_red) {
    Timed tm(ctx, "gram_reduce");
    HIP_OK(launch_gram_reduce(B.at<GramReduceDesc>(L.o_red), B.at<int>(L.b_red), (int)L.red.size(), L.n_red, s));
  }
  int ldmax = 0;
  for (const auto& e : L.eig) ldmax = std::max(ldmax, e.ld);
  for (const auto& e : L.eig_h) ldmax = std::max(ldmax, e.ld);
  if (!L.eig_h.empty()) {
    Timed tm(ctx, "eig_init");
    HIP_OK(launch_eig_init(B.at<EigDesc>(L.o_eig_h), (int)L.eig_h.size(), ldmax, s));
  }
  if (!L.eig.empty()) {
    Timed tm(ctx, "eig_init");
    HIP_OK(launch_eig_init(B.at<EigDesc>(L.o_eig), (int)L.eig.size(), ldmax, s));
  }
  between();
  if (!L.eig.empty()) {
    std::vector<int> at;
    for (int q : L.eig_jobs) at.push_back(4 * q);
    solve_eig(ctx, B.at<EigDesc>(L.o_eig), L.eig, B.at<int>(L.b_pair), B.at<int>(L.b_upd), L.n_pair, L.n_upd,
              flags, nflag_ints, at);
  }
  if (!L.htd.empty()) solve_htd(ctx, B.at<HtdDesc>(L.o_htd), L.htd);
  {
    Timed tm(ctx, "select");
    HIP_OK(launch_select(B.at<SelectDesc>(L.o_sel), np, s));
  }
  {
    Timed tm(ctx, "gather");
    HIP_OK(launch_gather(P, B.at<GatherDesc>(L.o_gat), B.at<int>(L.b_gat), np, L.n_gat, s));
  }
  {
    Timed tm(ctx, "project");
    HIP_OK(launch_gemm_nn(P, B.at<GemmDesc>(L.o_proj), B.at<int>(L.b_proj), np, L.n_proj, s));
  }
}

// Descriptors of split level t of job run r (index i in the caller's job
// list, which also indexes its convergence flags) appended to L; skr is the
// split's learned-sketch run or null.  Advances r's buffer parity.
void add_level(mps_ctx* ctx, LevelDescs& L, JobRun& r, int i, int t, const SkRun* skr) {
  L.jobs.push_back(i);
  const Level& lv = r.lv[t];
  const int m = lv.m;
  const Dim n2c = c_dim(ctx, r, t, 2);
  void* X = r.buf[r.cur];
  void* Y = r.buf[r.cur ^ 1];
  {
    GemmDesc d{};
    d.A = X;
    d.B = X;
    d.C = lv.ksplit > 1 ? (void*)r.part : (void*)r.G;
    d.M = n2c;
    d.N = n2c;
    d.K = fixed(lv.rows);
    d.lda = n2c;
    d.ldb = n2c;
    d.ldc = fixed(r.ld);
    d.batch = 1;
    d.tm = d.tn = ceil_div(2 * lv.c_bound, 64);
    d.ksplit = lv.ksplit;
    d.part = (int64_t)r.ld * r.ld;
    d.w = r.a > 0 ? ctx->lam[r.a - 1] : ctx->d_ones;
    d.wshift = m;
    d.alpha = 1.0;
    L.gram.push_back(d);
    if (lv.ksplit > 1) {
      GramReduceDesc g{};
      g.part = r.part;
      g.G = r.G;
      g.n = n2c;
      g.ld = fixed(r.ld);
      g.ksplit = lv.ksplit;
      g.stride = (int64_t)r.ld * r.ld;
      const int T = ceil_div(2 * lv.c_bound, 64);
      g.tiles = T * T;
      L.red.push_back(g);
    }
  }
  {
    const bool uh = level_htd(ctx, lv);
    EigDesc e{};
    e.G = r.G;
    e.V = r.V;
    e.J = r.J;
    e.Gw = r.G;
    e.Vw = r.V;
    e.pair_rot = r.pair_rot;
    e.flags = r.flags;
    e.scale = r.scale;
    e.work = ctx->timing ? ctx->d_work : nullptr;
    e.n = n2c;
    e.ld = r.ld;
    int nb = ceil_div(2 * lv.c_bound, JB);
    nb = std::max(nb, 2);
    nb += nb & 1;
    e.nb_max = nb;
    e.tol = 1e-13;
    if (uh) {
      L.eig_h.push_back(e);
      HtdDesc h = r.hw;
      h.A = r.G;
      h.V = r.V;
      h.n = n2c;
      h.ld = r.ld;
      h.rcap = lv.r_bound;
      h.skip = r.flags;
      L.htd.push_back(h);
    } else {
      L.nb_max_all = std::max(L.nb_max_all, nb);
      L.eig.push_back(e);
      L.eig_jobs.push_back(i);
    }
  }
  int* r_out = ctx->d_chi + (r.a + m - 1);
  {
    const bool uh = level_htd(ctx, lv);
    SelectDesc sd{};
    sd.G = r.G;
    sd.lam_in = uh ? r.hw.lam : nullptr;
    sd.ldg = r.ld;
    sd.n = n2c;
    sd.rows = lv.rows;
    sd.chi_max = ctx->chi_max;
    sd.eps_eff = ctx->eps_eff;
    sd.perm = r.perm;
    sd.r_out = r_out;
    sd.lam_out = ctx->lam[r.a + m - 1];
    sd.logf_acc = r.logf;
    sd.rec = r.rec + 4 * t;
    if (skr) {
      const SkRun& k = *skr;
      sd.use_sk = k.use;
      sd.lam_sk = k.lam;
      sd.tot_sk = r.scale;
      sd.s_sk = k.s;
    }
    L.sel.push_back(sd);
  }
  {
    GatherDesc g{};
    g.V = r.V;
    g.ldv = r.ld;
    g.perm = r.perm;
    g.r = r_out;
    g.n = n2c;
    g.B = ctx->site[r.a + m];
    g.Vr = r.Vr;
    g.tiles = ceil_div(lv.r_bound, 64) * ceil_div(2 * lv.c_bound, 64);
    if (skr) {
      const SkRun& k = *skr;
      g.use_sk = k.use;
      g.Vs = k.Vs;
      g.ld_sk = k.ld_s;
    }
    L.gat.push_back(g);
  }
  {
    GemmDesc d{};
    d.A = X;
    d.B = r.Vr;
    d.C = Y;
    d.M = fixed(lv.rows);
    d.K = n2c;
    d.N = Dim{1, r_out};
    d.lda = n2c;
    d.ldb = Dim{1, r_out};
    d.ldc = Dim{1, r_out};
    d.batch = 1;
    d.tm = ceil_div(lv.rows, 64);
    d.tn = ceil_div(lv.r_bound, 64);
    d.ksplit = 1;
    d.alpha = 1.0;
    L.proj.push_back(d);
  }
  r.cur ^= 1;
}

struct SkLevel {
  std::vector<int> ids;
  std::vector<SketchDesc> sd;
  std::vector<EigDesc> ea, eb;
  std::vector<GemmDesc> g[13];  // Y, Y^H Y, Q, G Q, H, Vs, C8, R1, R2, two Newton-Schulz steps
  size_t o_sd = 0, o_ea = 0, o_eb = 0, bp_a = 0, bu_a = 0, bp_b = 0, bu_b = 0;
  size_t o[13] = {0}, b[13] = {0};
  int n[13] = {0};
  int np_a = 0, nu_a = 0, np_b = 0, nu_b = 0;
  std::vector<int> flag_a, flag_b;
};

// Descriptors of one learned-sketch range finder (problem q of its level, its
// flags at 12 q of the level's flag array) on the Gram matrix G (leading
// dimension ld, size n2c, bound nb); trace: the device value of trace(G);
// exact_flags: set when the sketch is accepted (the exact solve is skipped).
void add_sketch(mps_ctx* ctx, SkLevel& S, SkRun& k, int q, double2* G, int ld, Dim n2c, int nb, double* trace,
                int* exact_flags) {
  const Dim fs = fixed(k.s), fls = fixed(k.ld_s), fly = fixed(k.ld_y), fld = fixed(ld), f8 = fixed(SK_PROBES);
  SketchDesc d{};
  d.n = n2c;
  d.s = k.s;
  d.ld_s = k.ld_s;
  d.ld_y = k.ld_y;
  d.seed = ctx->sketch_seed;
  d.stream = ctx->sketch_stream++;
  d.Omega = k.Omega;
  d.Probe = k.Probe;
  d.Bq = k.Bq;
  d.R1 = k.R1;
  d.R2 = k.R2;
  d.Gy = k.Gy;
  d.Uy = k.Uy;
  d.Hw = k.Hw;
  d.lam = k.lam;
  d.trace = trace;
  d.eps_eff = ctx->eps_eff;
  d.use = k.use;
  d.est = k.est;
  d.exact_flags = exact_flags;
  S.sd.push_back(d);
  S.g[0].push_back(gemm64(G, k.Omega, k.Y, n2c, fs, n2c, fld, fls, fls, nb, k.s));  // Y = G Omega
  {
    GemmDesc g = gemm64(k.Y, k.Y, k.Gy, fs, fs, n2c, fls, fls, fly, k.s, k.s);     // Y^H Y
    g.w = ctx->d_ones;
    g.wshift = 0;
    S.g[1].push_back(g);
  }
  S.g[2].push_back(gemm64(k.Y, k.Bq, k.Q, n2c, fs, fs, fls, fls, fls, nb, k.s));      // Q = Y Bq
  S.g[3].push_back(gemm64(G, k.Q, k.Y, n2c, fs, n2c, fld, fls, fls, nb, k.s));      // G Q (into Y)
  S.g[4].push_back(gemm64(k.Q, k.Y, k.Hw, fs, fs, n2c, fls, fls, fly, k.s, k.s));     // H = Q^H G Q
  S.g[5].push_back(gemm64(k.Q, k.Wh, k.Vs, n2c, fs, fs, fls, fly, fls, nb, k.s));     // Vs = Q W
  S.g[6].push_back(gemm64(k.Q, k.Probe, k.C8, fs, f8, n2c, fls, fls, fls, k.s, SK_PROBES));  // Q^H g
  S.g[7].push_back(gemm64(G, k.Probe, k.R1, n2c, f8, n2c, fld, fls, fls, nb, SK_PROBES));  // G g
  S.g[8].push_back(gemm64(k.Y, k.C8, k.R2, n2c, f8, fs, fls, fls, fls, nb, SK_PROBES));      // G Q Q^H g
  for (int it = 0; it < 2; ++it) {  // Newton-Schulz: S = X^H X, X' = X (1.5 I - 0.5 S)
    double2* from = it == 0 ? k.Q : k.Vs;
    double2* to = it == 0 ? k.Vs : k.Q;
    GemmDesc g = gemm64(from, from, k.Gy, fs, fs, n2c, fls, fls, fly, k.s, k.s);
    g.w = ctx->d_ones;
    g.wshift = 0;
    S.g[9 + 2 * it].push_back(g);
    S.g[10 + 2 * it].push_back(gemm64(from, k.Bq, to, n2c, fs, fs, fls, fls, fls, nb, k.s));
  }
  EigDesc ea{};
  ea.G = k.Gy;
  ea.V = k.Uy;
  ea.Gw = k.Gy;
  ea.Vw = k.Uy;
  ea.J = k.Ja;
  ea.pair_rot = k.pr_a;
  ea.flags = k.flags_a;
  ea.scale = k.scale_a;
  ea.work = ctx->timing ? ctx->d_work : nullptr;
  ea.n = fs;
  ea.ld = k.ld_y;
  ea.nb_max = k.nb;
  ea.tol = 1e-13;
  EigDesc eb = ea;
  eb.G = k.Hw;
  eb.V = k.Wh;
  eb.Gw = k.Hw;
  eb.Vw = k.Wh;
  eb.J = k.Jb;
  eb.pair_rot = k.pr_b;
  eb.flags = k.flags_b;
  eb.scale = k.scale_b;
  S.ea.push_back(ea);
  S.eb.push_back(eb);
  S.flag_a.push_back(12 * q);
  S.flag_b.push_back(12 * q + 4);
}

void upload_sketch(DescBlob& B, SkLevel& S) {
  S.o_sd = B.add_vec(S.sd);
  for (int g = 0; g < 13; ++g) S.n[g] = upload_gemms(B, S.g[g], S.o[g], S.b[g]);
  std::vector<int> pa{0}, ua{0};
  for (const auto& e : S.ea) {
    pa.push_back(pa.back() + e.nb_max / 2);
    ua.push_back(ua.back() + 2 * (e.nb_max / 2) * (e.nb_max / 2));
  }
  S.o_ea = B.add_vec(S.ea);
  S.o_eb = B.add_vec(S.eb);
  S.bp_a = B.add_vec(pa);
  S.bu_a = B.add_vec(ua);
  S.np_a = pa.back();
  S.nu_a = ua.back();
}

// Launches of one level's range finders; fill: draw the Gaussian test and
// probe matrices on the device (else they are already in place).
void launch_sketch(mps_ctx* ctx, DescBlob& B, SkLevel& S, const std::vector<SkRun>& sk, int* skflags_all, int nsk,
                   bool fill) {
  hipStream_t s = ctx->stream;
  // learned sketch of this level's predicted-low-rank splits
  const int ns = (int)S.ids.size();
  SketchDesc* dsk = B.at<SketchDesc>(S.o_sd);
  auto nn = [&](int g) { HIP_OK(launch_gemm_nn(Prec::FP64, B.at<GemmDesc>(S.o[g]), B.at<int>(S.b[g]), ns, S.n[g], s)); };
  auto cn = [&](int g) { HIP_OK(launch_gemm_cn(B.at<GemmDesc>(S.o[g]), B.at<int>(S.b[g]), ns, S.n[g], s)); };
  int ldy = 0;
  for (int q : S.ids) ldy = std::max(ldy, sk[q].ld_y);
  {
    Timed tm(ctx, "sketch");
    if (fill) {
      HIP_OK(launch_gauss_fill(dsk, ns, 0, s));
      HIP_OK(launch_gauss_fill(dsk, ns, 1, s));
    }
    nn(0);
    HIP_OK(launch_gram(Prec::FP64, B.at<GemmDesc>(S.o[1]), B.at<int>(S.b[1]), ns, S.n[1], s));
    HIP_OK(launch_eig_init(B.at<EigDesc>(S.o_ea), ns, ldy, s));
  }
  solve_eig(ctx, B.at<EigDesc>(S.o_ea), S.ea, B.at<int>(S.bp_a), B.at<int>(S.bu_a), S.np_a, S.nu_a,
            skflags_all, 12 * nsk, S.flag_a, true);
  {
    Timed tm(ctx, "sketch");
    HIP_OK(launch_orth_scale(dsk, ns, s));
    nn(2);
    for (int it = 0; it < 2; ++it) {
      HIP_OK(launch_gram(Prec::FP64, B.at<GemmDesc>(S.o[9 + 2 * it]), B.at<int>(S.b[9 + 2 * it]), ns,
                         S.n[9 + 2 * it], s));
      HIP_OK(launch_newton_schulz(dsk, ns, s));
      nn(10 + 2 * it);
    }
    nn(3);
    cn(4);
    HIP_OK(launch_eig_init(B.at<EigDesc>(S.o_eb), ns, ldy, s));
  }
  solve_eig(ctx, B.at<EigDesc>(S.o_eb), S.eb, B.at<int>(S.bp_a), B.at<int>(S.bu_a), S.np_a, S.nu_a,
            skflags_all, 12 * nsk, S.flag_b, true);
  {
    Timed tm(ctx, "sketch");
    nn(5);
    cn(6);
    nn(7);
    nn(8);
    HIP_OK(launch_sketch_accept(dsk, ns, s));
  }
}

void run_group(mps_ctx* ctx, std::vector<Job>& jobs, const std::vector<Site1QDesc>& sites1q, int nsub) {
  hipStream_t s = ctx->stream;
  const Prec P = ctx->prec;
  std::vector<JobRun> runs(jobs.size());
  size_t bytes = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    plan_job(ctx, jobs[i], runs[i]);
    bytes += job_bytes(ctx, runs[i]);
  }
  const int nj = (int)jobs.size();

  // ---- learned sketch: features of every split, predicted kept ranks
  std::vector<float> feats;
  std::vector<int> lv_job, lv_t;
  for (int i = 0; i < nj; ++i) {
    job_features(ctx, runs[i], jobs[i], nsub, feats);
    for (size_t t = 0; t < runs[i].lv.size(); ++t) {
      lv_job.push_back(i);
      lv_t.push_back((int)t);
    }
  }
  const int nlev = (int)lv_job.size();
  std::vector<SkRun> sk;
  std::vector<std::vector<int>> sk_of(nj);  // per job: sketch index per level or -1
  for (int i = 0; i < nj; ++i) sk_of[i].assign(runs[i].lv.size(), -1);
  if (ctx->opt.svd_mode == MPS_SVD_LEARNED && ctx->mlp_params && nlev > 0) {
    std::vector<float> pred(nlev);
    float *dX = nullptr, *dy = nullptr;
    HIP_OK(hipMalloc(&dX, feats.size() * sizeof(float)));
    HIP_OK(hipMalloc(&dy, nlev * sizeof(float)));
    HIP_OK(hipMemcpyAsync(dX, feats.data(), feats.size() * sizeof(float), hipMemcpyHostToDevice, s));
    {
      Timed tm(ctx, "mlp_forward");
      HIP_OK(launch_mlp_forward(ctx->mlp_params, dX, dy, nlev, s));
    }
    HIP_OK(hipMemcpyAsync(pred.data(), dy, nlev * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    (void)hipFree(dX);
    (void)hipFree(dy);
    for (int q = 0; q < nlev; ++q) {
      const Level& L = runs[lv_job[q]].lv[lv_t[q]];
      const int n = 2 * L.c_bound;
      const double rhat = std::exp2((double)std::min(pred[q], 30.f));
      int ssz = (int)std::ceil(rhat) + 8;  // oversampling p = 8
      if (n < 128 || ssz > n / 2 || rhat + 8 >= ctx->chi_max) continue;  // exact is cheaper or cap binds
      ssz = std::max(ssz, 16);
      SkRun k;
      k.job = lv_job[q];
      k.t = lv_t[q];
      k.s = ssz;
      k.ld_s = ((std::max(ssz, SK_PROBES) + 7) / 8) * 8;
      k.ld_y = ((ssz + 63) / 64) * 64;
      int nb = ceil_div(ssz, JB);
      nb = std::max(nb, 2);
      k.nb = nb + (nb & 1);
      sk_of[k.job][k.t] = (int)sk.size();
      sk.push_back(k);
      bytes += sk_bytes(n, k);
    }
  }
  const int nsk = (int)sk.size();

  bytes += (size_t)nj * (sizeof(double) + 4 * sizeof(int)) + (size_t)nsk * (12 * sizeof(int) + 2 * sizeof(double)) +
           8192;
  ctx->arena.reset();
  HIP_OK(ctx->arena.reserve(bytes));
  int* skflags_all = (int*)ctx->arena.take(std::max(1, nsk) * 12 * sizeof(int));
  double* skscale_all = (double*)ctx->arena.take(std::max(1, nsk) * 2 * sizeof(double));
  for (int q = 0; q < nsk; ++q)
    sk_assign(ctx->arena, sk[q], 2 * runs[sk[q].job].lv[sk[q].t].c_bound, skflags_all + 12 * q,
              skscale_all + 2 * q);
  double* logf_all = (double*)ctx->arena.take(std::max(1, nj) * sizeof(double));
  int* flags_all = (int*)ctx->arena.take(std::max(1, nj) * 4 * sizeof(int));
  for (int i = 0; i < nj; ++i) {
    assign_job(ctx, runs[i], ctx->arena);
    runs[i].logf = logf_all + i;
    runs[i].flags = flags_all + 4 * i;
    runs[i].flag_index = i;
  }
  if (nj) HIP_OK(hipMemsetAsync(logf_all, 0, nj * sizeof(double), s));
  if (ctx->timing) HIP_OK(hipMemsetAsync(ctx->d_work, 0, 4 * sizeof(unsigned long long), s));

  DescBlob& B = ctx->blob;
  B.host.clear();
  int kmax = 0;
  for (auto& r : runs) kmax = std::max(kmax, r.k);

  // ---- unitaries
  std::vector<UnitaryDesc> ud;
  std::vector<int> ubase{0};
  size_t ulds = 0;
  std::vector<size_t> gate_off(nj, 0);
  for (int i = 0; i < nj; ++i) {
    const Job& jb = jobs[i];
    if (!jb.U.empty()) continue;
    std::vector<UGate> ug;
    for (const auto& g : jb.gates) {
      UGate u{};
      u.nq = g.nq;
      u.q0 = g.q[0] - jb.a;
      u.q1 = g.nq > 1 ? g.q[1] - jb.a : 0;
      const int dd = 1 << (2 * g.nq);
      for (int e = 0; e < dd; ++e) {
        u.u[2 * e] = g.u[e].real();
        u.u[2 * e + 1] = g.u[e].imag();
      }
      ug.push_back(u);
    }
    gate_off[i] = ug.empty() ? 0 : B.add_vec(ug);
    UnitaryDesc d{};
    d.ngates = (int)ug.size();
    d.k = jb.k;
    d.U64 = (double2*)runs[i].U64;
    d.U32 = (P == Prec::FP64) ? nullptr : (float2*)runs[i].Uw;
    const int dim = 1 << jb.k;
    d.cols = std::max(1, std::min(16, 4096 / dim));
    d.blocks = ceil_div(dim, d.cols);
    ulds = std::max(ulds, (size_t)d.cols * dim * sizeof(double2));
    ud.push_back(d);
    ubase.push_back(ubase.back() + d.blocks);
  }
  std::vector<int> ud_job;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].U.empty()) ud_job.push_back(i);

  // ---- merges (j = 1..kmax-1), unitary application
  std::vector<std::vector<GemmDesc>> mg(kmax);
  for (auto& r : runs) {
    for (int j = 1; j < r.k; ++j) {
      GemmDesc d{};
      const int M = r.chi_l << j;
      const int K = r.mid[j - 1];
      const int N = 2 * ((j == r.k - 1) ? r.chi_r : r.mid[j]);
      d.A = (j == 1) ? ctx->site[r.a] : r.buf[(j - 1) & 1];
      d.B = ctx->site[r.a + j];
      d.C = r.buf[j & 1];
      d.M = fixed(M);
      d.N = fixed(N);
      d.K = fixed(K);
      d.lda = fixed(K);
      d.ldb = fixed(N);
      d.ldc = fixed(N);
      d.batch = 1;
      d.tm = ceil_div(M, 64);
      d.tn = ceil_div(N, 64);
      d.ksplit = 1;
      d.alpha = 1.0;
      mg[j].push_back(d);
    }
    r.cur = (r.k - 1) & 1;
  }
  std::vector<GemmDesc> ap;
  for (auto& r : runs) {
    GemmDesc d{};
    const int D = 1 << r.k;
    d.A = r.Uw;
    d.B = r.buf[r.cur];
    d.C = r.buf[r.cur ^ 1];
    d.M = fixed(D);
    d.N = fixed(r.chi_r);
    d.K = fixed(D);
    d.lda = fixed(D);
    d.ldb = fixed(r.chi_r);
    d.ldc = fixed(r.chi_r);
    d.sA = 0;
    d.sB = d.sC = (int64_t)D * r.chi_r;
    d.batch = r.chi_l;
    d.tm = ceil_div(D, 64);
    d.tn = ceil_div(r.chi_r, 64);
    d.ksplit = 1;
    d.alpha = 1.0;
    ap.push_back(d);
    r.cur ^= 1;
  }

  auto upload_gemm = [&](const std::vector<GemmDesc>& v, size_t& off, size_t& boff) {
    return upload_gemms(B, v, off, boff);
  };

  // Split levels: descriptors are built for every level up front.
  const int tmax = kmax - 1;
  std::vector<LevelDescs> LD(std::max(0, tmax));
  for (int t = 0; t < tmax; ++t) {
    LevelDescs& L = LD[t];
    L.nb_max_all = 0;
    for (int i = 0; i < nj; ++i) {
      if (t >= runs[i].k - 1) continue;
      add_level(ctx, L, runs[i], i, t, sk_of[i][t] >= 0 ? &sk[sk_of[i][t]] : nullptr);
    }
  }
  // Learned-sketch descriptors per level: range finder on G, two s x s solves,
  // residual probes, acceptance (see sketch.hip).
  std::vector<SkLevel> SL(std::max(0, tmax));
  for (int q = 0; q < nsk; ++q) {
    SkRun& k = sk[q];
    JobRun& r = runs[k.job];
    SL[k.t].ids.push_back(q);
    add_sketch(ctx, SL[k.t], k, q, r.G, r.ld, c_dim(ctx, r, k.t, 2), 2 * r.lv[k.t].c_bound, r.scale, r.flags);
  }

  std::vector<ScaleDesc> fin;
  std::vector<int> fbase{0};
  for (auto& r : runs) {
    ScaleDesc d{};
    d.X = r.buf[r.cur];
    d.B = ctx->site[r.a];
    d.count = Dim{2 * r.chi_l, ctx->d_chi + r.a};
    d.logf = r.logf;
    const int64_t bound = (int64_t)2 * r.chi_l * std::min(ctx->chi_max, 2 * r.chi_l);
    d.blocks = std::max(1, std::min(1024, ceil_div(bound, 256)));
    fin.push_back(d);
    fbase.push_back(fbase.back() + d.blocks);
  }
  std::vector<int> sbase{0};
  for (const auto& d : sites1q) sbase.push_back(sbase.back() + d.blocks);

  // ---- serialise descriptors
  size_t o_ud = 0, b_ud = 0;
  if (!ud.empty()) {
    o_ud = B.add_vec(ud);
    b_ud = B.add_vec(ubase);
  }
  std::vector<size_t> o_mg(kmax, 0), b_mg(kmax, 0);
  std::vector<int> n_mg(kmax, 0);
  for (int j = 1; j < kmax; ++j) n_mg[j] = upload_gemm(mg[j], o_mg[j], b_mg[j]);
  size_t o_ap = 0, b_ap = 0;
  const int n_ap = nj ? upload_gemm(ap, o_ap, b_ap) : 0;
  for (auto& L : LD) upload_level(B, L);
  for (auto& S : SL)
    if (!S.ids.empty()) upload_sketch(B, S);
  size_t o_fin = 0, b_fin = 0;
  if (nj) {
    o_fin = B.add_vec(fin);
    b_fin = B.add_vec(fbase);
  }
  size_t o_s1 = 0, b_s1 = 0;
  if (!sites1q.empty()) {
    o_s1 = B.add_vec(sites1q);
    b_s1 = B.add_vec(sbase);
  }
  HIP_OK(B.prepare());
  // gate pointers of the unitary descriptors, now that the blob has a device address
  for (size_t q = 0; q < ud.size(); ++q) {
    UnitaryDesc* d = B.host_at<UnitaryDesc>(o_ud) + q;
    d->gates = d->ngates ? B.at<UGate>(gate_off[ud_job[q]]) : nullptr;
  }
  HIP_OK(B.upload(s));

  // ---- launches
  if (!ud.empty()) {
    Timed tm(ctx, "unitary");
    HIP_OK(launch_build_unitary(B.at<UnitaryDesc>(o_ud), B.at<int>(b_ud), (int)ud.size(), ubase.back(), ulds, s));
  }
  for (int i = 0; i < nj; ++i) {
    if (jobs[i].U.empty()) continue;
    const size_t dimU = (size_t)1 << (2 * jobs[i].k);
    HIP_OK(hipMemcpyAsync(runs[i].U64, jobs[i].U.data(), dimU * sizeof(double2), hipMemcpyHostToDevice, s));
    if (P != Prec::FP64) HIP_OK(launch_convert_d2f((const double2*)runs[i].U64, (float2*)runs[i].Uw, dimU, s));
  }
  for (int j = 1; j < kmax; ++j) {
    Timed tm(ctx, "merge");
    HIP_OK(launch_gemm_nn(P, B.at<GemmDesc>(o_mg[j]), B.at<int>(b_mg[j]), (int)mg[j].size(), n_mg[j], s));
  }
  if (nj) {
    Timed tm(ctx, "apply");
    HIP_OK(launch_gemm_nn(P, B.at<GemmDesc>(o_ap), B.at<int>(b_ap), nj, n_ap, s));
  }
  for (int t = 0; t < tmax; ++t) {
    launch_level(ctx, B, LD[t], flags_all, 4 * nj, [&] {
      if (!SL[t].ids.empty()) launch_sketch(ctx, B, SL[t], sk, skflags_all, nsk, true);
    });
  }
  if (nj) {
    Timed tm(ctx, "finalize");
    HIP_OK(launch_finalize(P, B.at<ScaleDesc>(o_fin), B.at<int>(b_fin), nj, fbase.back(), s));
    HIP_OK(launch_accumulate(logf_all, nj, ctx->d_logf, s));
  }
  if (!sites1q.empty()) {
    Timed tm(ctx, "one_qubit");
    HIP_OK(launch_apply_1q(P, B.at<Site1QDesc>(o_s1), B.at<int>(b_s1), (int)sites1q.size(), sbase.back(), s));
  }
  // ---- end of step: bond dimensions and per-SVD records back to the host
  std::vector<double> rec;
  size_t nrec = 0;
  for (auto& r : runs) nrec += 4 * (r.k - 1);
  rec.resize(nrec);
  HIP_OK(hipMemcpyAsync(ctx->chi.data(), ctx->d_chi, (ctx->n - 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  {
    size_t off = 0;
    for (auto& r : runs) {
      HIP_OK(hipMemcpyAsync(rec.data() + off, r.rec, 4 * (r.k - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      off += 4 * (r.k - 1);
    }
  }
  unsigned long long eig_work[2] = {0, 0};
  if (ctx->timing)
    HIP_OK(hipMemcpyAsync(eig_work, ctx->d_work, sizeof(eig_work), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (ctx->timing) {
    collect_timing(ctx);
    account_flops(ctx, runs, (double)eig_work[0], (double)eig_work[1]);
  }
  for (size_t q = 0; q < nrec; q += 4) ctx->stats.discarded_weight += rec[q + 2];
  {
    size_t off = 0;
    for (auto& r : runs) {
      record_tails(ctx, r, rec.data() + off);
      off += 4 * (r.k - 1);
    }
  }
  if (nsk) {
    std::vector<int> skf(12 * nsk);
    HIP_OK(hipMemcpy(skf.data(), skflags_all, skf.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (int q = 0; q < nsk; ++q) {
      if (skf[12 * q + 8])
        ctx->stats.sketch_accepted += 1;
      else
        ctx->stats.sketch_fallback += 1;
    }
    if (kDebugTrace && std::getenv("CTEBD_SKETCH_TRACE")) {
      for (int q = 0; q < nsk; ++q) {
        double est[2];
        HIP_OK(hipMemcpy(est, sk[q].est, sizeof(est), hipMemcpyDeviceToHost));
        const JobRun& r = runs[sk[q].job];
        const Level& L = r.lv[sk[q].t];
        std::fprintf(stderr, "sketch n=%d s=%d kept=%d accepted=%d est/trace=%.3e\n", 2 * L.c_bound, sk[q].s,
                     ctx->chi[r.a + L.m - 1], skf[12 * q + 8], est[1] > 0 ? est[0] / est[1] : -1.0);
      }
    }
  }
  // (features, log2 kept rank) of every split, for training the network
  if (ctx->log_t.size() < (size_t)4000000) {
    for (int q = 0; q < nlev; ++q) {
      const JobRun& r = runs[lv_job[q]];
      const int rk = ctx->chi[r.a + r.lv[lv_t[q]].m - 1];
      ctx->log_x.insert(ctx->log_x.end(), feats.begin() + (size_t)q * N_FEAT, feats.begin() + (size_t)(q + 1) * N_FEAT);
      ctx->log_t.push_back(std::log2((float)rk));
    }
  }
  ctx->stats.cluster_updates += nj;
  for (auto& r : runs) ctx->stats.svds += r.k - 1;
  ctx->stats.site_updates += (int64_t)sites1q.size();
}

void run_jobs(mps_ctx* ctx, std::vector<Job>& jobs, const std::vector<Site1QDesc>& sites1q, int nsub) {
  if (ctx->opt.batch == MPS_BATCH_NONE && jobs.size() > 1) {
    for (size_t i = 0; i < jobs.size(); ++i) {
      std::vector<Job> one{jobs[i]};
      run_group(ctx, one, i + 1 == jobs.size() ? sites1q : std::vector<Site1QDesc>{}, nsub);
    }
  } else {
    run_group(ctx, jobs, sites1q, nsub);
  }
  ctx->stats.steps += 1;
}

int execute_step(mps_ctx* ctx, int end_hint);

// ------------------------------------------------ wavefront executor --
// The clusters of several consecutive steps (the "window") run as a
// dependency graph instead of step by step.  A cluster on sites a..a+k-1
// reads those sites and the Schmidt values of bond a-1 and writes the sites
// and its inner bonds a..a+k-2; it waits for the last earlier writer of each
// site and of bond a-1, and for every earlier reader of an inner bond (which
// still weights its Gram matrices with it).  One-qubit site updates wait for
// the last writer of their site.  Execution proceeds in rounds: every cluster
// whose inputs are final starts (unitary, merge chain, unitary application)
// and every running cluster takes its next split level, all in the same
// launches as the step executor builds them for one step, so each cluster
// computes exactly what the step executor computes (only the sum of log f is
// added up in another order).  A k-qubit cluster runs k-1 rounds.  The window
// is planned up front, which is exact because the plan does not depend on
// the bond dimensions when Eq. cond_cTEBD cannot bind (q_max at its default).
struct WaveTask {
  bool site = false;   // one-qubit update of site q (else a cluster)
  Job job;
  int q = -1;
  std::array<cplx, 4> u1{};
  int nsub = 0;        // sub-layers of the task's step (a feature of its splits)
  std::vector<int> deps;
  int state = 0;       // 0 waiting, 1 running, 2 done
  int level = 0;       // split level to run next
  JobRun run;
  char* ws = nullptr;  // workspace block of the pool
  size_t ws_cap = 0;
  std::vector<float> feats;
};

bool plan_is_chi_free(const mps_ctx* ctx) {
  return ctx->q_max_eff >= default_q_max(ctx->opt.k_max, ctx->chi_max);
}

// Tasks of the next `nsteps` planned steps (all buffered sub-layers when
// nsteps < 0); returns the number of sub-layers they consume.
int plan_window(mps_ctx* ctx, int nsteps, std::vector<WaveTask>& T, int* steps_out) {
  const int n = ctx->n;
  std::vector<int> last_site(n, -1), last_bond(std::max(0, n - 1), -1);
  std::vector<std::vector<int>> readers(std::max(0, n - 1));
  int start = 0, steps = 0;
  const int total = (int)ctx->pending.size();
  while (start < total && (nsteps < 0 || steps < nsteps)) {
    std::vector<Cluster> cl;
    const int end = plan_step(ctx->pending, start, n, ctx->chi, ctx->opt.k_max, ctx->q_max_eff,
                              ctx->l_max_eff, cl);
    std::vector<int> owner(n, -1);
    const int base = (int)T.size();
    for (size_t c = 0; c < cl.size(); ++c) {
      WaveTask w;
      w.job.a = cl[c].a;
      w.job.k = cl[c].k;
      w.nsub = end - start;
      T.push_back(std::move(w));
      for (int q = cl[c].a; q < cl[c].a + cl[c].k; ++q) owner[q] = base + (int)c;
    }
    std::vector<int> site_task(n, -1);
    for (int sl = start; sl < end; ++sl)
      for (const auto& g : ctx->pending[sl]) {
        const int o = owner[g.q[0]];
        if (o >= 0) {
          T[o].job.gates.push_back(g);
          continue;
        }
        const int q = g.q[0];
        if (site_task[q] < 0) {
          site_task[q] = (int)T.size();
          WaveTask w;
          w.site = true;
          w.q = q;
          w.u1 = {cplx(1), cplx(0), cplx(0), cplx(1)};
          T.push_back(std::move(w));
        }
        auto& m = T[site_task[q]].u1;
        std::array<cplx, 4> r;
        r[0] = g.u[0] * m[0] + g.u[1] * m[2];
        r[1] = g.u[0] * m[1] + g.u[1] * m[3];
        r[2] = g.u[2] * m[0] + g.u[3] * m[2];
        r[3] = g.u[2] * m[1] + g.u[3] * m[3];
        m = r;
      }
    for (int t = base; t < (int)T.size(); ++t) {
      WaveTask& w = T[t];
      auto dep = [&](int d) {
        if (d >= 0 && std::find(w.deps.begin(), w.deps.end(), d) == w.deps.end()) w.deps.push_back(d);
      };
      if (w.site) {
        dep(last_site[w.q]);
        last_site[w.q] = t;
        continue;
      }
      const int a = w.job.a, k = w.job.k;
      for (int q = a; q < a + k; ++q) dep(last_site[q]);
      if (a > 0) dep(last_bond[a - 1]);
      for (int b = a; b < a + k - 1; ++b)
        for (int rd : readers[b]) dep(rd);
      for (int q = a; q < a + k; ++q) last_site[q] = t;
      for (int b = a; b < a + k - 1; ++b) {
        last_bond[b] = t;
        readers[b].clear();
      }
      if (a > 0) readers[a - 1].push_back(t);
    }
    start = end;
    ++steps;
  }
  if (steps_out) *steps_out = steps;
  return start;
}

// One round: the site updates and cluster starts in `sites` / `starting`,
// the next split level of every task in `active` (the starting ones included),
// the final scaling of the tasks whose last level this is.
void wave_round(mps_ctx* ctx, std::vector<WaveTask>& T, const std::vector<int>& sites,
                const std::vector<int>& starting, const std::vector<int>& active) {
  hipStream_t s = ctx->stream;
  const Prec P = ctx->prec;
  // workspaces of the starting clusters
  for (int i : starting) {
    WaveTask& w = T[i];
    plan_job(ctx, w.job, w.run);
    const size_t bytes = job_bytes(ctx, w.run) + 4096;
    HIP_OK(ctx->pool.get(bytes, &w.ws, &w.ws_cap));
    DeviceArena view;
    view.base = w.ws;
    view.cap = w.ws_cap;
    assign_job(ctx, w.run, view);
    w.run.logf = (double*)view.take(sizeof(double));
    HIP_OK(hipMemsetAsync(w.run.logf, 0, sizeof(double), s));
    job_features(ctx, w.run, w.job, w.nsub, w.feats);
    if (ctx->timing) account_merge(ctx, w.run);
  }
  const int na = (int)active.size();
  ctx->arena.reset();
  HIP_OK(ctx->arena.reserve((size_t)std::max(1, na) * 4 * sizeof(int) + 4096));
  int* flags_round = (int*)ctx->arena.take((size_t)std::max(1, na) * 4 * sizeof(int));
  for (int p = 0; p < na; ++p) {
    JobRun& r = T[active[p]].run;
    r.flags = flags_round + 4 * p;
    r.flag_index = p;
  }
  if (ctx->timing) HIP_OK(hipMemsetAsync(ctx->d_work, 0, 4 * sizeof(unsigned long long), s));

  DescBlob& B = ctx->blob;
  B.host.clear();
  // one-qubit site updates
  std::vector<Site1QDesc> s1;
  std::vector<int> sbase{0};
  for (int i : sites) {
    const WaveTask& w = T[i];
    Site1QDesc d{};
    d.B = ctx->site[w.q];
    d.chi_l = bond_dim(ctx, w.q - 1);
    d.chi_r = bond_dim(ctx, w.q);
    for (int e = 0; e < 4; ++e) {
      d.u[2 * e] = w.u1[e].real();
      d.u[2 * e + 1] = w.u1[e].imag();
    }
    d.blocks = std::max(1, std::min(256, ceil_div((int64_t)d.chi_l * d.chi_r, 256)));
    s1.push_back(d);
    sbase.push_back(sbase.back() + d.blocks);
  }
  // unitaries, merge chains and unitary applications of the starting clusters
  int kmax = 0;
  for (int i : starting) kmax = std::max(kmax, T[i].job.k);
  std::vector<UnitaryDesc> ud;
  std::vector<int> ubase{0};
  std::vector<size_t> gate_off;
  size_t ulds = 0;
  for (int i : starting) {
    const Job& jb = T[i].job;
    std::vector<UGate> ug;
    for (const auto& g : jb.gates) {
      UGate u{};
      u.nq = g.nq;
      u.q0 = g.q[0] - jb.a;
      u.q1 = g.nq > 1 ? g.q[1] - jb.a : 0;
      const int dd = 1 << (2 * g.nq);
      for (int e = 0; e < dd; ++e) {
        u.u[2 * e] = g.u[e].real();
        u.u[2 * e + 1] = g.u[e].imag();
      }
      ug.push_back(u);
    }
    gate_off.push_back(ug.empty() ? 0 : B.add_vec(ug));
    UnitaryDesc d{};
    d.ngates = (int)ug.size();
    d.k = jb.k;
    d.U64 = (double2*)T[i].run.U64;
    d.U32 = (P == Prec::FP64) ? nullptr : (float2*)T[i].run.Uw;
    const int dim = 1 << jb.k;
    d.cols = std::max(1, std::min(16, 4096 / dim));
    d.blocks = ceil_div(dim, d.cols);
    ulds = std::max(ulds, (size_t)d.cols * dim * sizeof(double2));
    ud.push_back(d);
    ubase.push_back(ubase.back() + d.blocks);
  }
  std::vector<std::vector<GemmDesc>> mg(std::max(1, kmax));
  std::vector<GemmDesc> ap;
  for (int i : starting) {
    JobRun& r = T[i].run;
    for (int j = 1; j < r.k; ++j) {
      GemmDesc d{};
      const int M = r.chi_l << j;
      const int K = r.mid[j - 1];
      const int N = 2 * ((j == r.k - 1) ? r.chi_r : r.mid[j]);
      d.A = (j == 1) ? ctx->site[r.a] : r.buf[(j - 1) & 1];
      d.B = ctx->site[r.a + j];
      d.C = r.buf[j & 1];
      d.M = fixed(M);
      d.N = fixed(N);
      d.K = fixed(K);
      d.lda = fixed(K);
      d.ldb = fixed(N);
      d.ldc = fixed(N);
      d.batch = 1;
      d.tm = ceil_div(M, 64);
      d.tn = ceil_div(N, 64);
      d.ksplit = 1;
      d.alpha = 1.0;
      mg[j].push_back(d);
    }
    r.cur = (r.k - 1) & 1;
    GemmDesc d{};
    const int D = 1 << r.k;
    d.A = r.Uw;
    d.B = r.buf[r.cur];
    d.C = r.buf[r.cur ^ 1];
    d.M = fixed(D);
    d.N = fixed(r.chi_r);
    d.K = fixed(D);
    d.lda = fixed(D);
    d.ldb = fixed(r.chi_r);
    d.ldc = fixed(r.chi_r);
    d.sA = 0;
    d.sB = d.sC = (int64_t)D * r.chi_r;
    d.batch = r.chi_l;
    d.tm = ceil_div(D, 64);
    d.tn = ceil_div(r.chi_r, 64);
    d.ksplit = 1;
    d.alpha = 1.0;
    ap.push_back(d);
    r.cur ^= 1;
  }
  // split levels of every running cluster, final scaling of those that end
  LevelDescs L;
  L.nb_max_all = 0;
  std::vector<ScaleDesc> fin;
  std::vector<int> fbase{0};
  std::vector<const double*> fin_logf;
  for (int p = 0; p < na; ++p) {
    WaveTask& w = T[active[p]];
    JobRun& r = w.run;
    add_level(ctx, L, r, p, w.level, nullptr);
    if (w.level == r.k - 2) {
      ScaleDesc d{};
      d.X = r.buf[r.cur];
      d.B = ctx->site[r.a];
      d.count = Dim{2 * r.chi_l, ctx->d_chi + r.a};
      d.logf = r.logf;
      const int64_t bound = (int64_t)2 * r.chi_l * std::min(ctx->chi_max, 2 * r.chi_l);
      d.blocks = std::max(1, std::min(1024, ceil_div(bound, 256)));
      fin.push_back(d);
      fbase.push_back(fbase.back() + d.blocks);
      fin_logf.push_back(r.logf);
    }
  }
  // serialise
  size_t o_s1 = 0, b_s1 = 0, o_ud = 0, b_ud = 0, o_ap = 0, b_ap = 0, o_fin = 0, b_fin = 0, o_lf = 0;
  if (!s1.empty()) {
    o_s1 = B.add_vec(s1);
    b_s1 = B.add_vec(sbase);
  }
  if (!ud.empty()) {
    o_ud = B.add_vec(ud);
    b_ud = B.add_vec(ubase);
  }
  std::vector<size_t> o_mg(mg.size(), 0), b_mg(mg.size(), 0);
  std::vector<int> n_mg(mg.size(), 0);
  for (size_t j = 1; j < mg.size(); ++j) n_mg[j] = upload_gemms(B, mg[j], o_mg[j], b_mg[j]);
  const int n_ap = ap.empty() ? 0 : upload_gemms(B, ap, o_ap, b_ap);
  if (na) upload_level(B, L);
  if (!fin.empty()) {
    o_fin = B.add_vec(fin);
    b_fin = B.add_vec(fbase);
    o_lf = B.add_vec(fin_logf);
  }
  HIP_OK(B.prepare());
  for (size_t q = 0; q < ud.size(); ++q) {
    UnitaryDesc* d = B.host_at<UnitaryDesc>(o_ud) + q;
    d->gates = d->ngates ? B.at<UGate>(gate_off[q]) : nullptr;
  }
  HIP_OK(B.upload(s));
  // launches
  if (!s1.empty()) {
    Timed tm(ctx, "one_qubit");
    HIP_OK(launch_apply_1q(P, B.at<Site1QDesc>(o_s1), B.at<int>(b_s1), (int)s1.size(), sbase.back(), s));
  }
  if (!ud.empty()) {
    Timed tm(ctx, "unitary");
    HIP_OK(launch_build_unitary(B.at<UnitaryDesc>(o_ud), B.at<int>(b_ud), (int)ud.size(), ubase.back(), ulds, s));
  }
  for (size_t j = 1; j < mg.size(); ++j) {
    if (mg[j].empty()) continue;
    Timed tm(ctx, "merge");
    HIP_OK(launch_gemm_nn(P, B.at<GemmDesc>(o_mg[j]), B.at<int>(b_mg[j]), (int)mg[j].size(), n_mg[j], s));
  }
  if (!ap.empty()) {
    Timed tm(ctx, "apply");
    HIP_OK(launch_gemm_nn(P, B.at<GemmDesc>(o_ap), B.at<int>(b_ap), (int)ap.size(), n_ap, s));
  }
  if (na) launch_level(ctx, B, L, flags_round, 4 * na, [] {});
  if (!fin.empty()) {
    Timed tm(ctx, "finalize");
    HIP_OK(launch_finalize(P, B.at<ScaleDesc>(o_fin), B.at<int>(b_fin), (int)fin.size(), fbase.back(), s));
    HIP_OK(launch_accumulate_ptrs(B.at<const double*>(o_lf), (int)fin.size(), ctx->d_logf, s));
  }
  // end of round: bond dimensions and the finished clusters' records
  std::vector<double> rec;
  std::vector<int> ending;
  for (int i : active)
    if (T[i].level == T[i].run.k - 2) ending.push_back(i);
  size_t nrec = 0;
  for (int i : ending) nrec += 4 * (T[i].run.k - 1);
  rec.resize(nrec);
  HIP_OK(hipMemcpyAsync(ctx->chi.data(), ctx->d_chi, (ctx->n - 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  {
    size_t off = 0;
    for (int i : ending) {
      const JobRun& r = T[i].run;
      HIP_OK(hipMemcpyAsync(rec.data() + off, r.rec, 4 * (r.k - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      off += 4 * (r.k - 1);
    }
  }
  unsigned long long eig_work[2] = {0, 0};
  if (ctx->timing) HIP_OK(hipMemcpyAsync(eig_work, ctx->d_work, sizeof(eig_work), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (ctx->timing) {
    collect_timing(ctx);
    for (int i : active) account_level(ctx, T[i].run, T[i].level);
    ctx->timer.flop[ctx->timer.cls_of("eig_update")] += 8.0 * (double)eig_work[0];
    ctx->timer.flop[ctx->timer.cls_of("eig_pairs")] += (double)eig_work[1];
  }
  for (size_t q = 0; q < nrec; q += 4) ctx->stats.discarded_weight += rec[q + 2];
  {
    size_t off = 0;
    for (int i : ending) {
      record_tails(ctx, T[i].run, rec.data() + off);
      off += 4 * (T[i].run.k - 1);
    }
  }
  // (features, log2 kept rank) of the splits of this round
  for (int i : active) {
    const WaveTask& w = T[i];
    const int t = w.level;
    if (ctx->log_t.size() >= (size_t)4000000) break;
    const int rk = ctx->chi[w.run.a + w.run.lv[t].m - 1];
    ctx->log_x.insert(ctx->log_x.end(), w.feats.begin() + (size_t)t * N_FEAT,
                      w.feats.begin() + (size_t)(t + 1) * N_FEAT);
    ctx->log_t.push_back(std::log2((float)rk));
  }
  for (int i : active) {
    WaveTask& w = T[i];
    if (++w.level == w.run.k - 1) {
      w.state = 2;
      ctx->pool.put(w.ws, w.ws_cap);
      w.ws = nullptr;
      ctx->stats.cluster_updates += 1;
      ctx->stats.svds += w.run.k - 1;
    }
  }
  for (int i : sites) {
    T[i].state = 2;
    ctx->stats.site_updates += 1;
  }
}

void run_wave(mps_ctx* ctx, std::vector<WaveTask>& T) {
  std::vector<int> running;
  size_t done = 0;
  while (done < T.size()) {
    std::vector<int> sites, starting;
    for (int i = 0; i < (int)T.size(); ++i) {
      if (T[i].state != 0) continue;
      bool ready = true;
      for (int d : T[i].deps)
        if (T[d].state != 2) {
          ready = false;
          break;
        }
      if (!ready) continue;
      (T[i].site ? sites : starting).push_back(i);
    }
    for (int i : starting) {
      T[i].state = 1;
      running.push_back(i);
    }
    if (sites.empty() && running.empty()) fail(ctx, MPS_ESTATE, "wavefront executor: no task can run");
    wave_round(ctx, T, sites, starting, running);
    std::vector<int> still;
    for (int i : running)
      if (T[i].state != 2) still.push_back(i);
    running.swap(still);
    done = 0;
    for (const auto& w : T) done += w.state == 2;
  }
}

// Executes the next `nsteps` planned steps (every buffered one when nsteps < 0)
// with the wavefront executor; returns the number of steps.  Falls back to
// one step at a time where the window cannot be planned up front (a binding
// q_max) or where the step executor is the one asked for.
int execute_window(mps_ctx* ctx, int nsteps) {
  if (ctx->pending.empty() || nsteps == 0) return 0;
  const bool wave = ctx->opt.batch == MPS_BATCH_WAVE && ctx->opt.svd_mode == MPS_SVD_EXACT && plan_is_chi_free(ctx);
  if (!wave) {
    int done = 0;
    while (!ctx->pending.empty() && (nsteps < 0 || done < nsteps)) {
      execute_step(ctx, 0);
      ++done;
    }
    return done;
  }
  std::vector<WaveTask> T;
  int steps = 0;
  const int used = plan_window(ctx, nsteps, T, &steps);
  try {
    run_wave(ctx, T);
  } catch (...) {
    for (auto& w : T)
      if (w.ws) ctx->pool.put(w.ws, w.ws_cap);
    throw;
  }
  ctx->pending.erase(ctx->pending.begin(), ctx->pending.begin() + used);
  ctx->stats.steps += steps;
  return steps;
}

// Executes one planned step from the pending sub-layers; returns the number
// of sub-layers consumed.
int execute_step(mps_ctx* ctx, int end_hint) {
  std::vector<Cluster> cl;
  const int end = plan_step(ctx->pending, 0, ctx->n, ctx->chi, ctx->opt.k_max, ctx->q_max_eff,
                            ctx->l_max_eff, cl);
  (void)end_hint;
  std::vector<int> owner(ctx->n, -1);
  for (size_t c = 0; c < cl.size(); ++c)
    for (int q = cl[c].a; q < cl[c].a + cl[c].k; ++q) owner[q] = (int)c;
  std::vector<Job> jobs(cl.size());
  for (size_t c = 0; c < cl.size(); ++c) {
    jobs[c].a = cl[c].a;
    jobs[c].k = cl[c].k;
  }
  std::vector<std::array<cplx, 4>> u1(ctx->n);
  std::vector<char> has1(ctx->n, 0);
  for (int sl = 0; sl < end; ++sl) {
    for (const auto& g : ctx->pending[sl]) {
      const int o = owner[g.q[0]];
      if (o >= 0) {
        jobs[o].gates.push_back(g);
      } else {
        const int q = g.q[0];
        if (!has1[q]) {
          u1[q] = {cplx(1), cplx(0), cplx(0), cplx(1)};
          has1[q] = 1;
        }
        const auto& m = u1[q];
        std::array<cplx, 4> r;
        r[0] = g.u[0] * m[0] + g.u[1] * m[2];
        r[1] = g.u[0] * m[1] + g.u[1] * m[3];
        r[2] = g.u[2] * m[0] + g.u[3] * m[2];
        r[3] = g.u[2] * m[1] + g.u[3] * m[3];
        u1[q] = r;
      }
    }
  }
  std::vector<Site1QDesc> s1;
  for (int q = 0; q < ctx->n; ++q) {
    if (!has1[q]) continue;
    Site1QDesc d{};
    d.B = ctx->site[q];
    d.chi_l = bond_dim(ctx, q - 1);
    d.chi_r = bond_dim(ctx, q);
    for (int e = 0; e < 4; ++e) {
      d.u[2 * e] = u1[q][e].real();
      d.u[2 * e + 1] = u1[q][e].imag();
    }
    d.blocks = std::max(1, std::min(256, ceil_div((int64_t)d.chi_l * d.chi_r, 256)));
    s1.push_back(d);
  }
  run_jobs(ctx, jobs, s1, end);
  ctx->pending.erase(ctx->pending.begin(), ctx->pending.begin() + end);
  return end;
}

void flush_all(mps_ctx* ctx) { execute_window(ctx, -1); }

// Steps of the buffered sub-layers that can no longer grow (the last planned
// step may still take sub-layers of a later layer).
int complete_steps(mps_ctx* ctx) {
  int start = 0, cnt = 0;
  const int total = (int)ctx->pending.size();
  while (start < total) {
    std::vector<Cluster> cl;
    const int end = plan_step(ctx->pending, start, ctx->n, ctx->chi, ctx->opt.k_max, ctx->q_max_eff,
                              ctx->l_max_eff, cl);
    if (end >= total) break;
    ++cnt;
    start = end;
  }
  return cnt;
}

HostGate to_host_gate(const mps_gate& g) {
  HostGate h;
  h.nq = g.nq;
  h.q[0] = g.q[0];
  h.q[1] = g.nq > 1 ? g.q[1] : g.q[0];
  const int dd = 1 << (2 * g.nq);
  for (int e = 0; e < 16; ++e) h.u[e] = e < dd ? cplx(g.u[2 * e], g.u[2 * e + 1]) : cplx(0);
  return h;
}

// Why the gates of one layer are invalid on n qubits, or nullptr.
const char* gate_error(const mps_gate* gates, int ngates, int n) {
  std::vector<char> used(n, 0);
  for (int i = 0; i < ngates; ++i) {
    const mps_gate& g = gates[i];
    if (g.nq < 1 || g.nq > 2) return "gate with nq outside {1,2}";
    for (int j = 0; j < g.nq; ++j) {
      if (g.q[j] < 0 || g.q[j] >= n) return "gate qubit out of range";
      if (used[g.q[j]]) return "gates of one layer must act on disjoint qubits";
      used[g.q[j]] = 1;
    }
  }
  return nullptr;
}

mps_status check_gates(mps_ctx* ctx, const mps_gate* gates, int ngates, int n) {
  if (const char* why = gate_error(gates, ngates, n)) {
    ctx->err = why;
    return MPS_EINVAL;
  }
  return MPS_OK;
}

// ||U^H U - 1||_max <= 1e-10 for a dim x dim U (row-major).  The product
// costs dim^3 complex multiply-adds: on the host up to dim = 256 (tens of
// milliseconds), from dim = 512 on (a second and more on one host core, about
// 8 minutes at dim = 4096) on the FP64 matrix cores, the comparison with the
// identity on the host either way.  Synchronises the handle's stream.
bool is_unitary(mps_ctx* ctx, const std::vector<cplx>& U, int dim) {
  constexpr double tol = 1e-10;
  if (dim < 512) {
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j < dim; ++j) {
        cplx s = 0;
        for (int k = 0; k < dim; ++k) s += std::conj(U[(size_t)k * dim + i]) * U[(size_t)k * dim + j];
        if (std::abs(s - (i == j ? cplx(1) : cplx(0))) > tol) return false;
      }
    return true;
  }
  struct DevBuf {  // freed on every exit, errors included
    void* p = nullptr;
    ~DevBuf() {
      if (p) (void)hipFree(p);
    }
  } dU, dG;
  const size_t bytes = (size_t)dim * dim * sizeof(double2);
  hipStream_t s = ctx->stream;
  HIP_OK(hipStreamSynchronize(s));  // the descriptor blob may still feed queued launches
  HIP_OK(hipMalloc(&dU.p, bytes));
  HIP_OK(hipMalloc(&dG.p, bytes));
  HIP_OK(hipMemcpy(dU.p, U.data(), bytes, hipMemcpyHostToDevice));
  const Dim d = Dim{dim, nullptr};
  const GemmDesc g = gemm64(dU.p, dU.p, dG.p, d, d, d, d, d, d, dim, dim);  // G = U^H U
  DescBlob& B = ctx->blob;
  B.host.clear();
  const size_t og = B.add(&g, sizeof(g));
  const int tiles = gemm_tiles(g);
  const size_t ob = B.add_vec(std::vector<int>{0, tiles});
  HIP_OK(B.upload(s));
  HIP_OK(launch_gemm_cn(B.at<GemmDesc>(og), B.at<int>(ob), 1, tiles, s));
  std::vector<cplx> G((size_t)dim * dim);
  HIP_OK(hipMemcpyAsync(G.data(), dG.p, bytes, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j)
      if (std::abs(G[(size_t)i * dim + j] - (i == j ? cplx(1) : cplx(0))) > tol) return false;
  return true;
}

template <typename F>
mps_status guarded(mps_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return MPS_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return MPS_EINVAL;
  }
}

void destroy_ctx(mps_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  destroy_ctx(ctx->dmrg_scratch);
  ctx->dmrg_scratch = nullptr;
  if (ctx->htd_dev) (void)hipFree(ctx->htd_dev);
  ctx->arena.release();
  ctx->pool.release();
  ctx->blob.release();
  if (ctx->state_mem) (void)hipFree(ctx->state_mem);
  if (ctx->d_chi) (void)hipFree(ctx->d_chi);
  if (ctx->d_work) (void)hipFree(ctx->d_work);
  if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
  for (auto e : ctx->timer.pool) (void)hipEventDestroy(e);
  for (auto& p : ctx->timer.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

// ------------------------------------------------------------- DMRG --
// Adaptive-grouping DMRG step (Sec. III.B with the iteration of Sec. II.C) on
// the library's kernels, FP64: the virtual MPS of Eq. chi_est and the
// recursive bipartition of Eqs. cond_group1 / cond_group2 on the host; on the
// device the evolved state U |psi> of the segment (the cluster-TEBD executor
// on a scratch handle, nothing truncated beyond the Gram route's floor), its
// grouped tensors (merge GEMM chains), a grouped MPS M fitted to it (initial
// truncated-SVD compression at the group cuts, then sweeps of one-group
// updates M = F / ||F||, orthonormalised by polar factors), and M decomposed
// back into qubit tensors by Gram / eigen splits with chi_max and the cutoff.
// Every product is one launch of the library's GEMMs with a single problem
// (split along K when it has few output tiles); the stream is synchronised
// after each (the descriptor blob is reused).
struct DevOps {
  mps_ctx* ctx;
  std::vector<void*> mem;                       // every block, freed at the end
  std::unordered_map<void*, size_t> bytes_of;   // their sizes
  std::vector<std::pair<size_t, void*>> spare;  // released blocks
  double* d_scalar = nullptr;
  explicit DevOps(mps_ctx* c) : ctx(c) {}
  ~DevOps() {
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (void* p : mem) (void)hipFree(p);
  }
  // Blocks are recycled within the step: everything runs on one stream, so a
  // block released after its last use is only written again by work queued
  // after that use.  A spare block serves a request of up to twice its size.
  template <typename T>
  T* alloc(size_t n) {
    const size_t want = (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~size_t(255);
    size_t best = spare.size();
    for (size_t i = 0; i < spare.size(); ++i)
      if (spare[i].first >= want && spare[i].first <= 2 * want + (size_t(1) << 20) &&
          (best == spare.size() || spare[i].first < spare[best].first))
        best = i;
    if (best < spare.size()) {
      void* p = spare[best].second;
      spare.erase(spare.begin() + best);
      return (T*)p;
    }
    void* p = nullptr;
    HIP_OK(hipMalloc(&p, want));
    mem.push_back(p);
    bytes_of[p] = want;
    return (T*)p;
  }
  void release(void* p) {
    auto it = bytes_of.find(p);
    if (it == bytes_of.end()) return;
    for (const auto& e : spare)
      if (e.second == p) return;
    spare.push_back({it->second, p});
  }
  void run_gemm(const GemmDesc& d, bool cn) {
    DescBlob& B = ctx->blob;
    B.host.clear();
    const size_t o = B.add(&d, sizeof(d));
    const int tiles = gemm_tiles(d);
    const std::vector<int> base{0, tiles};
    const size_t ob = B.add_vec(base);
    HIP_OK(B.upload(ctx->stream));
    if (cn)
      HIP_OK(launch_gemm_cn(B.at<GemmDesc>(o), B.at<int>(ob), 1, tiles, ctx->stream));
    else
      HIP_OK(launch_gemm_nn(Prec::FP64, B.at<GemmDesc>(o), B.at<int>(ob), 1, tiles, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
  }
  // A product with few 64 x 64 output tiles and a long K (the environment
  // updates contract a group's whole physical index) is cut into K slices
  // whose partial products are summed afterwards, so that it fills more than
  // a handful of compute units.
  double2* parts = nullptr;
  size_t parts_cap = 0;
  void run_split(GemmDesc d, double2* C, int M, int N, int K, int ldc, bool cn) {
    const int tiles = d.tm * d.tn;
    int ks = 1;
    if (tiles < 128 && K >= 1024) ks = std::min({64, std::max(1, 256 / tiles), K / 512});
    if (ks <= 1) {
      run_gemm(d, cn);
      return;
    }
    const size_t need = (size_t)ks * M * N;
    if (need > parts_cap) {
      if (parts) release(parts);
      parts = alloc<double2>(need);
      parts_cap = need;
    }
    d.C = parts;
    d.ldc = fixed(N);
    d.ksplit = ks;
    d.part = (int64_t)M * N;
    run_gemm(d, cn);
    HIP_OK(launch_dense_sum_parts(parts, ks, (int64_t)M * N, M, N, C, ldc, ctx->stream));
  }
  // C (M x N) = A (M x K) B (K x N)
  void nn(const double2* A, const double2* B, double2* C, int M, int N, int K, int lda, int ldb, int ldc) {
    run_split(gemm64(A, B, C, fixed(M), fixed(N), fixed(K), fixed(lda), fixed(ldb), fixed(ldc), M, N), C, M, N, K,
              ldc, false);
  }
  // C (M x N) = A^H B, A: K x M, B: K x N
  void cn(const double2* A, const double2* B, double2* C, int M, int N, int K, int lda, int ldb, int ldc) {
    run_split(gemm64(A, B, C, fixed(M), fixed(N), fixed(K), fixed(lda), fixed(ldb), fixed(ldc), M, N), C, M, N, K,
              ldc, true);
  }
  double norm2(const double2* x, int64_t n) {
    if (!d_scalar) d_scalar = alloc<double>(1);
    HIP_OK(launch_dense_norm2(x, n, d_scalar, ctx->stream));
    double v = 0;
    HIP_OK(hipMemcpyAsync(&v, d_scalar, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return v;
  }
  void scale(double2* x, int64_t n, double a) { HIP_OK(launch_dense_scale(x, n, a, ctx->stream)); }
  // eigenpairs of the Hermitian n x n matrix G (ld), descending; V columns (ldv)
  struct Eig {
    double2* V;
    int ldv;
    std::vector<double> w;
    char* base;  // workspace holding V (release when done)
  };
  Eig eigh(const double2* G, int n, int ld) {
    if (n > HTD_MAX) fail(ctx, MPS_EINVAL, "DMRG: eigenproblem larger than 2048");
    const size_t lw = (size_t)ceil_div(n, 64) * 64;
    size_t bytes = 0;
    HtdDesc h{};
    auto count = [&](size_t x) -> void* {
      bytes = ((bytes + 255) & ~size_t(255)) + x;
      return nullptr;
    };
    count(lw * lw * sizeof(double2));
    count(lw * lw * sizeof(double2));
    htd_layout(lw, h, count);
    count(sizeof(HtdDesc));
    char* base = alloc<char>(bytes);
    size_t used = 0;
    auto take = [&](size_t x) -> void* {
      const size_t off = (used + 255) & ~size_t(255);
      used = off + x;
      return base + off;
    };
    h.A = (double2*)take(lw * lw * sizeof(double2));
    h.V = (double2*)take(lw * lw * sizeof(double2));
    htd_layout(lw, h, take);
    HtdDesc* dd = (HtdDesc*)take(sizeof(HtdDesc));
    h.n = Dim{n, nullptr};
    h.ld = (int)lw;
    h.rcap = n;
    h.skip = nullptr;
    HIP_OK(hipMemcpy2DAsync(h.A, lw * sizeof(double2), G, ld * sizeof(double2), n * sizeof(double2), n,
                            hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(dd, &h, sizeof(HtdDesc), hipMemcpyHostToDevice, ctx->stream));
    {
      // the solver reads no bond dimensions for fixed sizes
      struct Restore {
        mps_ctx* c;
        int n;
        ~Restore() { c->n = n; }
      } restore{ctx, ctx->n};
      ctx->n = 1;
      solve_htd(ctx, dd, std::vector<HtdDesc>{h});
    }
    Eig e;
    e.V = h.V;
    e.ldv = (int)lw;
    e.base = base;
    e.w.resize(n);
    HIP_OK(hipMemcpyAsync(e.w.data(), h.lam, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return e;
  }
  double* upload(const std::vector<double>& v) {
    double* d = alloc<double>(v.size());
    HIP_OK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return d;
  }
  // Polar factor of F (rows x cols): left (columns orthonormal, F (F^H F)^-1/2)
  // or right (rows orthonormal, (F F^H)^-1/2 F); directions below 1e-28 of the
  // largest eigenvalue are dropped
  double2* polar(const double2* F, int rows, int cols, bool left) {
    const int m = left ? cols : rows;
    double2* G = alloc<double2>((size_t)m * m);
    double2* Fh = nullptr;
    if (left) {
      cn(F, F, G, cols, cols, rows, cols, cols, cols);
    } else {
      Fh = alloc<double2>((size_t)rows * cols);
      HIP_OK(launch_dense_adjoint(F, rows, cols, cols, nullptr, Fh, rows, ctx->stream));
      cn(Fh, Fh, G, rows, rows, cols, rows, rows, rows);
    }
    Eig e = eigh(G, m, m);
    std::vector<double> d(m, 0.0);
    const double top = std::max(e.w[0], 1e-300);
    for (int i = 0; i < m; ++i) d[i] = e.w[i] > 1e-28 * top ? std::pow(e.w[i], -0.25) : 0.0;
    double* dd = upload(d);
    double2* Y = alloc<double2>((size_t)m * m);  // Y = diag(w^-1/4) V^H, P = Y^H Y = V w^-1/2 V^H
    HIP_OK(launch_dense_adjoint(e.V, m, m, e.ldv, dd, Y, m, ctx->stream));
    double2* P = alloc<double2>((size_t)m * m);
    cn(Y, Y, P, m, m, m, m, m, m);
    double2* Q = alloc<double2>((size_t)rows * cols);
    if (left)
      nn(F, P, Q, rows, cols, cols, cols, cols, cols);
    else
      nn(P, F, Q, rows, cols, rows, rows, cols, cols);
    release(e.base);
    release(G);
    release(Y);
    release(P);
    release(dd);
    if (Fh) release(Fh);
    return Q;
  }
};

struct Tensor3 {
  double2* p = nullptr;
  int l = 1, d = 1, r = 1;
  int64_t size() const { return (int64_t)l * d * r; }
};

int dmrg_truncation_rank(const std::vector<double>& w, int cap_rows, const mps_ctx* ctx, double* f) {
  double tot = 0;
  for (double x : w) tot += std::max(x, 0.0);
  int kept = 0;
  for (double x : w)
    if (tot > 0 && std::sqrt(std::max(x, 0.0) / tot) >= ctx->eps_eff) ++kept;
  kept = std::max(1, std::min({kept, ctx->chi_max, cap_rows, (int)w.size()}));
  double k = 0;
  for (int i = 0; i < kept; ++i) k += std::max(w[i], 0.0);
  *f = tot > 0 ? k / tot : 1.0;
  return kept;
}

// The step itself; `layers`: the segment's gates, layer by layer.  Returns f
// of the last update (the fit's fidelity) through *f_fit.
void dmrg_step(mps_ctx* ctx, const std::vector<std::vector<HostGate>>& layers, int chi_max_dmrg, int q_max,
               int sweeps, double* f_fit) {
  const int n = ctx->n;
  hipStream_t s = ctx->stream;
  // ---- Eq. chi_est and the grouping (host)
  std::vector<int> E(n - 1, 0);
  for (const auto& L : layers)
    for (const auto& g : L)
      if (g.nq == 2)
        for (int b = g.lo(); b < g.hi(); ++b) ++E[b];
  // chit: Eq. chi_est (each gate across a bond counted as doubling it);
  // chi_exact: a true bound for the evolved state, whose two-qubit gates
  // multiply a bond by their operator Schmidt rank, up to 4 (SWAP)
  std::vector<int64_t> chit(n - 1), chi_exact(n - 1);
  for (int b = 0; b < n - 1; ++b) {
    const int64_t cap = (int64_t)1 << std::min({b + 1, n - b - 1, 40});
    chit[b] = std::min({((int64_t)1 << std::min(E[b], 40)) * ctx->chi[b], cap, (int64_t)chi_max_dmrg});
    chi_exact[b] = std::min(((int64_t)1 << std::min(2 * E[b], 40)) * ctx->chi[b], cap);
  }
  std::vector<std::pair<int, int>> groups;
  std::function<void(int, int, int64_t, int64_t)> rec = [&](int lo, int hi, int64_t cl, int64_t cr) {
    const int N = hi - lo + 1;
    const bool fits = N <= 60 && (double)cl * (double)cr * std::ldexp(1.0, N) <= std::ldexp(1.0, q_max);
    if (lo == hi || fits) {
      groups.push_back({lo, hi});
      return;
    }
    int best = lo;
    for (int b = lo + 1; b < hi; ++b) {
      const auto key = [&](int c) { return std::make_tuple(chit[c], std::abs((c - lo + 1) - (hi - c)), c); };
      if (key(b) < key(best)) best = b;
    }
    rec(lo, best, cl, chit[best]);
    rec(best + 1, hi, chit[best], cr);
  };
  rec(0, n - 1, 1, 1);
  const int ng = (int)groups.size();
  // ---- the evolved state U |psi> on a scratch handle
  int64_t chi_t = 1;
  for (int b = 0; b < n - 1; ++b) chi_t = std::max(chi_t, chi_exact[b]);
  if (chi_t > HTD_MAX / 2) fail(ctx, MPS_EINVAL, "DMRG: the evolved state needs a bond dimension above 1024");
  mps_options to = ctx->opt;
  to.precision = MPS_PREC_FP64;
  to.batch = MPS_BATCH_STEP;
  to.svd_mode = MPS_SVD_EXACT;
  to.hip_stream = ctx->stream;
  // the scratch handle of the previous step serves again when its cap covers
  // chi_t and its options match (its cap only bounds, and never binds,
  // since chi_t bounds the exact state); it is created with chi_t rounded up
  // to a power of two so that a slowly growing chi_t rarely recreates it
  mps_handle T = ctx->dmrg_scratch;
  auto same = [](const mps_options& a, const mps_options& b) {
    return a.k_max == b.k_max && a.q_max == b.q_max && a.l_max == b.l_max && a.eig_method == b.eig_method &&
           a.floor_c == b.floor_c && a.hip_stream == b.hip_stream;
  };
  if (T && (T->n != n || T->chi_max < chi_t || !same(T->opt, to))) {
    destroy_ctx(T);
    T = ctx->dmrg_scratch = nullptr;
  }
  if (!T) {
    int64_t cap = 1;
    while (cap < chi_t) cap <<= 1;
    const mps_status cs = mps_create(n, (int)std::min<int64_t>(cap, HTD_MAX / 2), 0.0, &to, &T);
    if (cs != MPS_OK) fail(ctx, cs, "DMRG: could not create the scratch handle");
    ctx->dmrg_scratch = T;
  }
  T->pending.clear();
  for (int j = 0; j < n; ++j) {
    const int64_t cnt = (int64_t)bond_dim(ctx, j - 1) * 2 * bond_dim(ctx, j);
    HIP_OK(hipMemcpyAsync(T->site[j], ctx->site[j], cnt * 16, hipMemcpyDeviceToDevice, s));
  }
  for (int b = 0; b < n - 1; ++b)
    HIP_OK(hipMemcpyAsync(T->lam[b], ctx->lam[b], ctx->chi[b] * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_OK(hipMemcpyAsync(T->d_chi, ctx->d_chi, (n - 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  T->chi = ctx->chi;
  for (const auto& L : layers) legalize_layer(L, T->opt.k_max, T->pending);
  {
    const mps_status st = guarded(T, [&]() -> mps_status {
      while (!T->pending.empty()) execute_step(T, 0);
      return MPS_OK;
    });
    if (st != MPS_OK) fail(ctx, st, ("DMRG: evolving the segment: " + T->err).c_str());
  }
  HIP_OK(hipStreamSynchronize(s));
  DevOps D(ctx);
  // ---- grouped tensors of U |psi>
  std::vector<Tensor3> Tg(ng);
  for (int t = 0; t < ng; ++t) {
    const int a = groups[t].first, b = groups[t].second;
    Tensor3 cur{(double2*)T->site[a], bond_dim(T, a - 1), 2, bond_dim(T, a)};
    for (int j = a + 1; j <= b; ++j) {
      const int rn = bond_dim(T, j);
      double2* out = D.alloc<double2>((size_t)cur.l * cur.d * 2 * rn);
      D.nn(cur.p, (const double2*)T->site[j], out, cur.l * cur.d, 2 * rn, cur.r, cur.r, 2 * rn, 2 * rn);
      cur = Tensor3{out, cur.l, cur.d * 2, rn};
    }
    if (a == b) {  // own copy (the scratch handle's site stays valid until the end anyway)
      double2* out = D.alloc<double2>(cur.size());
      HIP_OK(hipMemcpyAsync(out, cur.p, cur.size() * 16, hipMemcpyDeviceToDevice, s));
      cur.p = out;
    }
    Tg[t] = cur;
  }
  // ---- initial M: truncated-SVD compression at the group cuts, left to right
  std::vector<Tensor3> M(ng);
  Tensor3 C = Tg[0];
  for (int t = 0; t + 1 < ng; ++t) {
    const int rows = C.l * C.d, r = C.r;
    double2* G = D.alloc<double2>((size_t)r * r);
    D.cn(C.p, C.p, G, r, r, rows, r, r, r);
    DevOps::Eig e = D.eigh(G, r, r);
    const double top = std::max(e.w[0], 1e-300);
    int k = 0;
    for (double w : e.w)
      if (w > 1e-20 * top) ++k;
    k = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)k, chit[groups[t].second], (int64_t)rows}));
    double2* CV = D.alloc<double2>((size_t)rows * k);
    D.nn(C.p, e.V, CV, rows, k, r, r, e.ldv, k);
    std::vector<double> inv(k);
    for (int i = 0; i < k; ++i) inv[i] = 1.0 / std::sqrt(e.w[i]);
    HIP_OK(launch_dense_scale_cols(CV, rows, k, k, D.upload(inv), s));
    M[t] = Tensor3{CV, C.l, C.d, k};
    D.release(e.base);
    D.release(G);
    double2* K = D.alloc<double2>((size_t)k * r);  // U^H C = S V^H
    D.cn(CV, C.p, K, k, r, rows, k, r, r);
    const Tensor3& Tn = Tg[t + 1];
    double2* Cn = D.alloc<double2>((size_t)k * Tn.d * Tn.r);
    D.nn(K, Tn.p, Cn, k, Tn.d * Tn.r, r, r, Tn.d * Tn.r, Tn.d * Tn.r);
    C = Tensor3{Cn, k, Tn.d, Tn.r};
  }
  {
    double2* last = D.alloc<double2>(C.size());
    HIP_OK(hipMemcpyAsync(last, C.p, C.size() * 16, hipMemcpyDeviceToDevice, s));
    D.scale(last, C.size(), 1.0 / std::sqrt(D.norm2(last, C.size())));
    M[ng - 1] = Tensor3{last, C.l, C.d, C.r};
  }
  // ---- sweeps of one-group updates
  std::vector<double2*> Lenv(ng + 1, nullptr), Renv(ng + 1, nullptr);  // Lenv[t]: chi_M x D (left of group t)
  std::vector<int> Lm(ng + 1, 1), Ld(ng + 1, 1), Rd(ng + 1, 1), Rm(ng + 1, 1);  // Renv[t]: D x chi_M (right of t-1)
  const double2 one = make_double2(1.0, 0.0);
  Lenv[0] = D.alloc<double2>(1);
  Renv[ng] = D.alloc<double2>(1);
  HIP_OK(hipMemcpyAsync(Lenv[0], &one, 16, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(Renv[ng], &one, 16, hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  auto left_env = [&](int t) {  // Lenv[t+1] from Lenv[t], M[t], Tg[t]
    const Tensor3 &m = M[t], &tg = Tg[t];
    double2* Z = D.alloc<double2>((size_t)m.l * tg.d * tg.r);
    D.nn(Lenv[t], tg.p, Z, m.l, tg.d * tg.r, tg.l, tg.l, tg.d * tg.r, tg.d * tg.r);
    double2* L2 = D.alloc<double2>((size_t)m.r * tg.r);
    D.cn(m.p, Z, L2, m.r, tg.r, m.l * m.d, m.r, tg.r, tg.r);
    D.release(Z);
    if (Lenv[t + 1]) D.release(Lenv[t + 1]);
    Lenv[t + 1] = L2;
    Lm[t + 1] = m.r;
    Ld[t + 1] = tg.r;
  };
  auto right_env = [&](int t) {  // Renv[t] from Renv[t+1], M[t], Tg[t]
    const Tensor3 &m = M[t], &tg = Tg[t];
    double2* W = D.alloc<double2>((size_t)tg.l * tg.d * m.r);
    D.nn(tg.p, Renv[t + 1], W, tg.l * tg.d, m.r, tg.r, tg.r, m.r, m.r);
    double2* Mh = D.alloc<double2>((size_t)m.d * m.r * m.l);
    HIP_OK(launch_dense_adjoint(m.p, m.l, m.d * m.r, m.d * m.r, nullptr, Mh, m.l, s));
    double2* R2 = D.alloc<double2>((size_t)tg.l * m.l);
    D.nn(W, Mh, R2, tg.l, m.l, tg.d * m.r, tg.d * m.r, m.l, m.l);
    D.release(W);
    D.release(Mh);
    if (Renv[t]) D.release(Renv[t]);
    Renv[t] = R2;
    Rd[t] = tg.l;
    Rm[t] = m.l;
  };
  auto update = [&](int t, double* f) {  // F = Lenv[t] Tg[t] Renv[t+1], normalised
    const Tensor3& tg = Tg[t];
    const int ml = Lm[t], mr = Rm[t + 1];
    double2* Z = D.alloc<double2>((size_t)ml * tg.d * tg.r);
    D.nn(Lenv[t], tg.p, Z, ml, tg.d * tg.r, tg.l, tg.l, tg.d * tg.r, tg.d * tg.r);
    double2* F = D.alloc<double2>((size_t)ml * tg.d * mr);
    D.nn(Z, Renv[t + 1], F, ml * tg.d, mr, tg.r, tg.r, mr, mr);
    D.release(Z);
    *f = D.norm2(F, (int64_t)ml * tg.d * mr);
    D.scale(F, (int64_t)ml * tg.d * mr, 1.0 / std::sqrt(*f));
    return Tensor3{F, ml, tg.d, mr};
  };
  for (int t = 0; t + 1 < ng; ++t) left_env(t);
  double f = 1.0;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int t = ng - 1; t >= 0; --t) {  // right to left
      Tensor3 F = update(t, &f);
      if (t > 0) {
        double2* Q = D.polar(F.p, F.l, F.d * F.r, false);
        D.release(F.p);
        F.p = Q;
      }
      D.release(M[t].p);
      M[t] = F;
      if (t > 0) right_env(t);
    }
    for (int t = 0; t < ng; ++t) {  // left to right
      Tensor3 F = update(t, &f);
      if (t + 1 < ng) {
        double2* Q = D.polar(F.p, F.l * F.d, F.r, true);
        D.release(F.p);
        F.p = Q;
      }
      D.release(M[t].p);
      M[t] = F;
      if (t + 1 < ng) left_env(t);
    }
  }
  if (sweeps == 0) {  // the compression alone: its fidelity is |<M|U psi>|^2
    for (int t = 0; t + 1 < ng; ++t) left_env(t);
    Tensor3 F = update(ng - 1, &f);
    D.release(F.p);
  }
  *f_fit = f;
  // ---- decomposition right to left into the handle's qubit tensors
  double log_f = std::log(f);
  std::vector<int> chi_new = ctx->chi;
  double2* X = Renv[ng];  // the 1 x 1 identity
  int Xr = 1, Xc = 1;
  for (int t = ng - 1; t >= 0; --t) {
    const int a = groups[t].first, b = groups[t].second;
    const Tensor3& m = M[t];
    double2* cur = D.alloc<double2>((size_t)m.l * m.d * Xc);
    D.nn(m.p, X, cur, m.l * m.d, Xc, Xr, Xr, Xc, Xc);
    int rows = m.l * m.d / 2, right = Xc;
    for (int q = b; q >= a; --q) {
      if (q == 0) {
        const double nrm = std::sqrt(D.norm2(cur, (int64_t)2 * right));
        D.scale(cur, 2 * right, 1.0 / nrm);
        HIP_OK(hipMemcpyAsync(ctx->site[0], cur, (size_t)2 * right * 16, hipMemcpyDeviceToDevice, s));
        break;
      }
      const int c2 = 2 * right;
      double2* G = D.alloc<double2>((size_t)c2 * c2);
      D.cn(cur, cur, G, c2, c2, rows, c2, c2, c2);
      DevOps::Eig e = D.eigh(G, c2, c2);
      double fq = 1.0;
      const int kk = dmrg_truncation_rank(e.w, rows, ctx, &fq);
      log_f += std::log(fq);
      // B_q = V_k^H as (kk, 2, right); Lambda_{q-1} = sqrt(w_k) normalised
      HIP_OK(launch_dense_adjoint(e.V, c2, kk, e.ldv, nullptr, (double2*)ctx->site[q], c2, s));
      std::vector<double> lam(kk);
      double kept = 0;
      for (int i = 0; i < kk; ++i) kept += std::max(e.w[i], 0.0);
      for (int i = 0; i < kk; ++i) lam[i] = std::sqrt(std::max(e.w[i], 0.0) / kept);
      HIP_OK(hipMemcpyAsync(ctx->lam[q - 1], lam.data(), kk * sizeof(double), hipMemcpyHostToDevice, s));
      chi_new[q - 1] = kk;
      double2* nxt = D.alloc<double2>((size_t)rows * kk);
      D.nn(cur, e.V, nxt, rows, kk, c2, c2, e.ldv, kk);
      D.release(cur);
      D.release(G);
      D.release(e.base);
      cur = nxt;
      right = kk;
      if (q > a) {
        rows /= 2;
      } else {
        X = cur;
        Xr = rows;
        Xc = kk;
      }
    }
  }
  HIP_OK(hipStreamSynchronize(s));
  ctx->chi = chi_new;
  HIP_OK(hipMemcpyAsync(ctx->d_chi, ctx->chi.data(), (n - 1) * sizeof(int), hipMemcpyHostToDevice, s));
  double lf0 = 0;
  HIP_OK(hipMemcpyAsync(&lf0, ctx->d_logf, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  lf0 += log_f;
  HIP_OK(hipMemcpyAsync(ctx->d_logf, &lf0, sizeof(double), hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  ctx->prev_dw.assign(n - 1, 0.f);
  ctx->prev_tail.assign(n - 1, 1.f);
  ctx->stats.steps += 1;
}

bool options_valid(const mps_options& o) {
  return o.k_max >= 2 && o.k_max <= 12 && o.precision >= 0 && o.precision <= 2 && o.svd_mode >= 0 &&
         o.svd_mode <= 1 && o.batch >= 0 && o.batch <= 2 && o.eig_method >= 0 && o.eig_method <= 2 &&
         o.floor_c >= 0.0;
}

// ---- saved-state files (mps_save / mps_load): little-endian fields in the
// order mps_save writes them, then a 64-bit FNV-1a checksum of the bytes before
constexpr char kSaveMagic[8] = {'C', 'T', 'E', 'B', 'D', 'M', 'P', 'S'};
constexpr uint32_t kSaveVersion = 2;

uint64_t fnv1a(const char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= (unsigned char)p[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct Writer {
  std::vector<char> buf;
  void raw(const void* p, size_t n) { buf.insert(buf.end(), (const char*)p, (const char*)p + n); }
  template <typename T>
  void put(T v) {
    raw(&v, sizeof(T));
  }
};

struct Reader {
  const char* data;
  size_t end;
  size_t pos = 0;
  bool ok = true;
  template <typename T>
  T get() {
    T v{};
    if (!ok || pos + sizeof(T) > end) {
      ok = false;
      return v;
    }
    std::memcpy(&v, data + pos, sizeof(T));
    pos += sizeof(T);
    return v;
  }
  const char* skip(size_t n) {
    if (!ok || pos + n > end) {
      ok = false;
      return data;
    }
    const char* p = data + pos;
    pos += n;
    return p;
  }
};

thread_local std::string g_err;  // message of the last failed call without a handle

// mps_load after its argument checks: the whole file is read and checked on
// the host before a handle exists.  Sub-layers must be as legalize_layer
// leaves them for the saved k_max (distinct qubits, disjoint two-qubit spans
// of at most k_max sites), so that the planner sees only clusters it can form.
mps_status load_checked(const char* path, mps_handle* out) {
  std::vector<char> buf;
  {
    std::ifstream f(path, std::ios::binary);
    if (!f) {
      g_err = "mps_load: cannot open the file";
      return MPS_EIO;
    }
    buf.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
  }
  Reader r{buf.data(), buf.size() >= 8 ? buf.size() - 8 : 0};
  auto bad = [&](const char* why) {
    g_err = std::string("mps_load: ") + why;
    return MPS_EIO;
  };
  if (buf.size() < 16 || std::memcmp(buf.data(), kSaveMagic, 8) != 0) return bad("not a saved state");
  uint64_t sum = 0;
  std::memcpy(&sum, buf.data() + buf.size() - 8, 8);
  if (sum != fnv1a(buf.data(), buf.size() - 8)) return bad("checksum mismatch");
  r.pos = 8;
  if (r.get<uint32_t>() != kSaveVersion) return bad("unknown version");
  const int n = r.get<int32_t>(), chi_max = r.get<int32_t>();
  const double eps = r.get<double>();
  mps_options o{};
  o.k_max = r.get<int32_t>();
  o.q_max = r.get<int32_t>();
  o.l_max = r.get<int32_t>();
  o.precision = r.get<int32_t>();
  o.svd_mode = r.get<int32_t>();
  o.batch = r.get<int32_t>();
  o.eig_method = r.get<int32_t>();
  o.floor_c = r.get<double>();
  o.hip_stream = nullptr;
  const double log_f = r.get<double>();
  mps_stats st{};
  st.steps = r.get<int64_t>();
  st.cluster_updates = r.get<int64_t>();
  st.svds = r.get<int64_t>();
  st.site_updates = r.get<int64_t>();
  st.sketch_accepted = r.get<int64_t>();
  st.sketch_fallback = r.get<int64_t>();
  st.jacobi_sweeps = r.get<int64_t>();
  st.discarded_weight = r.get<double>();
  const uint64_t sk_seed = r.get<uint64_t>();
  const uint32_t sk_stream = r.get<uint32_t>();
  if (!r.ok || n < 2 || n > (1 << 24) || chi_max < 1 || chi_max > 2048 || !(eps >= 0.0) || !options_valid(o))
    return bad("malformed header");
  std::vector<int> chi(n - 1);
  for (int b = 0; b < n - 1; ++b) {
    chi[b] = r.get<int32_t>();
    const int e = std::min(b + 1, n - b - 1);
    const int cap = e >= 30 ? chi_max : std::min(chi_max, 1 << e);
    if (!r.ok || chi[b] < 1 || chi[b] > cap) return bad("bond dimension out of range");
  }
  std::vector<float> pdw(n - 1), ptail(n - 1);
  for (int b = 0; b < n - 1; ++b) {
    pdw[b] = r.get<float>();
    ptail[b] = r.get<float>();
  }
  const size_t esz = o.precision == MPS_PREC_FP64 ? 16 : 8;
  std::vector<const char*> site_at(n), lam_at(n - 1);
  for (int j = 0; j < n; ++j) {
    const size_t bytes = (size_t)(j > 0 ? chi[j - 1] : 1) * 2 * (j < n - 1 ? chi[j] : 1) * esz;
    site_at[j] = r.skip(bytes);
  }
  for (int b = 0; b < n - 1; ++b) lam_at[b] = r.skip(chi[b] * sizeof(double));
  // counts are bounded by the bytes left before anything is sized by them
  const uint32_t nsub = r.get<uint32_t>();
  if (!r.ok || nsub > (r.end - r.pos) / sizeof(uint32_t)) return bad("malformed sub-layer count");
  std::vector<SubLayer> pending(nsub);
  std::vector<char> used(n, 0);
  std::vector<std::pair<int, int>> spans;
  constexpr size_t kGateBytes = 3 * sizeof(int32_t) + 32 * sizeof(double);
  for (auto& sl : pending) {
    const uint32_t ng = r.get<uint32_t>();
    if (!r.ok || ng > (uint32_t)n || ng > (r.end - r.pos) / kGateBytes) return bad("malformed sub-layer");
    sl.resize(ng);
    spans.clear();
    for (auto& g : sl) {
      g.nq = r.get<int32_t>();
      g.q[0] = r.get<int32_t>();
      g.q[1] = r.get<int32_t>();
      for (int e = 0; e < 16; ++e) {
        const double re = r.get<double>(), im = r.get<double>();
        g.u[e] = cplx(re, im);
      }
      // a one-qubit gate holds its qubit twice; a two-qubit gate two qubits
      if (g.nq < 1 || g.nq > 2 || g.q[0] < 0 || g.q[0] >= n || g.q[1] < 0 || g.q[1] >= n ||
          (g.q[0] == g.q[1]) != (g.nq == 1))
        return bad("malformed gate");
      if (g.hi() - g.lo() + 1 > o.k_max) return bad("gate span wider than the saved k_max");
      for (int i = 0; i < g.nq; ++i) {
        if (used[g.q[i]]) return bad("gates of one sub-layer share a qubit");
        used[g.q[i]] = 1;
      }
      if (g.nq == 2) spans.emplace_back(g.lo(), g.hi());
    }
    for (const auto& g : sl)
      for (int i = 0; i < g.nq; ++i) used[g.q[i]] = 0;
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
      if (spans[i].first <= spans[i - 1].second) return bad("two-qubit spans of one sub-layer overlap");
  }
  if (!r.ok || r.pos != buf.size() - 8) return bad("truncated or oversized file");
  mps_handle h = nullptr;
  mps_status cs = mps_create(n, chi_max, eps, &o, &h);
  if (cs != MPS_OK) {
    g_err = "mps_load: could not create the handle (" + g_err + ")";
    return cs;
  }
  mps_ctx* ctx = h;
  cs = guarded(ctx, [&]() -> mps_status {
    hipStream_t s = ctx->stream;
    ctx->chi = chi;
    for (int j = 0; j < n; ++j) {
      const size_t bytes = (size_t)bond_dim(ctx, j - 1) * 2 * bond_dim(ctx, j) * esz;
      HIP_OK(hipMemcpyAsync(ctx->site[j], site_at[j], bytes, hipMemcpyHostToDevice, s));
    }
    for (int b = 0; b < n - 1; ++b)
      HIP_OK(hipMemcpyAsync(ctx->lam[b], lam_at[b], chi[b] * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->d_chi, ctx->chi.data(), (n - 1) * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->d_logf, &log_f, sizeof(double), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));  // the host buffers above are released on return
    ctx->stats = st;
    ctx->prev_dw = pdw;
    ctx->prev_tail = ptail;
    ctx->sketch_seed = sk_seed;
    ctx->sketch_stream = sk_stream;
    ctx->pending.swap(pending);
    return MPS_OK;
  });
  if (cs != MPS_OK) {
    g_err = "mps_load: " + ctx->err;
    mps_destroy(h);
    return cs;
  }
  *out = h;
  return MPS_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

mps_status mps_default_options(mps_options* opt) {
  if (!opt) return MPS_EINVAL;
  opt->k_max = 4;
  opt->q_max = 0;
  opt->l_max = 0;
  opt->precision = MPS_PREC_FP32;
  opt->svd_mode = MPS_SVD_EXACT;
  opt->batch = MPS_BATCH_STEP;
  opt->eig_method = MPS_EIG_AUTO;
  opt->floor_c = 4.0;
  opt->hip_stream = nullptr;
  return MPS_OK;
}

mps_status mps_create(int n, int chi_max, double eps, const mps_options* opt, mps_handle* out) {
  if (!out || n < 2 || chi_max < 1 || chi_max > 2048 || !(eps >= 0.0)) {
    g_err = "mps_create: need n >= 2, 1 <= chi_max <= 2048, eps >= 0 and an output pointer";
    return MPS_EINVAL;
  }
  *out = nullptr;
  mps_ctx* ctx = new (std::nothrow) mps_ctx();
  if (!ctx) {
    g_err = "mps_create: host allocation failed";
    return MPS_ENOMEM;
  }
  mps_status st = guarded(ctx, [&]() -> mps_status {
    if (opt)
      ctx->opt = *opt;
    else
      mps_default_options(&ctx->opt);
    const mps_options& o = ctx->opt;
    if (!options_valid(o)) {
      ctx->err = "invalid options";
      return MPS_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      ctx->err = "no HIP device";
      return MPS_EDEVICE;
    }
    ctx->n = n;
    ctx->chi_max = chi_max;
    ctx->eps = eps;
    ctx->prec = (Prec)o.precision;
    ctx->esz = ctx->prec == Prec::FP64 ? 16 : 8;
    const double u = ctx->prec == Prec::FP64 ? std::pow(2.0, -26.5) : std::pow(2.0, -24.0);
    ctx->eps_eff = std::max(eps, o.floor_c * u);
    ctx->q_max_eff = o.q_max > 0 ? o.q_max : default_q_max(o.k_max, chi_max);
    ctx->l_max_eff = o.l_max > 0 ? o.l_max : (1 << 30);
    if (o.hip_stream) {
      ctx->stream = (hipStream_t)o.hip_stream;
    } else {
      HIP_OK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
      ctx->own_stream = true;
    }
    ctx->cap.resize(n - 1);
    ctx->chi.assign(n - 1, 1);
    ctx->prev_dw.assign(n - 1, 0.f);
    ctx->prev_tail.assign(n - 1, 1.f);
    for (int b = 0; b < n - 1; ++b) {
      const int e = std::min(b + 1, n - b - 1);
      ctx->cap[b] = e >= 30 ? chi_max : std::min(chi_max, 1 << e);
    }
    std::vector<size_t> soff(n), loff(n - 1);
    size_t total = 0;
    auto al = [&](size_t x) {
      const size_t o2 = (total + 255) & ~size_t(255);
      total = o2 + x;
      return o2;
    };
    for (int j = 0; j < n; ++j) {
      const size_t cl = j > 0 ? ctx->cap[j - 1] : 1, cr = j < n - 1 ? ctx->cap[j] : 1;
      soff[j] = al(cl * 2 * cr * ctx->esz);
    }
    for (int b = 0; b < n - 1; ++b) loff[b] = al(ctx->cap[b] * sizeof(double));
    const size_t ones_off = al(4096 * sizeof(double));
    const size_t logf_off = al(sizeof(double));
    HIP_OK(hipMalloc(&ctx->state_mem, total));
    HIP_OK(hipMemsetAsync(ctx->state_mem, 0, total, ctx->stream));
    ctx->site.resize(n);
    ctx->lam.resize(n - 1);
    for (int j = 0; j < n; ++j) ctx->site[j] = ctx->state_mem + soff[j];
    for (int b = 0; b < n - 1; ++b) ctx->lam[b] = (double*)(ctx->state_mem + loff[b]);
    ctx->d_ones = (double*)(ctx->state_mem + ones_off);
    ctx->d_logf = (double*)(ctx->state_mem + logf_off);
    HIP_OK(hipMalloc(&ctx->d_chi, (n - 1) * sizeof(int)));
    HIP_OK(hipMalloc(&ctx->d_work, 4 * sizeof(unsigned long long)));
    HIP_OK(hipHostMalloc(&ctx->h_flags, 4096 * 4 * sizeof(int), hipHostMallocDefault));
    // |0...0>: B_j = e_0 of shape (1, 2, 1); Lambda_b = [1]; ones for edge weights
    std::vector<double> one(4096, 1.0);
    HIP_OK(hipMemcpyAsync(ctx->d_ones, one.data(), 4096 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    const double c64[2] = {1.0, 0.0};
    const float c32[2] = {1.f, 0.f};
    for (int j = 0; j < n; ++j)
      HIP_OK(hipMemcpyAsync(ctx->site[j], ctx->prec == Prec::FP64 ? (const void*)c64 : (const void*)c32,
                            ctx->esz, hipMemcpyHostToDevice, ctx->stream));
    for (int b = 0; b < n - 1; ++b)
      HIP_OK(hipMemcpyAsync(ctx->lam[b], one.data(), sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(ctx->d_chi, ctx->chi.data(), (n - 1) * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return MPS_OK;
  });
  if (st != MPS_OK) {
    g_err = "mps_create: " + ctx->err;
    destroy_ctx(ctx);
    return st;
  }
  *out = ctx;
  return MPS_OK;
}

mps_status mps_destroy(mps_handle h) {
  destroy_ctx(h);
  return MPS_OK;
}

mps_status mps_apply_cluster(mps_handle ctx, const int* qubits, int k, const double* U) {
  if (!ctx || !qubits || !U || k < 1 || k > 12) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    for (int i = 0; i < k; ++i)
      if (qubits[i] < 0 || qubits[i] >= ctx->n || (i > 0 && qubits[i] <= qubits[i - 1])) {
        ctx->err = "qubits must be strictly ascending and in range";
        return MPS_ESPAN;
      }
    const int a = qubits[0], span = qubits[k - 1] - qubits[0] + 1;
    if (span > ctx->opt.k_max || span < 2) {
      ctx->err = "cluster span must be in [2, k_max]";
      return MPS_ESPAN;
    }
    const int dk = 1 << k;
    std::vector<cplx> Uk((size_t)dk * dk);
    for (size_t e = 0; e < Uk.size(); ++e) Uk[e] = cplx(U[2 * e], U[2 * e + 1]);
    if (!is_unitary(ctx, Uk, dk)) {
      ctx->err = "U is not unitary to 1e-10";
      return MPS_ENOTUNITARY;
    }
    flush_all(ctx);
    // embed U on the span: identity on the idle qubits (big-endian positions)
    const int ds = 1 << span;
    std::vector<int> pos(k);
    for (int i = 0; i < k; ++i) pos[i] = span - 1 - (qubits[i] - a);  // bit of qubit i
    int idle_mask = ds - 1;
    for (int i = 0; i < k; ++i) idle_mask &= ~(1 << pos[i]);
    auto sub = [&](int x) {
      int r = 0;
      for (int i = 0; i < k; ++i) r = (r << 1) | ((x >> pos[i]) & 1);
      return r;
    };
    Job job;
    job.a = a;
    job.k = span;
    job.U.assign((size_t)ds * ds, cplx(0));
    for (int i = 0; i < ds; ++i)
      for (int j = 0; j < ds; ++j)
        if ((i & idle_mask) == (j & idle_mask)) job.U[(size_t)i * ds + j] = Uk[(size_t)sub(i) * dk + sub(j)];
    std::vector<Job> jobs{job};
    run_jobs(ctx, jobs, {}, 0);
    return MPS_OK;
  });
}

mps_status mps_run_layer(mps_handle ctx, const mps_gate* gates, int ngates) {
  if (!ctx || ngates < 0 || (ngates > 0 && !gates)) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    const mps_status st = check_gates(ctx, gates, ngates, ctx->n);
    if (st != MPS_OK) return st;
    std::vector<HostGate> layer;
    for (int i = 0; i < ngates; ++i) layer.push_back(to_host_gate(gates[i]));
    legalize_layer(layer, ctx->opt.k_max, ctx->pending);
    // execute every step that can no longer grow
    if (ctx->opt.batch == MPS_BATCH_WAVE && plan_is_chi_free(ctx)) {
      execute_window(ctx, complete_steps(ctx));
      return MPS_OK;
    }
    while (!ctx->pending.empty()) {
      std::vector<Cluster> cl;
      const int end = plan_step(ctx->pending, 0, ctx->n, ctx->chi, ctx->opt.k_max, ctx->q_max_eff,
                                ctx->l_max_eff, cl);
      if (end >= (int)ctx->pending.size()) break;
      execute_step(ctx, end);
    }
    return MPS_OK;
  });
}

mps_status mps_flush(mps_handle ctx) {
  if (!ctx) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    flush_all(ctx);
    return MPS_OK;
  });
}

mps_status mps_queue_layer(mps_handle ctx, const mps_gate* gates, int ngates) {
  if (!ctx || ngates < 0 || (ngates > 0 && !gates)) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    const mps_status st = check_gates(ctx, gates, ngates, ctx->n);
    if (st != MPS_OK) return st;
    std::vector<HostGate> layer;
    for (int i = 0; i < ngates; ++i) layer.push_back(to_host_gate(gates[i]));
    legalize_layer(layer, ctx->opt.k_max, ctx->pending);
    return MPS_OK;
  });
}

mps_status mps_step(mps_handle ctx, int* clusters, int* remaining) {
  if (!ctx) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    const int64_t before = ctx->stats.cluster_updates;
    if (!ctx->pending.empty()) execute_step(ctx, 0);
    if (clusters) *clusters = (int)(ctx->stats.cluster_updates - before);
    if (remaining) *remaining = (int)ctx->pending.size();
    return MPS_OK;
  });
}

mps_status mps_run_steps(mps_handle ctx, int nsteps, int* clusters, int* remaining) {
  if (!ctx || nsteps < 0) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    const int64_t before = ctx->stats.cluster_updates;
    execute_window(ctx, nsteps);
    if (clusters) *clusters = (int)(ctx->stats.cluster_updates - before);
    if (remaining) *remaining = (int)ctx->pending.size();
    return MPS_OK;
  });
}

mps_status mps_clone(mps_handle src, const mps_options* opt, mps_handle* out) {
  if (!src || !opt || !out) return MPS_EINVAL;
  *out = nullptr;
  mps_handle dst = nullptr;
  mps_status st = mps_create(src->n, src->chi_max, src->eps, opt, &dst);
  if (st != MPS_OK) return st;
  mps_ctx* ctx = dst;
  st = guarded(ctx, [&]() -> mps_status {
    HIP_OK(hipStreamSynchronize(src->stream));
    hipStream_t s = dst->stream;
    const int n = src->n;
    for (int j = 0; j < n; ++j) {
      const int64_t cnt = (int64_t)bond_dim(src, j - 1) * 2 * bond_dim(src, j);
      if (src->prec == dst->prec || (src->prec != Prec::FP64 && dst->prec != Prec::FP64))
        HIP_OK(hipMemcpyAsync(dst->site[j], src->site[j], cnt * src->esz, hipMemcpyDeviceToDevice, s));
      else if (src->prec == Prec::FP64)
        HIP_OK(launch_convert_d2f((const double2*)src->site[j], (float2*)dst->site[j], cnt, s));
      else
        HIP_OK(launch_convert_f2d((const float2*)src->site[j], (double2*)dst->site[j], cnt, s));
    }
    for (int b = 0; b < n - 1; ++b)
      HIP_OK(hipMemcpyAsync(dst->lam[b], src->lam[b], src->chi[b] * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(dst->d_chi, src->d_chi, (n - 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(dst->d_logf, src->d_logf, sizeof(double), hipMemcpyDeviceToDevice, s));
    dst->chi = src->chi;
    dst->prev_dw = src->prev_dw;
    dst->prev_tail = src->prev_tail;
    if (dst->opt.k_max == src->opt.k_max) dst->pending = src->pending;
    HIP_OK(hipStreamSynchronize(s));
    return MPS_OK;
  });
  if (st != MPS_OK) {
    mps_destroy(dst);
    return st;
  }
  *out = dst;
  return MPS_OK;
}

mps_status mps_set_options(mps_handle ctx, const mps_options* opt) {
  if (!ctx || !opt) return MPS_EINVAL;
  if (!options_valid(*opt)) {
    ctx->err = "invalid options";
    return MPS_EINVAL;
  }
  return guarded(ctx, [&]() -> mps_status {
    // buffered sub-layers were routed for the current k_max: run them first
    if (opt->k_max != ctx->opt.k_max) flush_all(ctx);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    // the state goes into a handle built with the new options (site tensors
    // converted when the precision changes); the two handles then trade
    // contents, and what a clone does not copy comes along explicitly
    mps_handle fresh = nullptr;
    const mps_status st = mps_clone(ctx, opt, &fresh);
    if (st != MPS_OK) {
      ctx->err = "mps_set_options: the state could not be moved to the new options";
      return st;
    }
    fresh->pending = ctx->pending;
    fresh->stats = ctx->stats;
    fresh->timing = ctx->timing;
    std::swap(fresh->timer, ctx->timer);
    fresh->mlp_params = ctx->mlp_params;
    fresh->log_x.swap(ctx->log_x);
    fresh->log_t.swap(ctx->log_t);
    fresh->sketch_seed = ctx->sketch_seed;
    fresh->sketch_stream = ctx->sketch_stream;
    std::swap(*ctx, *fresh);
    destroy_ctx(fresh);  // now holds the previous state and stream
    return MPS_OK;
  });
}

mps_status mps_save(mps_handle ctx, const char* path) {
  if (!ctx || !path) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    Writer w;
    w.raw(kSaveMagic, 8);
    w.put<uint32_t>(kSaveVersion);
    w.put<int32_t>(ctx->n);
    w.put<int32_t>(ctx->chi_max);
    w.put<double>(ctx->eps);
    const mps_options& o = ctx->opt;
    for (int v : {o.k_max, o.q_max, o.l_max, o.precision, o.svd_mode, o.batch, o.eig_method}) w.put<int32_t>(v);
    w.put<double>(o.floor_c);
    double lf = 0;
    HIP_OK(hipMemcpy(&lf, ctx->d_logf, sizeof(double), hipMemcpyDeviceToHost));
    w.put<double>(lf);
    const mps_stats& st = ctx->stats;
    for (int64_t v : {st.steps, st.cluster_updates, st.svds, st.site_updates, st.sketch_accepted,
                      st.sketch_fallback, st.jacobi_sweeps})
      w.put<int64_t>(v);
    w.put<double>(st.discarded_weight);
    w.put<uint64_t>(ctx->sketch_seed);
    w.put<uint32_t>(ctx->sketch_stream);
    for (int b = 0; b < ctx->n - 1; ++b) w.put<int32_t>(ctx->chi[b]);
    for (int b = 0; b < ctx->n - 1; ++b) {
      w.put<float>(ctx->prev_dw[b]);
      w.put<float>(ctx->prev_tail[b]);
    }
    std::vector<char> tmp;
    for (int j = 0; j < ctx->n; ++j) {  // site tensors as stored (complex64 or complex128)
      const size_t bytes = (size_t)bond_dim(ctx, j - 1) * 2 * bond_dim(ctx, j) * ctx->esz;
      tmp.resize(bytes);
      HIP_OK(hipMemcpy(tmp.data(), ctx->site[j], bytes, hipMemcpyDeviceToHost));
      w.raw(tmp.data(), bytes);
    }
    for (int b = 0; b < ctx->n - 1; ++b) {
      tmp.resize(ctx->chi[b] * sizeof(double));
      HIP_OK(hipMemcpy(tmp.data(), ctx->lam[b], tmp.size(), hipMemcpyDeviceToHost));
      w.raw(tmp.data(), tmp.size());
    }
    w.put<uint32_t>((uint32_t)ctx->pending.size());
    for (const auto& sl : ctx->pending) {
      w.put<uint32_t>((uint32_t)sl.size());
      for (const auto& g : sl) {
        w.put<int32_t>(g.nq);
        w.put<int32_t>(g.q[0]);
        w.put<int32_t>(g.q[1]);
        for (int e = 0; e < 16; ++e) {
          w.put<double>(g.u[e].real());
          w.put<double>(g.u[e].imag());
        }
      }
    }
    w.put<uint64_t>(fnv1a(w.buf.data(), w.buf.size()));
    const std::string part = std::string(path) + ".part";
    {
      std::ofstream f(part, std::ios::binary | std::ios::trunc);
      if (!f) fail(ctx, MPS_EIO, "mps_save: cannot open the file for writing");
      f.write(w.buf.data(), (std::streamsize)w.buf.size());
      if (!f) fail(ctx, MPS_EIO, "mps_save: write failed");
    }
    if (std::rename(part.c_str(), path) != 0) fail(ctx, MPS_EIO, "mps_save: cannot move the file into place");
    return MPS_OK;
  });
}

mps_status mps_load(const char* path, mps_handle* out) {
  if (!path || !out) {
    g_err = "mps_load: null argument";
    return MPS_EINVAL;
  }
  *out = nullptr;
  try {
    return load_checked(path, out);
  } catch (const std::bad_alloc&) {
    g_err = "mps_load: host allocation failed";
    return MPS_ENOMEM;
  } catch (const std::exception& e) {
    g_err = std::string("mps_load: ") + e.what();
    return MPS_EIO;
  }
}

mps_status mps_sketch_range(mps_handle ctx, int n, int s, const double* G, const double* Omega,
                            const double* Probe, double* mu, double* V, double* est, int* accepted) {
  if (!ctx || n < 2 || n > HTD_MAX || s < 1 || s > n || !G || !Omega || !Probe || !mu || !V || !est)
    return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    hipStream_t st = ctx->stream;
    HIP_OK(hipStreamSynchronize(st));
    const size_t ld = (size_t)ceil_div(n, 64) * 64;
    SkRun k;
    k.s = s;
    k.ld_s = ((std::max(s, SK_PROBES) + 7) / 8) * 8;
    k.ld_y = ((s + 63) / 64) * 64;
    int nb = std::max(2, ceil_div(s, JB));
    k.nb = nb + (nb & 1);
    ctx->arena.reset();
    HIP_OK(ctx->arena.reserve(ld * ld * sizeof(double2) + sk_bytes(n, k) + 8192));
    DeviceArena& A = ctx->arena;
    double2* Gd = (double2*)A.take(ld * ld * sizeof(double2));
    int* flags = (int*)A.take(12 * sizeof(int));
    double* scales = (double*)A.take(2 * sizeof(double));
    double* trace = (double*)A.take(sizeof(double));
    int* exact = (int*)A.take(4 * sizeof(int));
    sk_assign(A, k, n, flags, scales);
    double tr = 0;
    for (int i = 0; i < n; ++i) tr += G[2 * ((size_t)i * n + i)];
    HIP_OK(hipMemcpy2DAsync(Gd, ld * sizeof(double2), G, n * sizeof(double2), n * sizeof(double2), n,
                            hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpy2DAsync(k.Omega, k.ld_s * sizeof(double2), Omega, s * sizeof(double2), s * sizeof(double2), n,
                            hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpy2DAsync(k.Probe, k.ld_s * sizeof(double2), Probe, SK_PROBES * sizeof(double2),
                            SK_PROBES * sizeof(double2), n, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(trace, &tr, sizeof(double), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemsetAsync(exact, 0, 4 * sizeof(int), st));
    SkLevel S;
    S.ids.push_back(0);
    const uint32_t stream_before = ctx->sketch_stream;
    add_sketch(ctx, S, k, 0, Gd, (int)ld, fixed(n), n, trace, exact);
    ctx->sketch_stream = stream_before;  // the random streams of the handle's own splits are not consumed
    DescBlob& B = ctx->blob;
    B.host.clear();
    upload_sketch(B, S);
    HIP_OK(B.prepare());
    HIP_OK(B.upload(st));
    std::vector<SkRun> sk{k};
    launch_sketch(ctx, B, S, sk, flags, 1, false);
    int use = 0;
    HIP_OK(hipMemcpyAsync(mu, k.lam, s * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpy2DAsync(V, s * sizeof(double2), k.Vs, k.ld_s * sizeof(double2), s * sizeof(double2), n,
                            hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(est, k.est, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&use, k.use, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (accepted) *accepted = use;
    return MPS_OK;
  });
}

mps_status mps_dmrg_step(mps_handle ctx, const mps_gate* gates, const int* layer_len, int nl, int chi_max_dmrg,
                         int q_max, int sweeps, double* f_fit) {
  if (!ctx) return MPS_EINVAL;
  if (nl < 0 || (nl > 0 && (!gates || !layer_len)) || chi_max_dmrg < 1 || q_max < 1 || sweeps < 0) {
    ctx->err = "mps_dmrg_step: invalid argument (nl >= 0, gates and layer_len, chi_max_dmrg >= 1, q_max >= 1, "
               "sweeps >= 0)";
    return MPS_EINVAL;
  }
  return guarded(ctx, [&]() -> mps_status {
    if (ctx->prec != Prec::FP64) {
      ctx->err = "mps_dmrg_step: needs an FP64 handle";
      return MPS_ESTATE;
    }
    std::vector<std::vector<HostGate>> layers(nl);
    int off = 0;
    for (int l = 0; l < nl; ++l) {
      if (layer_len[l] < 0) {
        ctx->err = "mps_dmrg_step: negative layer length";
        return MPS_EINVAL;
      }
      const mps_status st = check_gates(ctx, gates + off, layer_len[l], ctx->n);
      if (st != MPS_OK) return st;
      for (int i = 0; i < layer_len[l]; ++i) layers[l].push_back(to_host_gate(gates[off + i]));
      off += layer_len[l];
    }
    flush_all(ctx);
    double f = 1.0;
    dmrg_step(ctx, layers, chi_max_dmrg, q_max, sweeps, &f);
    if (f_fit) *f_fit = f;
    return MPS_OK;
  });
}

mps_status mps_overlap(mps_handle a, mps_handle b, double* re, double* im) {
  if (!a || !b || a->n != b->n) return MPS_EINVAL;
  mps_ctx* ctx = a;
  return guarded(ctx, [&]() -> mps_status {
    HIP_OK(hipStreamSynchronize(b->stream));
    HIP_OK(hipStreamSynchronize(a->stream));
    hipStream_t s = a->stream;
    const int n = a->n;
    int ca = 1, cb = 1;
    for (int j = 0; j < n - 1; ++j) {
      ca = std::max(ca, a->chi[j]);
      cb = std::max(cb, b->chi[j]);
    }
    const size_t cmax = std::max(ca, cb);
    ctx->arena.reset();
    HIP_OK(ctx->arena.reserve(8 * cmax * cmax * sizeof(double2) + 4096));
    double2* E[2] = {(double2*)ctx->arena.take(cmax * cmax * sizeof(double2)),
                     (double2*)ctx->arena.take(cmax * cmax * sizeof(double2))};
    double2* T = (double2*)ctx->arena.take(2 * cmax * cmax * sizeof(double2));
    double2* A64 = (double2*)ctx->arena.take(2 * cmax * cmax * sizeof(double2));
    double2* B64 = (double2*)ctx->arena.take(2 * cmax * cmax * sizeof(double2));
    const double2 one = make_double2(1.0, 0.0);
    HIP_OK(hipMemcpyAsync(E[0], &one, sizeof(one), hipMemcpyHostToDevice, s));
    DescBlob& Bl = ctx->blob;
    Bl.host.clear();
    std::vector<size_t> off(2 * n);
    std::vector<int> base{0, 0};
    for (int j = 0; j < n; ++j) {
      const int la = bond_dim(a, j - 1), ra = bond_dim(a, j), lb = bond_dim(b, j - 1), rb = bond_dim(b, j);
      GemmDesc t{};
      t.A = E[j & 1];
      t.B = (b->prec == Prec::FP64) ? b->site[j] : (void*)B64;
      t.C = T;
      t.M = fixed(la);
      t.K = fixed(lb);
      t.N = fixed(2 * rb);
      t.lda = fixed(lb);
      t.ldb = fixed(2 * rb);
      t.ldc = fixed(2 * rb);
      t.batch = 1;
      t.tm = ceil_div(la, 64);
      t.tn = ceil_div(2 * rb, 64);
      t.ksplit = 1;
      t.alpha = 1.0;
      GemmDesc e{};
      e.A = (a->prec == Prec::FP64) ? a->site[j] : (void*)A64;
      e.B = T;
      e.C = E[(j + 1) & 1];
      e.M = fixed(ra);
      e.N = fixed(rb);
      e.K = fixed(2 * la);
      e.lda = fixed(ra);
      e.ldb = fixed(rb);
      e.ldc = fixed(rb);
      e.batch = 1;
      e.tm = ceil_div(ra, 64);
      e.tn = ceil_div(rb, 64);
      e.ksplit = 1;
      e.alpha = 1.0;
      off[2 * j] = Bl.add(&t, sizeof(t));
      off[2 * j + 1] = Bl.add(&e, sizeof(e));
    }
    const size_t boff = Bl.add_vec(base);
    HIP_OK(Bl.upload(s));
    for (int j = 0; j < n; ++j) {
      const int la = bond_dim(a, j - 1), ra = bond_dim(a, j), lb = bond_dim(b, j - 1), rb = bond_dim(b, j);
      if (a->prec != Prec::FP64)
        HIP_OK(launch_convert_f2d((const float2*)a->site[j], A64, (int64_t)la * 2 * ra, s));
      if (b->prec != Prec::FP64)
        HIP_OK(launch_convert_f2d((const float2*)b->site[j], B64, (int64_t)lb * 2 * rb, s));
      HIP_OK(launch_gemm_nn(Prec::FP64, Bl.at<GemmDesc>(off[2 * j]), Bl.at<int>(boff), 1,
                            ceil_div(la, 64) * ceil_div(2 * rb, 64), s));
      HIP_OK(launch_gemm_cn(Bl.at<GemmDesc>(off[2 * j + 1]), Bl.at<int>(boff), 1,
                            ceil_div(ra, 64) * ceil_div(rb, 64), s));
    }
    double2 r;
    HIP_OK(hipMemcpyAsync(&r, E[n & 1], sizeof(r), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (re) *re = r.x;
    if (im) *im = r.y;
    return MPS_OK;
  });
}

mps_status mps_fidelity(mps_handle ctx, double* F_est, double* log_f) {
  if (!ctx) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    double lf = 0;
    HIP_OK(hipMemcpyAsync(&lf, ctx->d_logf, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (F_est) *F_est = std::exp(lf);
    if (log_f) *log_f = lf;
    return MPS_OK;
  });
}

mps_status mps_bond_dims(mps_handle ctx, int* chi) {
  if (!ctx || !chi) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    std::memcpy(chi, ctx->chi.data(), (ctx->n - 1) * sizeof(int));
    return MPS_OK;
  });
}

mps_status mps_schmidt(mps_handle ctx, int bond, double* sigma, int cap, int* len) {
  if (!ctx || bond < 0 || bond >= ctx->n - 1 || !len) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    const int c = ctx->chi[bond];
    *len = c;
    if (sigma && cap > 0)
      HIP_OK(hipMemcpy(sigma, ctx->lam[bond], std::min(c, cap) * sizeof(double), hipMemcpyDeviceToHost));
    return MPS_OK;
  });
}

mps_status mps_export_site(mps_handle ctx, int site, double* Bout, int64_t cap, int* dims) {
  if (!ctx || site < 0 || site >= ctx->n || !dims) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    const int cl = bond_dim(ctx, site - 1), cr = bond_dim(ctx, site);
    dims[0] = cl;
    dims[1] = 2;
    dims[2] = cr;
    const int64_t cnt = (int64_t)cl * 2 * cr;
    if (!Bout) return MPS_OK;
    if (cap < cnt) {
      ctx->err = "export buffer too small";
      return MPS_EINVAL;
    }
    if (ctx->prec == Prec::FP64) {
      HIP_OK(hipMemcpy(Bout, ctx->site[site], cnt * 16, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp(2 * cnt);
      HIP_OK(hipMemcpy(tmp.data(), ctx->site[site], cnt * 8, hipMemcpyDeviceToHost));
      for (int64_t e = 0; e < 2 * cnt; ++e) Bout[e] = tmp[e];
    }
    return MPS_OK;
  });
}

mps_status mps_import(mps_handle ctx, const int* chi, const double* const* sites, const double* const* lams,
                      double log_f) {
  if (!ctx || !chi || !sites || !lams) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    for (int b = 0; b < ctx->n - 1; ++b)
      if (chi[b] < 1 || chi[b] > ctx->cap[b]) {
        ctx->err = "bond dimension exceeds capacity";
        return MPS_EINVAL;
      }
    flush_all(ctx);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (int b = 0; b < ctx->n - 1; ++b) ctx->chi[b] = chi[b];
    for (int j = 0; j < ctx->n; ++j) {
      const int64_t cnt = (int64_t)bond_dim(ctx, j - 1) * 2 * bond_dim(ctx, j);
      if (ctx->prec == Prec::FP64) {
        HIP_OK(hipMemcpy(ctx->site[j], sites[j], cnt * 16, hipMemcpyHostToDevice));
      } else {
        std::vector<float> tmp(2 * cnt);
        for (int64_t e = 0; e < 2 * cnt; ++e) tmp[e] = (float)sites[j][e];
        HIP_OK(hipMemcpy(ctx->site[j], tmp.data(), cnt * 8, hipMemcpyHostToDevice));
      }
    }
    for (int b = 0; b < ctx->n - 1; ++b)
      HIP_OK(hipMemcpy(ctx->lam[b], lams[b], chi[b] * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(ctx->d_chi, ctx->chi.data(), (ctx->n - 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(ctx->d_logf, &log_f, sizeof(double), hipMemcpyHostToDevice));
    ctx->prev_dw.assign(ctx->n - 1, 0.f);
    ctx->prev_tail.assign(ctx->n - 1, 1.f);
    return MPS_OK;
  });
}

mps_status mps_amplitudes(mps_handle ctx, double* psi, int64_t cap) {
  if (!ctx || !psi || ctx->n > 24 || cap < ((int64_t)1 << ctx->n)) return MPS_EINVAL;
  return guarded(ctx, [&]() -> mps_status {
    flush_all(ctx);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    // host contraction B_0 B_1 ... B_{n-1} in FP64 (a read-out for tests)
    std::vector<cplx> cur(2), nxt;
    int cols = 1;
    int64_t rows = 1;
    std::vector<double> buf;
    for (int j = 0; j < ctx->n; ++j) {
      int dims[3];
      const int cl = bond_dim(ctx, j - 1), cr = bond_dim(ctx, j);
      buf.assign((size_t)2 * cl * 2 * cr, 0.0);
      mps_status st = mps_export_site(ctx, j, buf.data(), (int64_t)cl * 2 * cr, dims);
      if (st != MPS_OK) return st;
      if (j == 0) {
        cur.assign((size_t)2 * cr, cplx(0));
        for (int e = 0; e < 2 * cr; ++e) cur[e] = cplx(buf[2 * e], buf[2 * e + 1]);
        rows = 2;
        cols = cr;
        continue;
      }
      nxt.assign((size_t)rows * 2 * cr, cplx(0));
      for (int64_t r = 0; r < rows; ++r)
        for (int l = 0; l < cl; ++l) {
          const cplx x = cur[(size_t)r * cols + l];
          if (x == cplx(0)) continue;
          for (int e = 0; e < 2 * cr; ++e)
            nxt[(size_t)r * 2 * cr + e] += x * cplx(buf[2 * ((size_t)l * 2 * cr + e)], buf[2 * ((size_t)l * 2 * cr + e) + 1]);
        }
      rows *= 2;
      cols = cr;
      cur.swap(nxt);
    }
    for (int64_t i = 0; i < rows; ++i) {
      psi[2 * i] = cur[i].real();
      psi[2 * i + 1] = cur[i].imag();
    }
    return MPS_OK;
  });
}

mps_status mps_get_stats(mps_handle ctx, mps_stats* st) {
  if (!ctx || !st) return MPS_EINVAL;
  *st = ctx->stats;
  return MPS_OK;
}

mps_status mps_set_timing(mps_handle ctx, int on) {
  if (!ctx) return MPS_EINVAL;
  ctx->timing = on != 0;
  return MPS_OK;
}

mps_status mps_set_burst_timing(mps_handle ctx, const char* kernel_class, int stride, int reps) {
  if (!ctx) return MPS_EINVAL;
  if (!kernel_class || !*kernel_class) {
    ctx->timer.burst.clear();
    return MPS_OK;
  }
  const bool known = std::strcmp(kernel_class, "trd_hemv") == 0 || std::strcmp(kernel_class, "trd_col") == 0;
  if (!known || stride < 1 || reps < 0 || reps > 64) {
    ctx->err = "mps_set_burst_timing: only trd_col and trd_hemv, with stride >= 1 and 0 <= reps <= 64";
    return MPS_EINVAL;
  }
  auto& t = ctx->timer;
  const int c = t.cls_of(kernel_class);
  if (t.burst_seen.size() < t.names.size()) t.burst_seen.resize(t.names.size(), 0);
  t.burst[c] = {stride, reps};
  t.burst_seen[c] = 0;
  return MPS_OK;
}

mps_status mps_kernel_dispatches(mps_handle ctx, int64_t* dispatches, int cap, int* count) {
  if (!ctx || !count) return MPS_EINVAL;
  const int c = (int)ctx->timer.names.size();
  *count = c;
  for (int i = 0; i < c && i < cap; ++i)
    if (dispatches) dispatches[i] = ctx->timer.dispatches[i];
  return MPS_OK;
}

mps_status mps_kernel_times(mps_handle ctx, double* ms, int64_t* launches, double* flop, int cap, char* names,
                            int names_cap, int* count) {
  if (!ctx || !count) return MPS_EINVAL;
  const int c = (int)ctx->timer.names.size();
  *count = c;
  std::string all;
  for (int i = 0; i < c; ++i) {
    if (i < cap) {
      if (ms) ms[i] = ctx->timer.ms[i];
      if (launches) launches[i] = ctx->timer.launches[i];
      if (flop) flop[i] = ctx->timer.flop[i];
    }
    all += (i ? "," : "") + ctx->timer.names[i];
  }
  if (names && names_cap > 0) {
    std::strncpy(names, all.c_str(), names_cap - 1);
    names[names_cap - 1] = 0;
  }
  return MPS_OK;
}


mps_status mps_heev(int n, const double* A, double* w, double* V) {
  if (n < 1 || n > HTD_MAX || !A || !w || !V) {
    g_err = "mps_heev: need 1 <= n <= 2048 and non-null pointers";
    return MPS_EINVAL;
  }
  mps_ctx tmp;
  tmp.n = 1;
  char* mem = nullptr;
  mps_status st = guarded(&tmp, [&]() -> mps_status {
    mps_ctx* ctx = &tmp;
    HIP_OK(hipStreamCreateWithFlags(&tmp.stream, hipStreamNonBlocking));
    const size_t ld = (size_t)ceil_div(n, 64) * 64;
    HtdDesc h{};
    size_t bytes = 0;
    auto count = [&](size_t x) -> void* {
      bytes = ((bytes + 255) & ~size_t(255)) + x;
      return nullptr;
    };
    count(ld * ld * sizeof(double2));
    count(ld * ld * sizeof(double2));
    htd_layout(ld, h, count);
    count(sizeof(HtdDesc));
    HIP_OK(hipMalloc(&mem, bytes));
    size_t used = 0;
    auto take = [&](size_t x) -> void* {
      const size_t off = (used + 255) & ~size_t(255);
      used = off + x;
      return mem + off;
    };
    h.A = (double2*)take(ld * ld * sizeof(double2));
    h.V = (double2*)take(ld * ld * sizeof(double2));
    htd_layout(ld, h, take);
    h.n = Dim{n, nullptr};
    h.ld = (int)ld;
    h.rcap = n;
    h.skip = nullptr;
    hipStream_t s = tmp.stream;
    HIP_OK(hipMemcpy2DAsync(h.A, ld * sizeof(double2), A, n * sizeof(double2), n * sizeof(double2), n,
                            hipMemcpyHostToDevice, s));
    HtdDesc* dd = (HtdDesc*)take(sizeof(HtdDesc));
    HIP_OK(hipMemcpyAsync(dd, &h, sizeof(HtdDesc), hipMemcpyHostToDevice, s));
    solve_htd(ctx, dd, std::vector<HtdDesc>{h});
    HIP_OK(hipMemcpyAsync(w, h.lam, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpy2DAsync(V, n * sizeof(double2), h.V, ld * sizeof(double2), n * sizeof(double2), n,
                            hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    // the solver orders eigenpairs by descending eigenvalue; this entry point ascending
    std::reverse(w, w + n);
    for (int i = 0; i < n; ++i) {
      double2* row = reinterpret_cast<double2*>(V) + (size_t)i * n;
      std::reverse(row, row + n);
    }
    return MPS_OK;
  });
  if (tmp.stream) {
    (void)hipStreamSynchronize(tmp.stream);
    (void)hipStreamDestroy(tmp.stream);
  }
  if (mem) (void)hipFree(mem);
  if (st != MPS_OK) g_err = "mps_heev: " + tmp.err;
  return st;
}

}  // extern "C"

namespace {
// Workspace of mps_heev_noalloc: the working matrix, the eigenvector matrix,
// the tridiagonal solver's buffers and its descriptor for n <= 512 (15.2 MiB
// of the 16 MiB).  Every GPU that runs the call holds its own copy until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress gives on that device.
constexpr int HEEV_NOALLOC_MAX_N = 512;
constexpr size_t HEEV_SCRATCH_BYTES = size_t(16) << 20;
__device__ __align__(256) char scratch[HEEV_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_at[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_at[dev] = (char*)p;
  }
  *out = g_scratch_at[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

mps_status mps_heev_noalloc(int n, const double* A, double* w, double* V, void* stream) {
  if (n < 1 || n > HEEV_NOALLOC_MAX_N || !A || !w || !V) {
    g_err = "mps_heev_noalloc: need 1 <= n <= 512 and non-null device pointers";
    return MPS_EINVAL;
  }
  mps_ctx tmp;
  tmp.n = 1;
  tmp.stream = (hipStream_t)stream;
  const mps_status st = guarded(&tmp, [&]() -> mps_status {
    mps_ctx* ctx = &tmp;
    char* base = nullptr;
    HIP_OK(scratch_address(&base));
    const size_t ld = (size_t)ceil_div(n, 64) * 64;
    size_t used = 0;
    auto take = [&](size_t x) -> void* {
      const size_t off = (used + 255) & ~size_t(255);
      used = off + x;
      return base + off;
    };
    HtdDesc h{};
    h.A = (double2*)take(ld * ld * sizeof(double2));
    h.V = (double2*)take(ld * ld * sizeof(double2));
    htd_layout(ld, h, take);
    HtdDesc* dd = (HtdDesc*)take(sizeof(HtdDesc));
    if (used > HEEV_SCRATCH_BYTES) fail(ctx, MPS_EINVAL, "workspace larger than the scratch array");
    h.n = Dim{n, nullptr};
    h.ld = (int)ld;
    h.rcap = n;
    h.skip = nullptr;
    hipStream_t s = tmp.stream;
    HIP_OK(hipMemcpy2DAsync(h.A, ld * sizeof(double2), A, n * sizeof(double2), n * sizeof(double2), n,
                            hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(dd, &h, sizeof(HtdDesc), hipMemcpyHostToDevice, s));
    solve_htd(ctx, dd, std::vector<HtdDesc>{h});
    HIP_OK(launch_heev_out(h.V, (int)ld, h.lam, n, (double2*)V, w, s));
    HIP_OK(hipStreamSynchronize(s));
    return MPS_OK;
  });
  if (st != MPS_OK) g_err = "mps_heev_noalloc: " + tmp.err;
  tmp.stream = nullptr;  // the caller's stream
  return st;
}

mps_status mps_kernel_bytes(mps_handle ctx, double* bytes, int cap, int* count) {
  if (!ctx || !count) return MPS_EINVAL;
  const int c = (int)ctx->timer.names.size();
  *count = c;
  for (int i = 0; i < c && i < cap; ++i)
    if (bytes) bytes[i] = ctx->timer.bytes[i];
  return MPS_OK;
}

const char* mps_last_error(mps_handle ctx) {
  if (ctx) return ctx->err.c_str();
  return g_err.empty() ? "null handle" : g_err.c_str();
}

mps_status mps_plan(int n, int k_max, int q_max, int l_max, const int* chi, const mps_gate* gates,
                    const int* layer_len, int nl, int start, int* out_end, int* out_clusters, int cap,
                    int* out_count, int* n_sub) {
  if (n < 2 || k_max < 2 || !chi || !layer_len || nl < 0 || !out_end || !out_count || (cap > 0 && !out_clusters)) {
    g_err = "mps_plan: bad argument (n >= 2, k_max >= 2, non-null arrays)";
    return MPS_EINVAL;
  }
  try {
    std::vector<SubLayer> subs;
    int off = 0;
    for (int l = 0; l < nl; ++l) {
      if (layer_len[l] < 0 || (layer_len[l] > 0 && !gates)) {
        g_err = "mps_plan: bad layer length or null gates";
        return MPS_EINVAL;
      }
      if (const char* why = gate_error(gates + off, layer_len[l], n)) {
        g_err = std::string("mps_plan: ") + why;
        return MPS_EINVAL;
      }
      std::vector<HostGate> layer;
      for (int i = 0; i < layer_len[l]; ++i) layer.push_back(to_host_gate(gates[off + i]));
      off += layer_len[l];
      legalize_layer(layer, k_max, subs);
    }
    if (n_sub) *n_sub = (int)subs.size();
    if (start < 0 || start >= (int)subs.size()) {
      *out_end = start;
      *out_count = 0;
      if (subs.empty()) return MPS_OK;
      g_err = "mps_plan: start outside the sub-layers";
      return MPS_EINVAL;
    }
    std::vector<int> ch(chi, chi + n - 1);
    std::vector<Cluster> cl;
    const int qm = q_max > 0 ? q_max : 62;
    const int lm = l_max > 0 ? l_max : (1 << 30);
    *out_end = plan_step(subs, start, n, ch, k_max, qm, lm, cl);
    *out_count = (int)cl.size();
    for (int i = 0; i < (int)cl.size() && i < cap; ++i) {
      out_clusters[2 * i] = cl[i].a;
      out_clusters[2 * i + 1] = cl[i].k;
    }
    return MPS_OK;
  } catch (const std::bad_alloc&) {
    g_err = "mps_plan: host allocation failed";
    return MPS_ENOMEM;
  } catch (...) {
    g_err = "mps_plan: unexpected error";
    return MPS_EINVAL;
  }
}

}  // extern "C"
