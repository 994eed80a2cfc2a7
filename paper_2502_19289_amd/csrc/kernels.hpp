// Descriptors and launchers of the device kernels (all grouped: one launch
// serves a list of independent problems, one workgroup per output tile).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace ctebd {

// Every kernel of the library is launched through here.
template <typename... KArgs, typename... P>
inline void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shmem, hipStream_t s, P... args) {
  hipLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, s, args...);
}

// ---------------------------------------------------------------- GEMM ----
// C = alpha * A * B                         (mode NN)
// C = (W X)^H (W X), W = diag(w[row>>wshift])  (mode GRAM: A = B = X, FP64 out,
//                                            tiles with ti <= tj only, mirrored)
// Row-major complex matrices; batch b offsets A, B, C by b*sA, b*sB, b*sC.
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  Dim M, N, K, lda, ldb, ldc;
  int64_t sA, sB, sC;
  int batch;
  int tm, tn;       // tile counts the grid reserves (upper bounds)
  int ksplit;       // GRAM: K is cut into ksplit slices written to C + s*part
  int64_t part;     // element stride between the partial results of slices
  const double* w;  // GRAM row weights
  int wshift;
  double alpha;
  const int* skip;  // when non-null and *skip != 0 the problem is skipped
};

struct GramReduceDesc {
  const double2* part;  // ksplit partial results, stride `part` elements
  double2* G;
  Dim n, ld;
  int ksplit;
  int64_t stride;
  int tiles;            // element tiles of 64x64 reserved by the grid
};

enum class Prec : int { FP64 = 0, FP32 = 1, BF16X6 = 2 };

int gemm_tiles(const GemmDesc& d);  // blocks one problem needs

// Launches over `nprob` descriptors already in device memory (d_desc) with
// per-problem block offsets d_base (exclusive prefix, nprob+1 entries).
hipError_t launch_gemm_nn(Prec p, const GemmDesc* d_desc, const int* d_base, int nprob, int blocks,
                          hipStream_t s);
hipError_t launch_gram(Prec in_prec, const GemmDesc* d_desc, const int* d_base, int nprob,
                       int blocks, hipStream_t s);
hipError_t launch_gram_reduce(const GramReduceDesc* d_desc, const int* d_base, int nprob, int blocks,
                              hipStream_t s);
// complex64 C = A B as six BF16 matrix-core products per real product
hipError_t launch_gemm_bf16x6(const GemmDesc* d_desc, const int* d_base, int nprob, int blocks, hipStream_t s);
// C = A^H B in FP64 (A: K x M, B: K x N, row-major) -- overlaps of two states
hipError_t launch_gemm_cn(const GemmDesc* d_desc, const int* d_base, int nprob, int blocks, hipStream_t s);

// ------------------------------------------------------ eigen (Jacobi) ----
constexpr int JB = 32;        // Jacobi block size: subproblems are 2*JB square
constexpr int JP = 2 * JB;    // subproblem / update-tile size

struct EigDesc {
  double2* G;       // Hermitian Gram matrix (FP64), ld x ld
  double2* V;       // eigenvectors (columns, FP64), ld x ld
  void* Gw;         // working copy rotated to diagonal form (G itself, or the sketch's)
  void* Vw;         // working eigenvectors (V itself, or the sketch's)
  void* J;          // workspace: npair_max subproblem rotations of JP x JP
  int* pair_rot;    // per pair slot: rotation applied this round
  int* flags;       // [0] converged, [1] rotated during the current sweep
  double* scale;    // trace of G (set by eig_init)
  unsigned long long* work;  // complex MACs executed by eig_update (or null)
  Dim n;            // matrix size
  int ld;
  int nb_max;       // block count the grids reserve (even)
  double tol;       // relative off-diagonal threshold
};

hipError_t launch_eig_init(const EigDesc* d, int nprob, int ld_max, hipStream_t s);
hipError_t launch_eig_pairs(const EigDesc* d, const int* d_base, int nprob, int blocks, int round, hipStream_t s);
hipError_t launch_eig_update(const EigDesc* d, const int* d_base, int nprob, int blocks, int round, hipStream_t s);
hipError_t launch_eig_sweep_end(const EigDesc* d, int nprob, hipStream_t s);

// ------------------------------- tridiagonal divide-and-conquer eigen ----
// Hermitian G = Q T Q^H (Householder, T real tridiagonal), T = Z diag(w) Z^T
// (Cuppen divide and conquer), eigenvectors Q Z (blocked back-transformation).
constexpr int HTD_MAX = 2048;  // largest n: per-node lists are staged in LDS
constexpr int HTD_NB = 32;     // reflectors per back-transformation block
constexpr int HV_T = 64;       // edge of the HEMV tiles of the trailing block's lower triangle
constexpr int HV_TMAX = HTD_MAX / HV_T;  // tile rows at most
constexpr int HV_SLOTS = HV_TMAX + 2;    // y slots at most: one per tile column, two panel terms
constexpr int HV_PARTS = HV_TMAX * (HV_TMAX + 1) / 2 + 2 * HV_TMAX;  // HEMV workgroups at most
constexpr int HTD_KP = 2 + 2 * HTD_NB;  // per trd_col workgroup: (max, sum of squares), V^H x, W^H x
constexpr int KC_ROWS = 32;    // column rows per trd_col workgroup (8 per wavefront)
constexpr int BT_CH = 64;      // rows per split-K chunk of the back-transformation
constexpr int BT_NB = 32;      // reflectors per block of the back-transformation

struct HtdDesc {
  double2* A;       // n x n Hermitian (ld); the reduction keeps the lower triangle
                    // of the trailing block and the entries less than 64 above
                    // its diagonal up to date; row k keeps reflector v_k (cols > k)
  double2* V;       // out: eigenvectors as columns (ld), descending eigenvalues
  double* lam;      // out: eigenvalues, descending (n)
  Dim n;
  int ld;
  int rcap;         // eigenvectors needed: the first min(n, rcap) columns of V
  const int* skip;  // nonzero: the problem is solved elsewhere (accepted sketch)
  // reduction to tridiagonal form
  double* d;        // diagonal of T (n)
  double* e;        // off-diagonal of T (n - 1)
  double2* tau;     // reflector scalars (n - 1)
  double2* PV;      // panel reflectors V (n x HTD_NB, row-major)
  double2* PW;      // panel vectors W (n x HTD_NB, row-major), finalised
  double2* Y;       // HEMV partial sums of y (slot s, trailing row r at s * ld + r)
  double2* xb;      // the current column brought up to date (n)
  double2* kpart;   // per trd_col workgroup: HTD_KP partial results
  double2* part;    // per HEMV tile: its share of y^H v
  // divide and conquer (node lists are indexed by the node's first row)
  double* Q[2];     // n x n (ld) block-diagonal eigenvector matrices by level
                    // parity, stored by columns: Q[col * ld + row]
  double* D[2];     // eigenvalues of the nodes, ascending within a node
  double* unrm;     // 1 / norm of the rank-one problem's eigenvector of each root
  double* dl;       // non-deflated poles (ascending)
  double* w;        // their z components
  int* ndcol;       // their columns
  double* dval;     // deflated eigenvalues (sorted)
  int* dcol;        // their columns
  int* rot_a;       // deflation rotations: column pair, cosine, sine
  int* rot_b;
  double* rot_c;
  double* rot_s;
  int* origin;      // secular roots: lambda_k = dl[origin_k] + stau_k
  double* stau;
  double* zhat;     // recomputed z (Loewner)
  int* pos_nd;      // output position of root k within its node
  int* cnt;         // 4 ints per node: non-deflated, deflated, rotations, merged
  double* rho;      // per node: rank-one weight
  // back-transformation
  double2* T;       // per block of BT_NB reflectors: BT_NB x BT_NB upper triangle
  double2* Wp;      // split-K partials: ceil(ld / BT_CH) x BT_NB x ld
  double2* W;       // T (V_b^H Z): BT_NB x ld
};

// The columns from htd_tail_start(n) on (a panel boundary where the trailing
// size is at most HTD_TAIL) are reduced by trd_tail in one workgroup per
// problem; the blocked kernels stop there.
constexpr int HTD_TAIL = 128;
__host__ __device__ inline int htd_tail_start(int n) {
  return n <= HTD_TAIL ? 0 : ((n - HTD_TAIL + HTD_NB - 1) / HTD_NB) * HTD_NB;
}

// Per-problem workgroup counts of the launches (identical on host and device).
// HEMV: tile rows T of the trailing block; T (T + 1) / 2 workgroups for the
// tiles of its lower triangle and 2 T for the panel terms; T + 2 y slots.
// The tile grid of column k starts o = (k + 1) % 8 rows and columns before
// the trailing block (at absolute index (k + 1) - o), so that every row
// segment of a tile is whole 128-byte lines (ld is a multiple of 64); the
// first o rows and columns are read and masked.  m + o <= n keeps T <= HV_TMAX.
__host__ __device__ inline int htd_hemv_off(int k) { return (k + 1) & 7; }
__host__ __device__ inline int htd_hemv_rows(int n, int k) {
  const int m = n - k - 1;
  return m > 0 && k < htd_tail_start(n) ? (m + htd_hemv_off(k) + HV_T - 1) / HV_T : 0;
}
__host__ __device__ inline int htd_hemv_blocks(int n, int k) {
  const int t = htd_hemv_rows(n, k);
  return t * (t + 1) / 2 + 2 * t;
}
__host__ __device__ inline int htd_col_blocks(int n, int k) {
  const int m = n - k - 1;
  return m > 0 && k < htd_tail_start(n) ? (m + KC_ROWS - 1) / KC_ROWS : 0;
}
// panel starting at column p0: trailing matrix from p0 + min(HTD_NB, n - 1 - p0),
// the 64 x 64 tiles of its lower triangle and those just above the diagonal
__host__ __device__ inline int htd_her2k_blocks(int n, int p0) {
  const int nbp = n - 1 - p0 < HTD_NB ? n - 1 - p0 : HTD_NB;
  if (nbp <= 0 || p0 >= htd_tail_start(n)) return 0;
  const int t = (n - p0 - nbp + 63) / 64;
  return t * (t + 1) / 2 + t - 1;
}
__host__ __device__ inline int htd_rows(int n) { return (n + 255) / 256; }
__host__ __device__ inline int htd_waves(int n) { return (n + 3) / 4; }  // one wavefront per index
__host__ __device__ inline int htd_tiles64(int n) { return ((n + 63) / 64) * ((n + 63) / 64); }
__host__ __device__ inline int htd_nodes(int n, int L) { return (n + (1 << L) - 1) >> L; }
// dc_place: one workgroup per 64 columns of every node
__host__ __device__ inline int htd_place_blocks(int n, int L) { return htd_nodes(n, L) * (((1 << L) + 63) / 64); }
__host__ __device__ inline int htd_gemm_tiles(int n, int L) {
  const int t = ((1 << L) + 63) / 64;
  return htd_nodes(n, L) * t * t;
}
__host__ __device__ inline int htd_nblk(int n) { return n >= 2 ? (n - 2) / BT_NB + 1 : 0; }
__host__ __device__ inline int htd_bt_rows(int n, int b) { return n - BT_NB * b - 1; }
// nc: eigenvector columns back-transformed, min(n, rcap)
__host__ __device__ inline int htd_wpart_blocks(int n, int nc, int b) {
  return b < htd_nblk(n) ? ((htd_bt_rows(n, b) + BT_CH - 1) / BT_CH) * ((nc + 63) / 64) : 0;
}
constexpr int BT_WC = 8;  // columns of W per reduction workgroup (BT_NB x BT_WC = 256 entries)
__host__ __device__ inline int htd_wred_blocks(int n, int nc, int b) {
  return b < htd_nblk(n) ? (nc + BT_WC - 1) / BT_WC : 0;
}
__host__ __device__ inline int htd_update_blocks(int n, int nc, int b) {
  return b < htd_nblk(n) ? ((htd_bt_rows(n, b) + 63) / 64) * ((nc + 63) / 64) : 0;
}

// Sizes of the problems of one launch (at most HTD_GROUP), passed by value.
constexpr int HTD_GROUP = 64;
struct HtdSizes {
  int np;
  int n[HTD_GROUP];   // matrix sizes
  int nc[HTD_GROUP];  // eigenvector columns back-transformed: min(n, rcap)
};

// Buffers of the tridiagonal solver for Gram matrices of leading dim ld;
// take(bytes) returns device memory (or only counts it).  The buffers are
// taken in this order, each 256-byte aligned, so that a kernel can derive
// them from the first one (htd_view) without reading a descriptor.
template <typename F>
__host__ __device__ inline void htd_layout(size_t ld, HtdDesc& h, F take) {
  const size_t nd = ld * sizeof(double), ni = ld * sizeof(int), nc = ld * sizeof(double2);
  h.d = (double*)take(nd);
  h.e = (double*)take(nd);
  h.lam = (double*)take(nd);
  h.tau = (double2*)take(nc);
  h.PV = (double2*)take(HTD_NB * nc);
  h.PW = (double2*)take(HTD_NB * nc);
  h.Y = (double2*)take(((ld + HV_T - 1) / HV_T + 2) * nc);
  h.xb = (double2*)take(nc);
  h.kpart = (double2*)take((ld / KC_ROWS + 1) * HTD_KP * sizeof(double2));
  {
    const size_t t = (ld + HV_T - 1) / HV_T;
    h.part = (double2*)take((t * (t + 1) / 2 + 2 * t) * sizeof(double2));
  }
  for (int q = 0; q < 2; ++q) {
    h.Q[q] = (double*)take(ld * nd);
    h.D[q] = (double*)take(nd);
  }
  h.unrm = (double*)take(nd);
  h.dl = (double*)take(nd);
  h.w = (double*)take(nd);
  h.ndcol = (int*)take(ni);
  h.dval = (double*)take(nd);
  h.dcol = (int*)take(ni);
  h.rot_a = (int*)take(ni);
  h.rot_b = (int*)take(ni);
  h.rot_c = (double*)take(nd);
  h.rot_s = (double*)take(nd);
  h.origin = (int*)take(ni);
  h.stau = (double*)take(nd);
  h.zhat = (double*)take(nd);
  h.pos_nd = (int*)take(ni);
  h.cnt = (int*)take(4 * ni);
  h.rho = (double*)take(nd);
  h.T = (double2*)take((ld / BT_NB + 1) * BT_NB * BT_NB * sizeof(double2));
  h.Wp = (double2*)take(((ld + BT_CH - 1) / BT_CH) * BT_NB * nc);
  h.W = (double2*)take(BT_NB * nc);
}

// The problems of one launch of the column update and the HEMV, passed by
// value: with the sizes, the Gram matrix, the first workspace buffer (h.d)
// and the skip flag of each problem, the kernels reach every buffer without
// a dependent load of a descriptor (the launch-to-data latency of these short
// kernels is most of their run time).
// Kernel arguments live in memory that the scalar cache misses on every
// launch, so each problem's fields share one 32-byte record (one 64-byte
// line); the launches index the problems by blockIdx.y.
struct alignas(32) HtdProb {
  double2* A;
  char* ws;
  const int* skip;
  int n, ld;
};
struct HtdArgs {
  HtdProb pr[HTD_GROUP];
  int np;
};
// What a launch passes: the records of its problems only, in an argument
// block sized for at most N problems (N the smallest power of two >= the
// launch's problem count), which keeps the host's per-launch work small (a
// chain of empty launches with a 2.3 KB argument block enqueues 1.2 us per
// launch slower than with an 8-byte one on MI355X).
template <int N>
struct HtdProbs {
  HtdProb pr[N];
};

// The buffers of problem record q, laid out as htd_layout takes them.
__host__ __device__ inline HtdDesc htd_view(const HtdProb& q) {
  HtdDesc h{};
  char* base = q.ws;
  size_t off = 0;
  htd_layout((size_t)q.ld, h, [&](size_t x) -> void* {
    off = (off + 255) & ~size_t(255);
    void* r = base + off;
    off += x;
    return r;
  });
  h.A = q.A;
  h.ld = q.ld;
  h.skip = q.skip;
  return h;
}
__host__ __device__ inline HtdDesc htd_view(const HtdArgs& a, int p) { return htd_view(a.pr[p]); }

// launches over the problems of sz (descriptors in device memory; `blocks` is
// the sum of the per-problem counts above for the given step / level / block)
// or of a (grid blocks x a.np, `blocks` the largest per-problem count)
hipError_t launch_trd_col(const HtdArgs& a, int k, int blocks, hipStream_t s);
hipError_t launch_trd_tail(const HtdDesc* d, const HtdSizes& sz, hipStream_t s);
hipError_t launch_trd_hemv(const HtdArgs& a, int k, int blocks, hipStream_t s);
hipError_t launch_trd_her2k(const HtdDesc* d, const HtdSizes& sz, int p0, int blocks, hipStream_t s);
hipError_t launch_trd_finish(const HtdDesc* d, const HtdSizes& sz, hipStream_t s);
hipError_t launch_dc_init(const HtdDesc* d, const HtdSizes& sz, int blocks, hipStream_t s);
hipError_t launch_dc_prep(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s);
hipError_t launch_dc_rot(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s);
// stage 1: secular roots, 2: Loewner z, 3: eigenvector norms (one wavefront each)
hipError_t launch_dc_wave(int stage, const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s);
hipError_t launch_dc_place(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s);
hipError_t launch_dc_gemm(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s);
hipError_t launch_bt_init(const HtdDesc* d, const HtdSizes& sz, int Lmax, int blocks, hipStream_t s);
hipError_t launch_bt_larft(const HtdDesc* d, const HtdSizes& sz, int blocks, hipStream_t s);
hipError_t launch_bt_wpart(const HtdDesc* d, const HtdSizes& sz, int b, int blocks, hipStream_t s);
hipError_t launch_bt_wred(const HtdDesc* d, const HtdSizes& sz, int b, int blocks, hipStream_t s);
hipError_t launch_bt_update(const HtdDesc* d, const HtdSizes& sz, int b, int blocks, hipStream_t s);
// w ascending and V's columns to match, from one solve's descending output
hipError_t launch_heev_out(const double2* Vw, int ld, const double* lam, int n, double2* V, double* w,
                           hipStream_t s);

// ------------------------------------------------------ learned sketch ----
constexpr int SK_PROBES = 8;

// One randomized range finder on the Gram matrix G of a split (2c x 2c).
struct SketchDesc {
  Dim n;               // 2c
  int s;               // sketch size
  int ld_s;            // leading dim of the n x s (and n x SK_PROBES) panels
  int ld_y;            // leading dim of the s x s matrices
  uint64_t seed;
  uint32_t stream;
  double2* Omega;      // n x s Gaussian test matrix
  double2* Probe;      // n x SK_PROBES Gaussian probes
  double2* Bq;         // s x s: U Lambda^{-1/2}
  const double2* R1;   // n x SK_PROBES: G probes
  const double2* R2;   // n x SK_PROBES: (G Q)(Q^H probes); R1 - R2 = G (I - Q Q^H) probes
  const double2* Gy;   // diagonalised Y^H Y (eigenvalues on the diagonal)
  const double2* Uy;   // its eigenvectors
  const double2* Hw;   // diagonalised Q^H G Q
  double* lam;         // out: eigenvalues of Q^H G Q (s)
  const double* trace; // trace of G
  double eps_eff;
  int* use;            // out: 1 when the sketch is accepted
  double* est;         // out: [residual estimate, trace]
  int* exact_flags;    // the exact solve's flags (converged := 1 when accepted)
};
hipError_t launch_gauss_fill(const SketchDesc* d, int nprob, int which, hipStream_t s);
hipError_t launch_orth_scale(const SketchDesc* d, int nprob, hipStream_t s);
hipError_t launch_newton_schulz(const SketchDesc* d, int nprob, hipStream_t s);
hipError_t launch_sketch_accept(const SketchDesc* d, int nprob, hipStream_t s);

int mlp_param_count();
int mlp_chunk();
hipError_t launch_mlp_forward(const float* P, const float* X, float* y, int B, hipStream_t s);
hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const int* idx, int B, float tau,
                           float* part, float* loss_part, float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(float* P, const float* g, float* m, float* v, float lr, int t, hipStream_t s);

// ------------------------------------------------------- site kernels ----
// Truncation selection for one split (one workgroup per problem).
struct SelectDesc {
  const double2* G;     // diagonalised Gram matrix (eigenvalues on the diagonal)
  const double* lam_in; // eigenvalues given explicitly instead (or null)
  const int* use_sk;    // when *use_sk: take lam_sk (s_sk values) and total *tot_sk
  const double* lam_sk;
  const double* tot_sk;
  int s_sk;
  int ldg;
  Dim n;                // 2c
  int rows;             // chi_l 2^m: rank bound of X
  int chi_max;
  double eps_eff;       // threshold on normalised singular values
  int* perm;            // out: eigenvalue order, descending (n entries)
  int* r_out;           // out: kept rank (also the new bond dimension)
  double* lam_out;      // out: normalised kept singular values (Lambda)
  double* logf_acc;     // in/out: this cluster's sum of log f
  double* rec;          // out: [f, sigma_r/sigma_1, discarded weight, degenerate]
};
hipError_t launch_select(const SelectDesc* d, int nprob, hipStream_t s);

// B_site[i][col] = conj(V[col][perm[i]]) and Vr[col][i] = V[col][perm[i]]
struct GatherDesc {
  const double2* V;
  int ldv;
  const int* use_sk;    // when *use_sk: V := Vs with leading dim ld_sk
  const double2* Vs;
  int ld_sk;
  const int* perm;
  const int* r;
  Dim n;            // rows of V used (2c)
  void* B;          // site tensor (r x n) in working precision
  void* Vr;         // projection matrix (n x r) in working precision
  int tiles;        // 64 x 64 element tiles reserved
};
hipError_t launch_gather(Prec p, const GatherDesc* d, const int* d_base, int nprob, int blocks,
                         hipStream_t s);

// B_a = X / sqrt(exp(logf)) over `count` complex entries (count may be dynamic)
struct ScaleDesc {
  const void* X;
  void* B;
  Dim count;
  const double* logf;
  int blocks;
};
hipError_t launch_finalize(Prec p, const ScaleDesc* d, const int* d_base, int nprob, int blocks,
                           hipStream_t s);

// One-qubit gate products on sites outside every cluster.
struct Site1QDesc {
  void* B;
  int chi_l, chi_r;
  double u[8];  // 2x2 complex
  int blocks;
};
hipError_t launch_apply_1q(Prec p, const Site1QDesc* d, const int* d_base, int nprob, int blocks,
                           hipStream_t s);

// Cluster unitaries from gate lists: U = G_last ... G_first on k local qubits.
struct UGate {
  int nq;
  int q0, q1;     // local positions (q0 is the most significant of the gate)
  int pad;
  double u[32];   // 2^nq x 2^nq complex, row-major
};
struct UnitaryDesc {
  const UGate* gates;
  int ngates;
  int k;
  double2* U64;  // out: 2^k x 2^k FP64
  float2* U32;   // out (optional): the same in FP32
  int cols;      // columns per workgroup (cols * 2^k * 16 bytes of LDS)
  int blocks;    // column blocks
};
// lds_bytes: largest cols * 2^k * sizeof(double2) over the problems (<= 64 KiB)
hipError_t launch_build_unitary(const UnitaryDesc* d, const int* d_base, int nprob, int blocks,
                                size_t lds_bytes, hipStream_t s);

// Merge-kernel helper: copy with conversion (FP64 user unitary -> work precision)
hipError_t launch_convert_d2f(const double2* src, float2* dst, int64_t n, hipStream_t s);
hipError_t launch_convert_f2d(const float2* src, double2* dst, int64_t n, hipStream_t s);

// Log-f accumulation in a fixed order (deterministic): total += sum_i v[i]
hipError_t launch_accumulate(const double* v, int n, double* total, hipStream_t s);
// Dense FP64 complex helpers of the DMRG fit (row-major): sum |x|^2 into
// *out; x *= a; out = diag(d) conj(in)^T (d may be null); columns of x
// scaled by d.
hipError_t launch_dense_norm2(const double2* x, int64_t n, double* out, hipStream_t s);
hipError_t launch_dense_scale(double2* x, int64_t n, double a, hipStream_t s);
hipError_t launch_dense_adjoint(const double2* in, int rows, int cols, int ldi, const double* d, double2* out,
                                int ldo, hipStream_t s);
hipError_t launch_dense_scale_cols(double2* x, int rows, int cols, int ld, const double* d, hipStream_t s);
// C (M x N, ldc) = sum of `parts` partial products P + q stride (M x N each)
hipError_t launch_dense_sum_parts(const double2* P, int parts, int64_t stride, int M, int N, double2* C, int ldc,
                                  hipStream_t s);
// total += *v[0] + ... + *v[n-1] (v: device array of n device pointers)
hipError_t launch_accumulate_ptrs(const double* const* v, int n, double* total, hipStream_t s);

}  // namespace ctebd
