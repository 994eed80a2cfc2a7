// Descriptors and launchers of the device kernels (all grouped: one launch
// serves a list of independent problems, one workgroup per output tile).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace ctebd {

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
  void* Gw;         // working copy rotated to diagonal form (== G for FP64)
  void* Vw;         // working eigenvectors (== V for FP64)
  void* J;          // workspace: npair_max subproblem rotations of JP x JP
  double2* W;       // FP32 solve: G V for the Rayleigh quotients
  double* lam;      // FP32 solve: FP64 Rayleigh quotients (n entries)
  int* pair_rot;    // per pair slot: rotation applied this round
  int* flags;       // [0] converged, [1] rotated during the current sweep
  double* scale;    // trace of G (set by eig_init)
  unsigned long long* work;  // complex MACs executed by eig_update (or null)
  Dim n;            // matrix size
  int ld;
  int nb_max;       // block count the grids reserve (even)
  double tol;       // relative off-diagonal threshold
};

// fp32: the solve runs in FP32 on Gw/Vw (then eig_to64 + W = G V + rayleigh)
hipError_t launch_eig_init(bool fp32, const EigDesc* d, int nprob, int ld_max, hipStream_t s);
hipError_t launch_eig_pairs(bool fp32, const EigDesc* d, const int* d_base, int nprob, int blocks, int round,
                            hipStream_t s);
hipError_t launch_eig_update(bool fp32, const EigDesc* d, const int* d_base, int nprob, int blocks, int round,
                             hipStream_t s);
hipError_t launch_eig_sweep_end(const EigDesc* d, int nprob, hipStream_t s);
hipError_t launch_eig_to64(const EigDesc* d, int nprob, int ld_max, hipStream_t s);
hipError_t launch_eig_rayleigh(const EigDesc* d, int nprob, int n_max, hipStream_t s);

// ------------------------------- tridiagonal divide-and-conquer eigen ----
// Hermitian G = Q T Q^H (Householder, T real tridiagonal), T = Z diag(w) Z^T
// (Cuppen divide and conquer), eigenvectors Q Z (blocked back-transformation).
constexpr int HTD_MAX = 2048;  // largest n: per-node lists are staged in LDS
constexpr int HTD_NB = 32;     // reflectors per back-transformation block
constexpr int HV_ROWS = 8;     // trailing-matrix rows per HEMV workgroup
constexpr int BT_CH = 256;     // rows per split-K chunk of the back-transformation

struct HtdDesc {
  double2* A;       // n x n Hermitian (ld); row k keeps reflector v_k (cols > k)
  double2* V;       // out: eigenvectors as columns (ld)
  double* lam;      // out: eigenvalues, ascending (n)
  Dim n;
  int ld;
  const int* skip;  // nonzero: the problem is solved elsewhere (accepted sketch)
  // reduction to tridiagonal form
  double* d;        // diagonal of T (n)
  double* e;        // off-diagonal of T (n - 1)
  double2* tau;     // reflector scalars (n - 1)
  double2* v;       // current reflector (n)
  double2* y;       // tau G v of the current step (n)
  double2* part;    // per HEMV workgroup: sum of conj(y_i) v_i
  // divide and conquer (node lists are indexed by the node's first row)
  double* Q[2];     // n x n (ld) block-diagonal eigenvector matrices, by level parity
  double* D[2];     // eigenvalues of the nodes, ascending within a node
  double* DeltaT;   // ld x ld: DeltaT[lo+j][lo+k] = dl_j - lambda_k
  double* U;        // ld x ld: eigenvectors of the rank-one updated diagonal
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
  double2* T;       // per block of HTD_NB reflectors: HTD_NB x HTD_NB upper triangle
  double2* Wp;      // split-K partials: ceil(ld / BT_CH) x HTD_NB x ld
  double2* W;       // T (V_b^H Z): HTD_NB x ld
};

// Per-problem workgroup counts of the launches (identical on host and device).
__host__ __device__ inline int htd_hemv_blocks(int n, int k) {
  const int m = n - k - 1;
  return m > 0 ? (m + HV_ROWS - 1) / HV_ROWS : 0;
}
__host__ __device__ inline int htd_her2_blocks(int n, int k) {
  const int m = n - k - 1, t = (m + 63) / 64;
  return m > 0 ? t * t : 0;
}
__host__ __device__ inline int htd_rows(int n) { return (n + 255) / 256; }
__host__ __device__ inline int htd_nodes(int n, int L) { return (n + (1 << L) - 1) >> L; }
__host__ __device__ inline int htd_gemm_tiles(int n, int L) {
  const int t = ((1 << L) + 63) / 64;
  return htd_nodes(n, L) * t * t;
}
__host__ __device__ inline int htd_nblk(int n) { return n >= 2 ? (n - 2) / HTD_NB + 1 : 0; }
__host__ __device__ inline int htd_bt_rows(int n, int b) { return n - HTD_NB * b - 1; }
__host__ __device__ inline int htd_wpart_blocks(int n, int b) {
  return b < htd_nblk(n) ? ((htd_bt_rows(n, b) + BT_CH - 1) / BT_CH) * ((n + 63) / 64) : 0;
}
__host__ __device__ inline int htd_wred_blocks(int n, int b) { return b < htd_nblk(n) ? (n + 63) / 64 : 0; }
__host__ __device__ inline int htd_update_blocks(int n, int b) {
  return b < htd_nblk(n) ? ((htd_bt_rows(n, b) + 63) / 64) * ((n + 63) / 64) : 0;
}

// launches over np descriptors in device memory; `blocks` is the sum of the
// per-problem counts above for the given step / level / block
hipError_t launch_trd_hemv(const HtdDesc* d, int np, int k, int blocks, hipStream_t s);
hipError_t launch_trd_her2(const HtdDesc* d, int np, int k, int blocks, hipStream_t s);
hipError_t launch_trd_finish(const HtdDesc* d, int np, hipStream_t s);
hipError_t launch_dc_init(const HtdDesc* d, int np, int blocks, hipStream_t s);
hipError_t launch_dc_prep(const HtdDesc* d, int np, int L, int blocks, hipStream_t s);
// stage 0: deflation rotations, 1: secular roots, 2: Loewner z, 3: eigenvectors
hipError_t launch_dc_rows(int stage, const HtdDesc* d, int np, int L, int blocks, hipStream_t s);
hipError_t launch_dc_place(const HtdDesc* d, int np, int L, int blocks, hipStream_t s);
hipError_t launch_dc_gemm(const HtdDesc* d, int np, int L, int blocks, hipStream_t s);
hipError_t launch_bt_init(const HtdDesc* d, int np, int Lmax, int blocks, hipStream_t s);
hipError_t launch_bt_larft(const HtdDesc* d, int np, int blocks, hipStream_t s);
hipError_t launch_bt_wpart(const HtdDesc* d, int np, int b, int blocks, hipStream_t s);
hipError_t launch_bt_wred(const HtdDesc* d, int np, int b, int blocks, hipStream_t s);
hipError_t launch_bt_update(const HtdDesc* d, int np, int b, int blocks, hipStream_t s);

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

}  // namespace ctebd
