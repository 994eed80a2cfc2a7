/*
 * cluster_tebd.h -- C ABI of the MI355X cluster-TEBD library (libctebd.so).
 *
 * The library simulates an n-qubit circuit on a matrix-product state (MPS) with
 * the cluster-TEBD iteration of De Girolamo et al., arXiv:2502.19289, Sec. III.A:
 * qubits joined by entangling gates are grouped into entanglement clusters, the
 * gates of each cluster over several layers are merged into one exact
 * 2^k x 2^k unitary, the unitary is applied to the MPS block the cluster covers,
 * and the block is split back into k sites by a sweep of truncated SVDs with
 * cutoff eta and cap chi_max (Sec. II.B), whose discarded weights give the
 * fidelity estimate F = prod_i f_i (Eqs. f_i and approxF).
 *
 * Conventions shared by every call
 *   - Sites are 0..n-1, bond b joins sites b and b+1 (0 <= b < n-1).
 *   - Gate matrices are row-major complex128 stored as interleaved (re, im)
 *     doubles.  A matrix acting on qubits q[0..k-1] is big-endian in that list:
 *     q[0] is the most significant bit of its row/column index.
 *   - Statevector amplitudes use the same order (qubit 0 most significant).
 *   - Ownership: the caller owns every array it passes; the library copies what
 *     it needs before returning.  All device memory belongs to the handle and is
 *     released by mps_destroy.
 *   - Errors: every call returns an mps_status; nothing is thrown across the
 *     ABI.  Common to all calls: MPS_EINVAL for a NULL handle or a NULL
 *     pointer that the call writes through, MPS_EDEVICE / MPS_ENOMEM when a
 *     HIP call or an allocation fails (the handle stays valid and can be
 *     destroyed).  mps_last_error(h) gives a message for the last failed call on h;
 *     mps_last_error(NULL) for the calling thread's last failed call that
 *     takes no handle or creates one (mps_create, mps_load, ...).
 *   - Concurrency: one handle must not be used from two host threads at once.
 *     Work is queued on the handle's HIP stream; the calls documented as
 *     "synchronises" wait for it.
 */
#ifndef CLUSTER_TEBD_H
#define CLUSTER_TEBD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_ctx* mps_handle;

typedef enum {
  MPS_OK = 0,
  MPS_EINVAL = -1,       /* bad argument (size, index, null pointer)            */
  MPS_ENOMEM = -2,       /* device or host allocation failed                     */
  MPS_ESPAN = -3,        /* cluster wider than k_max or qubits not ascending     */
  MPS_ENOTUNITARY = -4,  /* ||U^dagger U - 1||_max > 1e-10                       */
  MPS_EDEVICE = -5,      /* a HIP call failed or no GPU is present               */
  MPS_ESTATE = -6,       /* call not valid in the handle's current state         */
  MPS_EIO = -7           /* file could not be read or written                    */
} mps_status;

/* Arithmetic of the contractions (merge, unitary application, projection).
 * The Gram matrices, the eigen-solver and every singular value stay FP64. */
enum {
  MPS_PREC_FP64 = 0,    /* complex128 site tensors, FP64 MFMA contractions      */
  MPS_PREC_FP32 = 1,    /* complex64 site tensors, FP32 MFMA contractions       */
  MPS_PREC_BF16X6 = 2   /* complex64 tensors, contractions as six BF16 MFMA
                           products of a three-way hi/mid/lo split, FP32 sums   */
};

/* How the truncated SVD of each split is obtained. */
enum {
  MPS_SVD_EXACT = 0,    /* FP64 Gram matrix + FP64 eigen-solver (eig_method)   */
  MPS_SVD_LEARNED = 1   /* randomized range finder with a sketch size chosen by
                           the kept-rank network; exact SVD when its residual
                           check fails                                          */
};

/* Eigen-solver of the exact split (the Gram matrix G is 2c x 2c, FP64).
 * Both reach FP64 accuracy; they differ in cost.  Block Jacobi needs about
 * 2 * 2c dependent rotation rounds per sweep and several sweeps; the
 * tridiagonal route (Householder reduction to a real tridiagonal, Cuppen
 * divide and conquer, back-transformation) needs 2 launches per column and
 * O(log 2c) merge levels. */
enum {
  MPS_EIG_AUTO = 0,     /* the faster route by size: at present tridiagonal
                           whenever 2c <= 2048 (as MPS_EIG_TRIDIAG), Jacobi
                           above                                                */
  MPS_EIG_JACOBI = 1,   /* FP64 block Jacobi                                    */
  MPS_EIG_TRIDIAG = 2   /* tridiagonal divide and conquer whenever 2c <= 2048   */
};

/* How the independent clusters are launched.  All three give the same site
 * tensors and Schmidt values bit for bit; the fidelity sum may differ in its
 * last bits (another summation order). */
enum {
  MPS_BATCH_NONE = 0,   /* one cluster per launch sequence, step by step        */
  MPS_BATCH_STEP = 1,   /* every cluster of a step in the same launches          */
  MPS_BATCH_WAVE = 2    /* the clusters of several steps as a dependency graph:
                           in every round each cluster whose sites and left
                           Schmidt values are final starts, each running cluster
                           takes its next split level, all in the same launches
                           (a k-qubit cluster runs k-1 rounds); mps_run_steps,
                           mps_flush and mps_run_layer hand it all the steps
                           they execute at once.  Needs the plan to be free of
                           bond dimensions (q_max at its default) and exact SVDs;
                           otherwise steps run as with MPS_BATCH_STEP            */
};

typedef struct {
  int k_max;        /* most qubits per cluster; wider gates are SWAP-routed    */
  int q_max;        /* Eq. cond_cTEBD: 2^k chi_l chi_r <= 2^q_max; <= 0 gives
                       k_max + 2 ceil(log2 chi_max), which never binds         */
  int l_max;        /* Eq. cond2_cTEBD: sub-layers per step; <= 0: unlimited  */
  int precision;    /* MPS_PREC_*                                              */
  int svd_mode;     /* MPS_SVD_*                                               */
  int batch;        /* MPS_BATCH_*                                             */
  int eig_method;   /* MPS_EIG_*                                               */
  double floor_c;   /* the kept-value threshold is max(eps, floor_c * u) with
                       u = 2^-24 for FP32/BF16X6 and 2^-26.5 for FP64; the
                       Gram route cannot resolve singular values below it    */
  void* hip_stream; /* hipStream_t to queue work on; NULL: a stream of its own */
} mps_options;

/* A one- or two-qubit gate: nq in {1,2}, q[0..nq-1] the qubits, u the
 * 2^nq x 2^nq matrix (row-major, interleaved re/im, big-endian in q). */
typedef struct {
  int nq;
  int q[2];
  double u[32];
} mps_gate;

/* Counters of the work done so far (all cumulative). */
typedef struct {
  int64_t steps;            /* cluster-TEBD iterations executed                  */
  int64_t cluster_updates;  /* clusters with k >= 2 contracted and split         */
  int64_t svds;             /* truncated SVDs (k-1 per cluster)                  */
  int64_t site_updates;     /* sites updated by one-qubit gates alone            */
  int64_t sketch_accepted;  /* learned-sketch SVDs that passed the residual test */
  int64_t sketch_fallback;  /* learned-sketch SVDs redone exactly                */
  int64_t jacobi_sweeps;    /* block-Jacobi sweeps launched                      */
  double discarded_weight;  /* sum over SVDs of (1 - f_i)                        */
} mps_stats;

/* Fills *opt with the defaults: k_max 4, q_max 0, l_max 0, FP32, exact SVD,
 * step batching, automatic eigen-solver choice, floor_c 4, library stream. */
mps_status mps_default_options(mps_options* opt);

/* Sec. II.B / IV.A: creates the product state |0...0> on n >= 2 qubits (every
 * bond of dimension one, F = 1) with bond cap chi_max >= 1 and cutoff eps >= 0
 * (singular values below eps, on the normalised spectrum, are dropped).
 * opt may be NULL (defaults).  Allocates the site tensors at their largest
 * possible size min(chi_max, 2^min(b+1, n-b-1)) per bond. */
mps_status mps_create(int n, int chi_max, double eps, const mps_options* opt,
                      mps_handle* out);
/* Releases the handle and all its device memory (NULL: nothing to do). */
mps_status mps_destroy(mps_handle h);

/* Sec. III.A steps "contract" and "decompose" for one cluster: applies the
 * 2^k x 2^k unitary U (interleaved complex128, row-major, big-endian in
 * qubits[]) to the sites qubits[0]..qubits[k-1], which must be strictly
 * ascending with qubits[k-1]-qubits[0]+1 <= k_max (else MPS_ESPAN); idle qubits
 * inside the span are padded with the identity.  The block is then split back
 * by k'-1 truncated SVDs (k' = span), adding log f_i of each to the fidelity
 * estimate.  Pending layers are flushed first.  2 <= k <= 12.  U must satisfy
 * ||U^H U - 1||_max <= 1e-10, else MPS_ENOTUNITARY and the state is left as
 * it was (the product U^H U is formed on the host for 2^k < 512 and on the
 * device, in FP64, from 512 on; either way the call waits for the handle's
 * stream). */
mps_status mps_apply_cluster(mps_handle h, const int* qubits, int k, const double* U);

/* Sec. III.A iteration driver: buffers one circuit layer (gates on disjoint
 * qubits, Sec. II.A).  Gates wider than k_max are routed by adjacent SWAPs.
 * When the buffered layers no longer fit the caps (k_max, Eq. cond_cTEBD,
 * Eq. cond2_cTEBD) the step made of the layers that do fit is contracted.
 * MPS_EINVAL (nothing buffered) for nq outside {1, 2}, a qubit out of range
 * or two gates sharing a qubit.  Gate matrices are taken as given. */
mps_status mps_run_layer(mps_handle h, const mps_gate* gates, int ngates);

/* Contracts every buffered layer (as many steps as the caps need). */
mps_status mps_flush(mps_handle h);

/* Buffers one layer like mps_run_layer but never executes a step. */
mps_status mps_queue_layer(mps_handle h, const mps_gate* gates, int ngates);

/* Sec. III.A, one iteration: plans the clusters of the buffered sub-layers
 * and contracts exactly one step.  *clusters receives the number of clusters
 * (k >= 2) of that step (0 when nothing is buffered) and *remaining the
 * sub-layers still buffered; either pointer may be NULL.  Synchronises. */
mps_status mps_step(mps_handle h, int* clusters, int* remaining);

/* Contracts the next nsteps planned steps (Sec. III.A) of the buffered
 * sub-layers, fewer when the buffer runs out; with MPS_BATCH_WAVE as one
 * dependency graph, else one step after the other.  *clusters receives the
 * number of clusters (k >= 2) contracted and *remaining the sub-layers still
 * buffered; either may be NULL.  Synchronises.  MPS_EINVAL for nsteps < 0. */
mps_status mps_run_steps(mps_handle h, int nsteps, int* clusters, int* remaining);

/* Copies the state (sites, Schmidt values, bond dimensions, fidelity sum and
 * buffered sub-layers) into a new handle whose options come from opt (the
 * precision may differ: tensors are converted on the device).  n, chi_max and
 * eps are those of h.  Synchronises. */
mps_status mps_clone(mps_handle h, const mps_options* opt, mps_handle* out);

/* Changes the options of a live handle (Sec. II.B's chi_max and eta stay
 * those given to mps_create).  When k_max changes, the buffered layers are
 * contracted first with the old options (they were routed for the old k_max).
 * A new precision converts the site tensors on the device (FP64 <-> FP32 is
 * a rounding; FP32 <-> BF16X6 keeps them as they are); a new hip_stream (NULL:
 * a stream of the handle's own) is used from the next call on.  Counters,
 * timing state, the attached sketch network and the fidelity sum carry over.
 * Synchronises.  MPS_EINVAL for invalid options (h unchanged). */
mps_status mps_set_options(mps_handle h, const mps_options* opt);

/* Writes the whole handle to the file `path` (replaced atomically through
 * path + ".part"): n, chi_max, eps, the options (hip_stream excepted), sum
 * log f, the counters, the sketch generator state, the bond dimensions, every
 * site tensor as stored (complex64 or complex128, bit for bit), the Schmidt
 * values and the buffered sub-layers, then a 64-bit FNV-1a checksum of the
 * preceding bytes; little-endian.  A handle loaded from the file continues
 * exactly as h would (the same kernels on the same bits).  Synchronises.
 * MPS_EIO when the file cannot be written. */
mps_status mps_save(mps_handle h, const char* path);

/* Creates a new handle from a file written by mps_save (its own stream; use
 * mps_set_options for another).  The file is read and checked on the host
 * first: MPS_EIO when it cannot be read, is truncated, fails its checksum,
 * holds out-of-range sizes, or holds buffered sub-layers that mps_run_layer
 * could not have left for the saved k_max (gates of one sub-layer sharing a
 * qubit, overlapping two-qubit spans, a span wider than k_max);
 * mps_last_error(NULL) then says why. */
mps_status mps_load(const char* path, mps_handle* out);

/* Sec. III.B, one step of the adaptive-grouping DMRG on an FP64 handle
 * (MPS_ESTATE otherwise): the nl layers (layer_len[i] gates each, flattened in
 * `gates`, disjoint qubits per layer) form the segment.  Buffered layers are
 * contracted first.  The virtual bond dimensions of Eq. chi_est (E(b) = the
 * segment's two-qubit gates crossing bond b, capped at chi_max_dmrg) are cut
 * recursively at their smallest bond (ties: the most balanced cut, then the
 * leftmost) until every part of N qubits between cuts chi~_L, chi~_R meets
 * N + log2 chi~_L + log2 chi~_R <= q_max (Eqs. cond_group1/2); a grouped MPS
 * with one site per part is fitted to the evolved state by `sweeps` sweeps of
 * one-group updates (right to left, then left to right), starting from the
 * evolved state compressed at the group cuts by truncated SVDs; it is then
 * split back into qubit tensors with the handle's chi_max and cutoff.
 * *f_fit (may be NULL) receives the fit's fidelity |<M|U psi>|^2; the
 * fidelity sum adds log f_fit and the log of the splits' kept weights.  The
 * evolved state's bond dimensions must stay <= 1024.  chi_max_dmrg >= 1,
 * q_max >= 1 (1: every group a single qubit), sweeps >= 0 (0: the
 * compression alone), else MPS_EINVAL.  The device memory that holds the
 * evolved segment (site tensors at bond cap 2^ceil(log2 chi), chi the
 * largest bound 4^E(b) chi_b) stays with the handle for the next DMRG step
 * and is released by mps_destroy.  Synchronises. */
mps_status mps_dmrg_step(mps_handle h, const mps_gate* gates, const int* layer_len, int nl, int chi_max_dmrg,
                         int q_max, int sweeps, double* f_fit);

/* <a|b> of the current states of two handles with the same n (buffered
 * layers are not applied), by a transfer-matrix sweep in FP64 on the device
 * (E <- sum_s A_s^dagger E B_s).  Synchronises.  MPS_EINVAL when n differs. */
mps_status mps_overlap(mps_handle a, mps_handle b, double* re, double* im);

/* Eq. approxF: synchronises and returns F_est = exp(sum log f_i) and
 * sum log f_i (either pointer may be NULL) of the steps executed so far;
 * buffered layers are not flushed (call mps_flush first for those). */
mps_status mps_fidelity(mps_handle h, double* F_est, double* log_f);

/* Synchronises; writes the n-1 current bond dimensions into chi. */
mps_status mps_bond_dims(mps_handle h, int* chi);

/* Synchronises; copies the normalised Schmidt values of bond b (descending,
 * FP64) into sigma[0..cap-1] and their count into *len (sigma may be NULL to
 * ask for the count).  MPS_EINVAL for a bond outside 0..n-2. */
mps_status mps_schmidt(mps_handle h, int bond, double* sigma, int cap, int* len);

/* Synchronises; copies site tensor B_j, shape (chi_{j-1}, 2, chi_j) row-major,
 * as interleaved complex128 into B[0..2*cap-1] (cap counts complex entries)
 * and its shape into dims[0..2] (B may be NULL to ask for the shape).  Sites
 * 1..n-1 are right-canonical up to the weight a truncation discarded while
 * the site was the leftmost of its cluster; the state is the contraction
 * B_0 B_1 ... B_{n-1}.  MPS_EINVAL for a site outside 0..n-1 or a cap below
 * the tensor's size. */
mps_status mps_export_site(mps_handle h, int site, double* B, int64_t cap, int* dims);

/* Replaces the whole state: sites[j] points at chi_{j-1}*2*chi_j interleaved
 * complex128 values (right-canonical for j >= 1), lams[b] at chi[b] Schmidt
 * values.  Bond dimensions must not exceed the handle's capacities
 * (MPS_EINVAL, state unchanged).  Buffered layers are contracted first. */
mps_status mps_import(mps_handle h, const int* chi, const double* const* sites,
                      const double* const* lams, double log_f);

/* Synchronises; writes the 2^n amplitudes (interleaved complex128) of the
 * state, buffered layers contracted first; n <= 24 and cap >= 2^n, else
 * MPS_EINVAL. */
mps_status mps_amplitudes(mps_handle h, double* psi, int64_t cap);

mps_status mps_get_stats(mps_handle h, mps_stats* st);

/* Device time (ms) spent in each kernel class since timing was switched on,
 * measured with HIP events on the handle's stream around every launch of that
 * class (mps_set_timing), the number of launches, and the algorithmic real
 * flops the class performed (8 per complex multiply-add; merges, unitary
 * products, Hermitian half of the Gram matrices, projections, and the
 * rotation tiles eig_update applied).  Arrays hold cap
 * entries; names receives the class names, comma-separated; *count the
 * number of classes. */
mps_status mps_set_timing(mps_handle h, int on);
mps_status mps_kernel_times(mps_handle h, double* ms, int64_t* launches, double* flop, int cap,
                            char* names, int names_cap, int* count);

/* Sec. III.A, the eigen-decomposition behind every exact split, on its own:
 * A (n x n Hermitian, interleaved complex128, row-major, host memory) =
 * V diag(w) V^H with w ascending and V[i*n + j] the i-th component of the
 * j-th eigenvector (unit norm).  Runs the tridiagonal divide-and-conquer
 * solver of the large splits on the current device; 1 <= n <= 2048.
 * Synchronous; allocates and frees its own device memory.  Both triangles
 * of A are read: A must be Hermitian.
 * MPS_EINVAL for a bad size or a null pointer, MPS_EDEVICE / MPS_ENOMEM for
 * HIP failures; mps_last_error(NULL) then describes the failure. */
mps_status mps_heev(int n, const double* A, double* w, double* V);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mps_heev on
 * caller-owned DEVICE buffers, with every intermediate in a 16 MiB array of
 * static device memory that the library holds on each GPU it runs on until
 * the process ends.  A: n x n Hermitian (interleaved complex128, row-major,
 * both triangles read, not modified); w: n eigenvalues, ascending; V: n x n,
 * V[i*n + j] the i-th component of the j-th eigenvector; the same kernels as
 * mps_heev, so the same results.  stream: hipStream_t to run on (NULL: the
 * null stream); the call returns after the stream has finished its work.
 * 1 <= n <= 512, else MPS_EINVAL (nothing runs); MPS_EDEVICE for HIP
 * failures; mps_last_error(NULL) says why.  No hipMalloc, hipFree or other
 * allocation of device memory happens in this call.  Every call on one GPU
 * uses the same array: calls that overlap on one GPU (two host threads, or
 * two streams) race and must be serialised by the caller. */
mps_status mps_heev_noalloc(int n, const double* A, double* w, double* V, void* stream);

/* Burst timing of one kernel class, for kernels too short for a pair of
 * events around each launch (on this GPU each event adds the latency of a
 * marker packet, several microseconds): every stride-th launch of the class
 * is followed by reps re-launches of the same kernel on the same inputs
 * (which it does not write, so the outputs are unchanged) and one pair of
 * events spans all reps + 1 launches; mps_kernel_times then reports for the
 * class the summed per-launch time of those bursts and their number, and
 * mps_kernel_bytes the algorithmic bytes of the sampled launches only.  The
 * other launches of the class run untimed.  Supported classes: "trd_col"
 * and "trd_hemv" (the column update and the Hermitian matrix-vector product
 * of the tridiagonal reduction); one call per class; stride >= 1,
 * 0 <= reps <= 64, else MPS_EINVAL.  kernel_class NULL or "" switches burst
 * timing off for all classes. */
mps_status mps_set_burst_timing(mps_handle h, const char* kernel_class, int stride, int reps);

/* Kernel dispatches of each kernel class since timing was switched on, the
 * re-launches of burst timing included (what a profiler of the same run
 * counts); classes in the order of mps_kernel_times. */
mps_status mps_kernel_dispatches(mps_handle h, int64_t* dispatches, int cap, int* count);

/* Algorithmic HBM bytes of each kernel class since timing was switched on,
 * for the classes bound by memory bandwidth (the HEMV and HER2 launches of
 * the tridiagonal reduction: the trailing Gram block read, and read and
 * written); 0 for the others.  Classes in the order of mps_kernel_times. */
mps_status mps_kernel_bytes(mps_handle h, double* bytes, int cap, int* count);

/* Message of the last failure of h; with h = NULL, of the last failed call
 * of this thread that takes no handle or creates one (mps_create, mps_load,
 * mps_heev, mps_heev_noalloc, mps_plan). */
const char* mps_last_error(mps_handle h);

/* ---- learned sketch -------------------------------------------------------
 * The paper does not sketch its SVDs; these calls serve the library's learned
 * sketch (svd_mode MPS_SVD_LEARNED): a network 12 -> 64 -> 64 -> 1 with GELU
 * (tanh form), FP32 on the device, predicts log2 of the rank a truncated SVD
 * keeps; the prediction sizes a randomized range finder on the split's Gram
 * matrix (Halko, Martinsson, Tropp, SIAM Rev. 53 (2011), Algs. 4.1/4.3/5.1),
 * accepted only when its 8-probe residual estimate shows that every
 * eigenvalue it missed lies below the truncation threshold, and otherwise
 * redone by the exact solve.  Features of a split (12 FP32): k, log2 chi_l,
 * log2 chi_r, m/k, log10 of the discarded weight of the bond's previous split,
 * log2 (2c bound), 2q gates crossing the bond, 2q gates of the cluster,
 * non-Clifford phase gates of the cluster, sub-layers of the step, log2 of
 * the bond's dimension before the step, log10 of the smallest kept over the
 * largest singular value of the bond's previous split.  Parameters are a flat FP32 vector: W1 (64x12), b1, W2
 * (64x64), b2, w3 (64), b3. */
typedef struct mlp_ctx* mlp_handle;

int mlp_num_params(void);
/* He-initialised weights (seeded), zero biases; MPS_EDEVICE without a GPU. */
mps_status mlp_create(int seed, mlp_handle* out);
mps_status mlp_destroy(mlp_handle h);
mps_status mlp_get_params(mlp_handle h, float* p);
mps_status mlp_set_params(mlp_handle h, const float* p);
/* y[i] = network(X[i, 0..11]) for n samples (host arrays). */
mps_status mlp_forward(mlp_handle h, const float* X, int n, float* y);
/* Gradient of the mean pinball loss (quantile tau in (0,1)) at targets t,
 * and the loss; grad may be NULL. */
mps_status mlp_grad(mlp_handle h, const float* X, const float* t, int n, float tau, float* grad,
                    float* loss);
/* Adam (lr, beta 0.9/0.999) on shuffled minibatches (seeded) for `epochs`;
 * *final_loss is the mean pinball loss over all n samples afterwards. */
mps_status mlp_train(mlp_handle h, const float* X, const float* t, int n, int epochs, int batch,
                     float lr, float tau, uint64_t seed, float* final_loss);
/* Attaches a network to a handle (NULL detaches); it must outlive that use. */
mps_status mps_set_sketch_model(mps_handle h, mlp_handle model);
/* The learned sketch's range finder on its own, for checking it against an
 * independent implementation: on the Hermitian Gram matrix G (n x n, host,
 * interleaved complex128, row-major) with the given Gaussian test matrix
 * Omega (n x s) and probes Probe (n x 8) instead of the device-drawn ones:
 * Y = G Omega, Q = an orthonormal basis of Y, H = Q^H G Q = W diag(mu) W^H,
 * V = Q W (n x s, row-major), est[0] = sqrt(mean_i ||G (I - Q Q^H) g_i||^2),
 * est[1] = trace(G); *accepted (may be NULL) tells whether est <= eps_eff^2
 * trace(G) with the handle's eps_eff (every eigenvalue left out below the
 * truncation threshold).  mu and the columns of V come in the order the
 * s x s solve leaves them.  2 <= n <= 2048, 1 <= s <= n.  Synchronises. */
mps_status mps_sketch_range(mps_handle h, int n, int s, const double* G, const double* Omega,
                            const double* Probe, double* mu, double* V, double* est, int* accepted);

/* Moves up to cap logged (features, log2 kept rank) pairs of the handle's
 * truncated SVDs into X (cap x 12) and t; *count = pairs held before the
 * call.  With X or t NULL only *count is set. */
mps_status mps_svd_log(mps_handle h, float* X, float* t, int cap, int* count);

/* Host-side planner of Sec. III.A, exposed for testing: legalises the layers
 * (SWAP routing, sub-layers of disjoint spans) and plans the first step from
 * sub-layer `start` with bond dimensions chi[0..n-2].
 *   layers: nl layers; layer_len[i] gates each; gates flattened in order.
 *   out_end: index (exclusive) of the last sub-layer of the step.
 *   out_clusters: pairs (first site, k) of the step's clusters, at most cap.
 *   n_sub: number of sub-layers after legalisation.
 * MPS_EINVAL for bad sizes or for gates that mps_run_layer would reject
 * (nq outside {1, 2}, a qubit out of range, two gates of a layer sharing a
 * qubit); mps_last_error(NULL) then says why. */
mps_status mps_plan(int n, int k_max, int q_max, int l_max, const int* chi,
                    const mps_gate* gates, const int* layer_len, int nl, int start,
                    int* out_end, int* out_clusters, int cap, int* out_count,
                    int* n_sub);

#ifdef __cplusplus
}
#endif

#endif /* CLUSTER_TEBD_H */
