// Learned sketch for the truncated SVD of the split sweep.
//
// The paper does not sketch; this is the library's accelerator for splits whose
// kept rank is far below the matrix size.  A small network (12 -> 64 -> 64 -> 1,
// GELU) predicts log2 of the rank the exact truncated SVD would keep; the
// prediction sets the size s of a randomized range finder (Halko, Martinsson,
// Tropp, SIAM Rev. 53, 217 (2011), Algs. 4.1/4.3/5.1) applied to the FP64 Gram
// matrix G of the split:
//   Y = G Omega,  Q = Y U Lambda^{-1/2} (Y^H Y = U Lambda U^H),
//   H = Q^H G Q = W M W^H,  V = Q W,  eigenvalues M,
// and accepted only when the a-posteriori estimate ||G (I - Q Q^H) g|| over 8
// Gaussian probes g says every eigenvalue it missed is below the truncation
// threshold; otherwise the exact block-Jacobi solve runs.
//
// This file holds the network (forward, backward, Adam, FP32) and the small
// kernels of the range finder; the products are the library's GEMMs.
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace ctebd {

namespace {

// ---------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): 10 rounds of multiply-high/low mixing with a Weyl key.
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// complex standard Gaussian (E|z|^2 = 1) number `idx` of stream (seed, stream)
__device__ __forceinline__ double2 gauss_c(uint64_t seed, uint32_t stream, uint64_t idx) {
  uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, 0x5EED5EEDu};
  philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = ((double)c[0] + 0.5) * 2.3283064365386963e-10;
  const double u2 = ((double)c[1] + 0.5) * 2.3283064365386963e-10;
  const double r = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586 * u2;
  return make_double2(r * cos(th) * 0.7071067811865476, r * sin(th) * 0.7071067811865476);
}

__global__ void gauss_fill_kernel(const SketchDesc* __restrict__ descs, int which) {
  const SketchDesc& d = descs[blockIdx.y];
  const int n = dim_value(d.n);
  const int cols = which == 0 ? d.s : SK_PROBES;
  double2* out = which == 0 ? d.Omega : d.Probe;
  const int64_t total = (int64_t)n * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / cols, col = e % cols;
    out[row * d.ld_s + col] = gauss_c(d.seed, (uint32_t)(2 * d.stream + which), e);
  }
}

// Bq[i][j] = U[i][j] / sqrt(lam_j) for lam_j above 64 n u of the largest, else 0
// (U: eigenvectors of Y^H Y with eigenvalues on the diagonal of the rotated
// copy).  One workgroup per problem.
__global__ __launch_bounds__(256) void orth_scale_kernel(const SketchDesc* __restrict__ descs) {
  const SketchDesc& d = descs[blockIdx.x];
  __shared__ double red[256];
  double mx = 0.0;
  for (int j = threadIdx.x; j < d.s; j += 256) mx = fmax(mx, d.Gy[(int64_t)j * d.ld_y + j].x);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  // eigenvalues of Y^H Y below its FP64 rounding level (about n u times the
  // largest) are noise, not directions of Y: their columns are set to zero
  const double thr = 64.0 * (double)dim_value(d.n) * 1.1102230246251565e-16 * red[0];
  for (int e = threadIdx.x; e < d.s * d.s; e += 256) {
    const int i = e / d.s, j = e % d.s;
    const double l = d.Gy[(int64_t)j * d.ld_y + j].x;
    const double sc = l > thr ? 1.0 / sqrt(l) : 0.0;
    const double2 u = d.Uy[(int64_t)i * d.ld_y + j];
    d.Bq[(int64_t)i * d.ld_s + j] = make_double2(u.x * sc, u.y * sc);
  }
}

// Newton-Schulz step towards an orthonormal Q: Bq = 1.5 I - 0.5 Q^H Q (the
// Gram S of Q is in Gy); Q <- Q Bq squares the orthogonality error.  The
// first basis comes from Y^H Y, whose conditioning is that of Y squared, so
// its columns are orthonormal only to u kappa(Y)^2 until these steps.
__global__ __launch_bounds__(256) void newton_schulz_kernel(const SketchDesc* __restrict__ descs) {
  const SketchDesc& d = descs[blockIdx.x];
  for (int e = threadIdx.x; e < d.s * d.s; e += 256) {
    const int i = e / d.s, j = e % d.s;
    const double2 g = d.Gy[(int64_t)i * d.ld_y + j];
    d.Bq[(int64_t)i * d.ld_s + j] = make_double2((i == j ? 1.5 : 0.0) - 0.5 * g.x, -0.5 * g.y);
  }
}

// est^2 = mean over probes of ||R[:, p]||^2 (R = G (I - Q Q^H) g); accept when
// est <= eps_eff^2 trace(G): every eigenvalue outside span(Q) is then below the
// truncation threshold (est estimates ||G (I - Q Q^H)||_F, which bounds the
// largest eigenvalue left out).  Also copies the H eigenvalues into lam (s entries).
__global__ __launch_bounds__(256) void accept_kernel(const SketchDesc* __restrict__ descs) {
  const SketchDesc& d = descs[blockIdx.x];
  __shared__ double red[256];
  const int n = dim_value(d.n);
  double s = 0.0;
  for (int e = threadIdx.x; e < n * SK_PROBES; e += 256) {
    const int i = e / SK_PROBES, p = e % SK_PROBES;
    const double2 a = d.R1[(int64_t)i * d.ld_s + p], b = d.R2[(int64_t)i * d.ld_s + p];
    const double x = a.x - b.x, y = a.y - b.y;
    s += x * x + y * y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  for (int j = threadIdx.x; j < d.s; j += 256) d.lam[j] = d.Hw[(int64_t)j * d.ld_y + j].x;
  if (threadIdx.x == 0) {
    const double est = sqrt(red[0] / SK_PROBES);
    const double tr = *d.trace;
    // the threshold of the exact route: an eigenvalue of G below
    // eps_eff^2 trace(G) is a singular value below eps_eff of the normalised
    // spectrum, which the exact split drops too.  FP64 rounding leaves about
    // u sqrt(n) lambda_1 in the estimate, so at large n an FP64 run (eps_eff^2
    // about 16 u) seldom accepts; FP32 / BF16X6 runs (eps_eff^2 about 1e-13)
    // do whenever the sketch holds every kept direction.
    const int ok = est <= d.eps_eff * d.eps_eff * tr ? 1 : 0;
    *d.use = ok;
    d.est[0] = est;
    d.est[1] = tr;
    if (ok) d.exact_flags[0] = 1;  // the exact solve of this split is skipped
  }
}

// ------------------------------------------------------------------- MLP --
constexpr int NI = 12, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH, NPARAM = OB3 + 1;

__device__ __forceinline__ float gelu(float x) {
  const float t = tanhf(0.7978845608028654f * (x + 0.044715f * x * x * x));
  return 0.5f * x * (1.f + t);
}
__device__ __forceinline__ float gelu_d(float x) {
  const float t = tanhf(0.7978845608028654f * (x + 0.044715f * x * x * x));
  const float dt = (1.f - t * t) * 0.7978845608028654f * (1.f + 3.f * 0.044715f * x * x);
  return 0.5f * (1.f + t) + 0.5f * x * dt;
}

// One wavefront per sample: lane j owns hidden unit j of both layers.
__global__ __launch_bounds__(64) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                         float* __restrict__ y, int B) {
  __shared__ float h1[NH];
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= B) return;
  const float* x = X + (int64_t)b * NI;
  float z = P[OB1 + j];
  for (int i = 0; i < NI; ++i) z += P[OW1 + j * NI + i] * x[i];
  h1[j] = gelu(z);
  __syncthreads();
  float z2 = P[OB2 + j];
  for (int i = 0; i < NH; ++i) z2 += P[OW2 + j * NH + i] * h1[i];
  float v = P[OW3 + j] * gelu(z2);
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (j == 0) y[b] = v + P[OB3];
}

// Mean pinball-loss gradient over samples idx[0..B-1]: each workgroup walks a
// contiguous chunk of samples, accumulating in registers (lane j owns row j of
// W1 and W2), and writes its partial gradient; mlp_reduce sums the partials in
// a fixed order.
constexpr int MLP_CHUNK = 64;

__global__ __launch_bounds__(64) void mlp_backward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                          const float* __restrict__ T, const int* __restrict__ idx,
                                                          int B, float tau, float* __restrict__ part,
                                                          float* __restrict__ loss_part) {
  __shared__ float xs[NI], h1[NH], z1s[NH], gz2[NH];
  const int j = threadIdx.x;
  float gW1[NI], gW2[NH];
  for (int i = 0; i < NI; ++i) gW1[i] = 0.f;
  for (int i = 0; i < NH; ++i) gW2[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
  const int b0 = blockIdx.x * MLP_CHUNK, b1 = min(B, b0 + MLP_CHUNK);
  const float invB = 1.f / (float)B;
  for (int b = b0; b < b1; ++b) {
    const int sidx = idx ? idx[b] : b;
    if (j < NI) xs[j] = X[(int64_t)sidx * NI + j];
    __syncthreads();
    float z = P[OB1 + j];
    for (int i = 0; i < NI; ++i) z += P[OW1 + j * NI + i] * xs[i];
    z1s[j] = z;
    h1[j] = gelu(z);
    __syncthreads();
    float z2 = P[OB2 + j];
    for (int i = 0; i < NH; ++i) z2 += P[OW2 + j * NH + i] * h1[i];
    const float h2 = gelu(z2);
    float v = P[OW3 + j] * h2;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const float yv = v + P[OB3];
    const float d = T[sidx] - yv;
    const float gy = (d >= 0.f ? -tau : 1.f - tau) * invB;
    lsum += (d >= 0.f ? tau * d : (tau - 1.f) * d) * invB;
    gw3 += gy * h2;
    gb3 += gy;
    const float g2 = gy * P[OW3 + j] * gelu_d(z2);
    gz2[j] = g2;
    gb2 += g2;
    for (int i = 0; i < NH; ++i) gW2[i] += g2 * h1[i];
    __syncthreads();
    float gh1 = 0.f;
    for (int q = 0; q < NH; ++q) gh1 += gz2[q] * P[OW2 + q * NH + j];
    const float g1 = gh1 * gelu_d(z1s[j]);
    gb1 += g1;
    for (int i = 0; i < NI; ++i) gW1[i] += g1 * xs[i];
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * NPARAM;
  for (int i = 0; i < NI; ++i) out[OW1 + j * NI + i] = gW1[i];
  out[OB1 + j] = gb1;
  for (int i = 0; i < NH; ++i) out[OW2 + j * NH + i] = gW2[i];
  out[OB2 + j] = gb2;
  out[OW3 + j] = gw3;
  if (j == 0) {
    out[OB3] = gb3;
    loss_part[blockIdx.x] = lsum;
  }
}

__global__ void mlp_reduce_kernel(const float* __restrict__ part, int nparts, float* __restrict__ grad,
                                  const float* __restrict__ loss_part, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) {
    float s = 0.f;
    for (int q = 0; q < nparts; ++q) s += part[(int64_t)q * NPARAM + p];
    grad[p] = s;
  }
  if (p == 0 && loss) {
    float s = 0.f;
    for (int q = 0; q < nparts; ++q) s += loss_part[q];
    *loss = s;
  }
}

__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m[p] = b1 * m[p] + (1.f - b1) * g[p];
  v[p] = b2 * v[p] + (1.f - b2) * g[p] * g[p];
  P[p] -= lr * (m[p] / c1) / (sqrtf(v[p] / c2) + eps);
}

}  // namespace

int mlp_param_count() { return NPARAM; }
int mlp_chunk() { return MLP_CHUNK; }

hipError_t launch_gauss_fill(const SketchDesc* d, int nprob, int which, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  launch(gauss_fill_kernel, dim3(64, nprob), dim3(256), 0, s, d, which);
  return hipGetLastError();
}

hipError_t launch_orth_scale(const SketchDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  launch(orth_scale_kernel, dim3(nprob), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_newton_schulz(const SketchDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  launch(newton_schulz_kernel, dim3(nprob), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_sketch_accept(const SketchDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  launch(accept_kernel, dim3(nprob), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, float* y, int B, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  launch(mlp_forward_kernel, dim3(B), dim3(64), 0, s, P, X, y, B);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const int* idx, int B, float tau,
                           float* part, float* loss_part, float* grad, float* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const int nparts = (B + MLP_CHUNK - 1) / MLP_CHUNK;
  launch(mlp_backward_kernel, dim3(nparts), dim3(64), 0, s, P, X, T, idx, B, tau, part, loss_part);
  launch(mlp_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, part, nparts, grad, loss_part, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* g, float* m, float* v, float lr, int t, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, (float)t), c2 = 1.f - powf(0.999f, (float)t);
  launch(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, g, m, v, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace ctebd
