// Per-site and per-split kernels of the cluster-TEBD step
// (arXiv:2502.19289, Secs. II.B and III.A):
//   build_unitary : U_c = G_last ... G_first for every cluster (FP64)
//   apply_1q      : one-qubit gate products on sites outside every cluster
//   select        : truncation rank r (cutoff, then cap chi_max, r >= 1),
//                   f = kept / total weight (Eq. f_i), Lambda = sigma[:r]/||.||
//   gather        : B_{a+m} = V_r^H and the projection matrix V_r
//   finalize      : B_a = X / sqrt(prod f)
#include <cfloat>

#include "common.hpp"
#include <algorithm>

#include "kernels.hpp"

namespace ctebd {

namespace {

template <typename C>
__device__ __forceinline__ C cscale(C v, double s) {
  v.x = (decltype(v.x))(v.x * s);
  v.y = (decltype(v.y))(v.y * s);
  return v;
}

// ------------------------------------------------------- build_unitary --
// One workgroup per (cluster, block of 16 columns): the columns are the images
// of basis vectors, propagated gate by gate in LDS.

__global__ __launch_bounds__(256) void build_unitary_kernel(const UnitaryDesc* __restrict__ descs,
                                                            const int* __restrict__ base, int nprob) {
  extern __shared__ double2 col[];  // [UCOLS][2^k]
  const int p = find_problem(base, nprob, blockIdx.x);
  const UnitaryDesc& d = descs[p];
  const int cb = blockIdx.x - base[p];
  const int k = d.k, dim = 1 << k;
  const int UCOLS = d.cols;
  const int c0 = cb * UCOLS;
  const int ncol = min(UCOLS, dim - c0);
  if (ncol <= 0) return;
  for (int e = threadIdx.x; e < UCOLS * dim; e += blockDim.x) {
    const int c = e / dim, i = e % dim;
    col[e] = make_double2((c < ncol && i == c0 + c) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int g = 0; g < d.ngates; ++g) {
    const UGate& G = d.gates[g];
    if (G.nq == 1) {
      const int bit = k - 1 - G.q0;
      const int half = dim >> 1;
      for (int e = threadIdx.x; e < ncol * half; e += blockDim.x) {
        const int c = e / half, j = e % half;
        const int lowmask = (1 << bit) - 1;
        const int i0 = ((j & ~lowmask) << 1) | (j & lowmask);
        const int i1 = i0 | (1 << bit);
        double2* v = col + c * dim;
        const double2 x0 = v[i0], x1 = v[i1];
        const double2 u00 = make_double2(G.u[0], G.u[1]), u01 = make_double2(G.u[2], G.u[3]);
        const double2 u10 = make_double2(G.u[4], G.u[5]), u11 = make_double2(G.u[6], G.u[7]);
        v[i0] = cadd(cmul(u00, x0), cmul(u01, x1));
        v[i1] = cadd(cmul(u10, x0), cmul(u11, x1));
      }
    } else {
      const int b0 = k - 1 - G.q0, b1 = k - 1 - G.q1;  // gate index = 2*bit(q0) + bit(q1)
      const int quarter = dim >> 2;
      const int lo = min(b0, b1), hi = max(b0, b1);
      for (int e = threadIdx.x; e < ncol * quarter; e += blockDim.x) {
        const int c = e / quarter;
        int j = e % quarter;
        // insert zero bits at positions lo and hi
        j = ((j >> lo) << (lo + 1)) | (j & ((1 << lo) - 1));
        j = ((j >> hi) << (hi + 1)) | (j & ((1 << hi) - 1));
        int idx[4];
        idx[0] = j;
        idx[1] = j | (1 << b1);
        idx[2] = j | (1 << b0);
        idx[3] = j | (1 << b0) | (1 << b1);
        double2* v = col + c * dim;
        double2 x[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = v[idx[a]];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          double2 s = make_double2(0.0, 0.0);
#pragma unroll
          for (int b = 0; b < 4; ++b) s = cadd(s, cmul(make_double2(G.u[2 * (4 * a + b)], G.u[2 * (4 * a + b) + 1]), x[b]));
          v[idx[a]] = s;
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < ncol * dim; e += blockDim.x) {
    const int c = e / dim, i = e % dim;
    const double2 v = col[c * dim + i];
    d.U64[(int64_t)i * dim + c0 + c] = v;
    if (d.U32) d.U32[(int64_t)i * dim + c0 + c] = make_float2((float)v.x, (float)v.y);
  }
}

// ------------------------------------------------------------- apply_1q --
template <typename C>
__global__ __launch_bounds__(256) void apply_1q_kernel(const Site1QDesc* __restrict__ descs,
                                                       const int* __restrict__ base, int nprob) {
  const int p = find_problem(base, nprob, blockIdx.x);
  const Site1QDesc& d = descs[p];
  const int b = blockIdx.x - base[p];
  const int64_t cols = (int64_t)d.chi_l * d.chi_r;
  C* B = (C*)d.B;
  const double2 u00 = make_double2(d.u[0], d.u[1]), u01 = make_double2(d.u[2], d.u[3]);
  const double2 u10 = make_double2(d.u[4], d.u[5]), u11 = make_double2(d.u[6], d.u[7]);
  for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < cols; e += (int64_t)d.blocks * 256) {
    const int64_t l = e / d.chi_r, r = e % d.chi_r;
    C* p0 = B + (l * 2) * d.chi_r + r;
    C* p1 = p0 + d.chi_r;
    const double2 x0 = to_d2(*p0), x1 = to_d2(*p1);
    *p0 = from_d2<C>(cadd(cmul(u00, x0), cmul(u01, x1)));
    *p1 = from_d2<C>(cadd(cmul(u10, x0), cmul(u11, x1)));
  }
}

// --------------------------------------------------------------- select --
constexpr int SEL_MAX = 4096;

__global__ __launch_bounds__(1024) void select_kernel(const SelectDesc* __restrict__ descs) {
  __shared__ double val[SEL_MAX];
  __shared__ int idx[SEL_MAX];
  __shared__ double red[1024];
  __shared__ int ired[1024];
  const SelectDesc& d = descs[blockIdx.x];
  const bool sk = d.use_sk && *d.use_sk;  // accepted learned sketch: its s eigenvalues
  const int n = sk ? d.s_sk : dim_value(d.n);
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  const int tid = threadIdx.x;
  for (int i = tid; i < np2; i += 1024) {
    if (i < n) {
      const double v = sk ? d.lam_sk[i] : d.lam_in ? d.lam_in[i] : d.G[(int64_t)i * d.ldg + i].x;
      val[i] = v > 0.0 ? v : 0.0;
    } else {
      val[i] = -1.0;
    }
    idx[i] = i;
  }
  __syncthreads();
  // bitonic sort, descending by value, ties by ascending index
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < np2; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = ((i & size) == 0);
          const double vi = val[i], vj = val[j];
          const int ii = idx[i], ij = idx[j];
          // "i before j" in the descending order
          const bool i_first = (vi > vj) || (vi == vj && ii < ij);
          if (desc ? !i_first : i_first) {
            val[i] = vj;
            val[j] = vi;
            idx[i] = ij;
            idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  // total weight (fixed-order tree reduction)
  double s = 0.0;
  for (int i = tid; i < n; i += 1024) s += val[i];
  red[tid] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  // the sketch misses eigenvalues below the threshold: the total is trace(G)
  const double tot = sk ? *d.tot_sk : red[0];
  __syncthreads();
  // count of normalised singular values >= eps_eff
  int c = 0;
  const double thr = d.eps_eff * d.eps_eff * tot;
  for (int i = tid; i < n; i += 1024) c += (val[i] >= thr && val[i] > 0.0) ? 1 : 0;
  ired[tid] = c;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) ired[tid] += ired[tid + w];
    __syncthreads();
  }
  int r = ired[0];
  r = min(r, min(d.chi_max, min(n, d.rows)));
  r = max(r, 1);
  __syncthreads();
  double k = 0.0;
  for (int i = tid; i < r; i += 1024) k += val[i];
  red[tid] = k;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double kept = red[0];
  for (int i = tid; i < n; i += 1024) d.perm[i] = idx[i];
  const double inv = kept > 0.0 ? 1.0 / kept : 0.0;
  for (int i = tid; i < r; i += 1024) d.lam_out[i] = kept > 0.0 ? sqrt(val[i] * inv) : (i == 0 ? 1.0 : 0.0);
  if (tid == 0) {
    *d.r_out = r;
    const double f = (tot > 0.0) ? kept / tot : 1.0;
    *d.logf_acc += log(f);
    if (d.rec) {
      d.rec[0] = f;
      d.rec[1] = (val[0] > 0.0) ? sqrt(val[r - 1] / val[0]) : 0.0;
      d.rec[2] = (tot > 0.0) ? (tot - kept) / tot : 0.0;
      const double next = (r < n) ? sqrt(val[r] > 0 ? val[r] : 0.0) : 0.0;
      d.rec[3] = (r < n && (sqrt(val[r - 1]) - next) < 1e-8 * sqrt(val[0])) ? 1.0 : 0.0;
    }
  }
}

// --------------------------------------------------------------- gather --
template <typename C>
__global__ __launch_bounds__(256) void gather_kernel(const GatherDesc* __restrict__ descs,
                                                     const int* __restrict__ base, int nprob) {
  __shared__ double2 tile[64][65];
  const int p = find_problem(base, nprob, blockIdx.x);
  const GatherDesc& d = descs[p];
  const int t = blockIdx.x - base[p];
  const int n = dim_value(d.n), r = *d.r;
  const int tcols = (n + 63) / 64;  // tiles along V's rows (= B's columns)
  const int tr = t / tcols, tc = t % tcols;  // tr: block of kept columns i, tc: block of V rows
  const int i0 = tr * 64, v0 = tc * 64;
  if (i0 >= r || v0 >= n) return;
  const bool sk = d.use_sk && *d.use_sk;  // accepted learned sketch: V = Q W
  const double2* V = sk ? d.Vs : d.V;
  const int ldv = sk ? d.ld_sk : d.ldv;
  // read V[v0 + a][perm[i0 + b]] -> tile[a][b]
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int a = e >> 6, b = e & 63;
    double2 v = make_double2(0.0, 0.0);
    if (v0 + a < n && i0 + b < r) v = V[(int64_t)(v0 + a) * ldv + d.perm[i0 + b]];
    tile[a][b] = v;
  }
  __syncthreads();
  C* B = (C*)d.B;
  C* Vr = (C*)d.Vr;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int a = e >> 6, b = e & 63;
    // Vr[v0 + a][i0 + b] = V[...][perm]  (coalesced along b)
    if (v0 + a < n && i0 + b < r) Vr[(int64_t)(v0 + a) * r + i0 + b] = from_d2<C>(tile[a][b]);
    // B[i0 + a][v0 + b] = conj(V[v0 + b][perm[i0 + a]])  (coalesced along b)
    if (i0 + a < r && v0 + b < n) {
      const double2 w = tile[b][a];
      B[(int64_t)(i0 + a) * n + v0 + b] = from_d2<C>(make_double2(w.x, -w.y));
    }
  }
}

// ------------------------------------------------------------- finalize --
template <typename C>
__global__ __launch_bounds__(256) void finalize_kernel(const ScaleDesc* __restrict__ descs,
                                                       const int* __restrict__ base, int nprob) {
  const int p = find_problem(base, nprob, blockIdx.x);
  const ScaleDesc& d = descs[p];
  const int b = blockIdx.x - base[p];
  const int64_t cnt = dim_value(d.count);
  const double s = exp(-0.5 * (*d.logf));
  const C* X = (const C*)d.X;
  C* B = (C*)d.B;
  for (int64_t e = (int64_t)b * 256 + threadIdx.x; e < cnt; e += (int64_t)d.blocks * 256)
    B[e] = cscale(X[e], s);
}

__global__ void convert_kernel(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

__global__ void convert_f2d_kernel(const float2* __restrict__ src, double2* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = make_double2(src[i].x, src[i].y);
}

__global__ void accumulate_kernel(const double* __restrict__ v, int n, double* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = *total;
    for (int i = 0; i < n; ++i) s += v[i];
    *total = s;
  }
}

// total += *v[0] + ... + *v[n-1], in that order (the log f of the clusters
// that finished in one round of the wavefront executor, each in its own
// workspace)
__global__ void accumulate_ptrs_kernel(const double* const* __restrict__ v, int n, double* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = *total;
    for (int i = 0; i < n; ++i) s += *v[i];
    *total = s;
  }
}

// ---- small dense helpers of the DMRG fit (FP64 complex, row-major)
// out[0] = sum |x_i|^2 (one workgroup, fixed order of the partial sums)
__global__ __launch_bounds__(256) void dense_norm2_kernel(const double2* __restrict__ x, int64_t n,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i].x * x[i].x + x[i].y * x[i].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void dense_scale_kernel(double2* __restrict__ x, int64_t n, double a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = make_double2(a * x[i].x, a * x[i].y);
}

// out (cols x rows, ldo) = conj(in (rows x cols, ldi))^T with row i of out
// scaled by d[i] when d is non-null
__global__ void dense_adjoint_kernel(const double2* __restrict__ in, int rows, int cols, int ldi,
                                     const double* __restrict__ d, double2* __restrict__ out, int ldo) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / rows), j = (int)(e % rows);  // out row i (input column), out column j (input row)
    const double2 v = in[(int64_t)j * ldi + i];
    const double sc = d ? d[i] : 1.0;
    out[(int64_t)i * ldo + j] = make_double2(sc * v.x, -sc * v.y);
  }
}

// columns j < cols of x (rows x cols, ld) scaled by d[j]
__global__ void dense_scale_cols_kernel(double2* __restrict__ x, int rows, int cols, int ld,
                                        const double* __restrict__ d) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    const double2 v = x[(int64_t)i * ld + j];
    x[(int64_t)i * ld + j] = make_double2(d[j] * v.x, d[j] * v.y);
  }
}

// C (M x N, ldc) = the sum of the `parts` partial products P + q stride
// (each M x N, row-major), in order q = 0, 1, ...
__global__ void dense_sum_parts_kernel(const double2* __restrict__ P, int parts, int64_t stride, int M, int N,
                                       double2* __restrict__ C, int ldc) {
  const int64_t total = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int q = 0; q < parts; ++q) {
      const double2 v = P[(int64_t)q * stride + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    C[(e / N) * ldc + e % N] = acc;
  }
}

}  // namespace

hipError_t launch_dense_sum_parts(const double2* P, int parts, int64_t stride, int M, int N, double2* C, int ldc,
                                  hipStream_t s) {
  const int64_t n = (int64_t)M * N;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  launch(dense_sum_parts_kernel, dim3(blocks), dim3(256), 0, s, P, parts, stride, M, N, C, ldc);
  return hipGetLastError();
}

hipError_t launch_dense_norm2(const double2* x, int64_t n, double* out, hipStream_t s) {
  launch(dense_norm2_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_dense_scale(double2* x, int64_t n, double a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  launch(dense_scale_kernel, dim3(blocks), dim3(256), 0, s, x, n, a);
  return hipGetLastError();
}

hipError_t launch_dense_adjoint(const double2* in, int rows, int cols, int ldi, const double* d, double2* out,
                                int ldo, hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  launch(dense_adjoint_kernel, dim3(blocks), dim3(256), 0, s, in, rows, cols, ldi, d, out, ldo);
  return hipGetLastError();
}

hipError_t launch_dense_scale_cols(double2* x, int rows, int cols, int ld, const double* d, hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  launch(dense_scale_cols_kernel, dim3(blocks), dim3(256), 0, s, x, rows, cols, ld, d);
  return hipGetLastError();
}

hipError_t launch_accumulate_ptrs(const double* const* v, int n, double* total, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch(accumulate_ptrs_kernel, dim3(1), dim3(64), 0, s, v, n, total);
  return hipGetLastError();
}

hipError_t launch_build_unitary(const UnitaryDesc* d, const int* d_base, int nprob, int blocks,
                                size_t lds_bytes, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  const size_t lds = lds_bytes;
  launch(build_unitary_kernel, dim3(blocks), dim3(256), lds, s, d, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_apply_1q(Prec p, const Site1QDesc* d, const int* d_base, int nprob, int blocks,
                           hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (p == Prec::FP64)
    launch(apply_1q_kernel<double2>, dim3(blocks), dim3(256), 0, s, d, d_base, nprob);
  else
    launch(apply_1q_kernel<float2>, dim3(blocks), dim3(256), 0, s, d, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_select(const SelectDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  launch(select_kernel, dim3(nprob), dim3(1024), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_gather(Prec p, const GatherDesc* d, const int* d_base, int nprob, int blocks,
                         hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (p == Prec::FP64)
    launch(gather_kernel<double2>, dim3(blocks), dim3(256), 0, s, d, d_base, nprob);
  else
    launch(gather_kernel<float2>, dim3(blocks), dim3(256), 0, s, d, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_finalize(Prec p, const ScaleDesc* d, const int* d_base, int nprob, int blocks,
                           hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (p == Prec::FP64)
    launch(finalize_kernel<double2>, dim3(blocks), dim3(256), 0, s, d, d_base, nprob);
  else
    launch(finalize_kernel<float2>, dim3(blocks), dim3(256), 0, s, d, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_convert_d2f(const double2* src, float2* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  launch(convert_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_convert_f2d(const float2* src, double2* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  launch(convert_f2d_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_accumulate(const double* v, int n, double* total, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch(accumulate_kernel, dim3(1), dim3(64), 0, s, v, n, total);
  return hipGetLastError();
}

}  // namespace ctebd
