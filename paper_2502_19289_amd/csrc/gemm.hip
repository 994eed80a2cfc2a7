// Grouped complex GEMMs on the matrix cores (FP32 and FP64 MFMA 16x16x4).
//
// Used for the block merge Theta_j = Theta_{j-1} B_j, the application of the
// cluster unitary Theta'_l = U Theta_l (batched over the left bond index l),
// the projection X <- X V_r of the split sweep, and the FP64 Gram matrix
// G = X^H D^2 X of every truncated SVD (arXiv:2502.19289, Secs. II.B, III.A).
//
// Tiling: a 256-thread workgroup computes a 64x64 complex output tile; its four
// wavefronts own 32x32 quadrants made of 2x2 MFMA blocks.  K advances in slices
// of 16 staged in LDS k-major (As[k][m], Bs[k][n]) so that the sixteen lanes
// that share a k read consecutive addresses.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace ctebd {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;


enum { MODE_NN = 0, MODE_GRAM = 1, MODE_CN = 2 };

template <typename CI, typename TM>
__device__ __forceinline__ typename cpx_of<TM>::type load_c(const CI* p) {
  const CI v = *p;
  typename cpx_of<TM>::type r;
  r.x = (TM)v.x;
  r.y = (TM)v.y;
  return r;
}

template <typename CI, typename CO, typename TM, int MODE>
__global__ __launch_bounds__(NT) void cgemm_kernel(const GemmDesc* __restrict__ descs,
                                                   const int* __restrict__ base, int nprob) {
  using CM = typename cpx_of<TM>::type;
  __shared__ CM As[2][BK][BM + 1];  // (rows padded: the staging writes of
  __shared__ CM Bs[2][BK][BN + 1];  // consecutive k rows fall in different banks)

  const int p = find_problem(base, nprob, blockIdx.x);
  const GemmDesc& d = descs[p];
  int t = blockIdx.x - base[p];
  const int M = dim_value(d.M), N = dim_value(d.N), K = dim_value(d.K);
  const int lda = dim_value(d.lda), ldb = dim_value(d.ldb), ldc = dim_value(d.ldc);
  const int tj = t % d.tn;
  t /= d.tn;
  const int ti = t % d.tm;
  t /= d.tm;
  const int split = t % d.ksplit;
  const int b = t / d.ksplit;
  const int m0 = ti * BM, n0 = tj * BN;
  if (b >= d.batch || m0 >= M || n0 >= N) return;
  if (d.skip && gld(d.skip)) return;
  if (MODE == MODE_GRAM && ti > tj) return;

  const CI* A = (const CI*)d.A + (int64_t)b * d.sA;
  const CI* Bm = (const CI*)d.B + (int64_t)b * d.sB;
  CO* C = (CO*)d.C + (int64_t)b * d.sC + (int64_t)split * d.part;

  int kbeg = 0, kend = K;
  if (d.ksplit > 1) {
    const int kc = ((K + d.ksplit - 1) / d.ksplit + BK - 1) / BK * BK;
    kbeg = split * kc;
    kend = min(K, kbeg + kc);
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  CAcc3<TM> acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j].clear();

  // Two LDS buffers: the loads of slice k0 + BK are issued before the
  // products of slice k0 (from one buffer) and staged into the other buffer
  // after them, so one barrier per slice separates the two.  The loads are
  // unconditional, at addresses clamped into the operands, and masked when
  // staged (a load guarded by its own branch would be waited for before the
  // next one is issued); they are kept in the input type until staged.
  CI ra[4], rb[4];
  TM wv = (TM)0;
  auto fetch = [&](int k0) __attribute__((always_inline)) {
    if (MODE == MODE_NN) {
      const int r = tid >> 2, c4 = (tid & 3) * 4;
      const int gm = min(m0 + r, M - 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) ra[i] = gld(A + (int64_t)gm * lda + min(k0 + c4 + i, kend - 1));
      const int kk = tid >> 4, n1 = tid & 15;
      const int gk = min(k0 + kk, kend - 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) rb[i] = gld(Bm + (int64_t)gk * ldb + min(n0 + n1 + 16 * i, N - 1));
    } else {
      // rows gk of A (K x M) and of B (K x N; A itself for a Gram matrix)
      const int kk = tid >> 4, c1 = tid & 15;
      const int gk = min(k0 + kk, kend - 1);
      const CI* Bk = MODE == MODE_GRAM ? A + (int64_t)gk * lda : Bm + (int64_t)gk * ldb;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ra[i] = gld(A + (int64_t)gk * lda + min(m0 + c1 + 16 * i, M - 1));
        rb[i] = gld(Bk + min(n0 + c1 + 16 * i, N - 1));
      }
      if (MODE == MODE_GRAM) wv = (TM)gld(d.w + (gk >> d.wshift));
    }
  };
  // ---- stage A (BM x BK) k-major and B (BK x BN) into buffer q; zero
  // outside the operands (component selects: a select of whole values would
  // take their addresses)
  auto stage = [&](int q, int k0) __attribute__((always_inline)) {
    auto cvt = [](bool in, CI v) {
      CM r;
      r.x = in ? (TM)v.x : (TM)0;
      r.y = in ? (TM)v.y : (TM)0;
      return r;
    };
    if (MODE == MODE_NN) {
      const int r = tid >> 2, c4 = (tid & 3) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) As[q][c4 + i][r] = cvt(m0 + r < M && k0 + c4 + i < kend, ra[i]);
      const int kk = tid >> 4, n1 = tid & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) Bs[q][kk][n1 + 16 * i] = cvt(k0 + kk < kend && n0 + n1 + 16 * i < N, rb[i]);
    } else {
      const int kk = tid >> 4, c1 = tid & 15;
      const bool kin = k0 + kk < kend;
      const TM wk = MODE == MODE_GRAM ? (kin ? wv : (TM)0) : (TM)1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        CM va = cvt(kin && m0 + c1 + 16 * i < M, ra[i]), vb = cvt(kin && n0 + c1 + 16 * i < N, rb[i]);
        va.x *= wk;
        va.y = -va.y * wk;  // conjugated (A^H)
        vb.x *= wk;
        vb.y *= wk;
        As[q][kk][c1 + 16 * i] = va;
        Bs[q][kk][c1 + 16 * i] = vb;
      }
    }
  };
  if (kbeg < kend) {
    fetch(kbeg);
    stage(0, kbeg);
  }
  __syncthreads();
  int q = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) fetch(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
      CM a0 = As[q][kr][wm * 32 + cl], a1 = As[q][kr][wm * 32 + 16 + cl];
      CM b0 = Bs[q][kr][wn * 32 + cl], b1 = Bs[q][kr][wn * 32 + 16 + cl];
      acc[0][0].mac(a0.x, a0.y, b0.x, b0.y);
      acc[0][1].mac(a0.x, a0.y, b1.x, b1.y);
      acc[1][0].mac(a1.x, a1.y, b0.x, b0.y);
      acc[1][1].mac(a1.x, a1.y, b1.x, b1.y);
    }
    if (more) stage(q ^ 1, k0 + BK);
    __syncthreads();
    q ^= 1;
  }

  const TM alpha = (TM)d.alpha;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 32 + bi * 16 + Mfma<TM>::row(lane, r);
        const int gn = n0 + wn * 32 + bj * 16 + (lane & 15);
        if (gm < M && gn < N) {
          CO v;
          v.x = acc_re(acc[bi][bj], r) * alpha;
          v.y = acc_im(acc[bi][bj], r) * alpha;
          gst(C + (int64_t)gm * ldc + gn, v);
          // a Gram matrix without split-K is complete here: mirror it
          if (MODE == MODE_GRAM && d.ksplit == 1 && ti < tj) {
            v.y = -v.y;
            gst(C + (int64_t)gn * ldc + gm, v);
          }
        }
      }
}

// Sums the split-K partial Gram matrices and fills the lower triangle from
// the upper one (G is Hermitian).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const GramReduceDesc* __restrict__ descs,
                                                          const int* __restrict__ base, int nprob) {
  const int p = find_problem(base, nprob, blockIdx.x);
  const GramReduceDesc& d = descs[p];
  const int n = dim_value(d.n), ld = dim_value(d.ld);
  const int t = blockIdx.x - base[p];
  const int nt = (n + 63) / 64;
  const int ti = t / nt, tj = t % nt;
  if (ti >= nt || ti > tj) return;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = ti * 64 + (e >> 6), j = tj * 64 + (e & 63);
    if (i >= n || j >= n) continue;
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < d.ksplit; ++q) s = cadd(s, gld(d.part + (int64_t)q * d.stride + (int64_t)i * ld + j));
    gst(d.G + (int64_t)i * ld + j, s);
    if (ti < tj) gst(d.G + (int64_t)j * ld + i, make_double2(s.x, -s.y));
  }
}

// ------------------------------------------------------------ BF16X6 ----
// C = A B for complex64 A, B with the BF16 matrix cores: every FP32 component
// x is split exactly into x = hi + mid + lo (three BF16 values, 24 mantissa
// bits in all) and each real product keeps the six partial products of order
// >= 2^-16 relative (hh, hm, mh, hl, lh, mm), accumulated in FP32.
// Cr = Ar Br - Ai Bi, Ci = Ar Bi + Ai Br.  64x64 complex output per workgroup,
// four wavefronts of 32x32 (2x2 blocks of v_mfma_f32_16x16x32_bf16), K slices
// of 32 staged in LDS as three planes per real component, k contiguous.
// Staging: a thread takes 8 consecutive k of one row of A and of one column
// of B, splits them in registers and writes each plane with one 16-byte LDS
// store; the next slice's loads are issued (unconditionally, at clamped
// addresses, masked when staged) before the current slice's products.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int XK = 32, XPAD = 40;  // K slice and padded LDS row (bf16 elements)

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// the three planes of 8 values (v masked to zero where !in)
__device__ __forceinline__ void split8(const float* v, bf16x8& h, bf16x8& m, bf16x8& l) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const __bf16 hh = (__bf16)v[i];
    const float r1 = v[i] - (float)hh;
    const __bf16 mm = (__bf16)r1;
    const float r2 = r1 - (float)mm;
    h[i] = hh;
    m[i] = mm;
    l[i] = (__bf16)r2;
  }
}

__global__ __launch_bounds__(256) void cgemm_bf16x6_kernel(const GemmDesc* __restrict__ descs,
                                                           const int* __restrict__ base, int nprob) {
  // planes [3 (hi,mid,lo)][2 (re,im)][64 rows][XPAD]; A as [m][k], B as [n][k]
  __shared__ __attribute__((aligned(16))) __bf16 As[3][2][64][XPAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[3][2][64][XPAD];

  const int p = find_problem(base, nprob, blockIdx.x);
  const GemmDesc& d = descs[p];
  int t = blockIdx.x - base[p];
  const int M = dim_value(d.M), N = dim_value(d.N), K = dim_value(d.K);
  const int lda = dim_value(d.lda), ldb = dim_value(d.ldb), ldc = dim_value(d.ldc);
  const int tj = t % d.tn;
  t /= d.tn;
  const int ti = t % d.tm;
  t /= d.tm;
  const int b = t;
  const int m0 = ti * 64, n0 = tj * 64;
  if (b >= d.batch || m0 >= M || n0 >= N) return;
  if (d.skip && gld(d.skip)) return;
  const float2* A = (const float2*)d.A + (int64_t)b * d.sA;
  const float2* Bm = (const float2*)d.B + (int64_t)b * d.sB;
  float2* C = (float2*)d.C + (int64_t)b * d.sC;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  // Ar Br, Ai Bi, Ar Bi, Ai Br: four independent accumulator chains per block
  f32x4 arr[2][2], ari[2][2], aib[2][2], aia[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      arr[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      ari[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      aib[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      aia[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  // staging roles: A row ra, k offset ka; B column nb, k offset kb
  const int ra = tid >> 2, ka = (tid & 3) * 8;
  const int nb = tid & 63, kb = (tid >> 6) * 8;
  const bool rowok = m0 + ra < M, colok = n0 + nb < N;
  const float2* Arow = A + (int64_t)min(m0 + ra, M - 1) * lda;
  const float2* Bcol = Bm + min(n0 + nb, N - 1);
  float2 va[8], vb[8];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 8; ++i) va[i] = gld(Arow + min(k0 + ka + i, K - 1));
#pragma unroll
    for (int i = 0; i < 8; ++i) vb[i] = gld(Bcol + (int64_t)min(k0 + kb + i, K - 1) * ldb);
  };
  auto stage = [&](int k0) __attribute__((always_inline)) {
    float re[8], im[8];
    bf16x8 h, m, l;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bool in = rowok && k0 + ka + i < K;
      re[i] = in ? va[i].x : 0.f;
      im[i] = in ? va[i].y : 0.f;
    }
    split8(re, h, m, l);
    *(bf16x8*)&As[0][0][ra][ka] = h;
    *(bf16x8*)&As[1][0][ra][ka] = m;
    *(bf16x8*)&As[2][0][ra][ka] = l;
    split8(im, h, m, l);
    *(bf16x8*)&As[0][1][ra][ka] = h;
    *(bf16x8*)&As[1][1][ra][ka] = m;
    *(bf16x8*)&As[2][1][ra][ka] = l;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bool in = colok && k0 + kb + i < K;
      re[i] = in ? vb[i].x : 0.f;
      im[i] = in ? vb[i].y : 0.f;
    }
    split8(re, h, m, l);
    *(bf16x8*)&Bs[0][0][nb][kb] = h;
    *(bf16x8*)&Bs[1][0][nb][kb] = m;
    *(bf16x8*)&Bs[2][0][nb][kb] = l;
    split8(im, h, m, l);
    *(bf16x8*)&Bs[0][1][nb][kb] = h;
    *(bf16x8*)&Bs[1][1][nb][kb] = m;
    *(bf16x8*)&Bs[2][1][nb][kb] = l;
  };

  if (K > 0) {
    fetch(0);
    stage(0);
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4), cl = lane & 15;
  for (int k0 = 0; k0 < K; k0 += XK) {
    const bool more = k0 + XK < K;
    if (more) fetch(k0 + XK);
    bf16x8 br[2][3], bi[2][3];  // the B planes of both column blocks, read once
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) {
        br[j][pl] = *(const bf16x8*)&Bs[pl][0][wn * 32 + j * 16 + cl][kq];
        bi[j][pl] = *(const bf16x8*)&Bs[pl][1][wn * 32 + j * 16 + cl][kq];
      }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      bf16x8 ar[3], ai[3];
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) {
        ar[pl] = *(const bf16x8*)&As[pl][0][wm * 32 + i * 16 + cl][kq];
        ai[pl] = *(const bf16x8*)&As[pl][1][wm * 32 + i * 16 + cl][kq];
      }
      // the six plane products (hh, hm, mh, hl, lh, mm), each across the
      // eight chains of this row block before the next
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int pa = q == 2 ? 1 : q == 4 ? 2 : q == 5 ? 1 : 0;
        const int pb = q == 1 ? 1 : q == 3 ? 2 : q == 5 ? 1 : 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          arr[i][j] = mfma_bf16(ar[pa], br[j][pb], arr[i][j]);
          ari[i][j] = mfma_bf16(ai[pa], bi[j][pb], ari[i][j]);
          aib[i][j] = mfma_bf16(ar[pa], bi[j][pb], aib[i][j]);
          aia[i][j] = mfma_bf16(ai[pa], br[j][pb], aia[i][j]);
        }
      }
    }
    __syncthreads();
    if (more) {
      stage(k0 + XK);
      __syncthreads();
    }
  }
  const float alpha = (float)d.alpha;
#pragma unroll
  for (int bi2 = 0; bi2 < 2; ++bi2)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 32 + bi2 * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wn * 32 + bj * 16 + (lane & 15);
        if (gm < M && gn < N)
          gst(C + (int64_t)gm * ldc + gn,
              make_float2((arr[bi2][bj][r] - ari[bi2][bj][r]) * alpha, (aib[bi2][bj][r] + aia[bi2][bj][r]) * alpha));
      }
}

}  // namespace

int gemm_tiles(const GemmDesc& d) { return d.tm * d.tn * d.ksplit * d.batch; }

hipError_t launch_gemm_bf16x6(const GemmDesc* d_desc, const int* d_base, int nprob, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(cgemm_bf16x6_kernel, dim3(blocks), dim3(256), 0, s, d_desc, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(Prec p, const GemmDesc* d_desc, const int* d_base, int nprob, int blocks,
                          hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (p == Prec::FP64)
    launch(cgemm_kernel<double2, double2, double, MODE_NN>, dim3(blocks), dim3(NT), 0, s, d_desc, d_base, nprob);
  else if (p == Prec::BF16X6)
    return launch_gemm_bf16x6(d_desc, d_base, nprob, blocks, s);
  else
    launch(cgemm_kernel<float2, float2, float, MODE_NN>, dim3(blocks), dim3(NT), 0, s, d_desc, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_gram(Prec in_prec, const GemmDesc* d_desc, const int* d_base, int nprob, int blocks,
                       hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (in_prec == Prec::FP64)
    launch(cgemm_kernel<double2, double2, double, MODE_GRAM>, dim3(blocks), dim3(NT), 0, s, d_desc, d_base, nprob);
  else
    launch(cgemm_kernel<float2, double2, double, MODE_GRAM>, dim3(blocks), dim3(NT), 0, s, d_desc, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_gemm_cn(const GemmDesc* d_desc, const int* d_base, int nprob, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(cgemm_kernel<double2, double2, double, MODE_CN>, dim3(blocks), dim3(NT), 0, s, d_desc, d_base, nprob);
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const GramReduceDesc* d_desc, const int* d_base, int nprob, int blocks,
                              hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(gram_reduce_kernel, dim3(blocks), dim3(256), 0, s, d_desc, d_base, nprob);
  return hipGetLastError();
}

}  // namespace ctebd
