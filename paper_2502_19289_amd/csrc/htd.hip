// Dense Hermitian eigen-solver of the large splits.  The truncated SVD of a
// split is read off the eigen-decomposition of its Gram matrix (Sec. III.A);
// for Gram matrices of a few hundred rows and more this path replaces block
// Jacobi, whose sweeps each take about 2n dependent rotation rounds:
//
//  1. Householder reduction G = Q T Q^H with T real symmetric tridiagonal,
//     Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^H; per column one
//     launch forms the reflector and y = tau G v (every workgroup rebuilds
//     the reflector from row k, so no launch is spent on it), one launch
//     applies the rank-two update G -= v w^H + w v^H;
//  2. Cuppen's divide and conquer on T: T is torn into 1x1 blocks by rank-one
//     corrections at every off-diagonal entry, then merged level by level:
//     per merge a deflation scan, the secular equation per root, z recomputed
//     from the roots (Loewner formula, which keeps the eigenvectors orthogonal
//     whatever the root accuracy) and a GEMM with the children's eigenvectors;
//  3. back-transformation V = Q Z in blocks of HTD_NB reflectors written as
//     I - V_b T_b V_b^H (compact WY).
//
// Everything is FP64.  All kernels serve the problems of one split level at
// once; each computes its problem and block from the same per-problem counts
// as the host (kernels.hpp), and problems whose learned sketch was accepted
// (skip flag) return at once.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "kernels.hpp"
#include "mfma.hpp"

namespace ctebd {
namespace {

constexpr double EPS53 = 1.1102230246251565e-16;  // unit roundoff of FP64

struct Loc {
  int p, b;
};

// problem and problem-local block of flat block `bid`; the sizes come with
// the launch (kernel arguments), so finding the problem costs no memory access
template <typename S, typename F>
__device__ __forceinline__ Loc locate(const S& sz, int bid, F count) {
  for (int p = 0; p < sz.np; ++p) {
    const int c = count(sz.n[p]);
    if (bid < c) return Loc{p, bid};
    bid -= c;
  }
  return Loc{-1, 0};
}
// the same with counts that also depend on the back-transformed columns
template <typename F>
__device__ __forceinline__ Loc locate_d(const HtdSizes& sz, int bid, F count) {
  for (int p = 0; p < sz.np; ++p) {
    const int c = count(sz.n[p], sz.nc[p]);
    if (bid < c) return Loc{p, bid};
    bid -= c;
  }
  return Loc{-1, 0};
}

__device__ __forceinline__ bool skipped(const HtdDesc& d) { return d.skip && gld(d.skip); }

__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// ======================================================= tridiagonalisation
// Block reductions over the four wavefronts of a 256-thread workgroup: wave
// shuffles, then the wave results combined in a fixed order (deterministic).
// Wavefront sum on the DPP paths (no LDS permutes): pairs and quads
// (quad_perm), 8- and 16-lane rows (row_half_mirror, row_mirror), then rows
// 0+1 and 0..3 through row_bcast15 / row_bcast31, which leaves the total in
// lane 63; read back as a scalar, so every lane returns the same bits.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_take<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_take<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_take<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_take<0x140, 0xf>(v);  // row_mirror
  v += dpp_take<0x142, 0xa>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_take<0x143, 0xc>(v);  // row_bcast31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// N wavefront sums at once, stage by stage, so that the DPP steps of the
// different values are independent and issue back to back.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_take<0xb1, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_take<0x4e, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_take<0x141, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_take<0x140, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_take<0x142, 0xa>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_take<0x143, 0xc>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const long long b = __double_as_longlong(v[i]);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    v[i] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
}
// Orders a wavefront's LDS writes before its later LDS reads of the values
// other lanes of the same wavefront wrote (the hardware executes a
// wavefront's LDS operations in order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// lane q's value in every lane (q the same in all lanes)
__device__ __forceinline__ double lane_at(double v, int q) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, q);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), q);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// v + (v of lane c ^ 16) and v + (v of lane c ^ 32) with the lane-swap
// instructions: swapping a register with itself leaves lanes c and c ^ 16
// (c ^ 32) holding the pair's two values in its two results, so their sum
// is the pair sum in both lanes, the same value a shuffle gives, without the
// LDS crossbar.
__device__ __forceinline__ double pair_sum16(double v) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)b, (int)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(b >> 32), (int)(b >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]) +
         __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
}
__device__ __forceinline__ double pair_sum32(double v) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)b, (int)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(b >> 32), (int)(b >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]) +
         __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
}
// Wavefront maximum on the same DPP paths as wave_sum.
// lane 0's value in every lane
__device__ __forceinline__ double lane0(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_take<0xb1, 0xf>(v));
  v = fmax(v, dpp_take<0x4e, 0xf>(v));
  v = fmax(v, dpp_take<0x141, 0xf>(v));
  v = fmax(v, dpp_take<0x140, 0xf>(v));
  v = fmax(v, dpp_take<0x142, 0xa>(v));
  v = fmax(v, dpp_take<0x143, 0xc>(v));
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double block4_max(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}
__device__ __forceinline__ double block4_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Blocked (panel) form of the Householder reduction.  Within a panel of
// HTD_NB columns the trailing matrix stays as it was at the panel start; for
// column k (panel column j) with the panel's earlier reflectors V[:, <j] and
// vectors W[:, <j]:
//   trd_col:   x = G[k+1:, k] - V W[k, :]^H - W V[k, :]^H (the up-to-date
//              column), its scaled norm and the dots V^H x, W^H x; it also
//              finalises w_{j-1} = y_{j-1} - (tau/2)(y_{j-1}^H v_{j-1}) v_{j-1}
//              from y_{j-1} (summed from the HEMV's slots; neither kernel
//              writes what it reads, so each can be launched again on the
//              same inputs)
//   trd_hemv:  the reflector H^H (alpha, x1)^T = (beta, 0)^T (beta real) and
//              y = tau (G v - V (W^H v) - W (V^H v)) from the lower triangle
//              of G, as partial sums per 64 x 64 tile (slots)
// and at the end of the panel trd_her2k applies G -= V W^H + W V^H to the
// trailing matrix on the matrix cores.  One triangle of the trailing matrix
// is thus read once per column (HEMV); all of it is read and written once per
// panel.
// acc += a b and acc += conj(a) b as four fused multiply-adds each (the
// product formed with separate multiplies and the sum with a separate add
// takes half as many instructions again)
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cfmac(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// dlassq-style running (scale, sum of squares): sum a^2 = scale^2 * ssq
__device__ __forceinline__ void lassq(double a, double& scale, double& ssq) {
  a = fabs(a);
  if (a == 0.0) return;
  if (scale < a) {
    ssq = 1.0 + ssq * (scale / a) * (scale / a);
    scale = a;
  } else {
    ssq += (a / scale) * (a / scale);
  }
}

// The reflector H = I - tau v v^H with H^H (alpha, x1)^T = (beta, 0)^T, beta
// real, v = (1, scale x1), from alpha and the scaled norm of x1
// (||x1||^2 = smax^2 ssq); tau = 0 (H = I) when x1 = 0 and alpha is real.
// Worked in units of amax = max(smax, |alpha|): with a = alpha / amax the norm
// nrm = |(a, x1 / amax)| is at least 1, b = beta / amax = -sign(Re a) nrm,
// d = a - b has |Re d| = |Re a| + nrm >= 1, so tau = (b - a) / b and
// scale = 1 / (amax d) = conj(d) / (amax |d|^2) need one reciprocal each
// (|d|^2 lies in [1, 4 nrm^2]).  Below 2^-1000 (where 1 / amax could
// overflow) the same quantities are formed by division.
__device__ __forceinline__ void householder(double2 alpha, double smax, double ssq, double& beta, double2& tau,
                                            double2& scale) {
  const double amax = fmax(smax, fmax(fabs(alpha.x), fabs(alpha.y)));
  tau = make_double2(0.0, 0.0);
  scale = make_double2(0.0, 0.0);
  beta = alpha.x;
  if (amax > 0.0) {
    const bool tiny = amax < 0x1p-1000;
    const double ia = tiny ? 0.0 : 1.0 / amax;
    const double sr = tiny ? smax / amax : smax * ia;
    const double xs2 = ssq * sr * sr;
    if (xs2 > 0.0 || alpha.y != 0.0) {
      const double ar = tiny ? alpha.x / amax : alpha.x * ia, ai = tiny ? alpha.y / amax : alpha.y * ia;
      const double nrm = sqrt(ar * ar + ai * ai + xs2);
      const double b = -copysign(nrm, alpha.x);
      beta = amax * b;
      const double dr = ar - b, den = dr * dr + ai * ai;
      if (tiny) {
        tau = make_double2((b - ar) / b, -ai / b);
        scale = make_double2(dr / den / amax, -ai / den / amax);
      } else {
        const double ib = 1.0 / b, q = 1.0 / (den * amax);
        tau = make_double2((b - ar) * ib, -ai * ib);
        scale = make_double2(dr * q, -ai * q);
      }
    }
  }
}

// KC_ROWS rows per 256-thread workgroup.  Lane c of every wavefront owns
// column c of [V | W] (c < HTD_NB: V[:, c], else W[:, c - HTD_NB]) and the
// wavefront owns rows wv, wv + 4, ... of the workgroup's rows, so that each
// load reads whole panel rows.  The column entry of row r is the sum of the
// lanes' terms (through LDS); the dots V^H x, W^H x are per-lane sums over the
// rows, added over the four wavefronts in LDS.
template <int N>
__global__ __launch_bounds__(256) void trd_col_kernel(const HtdProbs<N> sz, int k) {
  constexpr int RPW = KC_ROWS / 4;  // rows per wavefront
  __shared__ double2 dsum[4][2 * HTD_NB];
  __shared__ double2 kv[2 * HTD_NB];  // row k: w_k (V lanes), v_k (W lanes)
  __shared__ double2 psum[4];
  __shared__ double2 tx[KC_ROWS][64];  // the terms of x, row by row
  __shared__ double2 xr[KC_ROWS];
  // problem blockIdx.y: its record is the only argument line read before the data
  const Loc lc{(int)blockIdx.y, (int)blockIdx.x};
  const int n = sz.pr[lc.p].n;
  if (lc.b >= htd_col_blocks(n, k)) return;
  const HtdDesc d = htd_view(sz.pr[lc.p]);
  if (skipped(d)) return;
  const int m = n - k - 1, ld = d.ld, tid = threadIdx.x;
  const int j = k & (HTD_NB - 1);
  const int c = tid & 63, wv = tid >> 6;
  const int u = c & (HTD_NB - 1);
  const bool isv = c < HTD_NB;
  const bool live = u < j;                 // panel column u exists
  const bool vfin = isv && u == j - 1;     // holds w_k[j-1], finalised here
  const bool fin = !isv && u == j - 1;     // W column j-1, finalised here
  // independent loads, the small ones first (memory operations complete in
  // issue order): partials of alpha, row k, then this wavefront's rows
  const int nbp = j > 0 ? htd_hemv_blocks(n, k - 1) : 0;
  constexpr int PQ = (HV_PARTS + 255) / 256;
  // (loads are unconditional at clamped, always valid indexes and masked at
  // their use, so that no use is folded into a branch right after its load,
  // which would wait for it before the later loads are issued)
  double2 pq[PQ];
#pragma unroll
  for (int t = 0; t < PQ; ++t) {
    const int q = tid + 256 * t;
    pq[t] = d.part[q < nbp ? q : 0];
  }
  const double2 tpl = d.tau[k > 0 ? k - 1 : 0];
  // lane of V column u: w_k[u]; lane of W column u: v_k[u]
  double2 rk = make_double2(0.0, 0.0), rkv = make_double2(0.0, 0.0);
  if (live && !vfin) rk = isv ? d.PW[(int64_t)k * HTD_NB + u] : d.PV[(int64_t)k * HTD_NB + u];
  if (vfin) rkv = d.PV[(int64_t)k * HTD_NB + u];
  const double akk = lc.b == 0 && tid == 64 ? d.A[(int64_t)k * ld + k].x : 0.0;
  double2 a[RPW], pv[RPW], pf[RPW];
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int i = lc.b * KC_ROWS + wv + 4 * q;
    const bool own = i < m;
    const int64_t r = k + 1 + i;
    a[q] = own && c == 0 ? d.A[r * ld + k] : make_double2(0.0, 0.0);  // G[r][k], lower triangle
    pv[q] = make_double2(0.0, 0.0);
    pf[q] = make_double2(0.0, 0.0);
    if (own && live && !fin) pv[q] = isv ? d.PV[r * HTD_NB + u] : d.PW[r * HTD_NB + u];
    if (own && fin) pf[q] = d.PV[r * HTD_NB + u];
  }
  // y_{j-1}: the sums of the HEMV's slots over the rows of column k-1's
  // trailing block (which starts at row k), per wavefront: lane c takes
  // slots c / 8 + 8 u of the wavefront's row q = c % 8, and slot c of row k
  static_assert(RPW == 8, "one row of the wavefront per lane residue mod 8");
  constexpr int YU = (HV_SLOTS + 7) / 8;
  const int ty = j > 0 ? htd_hemv_rows(n, k - 1) + 2 : 0, tyc = ty > 0 ? ty : 1;
  const int yrow = min(1 + lc.b * KC_ROWS + wv + 4 * (c & 7), m);  // m: last row of that block
  double2 ys[YU];
#pragma unroll
  for (int q = 0; q < YU; ++q) ys[q] = d.Y[(int64_t)min((c >> 3) + 8 * q, tyc - 1) * ld + yrow];
  const double2 y0l = d.Y[(int64_t)min(c, tyc - 1) * ld];
  // alpha = -(tau/2) y^H v of panel column j-1 (its HEMV's partial sums)
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int t = 0; t < PQ; ++t) {
    const bool okq = tid + 256 * t < nbp;
    sx += okq ? pq[t].x : 0.0;
    sy += okq ? pq[t].y : 0.0;
  }
  {
    double sp[2] = {sx, sy};
    wave_sum_n(sp);
    sx = sp[0];
    sy = sp[1];
  }
  if (c == 0) psum[wv] = make_double2(sx, sy);
  {
    // row q = c % 8: the 8 lanes with that residue (c ^ 8 by DPP row_ror:8,
    // c ^ 16 and c ^ 32 by shuffles); row k: the whole wavefront
    double ya[2] = {0.0, 0.0}, y0[2];
#pragma unroll
    for (int q = 0; q < YU; ++q)
      if ((c >> 3) + 8 * q < ty) {
        ya[0] += ys[q].x;
        ya[1] += ys[q].y;
      }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      ya[x] += dpp_take<0x128, 0xf>(ya[x]);
      ya[x] = pair_sum16(ya[x]);
      ya[x] = pair_sum32(ya[x]);
    }
    y0[0] = c < ty ? y0l.x : 0.0;
    y0[1] = c < ty ? y0l.y : 0.0;
    wave_sum_n(y0);
    if (vfin) rk = make_double2(y0[0], y0[1]);
#pragma unroll
    for (int q = 0; q < RPW; ++q) {  // row q's sum from lane q, in every lane
      const double2 yq = make_double2(lane_at(ya[0], q), lane_at(ya[1], q));
      if (fin) pv[q] = yq;
    }
  }
  __syncthreads();
  double2 al = make_double2(0.0, 0.0);
  if (j > 0) {
    const double2 ps = cadd(cadd(psum[0], psum[1]), cadd(psum[2], psum[3]));
    al = cmul(make_double2(-0.5 * tpl.x, -0.5 * tpl.y), ps);
  }
  // w_{j-1} = y_{j-1} + alpha v_{j-1}, on row k and on this wavefront's rows
  if (vfin) cfma(rk, al, rkv);
  kv[c] = rk;
  if (fin) {
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const int i = lc.b * KC_ROWS + wv + 4 * q;
      cfma(pv[q], al, pf[q]);
      if (i < m) d.PW[(int64_t)(k + 1 + i) * HTD_NB + u] = pv[q];
    }
  }
  // x_r = G[r][k] - sum_u V[r][u] conj(w_k[u]) + W[r][u] conj(v_k[u]):
  // lane c of the row's wavefront contributes pv conj(rk), lane 0 also
  // G[r][k].  The sums over the 64 lanes go through LDS (the terms of the
  // wavefront's 8 rows, then 8 lanes per row with 8 terms each and an 8-lane
  // DPP sum): far fewer instructions than 16 full wavefront reductions.  Each
  // wavefront sums the rows it owns and reads back only what it wrote itself
  // (a wavefront's LDS operations execute in order), so no workgroup barrier
  // separates the terms, the sums and the dots.
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    double2 xq = a[q];  // a - pv conj(rk) = a + pv (-conj(rk))
    if (live) cfma(xq, pv[q], make_double2(-rk.x, rk.y));
    tx[wv + 4 * q][c] = xq;
  }
  wave_lds_order();
  const int i0 = lc.b * KC_ROWS;  // row r of the workgroup is row i0 + r of the column
  {
    const int wr = wv + 4 * (c >> 3), part = c & 7;
    double2 sxy = make_double2(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < 8; ++e) sxy = cadd(sxy, tx[wr][part * 8 + e]);
    sxy.x += dpp_take<0xb1, 0xf>(sxy.x);
    sxy.y += dpp_take<0xb1, 0xf>(sxy.y);
    sxy.x += dpp_take<0x4e, 0xf>(sxy.x);
    sxy.y += dpp_take<0x4e, 0xf>(sxy.y);
    sxy.x += dpp_take<0x141, 0xf>(sxy.x);
    sxy.y += dpp_take<0x141, 0xf>(sxy.y);
    if (part == 0) {
      xr[wr] = sxy;
      if (i0 + wr < m) d.xb[i0 + wr] = sxy;
    }
  }
  wave_lds_order();
  // the dots V^H x_1, W^H x_1: lane c sums its column over the wavefront's rows
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int i = i0 + wv + 4 * q;
    if (live && i > 0 && i < m) cfmac(acc, pv[q], xr[wv + 4 * q]);
  }
  dsum[wv][c] = acc;
  __syncthreads();
  double2* rec = d.kpart + (int64_t)lc.b * HTD_KP;
  if (wv == 0) {  // scaled norm of x_1 (rows i > 0) over the workgroup's rows; the dots
    const int i = i0 + c;
    const double2 xv = c < KC_ROWS && i > 0 && i < m ? xr[c] : make_double2(0.0, 0.0);
    const double amax = wave_max(fmax(fabs(xv.x), fabs(xv.y)));
    double ss = 0.0;
    if (amax > 0.0) {
      const double inv = 1.0 / amax;
      ss = (xv.x * inv) * (xv.x * inv) + (xv.y * inv) * (xv.y * inv);
    }
    ss = wave_sum(ss);
    if (c == 0) rec[0] = make_double2(amax, ss);
    rec[2 + c] = cadd(cadd(dsum[0][c], dsum[1][c]), cadd(dsum[2][c], dsum[3][c]));
  }
  if (lc.b == 0 && wv == 1) {  // d_k = G[k][k] - 2 sum_q Re(conj(v_k[q]) w_k[q])
    double t = 0.0;
    if (c < j) t = kv[HTD_NB + c].x * kv[c].x + kv[HTD_NB + c].y * kv[c].y;
    t = wave_sum(t);
    if (c == 0) d.d[k] = akk - 2.0 * t;
  }
}

// The product with the trailing block from its lower triangle (G is
// Hermitian).  Workgroups t < T (T + 1) / 2 take the 64 x 64 tiles (I, J),
// J <= I, of the trailing rows and columns: a tile adds tau G[I, J] v_J to
// y_I and, below the diagonal, tau G[I, J]^H v_I to y_J.  The next 2 T
// workgroups take the panel term -tau (V (W^H v) + W (V^H v)) of 64 rows,
// the V half or the W half (the V half also writes the reflector).  Each sum
// goes to a slot of its own: y_I's share of tile (I, J) to slot J, y_J's
// share to slot I, the panel halves to slots T and T + 1, so y_r is the sum
// of the T + 2 slots of row r, formed where y is used (trd_col, trd_her2k);
// every workgroup also leaves its share of y^H v.  All rebuild the reflector
// from the trd_col records (same operations, same values) while their loads
// are in flight; the products with x (v = (1, scale x[1:])) come first.
// Thread layout: wavefront w, lane 16 s + c holds rows 16 w + 4 q + s (q < 4)
// and columns 16 p + c of the tile (p < 4) or of the panel half (p < 2): a
// load instruction reads four row segments of 256 bytes, a row's sum is a
// 16-lane DPP reduction, a column's sum runs over 4 rows in registers, then
// through LDS.
template <int N>
__global__ __launch_bounds__(256) void trd_hemv_kernel(const HtdProbs<N> sz, int k) {
  __shared__ double2 hsum[8][HTD_NB];    // panel: record sums by group
  __shared__ double2 cpart[16][64 + 1];  // tile: column sums of (wavefront, s)
  __shared__ double2 wred[4];
  // problem blockIdx.y: its record is the only argument line read before the data
  const int p = blockIdx.y, t = blockIdx.x;
  const int n = sz.pr[p].n;
  const int T = htd_hemv_rows(n, k), NT = T * (T + 1) / 2;
  if (t >= NT + 2 * T) return;
  const HtdDesc d = htd_view(sz.pr[p]);
  if (skipped(d)) return;
  const bool panel = t >= NT;
  int I = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);  // t = I (I + 1) / 2 + J
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  int J = t - I * (I + 1) / 2;
  const int h = (t - NT) & 1;  // panel half: 0 V, 1 W
  if (panel) I = J = (t - NT) >> 1;
  const bool diag = I == J;
  const int m = n - k - 1, ld = d.ld, tid = threadIdx.x;
  const int j = k & (HTD_NB - 1);
  const int wave = tid >> 6, lane = tid & 63, s4 = lane >> 4, cl = lane & 15;
  const int o = htd_hemv_off(k);
  const int i0 = I * HV_T - o, c0 = J * HV_T - o;  // offsets in the trailing block (>= -o)
  auto rowof = [&](int q) { return i0 + 16 * wave + 4 * q + s4; };
  auto colof = [&](int pp) { return c0 + 16 * pp + cl; };
  // small loads first (memory operations complete in issue order), all
  // unconditional at clamped, valid indexes and masked at their use (a use
  // folded into a branch right after its load would wait for it before the
  // later loads are issued)
  const int nka = htd_col_blocks(n, k);
  static_assert(HTD_MAX / KC_ROWS <= 64, "the norm records are reduced by one wavefront");
  // every wavefront reads all the records and forms the reflector itself
  // (same operations, same values), so no workgroup barrier precedes it
  const double2 rq0 = d.kpart[(int64_t)(lane < nka ? lane : 0) * HTD_KP];
  const double2 rq = lane < nka ? rq0 : make_double2(0.0, 0.0);
  const double2 alpha = d.xb[0];
  double2 xr[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) xr[q] = d.xb[min(max(rowof(q), 0), m - 1)];
  double2 tau, scale;
  double beta;
  auto reflector = [&]() {
    const double rm = rq.x, rs = rq.y;
    const double smax = wave_max(rm);
    const double c = (rm > 0.0 && smax > 0.0) ? rs * (rm / smax) * (rm / smax) : 0.0;
    const double ssq = wave_sum(c);
    householder(alpha, smax, ssq, beta, tau, scale);
  };
  double2 dot = make_double2(0.0, 0.0);
  if (!panel) {
    double2 xc[4];
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) xc[pp] = d.xb[min(max(colof(pp), 0), m - 1)];
    const double2 xcol = d.xb[min(max(c0 + lane, 0), m - 1)];
    const double2* g0 = d.A + (int64_t)(k + 1) * ld + (k + 1);
    // (the lower triangle and the band of 64 above the diagonal are up to
    // date, which covers a diagonal tile; rows and columns -o..-1 are valid
    // memory before the block, read whole and masked)
    double2 a[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) a[q][pp] = g0[(int64_t)min(rowof(q), m - 1) * ld + min(colof(pp), m - 1)];
    reflector();
    const bool ident = tau.x == 0.0 && tau.y == 0.0;
    // row sums over this thread's columns (x_0 = alpha left out: v_0 = 1 is
    // added through G[r][0] itself); column sums over its rows (rows > 0
    // below the diagonal)
    double2 gr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        const int c = colof(pp);
        cfma(acc, a[q][pp], c > 0 && c < m ? xc[pp] : make_double2(0.0, 0.0));
      }
      gr[q] = acc;
    }
    if (!diag)
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) cfmac(acc, a[q][pp], rowof(q) < m ? xr[q] : make_double2(0.0, 0.0));
        cpart[wave * 4 + s4][16 * pp + cl] = acc;
      }
    // the rows' y: this wavefront's own rows, before the barrier the column
    // sums need
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2 acc = cmul(scale, gr[q]);
      acc.x += dpp_take<0xb1, 0xf>(acc.x);
      acc.y += dpp_take<0xb1, 0xf>(acc.y);
      acc.x += dpp_take<0x4e, 0xf>(acc.x);
      acc.y += dpp_take<0x4e, 0xf>(acc.y);
      acc.x += dpp_take<0x141, 0xf>(acc.x);
      acc.y += dpp_take<0x141, 0xf>(acc.y);
      acc.x += dpp_take<0x140, 0xf>(acc.x);
      acc.y += dpp_take<0x140, 0xf>(acc.y);
      double2 g_r0 = make_double2(0.0, 0.0);  // G[r][0]: column 0 of the block is tile column o
      if (J == 0) {
        g_r0.x = __shfl(a[q][0].x, (lane & 48) | o);
        g_r0.y = __shfl(a[q][0].y, (lane & 48) | o);
      }
      const int r = rowof(q);
      if (cl == 0 && r >= 0 && r < m) {
        if (J == 0) acc = cadd(acc, g_r0);  // G[r][0] v_0
        const double2 y = ident ? make_double2(0.0, 0.0) : cmul(tau, acc);
        const double2 vi = r == 0 ? make_double2(1.0, 0.0) : (ident ? make_double2(0.0, 0.0) : cmul(xr[q], scale));
        d.Y[(int64_t)J * ld + r] = y;
        cfmac(dot, y, vi);
      }
    }
    __syncthreads();
    if (!diag && tid < 64 && c0 + tid >= 0 && c0 + tid < m) {  // column c = c0 + tid
      const int c = c0 + tid;
      double2 cs = make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < 16; ++r) cs = cadd(cs, cpart[r][tid]);
      const double2 y = ident ? make_double2(0.0, 0.0) : cmul(tau, cmul(scale, cs));
      const double2 vc = c == 0 ? make_double2(1.0, 0.0) : (ident ? make_double2(0.0, 0.0) : cmul(xcol, scale));
      d.Y[(int64_t)I * ld + c] = y;
      cfmac(dot, y, vc);
    }
  } else {
    // half h: sum_l P[r][l] c_l over the panel columns l < j, P = V (h = 0) or
    // W (h = 1), c = W^H v or V^H v = conj(Q[k+1, l]) + scale (Q^H x[1:])_l
    // with Q the other one; (Q^H x[1:])_l from the records of trd_col
    const double2* P = h == 0 ? d.PV : d.PW;
    const double2* Q = h == 0 ? d.PW : d.PV;
    const int e = tid & 31, g = tid >> 5;
    constexpr int RQ = HTD_MAX / KC_ROWS / 8;  // records per group
    double2 rv[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      const int q = g + 8 * u;
      rv[u] = d.kpart[(int64_t)(q < nka ? q : 0) * HTD_KP + 2 + (h == 0 ? HTD_NB : 0) + e];
    }
    double2 q1[2], pe[4][2];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) q1[pp] = Q[(int64_t)(k + 1) * HTD_NB + 16 * pp + cl];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) pe[q][pp] = P[(int64_t)(k + 1 + min(rowof(q), m - 1)) * HTD_NB + 16 * pp + cl];
    // (columns l >= j are not written yet in this panel: masked by selects,
    // never by a zero factor)
    {
      double2 tt = make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < RQ; ++u)
        if (g + 8 * u < nka) tt = cadd(tt, rv[u]);
      hsum[g][e] = tt;
    }
    reflector();
    __syncthreads();
    // the two parts of each row's sum: with conj(Q[k+1, l]) and with (Q^H x[1:])_l
    double2 h1[4], h2[4];
    {
      double2 c1[2], c2[2];
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) {
        const int l = 16 * pp + cl;
        double2 sgl = make_double2(0.0, 0.0);
#pragma unroll
        for (int gg = 0; gg < 8; ++gg) sgl = cadd(sgl, hsum[gg][l]);
        c1[pp] = l < j ? make_double2(q1[pp].x, -q1[pp].y) : make_double2(0.0, 0.0);
        c2[pp] = l < j ? sgl : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int pp = 0; pp < 2; ++pp)
          if (16 * pp + cl >= j) pe[q][pp] = make_double2(0.0, 0.0);
        h1[q] = make_double2(0.0, 0.0);
        h2[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int pp = 0; pp < 2; ++pp) {
          cfma(h1[q], pe[q][pp], c1[pp]);
          cfma(h2[q], pe[q][pp], c2[pp]);
        }
      }
    }
    const bool ident = tau.x == 0.0 && tau.y == 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2 acc = h1[q];
      cfma(acc, scale, h2[q]);
      acc.x += dpp_take<0xb1, 0xf>(acc.x);
      acc.y += dpp_take<0xb1, 0xf>(acc.y);
      acc.x += dpp_take<0x4e, 0xf>(acc.x);
      acc.y += dpp_take<0x4e, 0xf>(acc.y);
      acc.x += dpp_take<0x141, 0xf>(acc.x);
      acc.y += dpp_take<0x141, 0xf>(acc.y);
      acc.x += dpp_take<0x140, 0xf>(acc.x);
      acc.y += dpp_take<0x140, 0xf>(acc.y);
      const int r = rowof(q);
      if (cl == 0 && r >= 0 && r < m) {
        const double2 y = ident ? make_double2(0.0, 0.0) : cmul(make_double2(-tau.x, -tau.y), acc);
        const double2 vi = r == 0 ? make_double2(1.0, 0.0) : (ident ? make_double2(0.0, 0.0) : cmul(xr[q], scale));
        d.Y[(int64_t)(T + h) * ld + r] = y;
        cfmac(dot, y, vi);
        if (h == 0) {  // the reflector: panel column j and row k of A
          d.PV[(int64_t)(k + 1 + r) * HTD_NB + j] = vi;
          d.A[(int64_t)k * ld + (k + 1 + r)] = vi;
        }
      }
    }
  }
  double sd[2] = {dot.x, dot.y};
  wave_sum_n(sd);
  if (lane == 0) wred[wave] = make_double2(sd[0], sd[1]);
  __syncthreads();
  if (tid == 0) {
    d.part[t] = cadd(cadd(wred[0], wred[1]), cadd(wred[2], wred[3]));
    if (t == 0) {
      d.tau[k] = tau;
      d.e[k] = beta;
    }
  }
}

// End of a panel: G[p1:, p1:] -= V W^H + W V^H (p1 = first column after the
// panel) as C = [V | W] [W | V]^H with K = 2 HTD_NB, on 64 x 64 tiles, in
// K slices of 16 staged through LDS.  The loads of slice s + 1 (and, during
// the last slice, the tile of G) are issued before the products of slice s;
// all are unconditional at clamped addresses and masked when staged.  The
// panel's last w, y + alpha v, is formed once per row in LDS.
__global__ __launch_bounds__(256) void trd_her2k_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int p0) {
  constexpr int KS = 16, NS = 2 * HTD_NB / KS, EPT = KS * 64 / 256;
  constexpr int PQ = (HV_PARTS + 255) / 256, YU = (HV_SLOTS + 1) / 2;
  __shared__ double2 As[KS][64 + 1];
  __shared__ double2 Bs[KS][64 + 1];
  __shared__ double2 wl[128];  // last w at rows r0.. (0..63) and c0.. (64..127)
  __shared__ double2 yh[2][128];
  __shared__ double sh[4];
  const Loc lc = locate(sz, blockIdx.x, [p0](int n) { return htd_her2k_blocks(n, p0); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], ld = d.ld, tid = threadIdx.x;
  const int nbp = min(HTD_NB, n - 1 - p0), p1 = p0 + nbp, mt = n - p1;
  // tile (ti, tj): b < T (T + 1) / 2 the lower triangle, b = ti (ti + 1) / 2 + tj;
  // then the tiles (u, u + 1) just above the diagonal, so that every entry
  // less than 64 above the diagonal is up to date too (whatever the tiles'
  // anchoring, such an entry lies in a diagonal or superdiagonal tile)
  const int T = (mt + 63) / 64, NL = T * (T + 1) / 2;
  int ti = (int)((sqrtf(8.0f * (float)lc.b + 1.0f) - 1.0f) * 0.5f);
  while (ti * (ti + 1) / 2 > lc.b) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= lc.b) ++ti;
  int tj = lc.b - ti * (ti + 1) / 2;
  if (lc.b >= NL) {
    ti = lc.b - NL;
    tj = ti + 1;
  }
  const int kl = p1 - 1;
  const int nb = htd_hemv_blocks(n, kl);
  const int r0 = p1 + ti * 64, c0 = p1 + tj * 64;
  const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  auto clampr = [n](int r) { return r < n ? r : n - 1; };
  // entry i of this thread in a slice: row e / KS of the tile, index e % KS
  double2 sa[EPT], sb[EPT];
  // slice s: As = [V | W] at rows r0.., Bs = [W | V] at rows c0..
  auto fetch = [&](int s) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + 256 * i, row = e / KS, l = s * KS + e % KS;
      const int q = l & (HTD_NB - 1);
      const int qq = q < nbp ? q : 0;
      const bool av = l < HTD_NB;
      sa[i] = gld((av ? d.PV : d.PW) + (int64_t)clampr(r0 + row) * HTD_NB + qq);
      sb[i] = gld((av ? d.PW : d.PV) + (int64_t)clampr(c0 + row) * HTD_NB + qq);
    }
  };
  fetch(0);
  double2 pq[PQ];
#pragma unroll
  for (int u = 0; u < PQ; ++u) pq[u] = gld(d.part + (tid + 256 * u < nb ? tid + 256 * u : 0));
  const double2 tl = gld(d.tau + kl);
  // the last column's y at this thread's row (rows r0.., then c0..) from the
  // HEMV's slots (its trailing block starts at row p1): YU slots per thread
  const int wr = clampr((tid & 127) < 64 ? r0 + (tid & 127) : c0 + (tid & 127) - 64);
  const int ty = htd_hemv_rows(n, kl) + 2;
  double2 ys[YU];
#pragma unroll
  for (int u = 0; u < YU; ++u) ys[u] = gld(d.Y + (int64_t)min((tid >> 7) + 2 * u, ty - 1) * ld + (wr - p1));
  const double2 vl = gld(d.PV + (int64_t)wr * HTD_NB + nbp - 1);
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int u = 0; u < PQ; ++u) {
    sx += tid + 256 * u < nb ? pq[u].x : 0.0;
    sy += tid + 256 * u < nb ? pq[u].y : 0.0;
  }
  {
    double2 ya = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < YU; ++u)
      if ((tid >> 7) + 2 * u < ty) ya = cadd(ya, ys[u]);
    yh[tid >> 7][tid & 127] = ya;
  }
  sx = block4_sum(sx, sh);
  sy = block4_sum(sy, sh);
  const double2 al = cmul(make_double2(-0.5 * tl.x, -0.5 * tl.y), make_double2(sx, sy));
  if (tid < 128) wl[tid] = cadd(cadd(yh[0][tid], yh[1][tid]), cmul(al, vl));
  __syncthreads();
  CAcc3<double> acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y].clear();
  double2 at[2][2][4];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + 256 * i, row = e / KS, kk = e % KS, l = s * KS + kk;
      const int q = l & (HTD_NB - 1);
      const bool av = l < HTD_NB, last = q == nbp - 1;
      double2 a = (!av && last) ? wl[row] : sa[i];
      double2 b = (av && last) ? wl[64 + row] : sb[i];
      a = q < nbp && r0 + row < n ? a : make_double2(0.0, 0.0);
      b = q < nbp && c0 + row < n ? b : make_double2(0.0, 0.0);
      As[kk][row] = a;
      Bs[kk][row] = make_double2(b.x, -b.y);
    }
    __syncthreads();
    if (s + 1 < NS) {
      fetch(s + 1);
    } else {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = r0 + wm * 32 + x * 16 + Mfma<double>::row(lane, q);
            const int c = c0 + wn * 32 + y * 16 + (lane & 15);
            at[x][y][q] = gld(d.A + (int64_t)clampr(r) * ld + clampr(c));
          }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
      const double2 a0 = As[kr][wm * 32 + cl], a1 = As[kr][wm * 32 + 16 + cl];
      const double2 b0 = Bs[kr][wn * 32 + cl], b1 = Bs[kr][wn * 32 + 16 + cl];
      acc[0][0].mac(a0.x, a0.y, b0.x, b0.y);
      acc[0][1].mac(a0.x, a0.y, b1.x, b1.y);
      acc[1][0].mac(a1.x, a1.y, b0.x, b0.y);
      acc[1][1].mac(a1.x, a1.y, b1.x, b1.y);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wm * 32 + x * 16 + Mfma<double>::row(lane, q);
        const int c = c0 + wn * 32 + y * 16 + (lane & 15);
        if (r < n && c < n)
          gst(d.A + (int64_t)r * ld + c,
              make_double2(at[x][y][q].x - acc_re(acc[x][y], q), at[x][y][q].y - acc_im(acc[x][y], q)));
      }
}

// The last columns of the reduction, from k0 = htd_tail_start(n) on (all of
// them when n <= HTD_TAIL): the trailing block, mt = n - k0 <= HTD_TAIL rows,
// is up to date there (the last panel's trd_her2k ran) and is held in the
// registers of one 512-thread workgroup as 4 x 8 tiles: thread t owns rows
// 4 (t / 16) .. +3 and columns 8 (t % 16) .. +7, so that a row is spread over
// the 16 lanes of one DPP row.  Column by column (unblocked): the column below
// the diagonal is the conjugated row, the reflector comes from its scaled
// norm, y = tau A v, w = y - (tau/2)(y^H v) v and A -= v w^H + w v^H; d, e,
// tau and the reflectors (row k of A) are written as the blocked kernels
// write them.  Per column two barriers: one after the row is staged, one
// after y; every wavefront forms the reflector and y^H v itself (same
// operations in the same order, so the same values) and reads v and w from
// the staged x and y.  x and y alternate between two buffers, so the next
// column's staging needs no barrier of its own.
__global__ __launch_bounds__(512) void trd_tail_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz) {
  constexpr int TR = 4, TC = 8, CG = HTD_TAIL / TC;  // tile rows, tile columns, column groups
  static_assert(CG == 16 && (HTD_TAIL / TR) * CG == 512, "tail tiling");
  static_assert(HTD_TAIL == 128, "two column entries per lane");
  __shared__ double2 xs[2][HTD_TAIL], ys[2][HTD_TAIL];
  const int p = blockIdx.x;
  if (p >= sz.np) return;
  const HtdDesc& d = ds[p];
  if (skipped(d)) return;
  const int n = sz.n[p], k0 = htd_tail_start(n), mt = n - k0, ld = d.ld, tid = threadIdx.x;
  const int lane = tid & 63;
  const int r0 = (tid / CG) * TR, c0 = (tid % CG) * TC;
  // (unconditional loads at clamped, valid addresses, masked afterwards: no
  // load waits for the one before it)
  // (the panel updates keep the lower triangle and only a band above the
  // diagonal up to date: upper entries as conj(G[c][r]))
  double2 a[TR][TC];
  const double2* blk = d.A + (int64_t)k0 * ld + k0;
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int rr = r0 + i < mt ? r0 + i : 0;
#pragma unroll
    for (int j = 0; j < TC; ++j) {
      const int cc = c0 + j < mt ? c0 + j : 0;
      a[i][j] = gld(blk + (cc > rr ? (int64_t)cc * ld + rr : (int64_t)rr * ld + cc));
    }
  }
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TC; ++j) {
      if (c0 + j > r0 + i) a[i][j].y = -a[i][j].y;
      if (!(r0 + i < mt && c0 + j < mt)) a[i][j] = make_double2(0.0, 0.0);
    }
  if (tid < 2 * HTD_TAIL) {  // entries past mt are read as zeros
    xs[tid >> 7][tid & (HTD_TAIL - 1)] = make_double2(0.0, 0.0);
    ys[tid >> 7][tid & (HTD_TAIL - 1)] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int kk = 0; kk + 1 < mt; ++kk) {
    const int k = k0 + kk, b = kk & 1;
    const double2* x = xs[b];
    // column kk below the diagonal = conj(row kk) (entries past mt are zero
    // and stay zero; entries up to kk are read by no one); the diagonal is final
#pragma unroll
    for (int i = 0; i < TR; ++i)
      if (r0 + i == kk)
#pragma unroll
        for (int j = 0; j < TC; ++j) xs[b][c0 + j] = make_double2(a[i][j].x, -a[i][j].y);
    __syncthreads();
    // the reflector from alpha = x[kk+1] and the scaled norm of x[kk+2:], in every wavefront
    double2 tau, scale;
    {
      const int ca = kk + 2 + lane, cb = ca + 64;
      const double2 xa = x[ca < HTD_TAIL ? ca : 0], xb = x[cb < HTD_TAIL ? cb : 0];
      const bool ia = ca < mt, ib = cb < mt;
      const double am = fmax(ia ? fmax(fabs(xa.x), fabs(xa.y)) : 0.0, ib ? fmax(fabs(xb.x), fabs(xb.y)) : 0.0);
      const double smax = wave_max(am);
      const double rs = smax > 0.0 ? 1.0 / smax : 0.0;
      const double ss = (ia ? (xa.x * rs) * (xa.x * rs) + (xa.y * rs) * (xa.y * rs) : 0.0) +
                        (ib ? (xb.x * rs) * (xb.x * rs) + (xb.y * rs) * (xb.y * rs) : 0.0);
      const double ssq = wave_sum(ss);
      double beta;
      householder(x[kk + 1], smax, ssq, beta, tau, scale);
      if (tid == 0) {
        gst(d.d + k, x[kk].x);
        gst(d.tau + k, tau);
        gst(d.e + k, beta);
      }
    }
    const bool ident = tau.x == 0.0 && tau.y == 0.0;
    // v = (1 at kk+1, scale x past it), zero elsewhere
    auto vat = [&](int c) {
      return c == kk + 1 ? make_double2(1.0, 0.0)
                         : (c > kk + 1 && !ident ? cmul(x[c], scale) : make_double2(0.0, 0.0));
    };
    if (tid > kk && tid < mt) gst(d.A + (int64_t)k * ld + k0 + tid, vat(tid));
    if (ident) continue;  // H = I: the trailing block is unchanged
    // y = tau A v on the rows below kk (each row summed over its 16 lanes)
    double2 vc[TC];
#pragma unroll
    for (int j = 0; j < TC; ++j) vc[j] = vat(c0 + j);
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < TC; ++j) cfma(acc, a[i][j], vc[j]);
      acc.x += dpp_take<0xb1, 0xf>(acc.x);
      acc.y += dpp_take<0xb1, 0xf>(acc.y);
      acc.x += dpp_take<0x4e, 0xf>(acc.x);
      acc.y += dpp_take<0x4e, 0xf>(acc.y);
      acc.x += dpp_take<0x141, 0xf>(acc.x);
      acc.y += dpp_take<0x141, 0xf>(acc.y);
      acc.x += dpp_take<0x140, 0xf>(acc.x);
      acc.y += dpp_take<0x140, 0xf>(acc.y);
      const int r = r0 + i;
      if (c0 == 0 && r < mt) ys[b][r] = r > kk ? cmul(tau, acc) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const double2* y = ys[b];
    // alpha = -(tau/2) y^H v in every wavefront, then w = y + alpha v
    double2 al;
    {
      const int ca = kk + 1 + lane, cb = ca + 64;
      const double2 ya = y[ca < HTD_TAIL ? ca : 0], yb = y[cb < HTD_TAIL ? cb : 0];
      const double2 ta = ca < mt ? cmulc(ya, vat(ca < HTD_TAIL ? ca : 0)) : make_double2(0.0, 0.0);
      const double2 tb = cb < mt ? cmulc(yb, vat(cb < HTD_TAIL ? cb : 0)) : make_double2(0.0, 0.0);
      double su[2] = {ta.x + tb.x, ta.y + tb.y};
      wave_sum_n(su);
      al = cmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), make_double2(su[0], su[1]));
    }
    if (r0 + TR - 1 > kk) {  // A -= v w^H + w v^H (v, w vanish at indexes <= kk and >= mt)
      double2 vr[TR], wr[TR];
#pragma unroll
      for (int i = 0; i < TR; ++i) {
        vr[i] = vat(r0 + i);
        wr[i] = cadd(y[r0 + i], cmul(al, vr[i]));
      }
#pragma unroll
      for (int j = 0; j < TC; ++j) {  // one column at a time keeps the live registers few
        const double2 vj = vc[j];
        const double2 wj = cadd(y[c0 + j], cmul(al, vj));
        // a -= v_r conj(w_j) + w_r conj(v_j): the same conjugate products with
        // the minus folded in, conj(w_j) (-v_r) + conj(v_j) (-w_r)
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          cfmac(a[i][j], wj, make_double2(-vr[i].x, -vr[i].y));
          cfmac(a[i][j], vj, make_double2(-wr[i].x, -wr[i].y));
        }
      }
    }
  }
  // the last diagonal entry, also back into A for trd_finish
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TC; ++j)
      if (r0 + i == mt - 1 && c0 + j == mt - 1) {
        gst(d.d + (n - 1), a[i][j].x);
        gst(d.A + (int64_t)(n - 1) * ld + (n - 1), a[i][j]);
      }
  if (tid == 0) gst(d.e + (n - 1), 0.0);
}

__global__ void trd_finish_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= sz.np) return;
  const HtdDesc& d = ds[p];
  if (skipped(d)) return;
  const int n = sz.n[p];
  if (n < 1) return;
  d.d[n - 1] = d.A[(int64_t)(n - 1) * d.ld + (n - 1)].x;
  d.e[n - 1] = 0.0;
}

// ======================================================= divide and conquer
// The eigenvector matrices of the nodes are stored by columns: Q[col * ld +
// row], so that deflation rotations and column copies read whole columns.
//
// Level 0: T torn at every off-diagonal entry (d_i -= |e_{i-1}| + |e_i|),
// 1 x 1 blocks with eigenvector 1.  Both eigenvector buffers start at zero:
// a merge multiplies whole columns of its node, so the quadrants outside the
// children's blocks must hold exact zeros (later levels only ever write
// inside their own node blocks).
__global__ __launch_bounds__(256) void dc_init_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz) {
  const Loc lc = locate(sz, blockIdx.x, [](int n) { return n; });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], i = lc.b, ld = d.ld;
  double* q0 = d.Q[0] + (int64_t)i * ld;
  double* q1 = d.Q[1] + (int64_t)i * ld;
  for (int c = threadIdx.x; c < n; c += 256) {
    q0[c] = c == i ? 1.0 : 0.0;
    q1[c] = 0.0;
  }
  if (threadIdx.x == 0) {
    double v = d.d[i];
    if (i > 0) v -= fabs(d.e[i - 1]);
    if (i < n - 1) v -= fabs(d.e[i]);
    d.D[0][i] = v;
  }
}

__device__ __forceinline__ double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r = fmax(r, red[w]);
  return r;
}

// Exclusive prefix, over a 1024-thread workgroup, of two ordered flags per
// thread (entries 2 tid and 2 tid + 1); *total receives the count of all set
// flags.  Ballots and bit counts within each wavefront, then the 16
// wavefront totals through LDS.
__device__ __forceinline__ int block_prefix2(bool f0, bool f1, int* wsum, int& total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const unsigned long long b0 = __ballot(f0), b1 = __ballot(f1);
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int pre = __popcll(b0 & lt) + __popcll(b1 & lt);
  if (lane == 0) wsum[w] = __popcll(b0) + __popcll(b1);
  __syncthreads();
  int base = 0, tot = 0;
  for (int q = 0; q < 16; ++q) {
    const int v = wsum[q];
    if (q < w) base += v;
    tot += v;
  }
  total = tot;
  __syncthreads();  // wsum is reused by the next call
  return base + pre;
}

// Merge of node [lo, hi) at level L (children [lo, mid), [mid, hi)):
// T_node = diag(Q1, Q2) (diag(D1, D2) + rho z z^T) diag(Q1, Q2)^T with
// z = (last row of Q1, sign(e) first row of Q2) / sqrt(2), rho = 2 |e_{mid-1}|.
// Sorts the poles, deflates small z components and (after a rotation)
// close poles, and lists the non-deflated poles for the secular equation.
__global__ __launch_bounds__(1024) void dc_prep_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int L) {
  __shared__ double Ds[HTD_MAX];
  __shared__ double zs[HTD_MAX];
  __shared__ int col[HTD_MAX];
  __shared__ int ndl[HTD_MAX];
  __shared__ int fl[HTD_MAX];
  __shared__ unsigned char rf[HTD_MAX];
  __shared__ int wsum[16];
  __shared__ double red[16];
  __shared__ int sh_ndef;
  const Loc lc = locate(sz, blockIdx.x, [L](int n) { return htd_nodes(n, L); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], s = 1 << L, tid = threadIdx.x;
  const int lo = lc.b * s, mid = lo + s / 2, hi = min(lo + s, n);
  int* cnt = d.cnt + 4 * lo;
  if (mid >= hi) {
    if (tid == 0) cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
    return;
  }
  const int K = hi - lo, nl = mid - lo, nr = hi - mid, ld = d.ld;
  const double* Din = d.D[(L - 1) & 1];
  const double* Qin = d.Q[(L - 1) & 1];
  const double eb = d.e[mid - 1];
  const double rho = 2.0 * fabs(eb), sg = eb >= 0.0 ? 1.0 : -1.0;
  const double r2 = 0.70710678118654752440;
  // Every slot starts valid: with NaN values (a corrupted input) the ranks
  // below can collide and leave slots unwritten, and their columns are used
  // as indexes by the later kernels of the merge.
  for (int t = tid; t < K; t += 1024) {
    Ds[t] = 0.0;
    zs[t] = 0.0;
    col[t] = lo + t;
  }
  __syncthreads();
  for (int t = tid; t < K; t += 1024) {
    double val, z;
    int rank;
    if (t < nl) {
      val = Din[lo + t];
      int a = 0, b = nr;  // right values below val
      while (a < b) {
        const int mm = (a + b) >> 1;
        if (Din[mid + mm] < val)
          a = mm + 1;
        else
          b = mm;
      }
      rank = t + a;
      z = Qin[(int64_t)(lo + t) * ld + (mid - 1)];
    } else {
      const int q = t - nl;
      val = Din[mid + q];
      int a = 0, b = nl;  // left values at or below val
      while (a < b) {
        const int mm = (a + b) >> 1;
        if (Din[lo + mm] <= val)
          a = mm + 1;
        else
          b = mm;
      }
      rank = q + a;
      z = sg * Qin[(int64_t)(mid + q) * ld + mid];
    }
    Ds[rank] = val;
    zs[rank] = z * r2;
    col[rank] = lo + t;
  }
  __syncthreads();
  double md = 0.0, mz = 0.0;
  for (int t = tid; t < K; t += 1024) {
    md = fmax(md, fabs(Ds[t]));
    mz = fmax(mz, fabs(zs[t]));
  }
  md = block_max(md, red);
  mz = block_max(mz, red);
  const double tol = 8.0 * EPS53 * fmax(md, mz);
  // The deflation scan (ascending poles; a pole with small rho |z| deflates;
  // two consecutive remaining poles pj < t too close for the secular equation
  // are rotated so that z_pj = 0, pj deflates and t carries on with the
  // rotated value and z) in parallel wherever it can be.  A pair's test only
  // depends on values a rotation changed when the pair before it rotated, so
  // the pairs whose test on the unmodified values fails and whose
  // predecessor pair did not rotate are settled at once.  One thread walks
  // from each flagged pair (in order) through the rotations that follow it,
  // exactly as the sequential scan would; everything else is written in
  // parallel.  With no rotation at all the lists are final here: the
  // remaining poles in order and the deflated values ascending with ties by
  // column (no sort).
  const bool alldef = rho * mz <= tol;
  const int t0 = 2 * tid, t1 = t0 + 1;
  const bool nd0 = t0 < K && !alldef && rho * fabs(zs[t0]) > tol;
  const bool nd1 = t1 < K && !alldef && rho * fabs(zs[t1]) > tol;
  int knd = 0;
  const int p = block_prefix2(nd0, nd1, wsum, knd);
  if (nd0) ndl[p] = t0;
  if (nd1) ndl[p + (nd0 ? 1 : 0)] = t1;
  const bool df0 = t0 < K && !nd0, df1 = t1 < K && !nd1;
  int kdef = 0;
  const int q = block_prefix2(df0, df1, wsum, kdef);
  if (df0) {
    d.dval[lo + q] = Ds[t0];
    d.dcol[lo + q] = col[t0];
  }
  if (df1) {
    d.dval[lo + q + (df0 ? 1 : 0)] = Ds[t1];
    d.dcol[lo + q + (df0 ? 1 : 0)] = col[t1];
  }
  __syncthreads();
  // pair i = (ndl[i-1], ndl[i]), 1 <= i < knd; this thread's pairs 2 tid, 2 tid + 1
  auto close = [&](int pj, int t, double& cs, double& sn, double& tau) {
    sn = zs[pj];
    cs = zs[t];
    tau = hypot(cs, sn);
    const double tt = Ds[t] - Ds[pj];
    cs /= tau;
    sn = -sn / tau;
    return fabs(tt * cs * sn) <= tol;
  };
  bool f0 = false, f1 = false;
  {
    double cs, sn, tau;
    if (t0 >= 1 && t0 < knd) f0 = close(ndl[t0 - 1], ndl[t0], cs, sn, tau);
    if (t1 < knd) f1 = close(ndl[t1 - 1], ndl[t1], cs, sn, tau);
  }
  int nf = 0;
  const int pf = block_prefix2(f0, f1, wsum, nf);
  // flagged pairs in order to fl[]; rf[i] marks a rotation at pair i
  if (f0) fl[pf] = t0;
  if (f1) fl[pf + (f0 ? 1 : 0)] = t1;
  for (int i = tid; i < knd; i += 1024) rf[i] = 0;
  __syncthreads();
  if (tid == 0 && nf > 0) {
    int pos = 1, nrot = 0;  // pairs below pos are settled
    for (int u = 0; u < nf; ++u) {
      const int i = fl[u];
      if (i < pos) continue;
      int pj = ndl[i - 1], r = i;
      for (; r < knd; ++r) {
        const int t = ndl[r];
        double cs, sn, tau;
        if (!close(pj, t, cs, sn, tau)) break;
        zs[t] = tau;
        zs[pj] = 0.0;
        d.rot_a[lo + nrot] = col[pj];
        d.rot_b[lo + nrot] = col[t];
        d.rot_c[lo + nrot] = cs;
        d.rot_s[lo + nrot] = sn;
        const double v1 = Ds[pj] * cs * cs + Ds[t] * sn * sn;
        Ds[t] = Ds[pj] * sn * sn + Ds[t] * cs * cs;
        Ds[pj] = v1;
        d.dval[lo + kdef + nrot] = v1;
        d.dcol[lo + kdef + nrot] = col[pj];
        ++nrot;
        rf[r] = 1;
        pj = t;
      }
      pos = r + 1;
    }
    sh_ndef = nrot;
  }
  if (nf == 0 && tid == 0) sh_ndef = 0;
  __syncthreads();
  const int nrot = sh_ndef;
  // remaining pole j of the chain survives unless pair j + 1 rotated it away
  const bool s0 = t0 < knd && (t0 == knd - 1 || !rf[t0 + 1]);
  const bool s1 = t1 < knd && (t1 == knd - 1 || !rf[t1 + 1]);
  int K2 = 0;
  const int ps = block_prefix2(s0, s1, wsum, K2);
  if (s0) {
    d.dl[lo + ps] = Ds[ndl[t0]];
    d.w[lo + ps] = zs[ndl[t0]];
    d.ndcol[lo + ps] = col[ndl[t0]];
  }
  if (s1) {
    const int o = ps + (s0 ? 1 : 0);
    d.dl[lo + o] = Ds[ndl[t1]];
    d.w[lo + o] = zs[ndl[t1]];
    d.ndcol[lo + o] = col[ndl[t1]];
  }
  const int ndef = kdef + nrot;
  if (tid == 0) {
    cnt[0] = K2;
    cnt[1] = ndef;
    cnt[2] = nrot;
    cnt[3] = 1;
    d.rho[lo] = rho;
  }
  if (nrot == 0) return;
  __syncthreads();
  // deflated eigenvalues ascending (bitonic sort, ties by column): the
  // values rotated away were appended after the others
  if (ndef > 1) {
    int p2 = 1;
    while (p2 < ndef) p2 <<= 1;
    for (int t = tid; t < p2; t += 1024) {
      Ds[t] = t < ndef ? d.dval[lo + t] : INFINITY;
      col[t] = t < ndef ? d.dcol[lo + t] : INT_MAX;
    }
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = tid; i < p2; i += 1024) {
          const int j = i ^ stride;
          if (j > i) {
            const bool up = (i & size) == 0;
            const bool i_first = Ds[i] < Ds[j] || (Ds[i] == Ds[j] && col[i] < col[j]);
            if (up ? !i_first : i_first) {
              const double tv = Ds[i];
              Ds[i] = Ds[j];
              Ds[j] = tv;
              const int tc = col[i];
              col[i] = col[j];
              col[j] = tc;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int t = tid; t < ndef; t += 1024) {
      d.dval[lo + t] = Ds[t];
      d.dcol[lo + t] = col[t];
    }
  }
}

// dl_j - lambda_k, formed as (dl_j - dl_origin) - tau so that it keeps full
// relative accuracy next to either pole
__device__ __forceinline__ double delta_jk(const double* dl, int j, int o, double tau) {
  return (dl[j] - dl[o]) - tau;
}

// Root k of the secular equation 1 + rho sum_j w_j^2 / (dl_j - lambda) = 0 in
// (dl_k, dl_{k+1}) (last root: (dl_k, dl_k + rho |w|^2]), computed by one
// wavefront (the sums over j are split across the lanes; every lane ends with
// the same sums, so control flow is uniform).  lambda is kept as
// dl_origin + tau with the origin at the nearer pole.  Iteration: each step
// replaces the two poles' terms by the rational model of Li's middle way
// (value and slope of both sums matched at the current point) and takes the
// root of the resulting quadratic; a bracket on the sign of f guards every
// step and falls back to bisection (geometric when the bracket spans a
// decade or more).
__device__ void secular_root(const double* dl, const double* w, int K2, double rho, int k, int lane, int& origin,
                             double& tau_out) {
  if (K2 == 1) {
    origin = 0;
    tau_out = rho * w[0] * w[0];
    return;
  }
  const bool last = k == K2 - 1;
  int o;
  double tlo, thi;
  if (!last) {
    const double mid = 0.5 * (dl[k + 1] - dl[k]);
    double f = 0.0;
    for (int j = lane; j < K2; j += 64) f += w[j] * w[j] / ((dl[j] - dl[k]) - mid);
    f = 1.0 + rho * wave_sum(f);
    if (f >= 0.0) {
      o = k;
      tlo = 0.0;
      thi = mid;
    } else {
      o = k + 1;
      tlo = -mid;
      thi = 0.0;
    }
  } else {
    o = k;
    double s = 0.0;
    for (int j = lane; j < K2; j += 64) s += w[j] * w[j];
    tlo = 0.0;
    thi = rho * wave_sum(s);
  }
  double tau = 0.5 * (tlo + thi);
  for (int it = 0; it < 200; ++it) {
    double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
    for (int j = lane; j < K2; j += 64) {
      const double t = w[j] / delta_jk(dl, j, o, tau);
      if (j <= k) {
        psi += w[j] * t;
        dpsi += t * t;
      } else {
        phi += w[j] * t;
        dphi += t * t;
      }
    }
    psi = rho * wave_sum(psi);
    phi = rho * wave_sum(phi);
    dpsi = rho * wave_sum(dpsi);
    dphi = rho * wave_sum(dphi);
    const double f = 1.0 + psi + phi;
    if (f == 0.0) break;
    if (f < 0.0)
      tlo = tau;
    else
      thi = tau;
    const double err = 8.0 * EPS53 * K2 * (1.0 + fabs(psi) + fabs(phi));
    if (fabs(f) <= err || thi - tlo <= 4.0 * EPS53 * fmax(fabs(tlo), fabs(thi))) break;
    const double di = delta_jk(dl, k, o, tau);
    double eta;
    if (!last) {
      const double dj = delta_jk(dl, k + 1, o, tau);
      const double c = f - di * dpsi - dj * dphi;
      const double a = (di + dj) * f - di * dj * (dpsi + dphi);
      const double b = di * dj * f;
      const double disc = sqrt(fabs(a * a - 4.0 * b * c));
      if (c == 0.0)
        eta = a != 0.0 ? b / a : NAN;
      else if (a <= 0.0)
        eta = (a - disc) / (2.0 * c);
      else
        eta = 2.0 * b / (a + disc);
    } else {
      const double c = f - di * dpsi;
      eta = c != 0.0 ? di + di * di * dpsi / c : NAN;
    }
    double nt = tau + eta;
    if (!(nt > tlo && nt < thi)) {
      if (tlo > 0.0 && thi > 4.0 * tlo)
        nt = sqrt(tlo * thi);
      else if (thi < 0.0 && tlo < 4.0 * thi)
        nt = -sqrt(tlo * thi);
      else
        nt = 0.5 * (tlo + thi);
      if (!(nt > tlo && nt < thi)) break;
    }
    tau = nt;
  }
  origin = o;
  tau_out = tau;
}

// Deflation rotations of a merge level on the children's eigenvector
// columns, one thread per row.
__global__ __launch_bounds__(256) void dc_rot_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int L) {
  const Loc lc = locate(sz, blockIdx.x, [](int n) { return htd_rows(n); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], i = lc.b * 256 + threadIdx.x;
  if (i >= n) return;
  const int lo = (i >> L) << L, ld = d.ld;
  const int* cnt = d.cnt + 4 * lo;
  if (!cnt[3]) return;
  double* q = d.Q[(L - 1) & 1] + i;
  const int nrot = cnt[2];
  for (int r = 0; r < nrot; ++r) {
    const int a = d.rot_a[lo + r], b = d.rot_b[lo + r];
    const double c = d.rot_c[lo + r], s = d.rot_s[lo + r];
    const double x = q[(int64_t)a * ld], y = q[(int64_t)b * ld];
    q[(int64_t)a * ld] = c * x + s * y;
    q[(int64_t)b * ld] = c * y - s * x;
  }
}

// One wavefront per root / pole of a merge level: stage 1 solves the secular
// equation of root k, stage 2 recomputes z_j from all roots (Loewner:
// zhat_j^2 = prod_k (lambda_k - dl_j) / (rho prod_{k != j} (dl_k - dl_j))),
// stage 3 the norm of eigenvector k, u_j = zhat_j / (dl_j - lambda_k).
__global__ __launch_bounds__(256) void dc_wave_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int L, int stage) {
  const Loc lc = locate(sz, blockIdx.x, [](int n) { return htd_waves(n); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], lane = threadIdx.x & 63;
  const int i = lc.b * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int lo = (i >> L) << L;
  const int* cnt = d.cnt + 4 * lo;
  if (!cnt[3]) return;
  const int K2 = cnt[0], k = i - lo;
  if (k >= K2) return;
  const double* dl = d.dl + lo;
  const double* w = d.w + lo;
  const int* org = d.origin + lo;
  const double* st = d.stau + lo;
  if (stage == 1) {
    int o;
    double tau;
    secular_root(dl, w, K2, d.rho[lo], k, lane, o, tau);
    if (lane == 0) {
      d.origin[lo + k] = o;
      d.stau[lo + k] = tau;
    }
  } else if (stage == 2) {
    const int j = k;
    double v = 1.0;
    for (int q = lane; q < K2; q += 64)
      if (q != j) v *= (-delta_jk(dl, j, org[q], st[q])) / (dl[q] - dl[j]);
    for (int off = 32; off > 0; off >>= 1) v *= __shfl_xor(v, off);
    v *= -delta_jk(dl, j, org[j], st[j]) / d.rho[lo];
    if (lane == 0) d.zhat[lo + j] = copysign(sqrt(fmax(v, 0.0)), w[j]);
  } else {
    const double* zh = d.zhat + lo;
    double s2 = 0.0;
    for (int j = lane; j < K2; j += 64) {
      const double u = zh[j] / delta_jk(dl, j, org[k], st[k]);
      s2 += u * u;
    }
    s2 = wave_sum(s2);
    if (lane == 0) d.unrm[lo + k] = 1.0 / sqrt(s2);
  }
}

// Places the merged node's values (ascending: roots and deflated values
// interleaved) and copies the deflated columns to their places.  One
// workgroup per 64 columns of a node (the copy of a node of 2048 deflated
// columns would take one workgroup hundreds of microseconds); the first
// workgroup of a node also places the roots (dc_gemm writes their columns).
__global__ __launch_bounds__(256) void dc_place_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int L) {
  __shared__ double lamv[HTD_MAX];
  __shared__ double dv[HTD_MAX];
  __shared__ int pdef[64], srcc[64];
  const Loc lc = locate(sz, blockIdx.x, [L](int n) { return htd_place_blocks(n, L); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], s = 1 << L, tid = threadIdx.x, ld = d.ld;
  const int per = (s + 63) / 64, node = lc.b / per, c0 = (lc.b % per) * 64;
  const int lo = node * s, hi = min(lo + s, n), K = hi - lo;
  if (c0 >= K) return;
  const double* Din = d.D[(L - 1) & 1];
  const double* Qin = d.Q[(L - 1) & 1];
  double* Dout = d.D[L & 1];
  double* Qout = d.Q[L & 1];
  const int* cnt = d.cnt + 4 * lo;
  const int cw = min(64, K - c0);
  const int wave = tid >> 6, lane = tid & 63;
  // one column of K rows by one wavefront, 4 loads per lane in flight
  // (clamped, the stores guarded)
  auto copy_col = [&](const double* src, double* dst) {
    for (int r0 = 0; r0 < K; r0 += 256) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = src[min(r0 + 64 * u + lane, K - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (r0 + 64 * u + lane < K) dst[r0 + 64 * u + lane] = v[u];
    }
  };
  if (!cnt[3]) {  // nothing merged: the node's block as it was
    for (int t = wave; t < cw; t += 4)
      copy_col(Qin + (int64_t)(lo + c0 + t) * ld + lo, Qout + (int64_t)(lo + c0 + t) * ld + lo);
    if (tid < cw) Dout[lo + c0 + tid] = Din[lo + c0 + tid];
    return;
  }
  const int K2 = cnt[0], ndef = cnt[1];
  const bool roots = c0 == 0;  // this workgroup also places the roots
  if (!roots && c0 >= ndef) return;
  for (int k = tid; k < K2; k += 256) lamv[k] = d.dl[lo + d.origin[lo + k]] + d.stau[lo + k];
  if (roots)
    for (int q = tid; q < ndef; q += 256) dv[q] = d.dval[lo + q];
  __syncthreads();
  if (roots)
    for (int k = tid; k < K2; k += 256) {
      const double x = lamv[k];
      int a = 0, b = ndef;  // deflated values below x
      while (a < b) {
        const int mm = (a + b) >> 1;
        if (dv[mm] < x)
          a = mm + 1;
        else
          b = mm;
      }
      d.pos_nd[lo + k] = k + a;
      Dout[lo + k + a] = x;
    }
  const int qn = max(0, min(64, ndef - c0));  // deflated columns c0 .. c0 + qn - 1
  if (tid < qn) {
    const int q = c0 + tid;
    const double x = d.dval[lo + q];
    int a = 0, b = K2;  // roots at or below x
    while (a < b) {
      const int mm = (a + b) >> 1;
      if (lamv[mm] <= x)
        a = mm + 1;
      else
        b = mm;
    }
    pdef[tid] = q + a;
    srcc[tid] = d.dcol[lo + q];
    Dout[lo + q + a] = x;
  }
  __syncthreads();
  for (int t = wave; t < qn; t += 4)
    copy_col(Qin + (int64_t)srcc[t] * ld + lo, Qout + (int64_t)(lo + pdef[t]) * ld + lo);
}

// Eigenvector of root k = Q_in[:, ndcol] u_k, written to column lo + pos_k:
// with columns stored contiguously this is C = U^T B, C[k][r] =
// sum_j u_k[j] Q_in[ndcol_j][r]; u_k[j] = zhat_j / (dl_j - lambda_k) / |.|
// is formed while staging.  Matrix cores (f64 16x16x4), each of the four
// wavefronts owns a 32 x 32 quadrant of the 64 x 64 tile (roots x rows).
__global__ __launch_bounds__(256) void dc_gemm_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int L) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const Loc lc = locate(sz, blockIdx.x, [L](int n) { return htd_gemm_tiles(n, L); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], s = 1 << L, ld = d.ld;
  const int T = (s + 63) / 64, per = T * T;
  const int node = lc.b / per, t = lc.b % per, ti = t / T, tj = t % T;
  const int lo = node * s, hi = min(lo + s, n), K = hi - lo;
  const auto cnt = gp(d.cnt + 4 * lo);
  if (!cnt[3]) return;
  const int K2 = cnt[0];
  const int k0 = ti * 64, r0 = tj * 64;  // roots k0.., rows r0..
  if (k0 >= K2 || r0 >= K) return;
  const auto Qin = gp((const double*)d.Q[(L - 1) & 1]);
  const auto Qout = gp(d.Q[L & 1]);
  const auto pos = gp((const int*)d.pos_nd + lo);
  const auto ndc = gp((const int*)d.ndcol + lo);
  const auto dl = gp((const double*)d.dl + lo);
  const auto zh = gp((const double*)d.zhat + lo);
  const auto org = gp((const int*)d.origin + lo);
  const auto st = gp((const double*)d.stau + lo);
  const auto un = gp((const double*)d.unrm + lo);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<double>::zero();
  // this thread stages column c = tid % 64 (root k0 + c, row r0 + c) of rows
  // kk = tid / 64 + 4 i (pole j0 + kk): the root's values are loaded once;
  // the next slice's pole values and Q_in entries are loaded (unconditionally,
  // at clamped indexes) before the products of the current one
  const int c = tid & 63, kk0 = tid >> 6;
  const int kc = min(k0 + c, K2 - 1), rc = min(r0 + c, K - 1);
  const int ok = org[kc];
  const double dlo = dl[ok], stk = st[kc], unk = un[kc];
  double pz[4], pd[4], pq[4];
  auto fetch = [&](int j0) {
    int nj[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = min(j0 + kk0 + 4 * i, K2 - 1);
      pz[i] = zh[j];
      pd[i] = dl[j];
      nj[i] = ndc[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) pq[i] = Qin[(int64_t)nj[i] * ld + lo + rc];
  };
  fetch(0);
  for (int j0 = 0; j0 < K2; j0 += 16) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = kk0 + 4 * i, j = j0 + kk;
      // u_k[j] = zhat_j / (dl_j - lambda_k) / |.|, lambda_k = dl[origin_k] + stau_k
      As[kk][c] = (j < K2 && k0 + c < K2) ? pz[i] / ((pd[i] - dlo) - stk) * unk : 0.0;
      Bs[kk][c] = (j < K2 && r0 + c < K) ? pq[i] : 0.0;
    }
    __syncthreads();
    if (j0 + 16 < K2) fetch(j0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
      const double a0 = As[kr][wm * 32 + cl], a1 = As[kr][wm * 32 + 16 + cl];
      const double b0 = Bs[kr][wn * 32 + cl], b1 = Bs[kr][wn * 32 + 16 + cl];
      acc[0][0] = Mfma<double>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<double>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<double>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<double>::mac(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + wm * 32 + x * 16 + Mfma<double>::row(lane, q);
        const int r = r0 + wn * 32 + y * 16 + (lane & 15);
        if (k < K2 && r < K) Qout[(int64_t)(lo + pos[k]) * ld + lo + r] = acc[x][y][q];
      }
}

// ======================================================= back-transformation
// V = Z (real eigenvectors of T from the last level's column-stored buffer,
// transposed through LDS in 64 x 64 tiles) and lam, both in descending
// eigenvalue order: the eigenvectors a split keeps are the first columns
// (equal eigenvalues are taken lowest index first), so only min(n, rcap)
// columns need the back-transformation.
__global__ __launch_bounds__(256) void bt_init_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int Lmax) {
  __shared__ double tile[64][64 + 1];
  const Loc lc = locate(sz, blockIdx.x, [](int n) { return htd_tiles64(n); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], ld = d.ld, tid = threadIdx.x;
  const int T = (n + 63) / 64, tr = lc.b / T, tc = lc.b % T;  // rows j, columns c of V
  const double* Z = d.Q[Lmax & 1];
  for (int e = tid; e < 64 * 64; e += 256) {
    const int cc = e >> 6, jj = e & 63;
    const int c = tc * 64 + cc, j = tr * 64 + jj;
    tile[cc][jj] = (c < n && j < n) ? Z[(int64_t)(n - 1 - c) * ld + j] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int jj = e >> 6, cc = e & 63;
    const int c = tc * 64 + cc, j = tr * 64 + jj;
    if (c < n && j < n) d.V[(int64_t)j * ld + c] = make_double2(tile[cc][jj], 0.0);
  }
  if (tr == 0)
    for (int cc = tid; cc < 64; cc += 256) {
      const int c = tc * 64 + cc;
      if (c < n) d.lam[c] = d.D[Lmax & 1][n - 1 - c];
    }
}

// reflector i of block b (k = BT_NB b + i) at row j: 0 for j <= k, else row k of A
__device__ __forceinline__ double2 refl(const HtdDesc& d, int k, int j) {
  return j > k ? gld(d.A + (int64_t)k * d.ld + j) : make_double2(0.0, 0.0);
}

// T of each block: H_k0 ... H_k0+nb-1 = I - V_b T V_b^H (upper triangular T,
// T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] S[0:i, i], S = V_b^H V_b).  S is
// accumulated over 16-row chunks of the reflectors staged in LDS, each thread
// owning BT_NB^2 / 256 entries; T then replaces S column by column.
__global__ __launch_bounds__(256) void bt_larft_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz) {
  constexpr int PPT = BT_NB * BT_NB / 256;  // entries of S per thread
  __shared__ double2 Vs[16][BT_NB + 1];
  __shared__ double2 Ts[BT_NB][BT_NB + 1];
  __shared__ double2 tv[BT_NB];
  const Loc lc = locate(sz, blockIdx.x, [](int n) { return htd_nblk(n); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], b = lc.b, k0 = BT_NB * b, tid = threadIdx.x;
  const int nb = min(BT_NB, (n - 1) - k0);
  double2 acc[PPT];
#pragma unroll
  for (int t = 0; t < PPT; ++t) acc[t] = make_double2(0.0, 0.0);
  for (int j0 = k0 + 1; j0 < n; j0 += 16) {
    for (int e = tid; e < 16 * BT_NB; e += 256) {
      const int jj = e / BT_NB, i = e % BT_NB, j = j0 + jj;
      Vs[jj][i] = i < nb && j < n ? refl(d, k0 + i, j) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
#pragma unroll
      for (int t = 0; t < PPT; ++t) {
        const int e = tid + 256 * t, a = e / BT_NB, i = e % BT_NB;
        acc[t] = cadd(acc[t], cmulc(Vs[jj][a], Vs[jj][i]));
      }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const int e = tid + 256 * t, a = e / BT_NB, i = e % BT_NB;
    Ts[a][i] = a < i ? acc[t] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const double2 ti = gld(d.tau + k0 + i);
    if (tid < i) {
      const double2 t = cmul(ti, Ts[tid][i]);
      tv[tid] = make_double2(-t.x, -t.y);
    }
    __syncthreads();
    if (tid < i) {  // reads columns < i of T, writes column i
      double2 s2 = make_double2(0.0, 0.0);
      for (int l = tid; l < i; ++l) s2 = cadd(s2, cmul(Ts[tid][l], tv[l]));
      Ts[tid][i] = s2;
    }
    if (tid == 0) Ts[i][i] = ti;
    __syncthreads();
  }
  double2* out = d.T + (int64_t)b * BT_NB * BT_NB;
  for (int e = tid; e < BT_NB * BT_NB; e += 256) gst(out + e, Ts[e / BT_NB][e % BT_NB]);
}

// partial W = V_b^H Z over a chunk of BT_CH rows (rows from k0 + 1) and 64
// eigenvector columns, on the matrix cores: the BT_NB x 64 output is
// (BT_NB / 16) x 4 blocks of 16 x 16, BT_NB / 16 per wavefront.  The chunk
// goes through LDS in slices of 16 rows; the loads of slice s + 1 are issued
// before the products of slice s, unconditionally at clamped addresses and
// masked when staged.
__global__ __launch_bounds__(256) void bt_wpart_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int b) {
  constexpr int BPW = BT_NB / 16;         // output blocks per wavefront
  constexpr int EA = 16 * BT_NB / 256, EB = 16 * 64 / 256;
  __shared__ double2 As[16][BT_NB + 1];   // conj(v_i[j]), k-major
  __shared__ double2 Bs[16][64 + 1];      // Z[j][c]
  const Loc lc = locate_d(sz, blockIdx.x, [b](int n, int nc) {
    return htd_wpart_blocks(n, nc, b);
  });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], nc = sz.nc[lc.p], ld = d.ld, tid = threadIdx.x, k0 = BT_NB * b;
  const int nb = min(BT_NB, (n - 1) - k0);
  const int ct = (nc + 63) / 64, ch = lc.b / ct, c0 = (lc.b % ct) * 64;
  const int rbeg = k0 + 1 + ch * BT_CH, rend = min(n, rbeg + BT_CH);
  const int lane = tid & 63, wave = tid >> 6;
  double2 ra[EA], rb[EB];
  auto fetch = [&](int j0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + 256 * u, i = e >> 4, j = j0 + (e & 15);
      ra[u] = gld(d.A + (int64_t)(k0 + min(i, nb - 1)) * ld + min(j, rend - 1));
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + 256 * u, j = j0 + (e >> 6), c = e & 63;
      rb[u] = gld(d.V + (int64_t)min(j, rend - 1) * ld + min(c0 + c, nc - 1));
    }
  };
  CAcc3<double> acc[BPW];
#pragma unroll
  for (int q = 0; q < BPW; ++q) acc[q].clear();
  fetch(rbeg);
  for (int j0 = rbeg; j0 < rend; j0 += 16) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + 256 * u, i = e >> 4, kk = e & 15, j = j0 + kk;
      const bool in = i < nb && j < rend && j > k0 + i;  // v_i is zero up to row k0 + i
      As[kk][i] = make_double2(in ? ra[u].x : 0.0, in ? -ra[u].y : 0.0);
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + 256 * u, kk = e >> 6, c = e & 63;
      const bool in = j0 + kk < rend && c0 + c < nc;
      Bs[kk][c] = make_double2(in ? rb[u].x : 0.0, in ? rb[u].y : 0.0);
    }
    __syncthreads();
    if (j0 + 16 < rend) fetch(j0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int q = 0; q < BPW; ++q) {
        const int blk = wave * BPW + q, bi = blk >> 2, bj = blk & 3;
        const double2 a = As[kr][bi * 16 + cl], bb = Bs[kr][bj * 16 + cl];
        acc[q].mac(a.x, a.y, bb.x, bb.y);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < BPW; ++q) {
    const int blk = wave * BPW + q, bi = blk >> 2, bj = blk & 3;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = bi * 16 + Mfma<double>::row(lane, r);
      const int c = c0 + bj * 16 + (lane & 15);
      if (c < nc) gst(d.Wp + ((int64_t)ch * BT_NB + i) * ld + c, make_double2(acc_re(acc[q], r), acc_im(acc[q], r)));
    }
  }
}

// W = T (sum of the partials) for BT_WC columns per workgroup: one entry
// (i, c) per thread, all its chunk partials loaded at once (clamped, masked)
// and T staged in LDS.
__global__ __launch_bounds__(256) void bt_wred_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int b) {
  constexpr int NCH = HTD_MAX / BT_CH;  // chunks at most
  static_assert(BT_NB * BT_WC == 256, "one entry of W per thread");
  __shared__ double2 Ws[BT_NB][BT_WC];
  __shared__ double2 Ts[BT_NB][BT_NB + 1];
  const Loc lc = locate_d(sz, blockIdx.x, [b](int n, int nc) {
    return htd_wred_blocks(n, nc, b);
  });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], nc = sz.nc[lc.p], ld = d.ld, tid = threadIdx.x, c0 = lc.b * BT_WC;
  const int nch = (htd_bt_rows(n, b) + BT_CH - 1) / BT_CH;
  const double2* Tb = d.T + (int64_t)b * BT_NB * BT_NB;
  const int i = tid / BT_WC, c = tid % BT_WC;
  const double2* w = d.Wp + (int64_t)i * ld + min(c0 + c, nc - 1);
  double2 v[NCH];
#pragma unroll
  for (int q = 0; q < NCH; ++q) v[q] = gld(w + (int64_t)(q < nch ? q : 0) * BT_NB * ld);
#pragma unroll
  for (int e = tid; e < BT_NB * BT_NB; e += 256) Ts[e / BT_NB][e % BT_NB] = gld(Tb + e);
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int q = 0; q < NCH; ++q) {
    sx += q < nch ? v[q].x : 0.0;
    sy += q < nch ? v[q].y : 0.0;
  }
  Ws[i][c] = make_double2(sx, sy);
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  for (int l = i; l < BT_NB; ++l) s = cadd(s, cmul(Ts[i][l], Ws[l][c]));
  if (c0 + c < nc) gst(d.W + (int64_t)i * ld + c0 + c, s);
}

// Z[j][c] -= sum_i v_i[j] W[i][c] on 64 x 64 tiles of rows k0 + 1 ...; each
// wavefront owns a 32 x 32 quadrant (2 x 2 blocks of 16 x 16), K = BT_NB in
// slices of 16.  As in the partial product, the next slice (and during the
// last slice the tile of Z) is loaded before the products of the current one.
__global__ __launch_bounds__(256) void bt_update_kernel(const HtdDesc* __restrict__ ds, const HtdSizes sz, int b) {
  constexpr int EPT = 16 * 64 / 256;
  __shared__ double2 As[16][64 + 1];  // v_i[j], k-major
  __shared__ double2 Bs[16][64 + 1];  // W[i][c]
  const Loc lc = locate_d(sz, blockIdx.x, [b](int n, int nc) {
    return htd_update_blocks(n, nc, b);
  });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = sz.n[lc.p], nc = sz.nc[lc.p], ld = d.ld, tid = threadIdx.x, k0 = BT_NB * b;
  const int nb = min(BT_NB, (n - 1) - k0);
  const int ct = (nc + 63) / 64, rt = lc.b / ct, c0 = (lc.b % ct) * 64;
  const int j0 = k0 + 1 + rt * 64;
  const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  double2 ra[EPT], rb[EPT];
  auto fetch = [&](int i0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u, i = min(i0 + (e >> 6), nb - 1), x = e & 63;
      ra[u] = gld(d.A + (int64_t)(k0 + i) * ld + min(j0 + x, n - 1));
      rb[u] = gld(d.W + (int64_t)i * ld + min(c0 + x, nc - 1));
    }
  };
  CAcc3<double> acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y].clear();
  double2 zt[2][2][4];
  fetch(0);
#pragma unroll
  for (int i0 = 0; i0 < BT_NB; i0 += 16) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u, ii = e >> 6, x = e & 63;
      const int i = i0 + ii, j = j0 + x;
      const bool ina = i < nb && j < n && j > k0 + i, inb = i < nb && c0 + x < nc;
      As[ii][x] = make_double2(ina ? ra[u].x : 0.0, ina ? ra[u].y : 0.0);
      Bs[ii][x] = make_double2(inb ? rb[u].x : 0.0, inb ? rb[u].y : 0.0);
    }
    __syncthreads();
    if (i0 + 16 < BT_NB) {
      fetch(i0 + 16);
    } else {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + wm * 32 + x * 16 + Mfma<double>::row(lane, r);
            const int c = c0 + wn * 32 + y * 16 + (lane & 15);
            zt[x][y][r] = gld(d.V + (int64_t)min(j, n - 1) * ld + min(c, nc - 1));
          }
    }
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
      const double2 a0 = As[kr][wm * 32 + cl], a1 = As[kr][wm * 32 + 16 + cl];
      const double2 b0 = Bs[kr][wn * 32 + cl], b1 = Bs[kr][wn * 32 + 16 + cl];
      acc[0][0].mac(a0.x, a0.y, b0.x, b0.y);
      acc[0][1].mac(a0.x, a0.y, b1.x, b1.y);
      acc[1][0].mac(a1.x, a1.y, b0.x, b0.y);
      acc[1][1].mac(a1.x, a1.y, b1.x, b1.y);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + wm * 32 + x * 16 + Mfma<double>::row(lane, r);
        const int c = c0 + wn * 32 + y * 16 + (lane & 15);
        if (j < n && c < nc)
          gst(d.V + (int64_t)j * ld + c,
              make_double2(zt[x][y][r].x - acc_re(acc[x][y], r), zt[x][y][r].y - acc_im(acc[x][y], r)));
      }
}

}  // namespace

// The records of a's problems in the smallest argument block that holds them.
template <template <int> class K, int N>
hipError_t launch_probs(const HtdArgs& a, int k, int blocks, hipStream_t s) {
  if (a.np > N) return launch_probs<K, (N < HTD_GROUP ? 2 * N : N)>(a, k, blocks, s);
  HtdProbs<N> b;
  for (int q = 0; q < a.np; ++q) b.pr[q] = a.pr[q];
  for (int q = a.np; q < N; ++q) b.pr[q] = HtdProb{};
  launch(K<N>::kernel, dim3(blocks, a.np), dim3(256), 0, s, b, k);
  return hipGetLastError();
}
template <int N>
struct HemvK {
  static constexpr auto kernel = trd_hemv_kernel<N>;
};
template <int N>
struct ColK {
  static constexpr auto kernel = trd_col_kernel<N>;
};

hipError_t launch_trd_hemv(const HtdArgs& a, int k, int blocks, hipStream_t s) {
  if (blocks <= 0 || a.np <= 0) return hipSuccess;
  if (a.np > HTD_GROUP) return hipErrorInvalidValue;
  return launch_probs<HemvK, 1>(a, k, blocks, s);
}
hipError_t launch_trd_tail(const HtdDesc* d, const HtdSizes& sz, hipStream_t s) {
  if (sz.np <= 0) return hipSuccess;
  launch(trd_tail_kernel, dim3(sz.np), dim3(512), 0, s, d, sz);
  return hipGetLastError();
}
hipError_t launch_trd_col(const HtdArgs& a, int k, int blocks, hipStream_t s) {
  if (blocks <= 0 || a.np <= 0) return hipSuccess;
  if (a.np > HTD_GROUP) return hipErrorInvalidValue;
  return launch_probs<ColK, 1>(a, k, blocks, s);
}
hipError_t launch_trd_her2k(const HtdDesc* d, const HtdSizes& sz, int p0, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(trd_her2k_kernel, dim3(blocks), dim3(256), 0, s, d, sz, p0);
  return hipGetLastError();
}
hipError_t launch_trd_finish(const HtdDesc* d, const HtdSizes& sz, hipStream_t s) {
  if (sz.np <= 0) return hipSuccess;
  launch(trd_finish_kernel, dim3((sz.np + 63) / 64), dim3(64), 0, s, d, sz);
  return hipGetLastError();
}
hipError_t launch_dc_init(const HtdDesc* d, const HtdSizes& sz, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(dc_init_kernel, dim3(blocks), dim3(256), 0, s, d, sz);
  return hipGetLastError();
}
hipError_t launch_dc_prep(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(dc_prep_kernel, dim3(blocks), dim3(1024), 0, s, d, sz, L);
  return hipGetLastError();
}
hipError_t launch_dc_rot(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(dc_rot_kernel, dim3(blocks), dim3(256), 0, s, d, sz, L);
  return hipGetLastError();
}
hipError_t launch_dc_wave(int stage, const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(dc_wave_kernel, dim3(blocks), dim3(256), 0, s, d, sz, L, stage);
  return hipGetLastError();
}
hipError_t launch_dc_place(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(dc_place_kernel, dim3(blocks), dim3(256), 0, s, d, sz, L);
  return hipGetLastError();
}
hipError_t launch_dc_gemm(const HtdDesc* d, const HtdSizes& sz, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(dc_gemm_kernel, dim3(blocks), dim3(256), 0, s, d, sz, L);
  return hipGetLastError();
}
hipError_t launch_bt_init(const HtdDesc* d, const HtdSizes& sz, int Lmax, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(bt_init_kernel, dim3(blocks), dim3(256), 0, s, d, sz, Lmax);
  return hipGetLastError();
}
hipError_t launch_bt_larft(const HtdDesc* d, const HtdSizes& sz, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(bt_larft_kernel, dim3(blocks), dim3(256), 0, s, d, sz);
  return hipGetLastError();
}
hipError_t launch_bt_wpart(const HtdDesc* d, const HtdSizes& sz, int b, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(bt_wpart_kernel, dim3(blocks), dim3(256), 0, s, d, sz, b);
  return hipGetLastError();
}
hipError_t launch_bt_wred(const HtdDesc* d, const HtdSizes& sz, int b, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(bt_wred_kernel, dim3(blocks), dim3(256), 0, s, d, sz, b);
  return hipGetLastError();
}
hipError_t launch_bt_update(const HtdDesc* d, const HtdSizes& sz, int b, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(bt_update_kernel, dim3(blocks), dim3(256), 0, s, d, sz, b);
  return hipGetLastError();
}

// Eigenpairs of one solve in ascending order into caller buffers: w[j] and
// column j of V (row-major n x n) from the solver's descending lam / columns
// of Vw (leading dimension ld).
__global__ void heev_out_kernel(const double2* __restrict__ Vw, int ld, const double* __restrict__ lam, int n,
                                double2* __restrict__ V, double* __restrict__ w) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    V[e] = Vw[(int64_t)i * ld + (n - 1 - j)];
    if (i == 0) w[j] = lam[n - 1 - j];
  }
}

hipError_t launch_heev_out(const double2* Vw, int ld, const double* lam, int n, double2* V, double* w,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, ((int64_t)n * n + 255) / 256);
  hipLaunchKernelGGL(heev_out_kernel, dim3(blocks), dim3(256), 0, s, Vw, ld, lam, n, V, w);
  return hipGetLastError();
}

}  // namespace ctebd
