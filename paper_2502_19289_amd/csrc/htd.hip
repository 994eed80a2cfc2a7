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

// problem and problem-local block of flat block `bid`
template <typename F>
__device__ __forceinline__ Loc locate(const HtdDesc* ds, int np, int bid, F count) {
  for (int p = 0; p < np; ++p) {
    const int c = count(dim_value(ds[p].n));
    if (bid < c) return Loc{p, bid};
    bid -= c;
  }
  return Loc{-1, 0};
}

__device__ __forceinline__ bool skipped(const HtdDesc& d) { return d.skip && *d.skip; }

__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// ======================================================= tridiagonalisation
// Step k: x = G[k+1:, k] (read as the conjugate of row k), reflector with
// H^H (alpha, x1)^T = (beta, 0)^T, beta real; y = tau G22 v for this
// workgroup's HV_ROWS rows; part = sum over them of conj(y_i) v_i.
__global__ __launch_bounds__(256) void trd_hemv_kernel(const HtdDesc* __restrict__ ds, int np, int k) {
  __shared__ double2 vs[HTD_MAX];
  __shared__ double red[256];
  __shared__ double2 wred[4];
  const Loc lc = locate(ds, np, blockIdx.x, [k](int n) { return htd_hemv_blocks(n, k); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), m = n - k - 1, ld = d.ld, tid = threadIdx.x;
  const double2* rowk = d.A + (int64_t)k * ld + (k + 1);
  // norms are formed on entries divided by the largest one, so that neither
  // tiny nor huge Gram entries under- or overflow in the squares
  double mx = 0.0;
  for (int j = tid; j < m; j += 256) {
    const double2 a = rowk[j];
    vs[j] = make_double2(a.x, -a.y);
    mx = fmax(mx, fmax(fabs(a.x), fabs(a.y)));
  }
  red[tid] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double amax = red[0];
  __syncthreads();
  double s = 0.0;  // |x_1..|^2 / amax^2 (alpha = x_0 excluded)
  if (amax > 0.0)
    for (int j = tid; j < m; j += 256) {
      if (j == 0) continue;
      const double2 x = vs[j];
      s += (x.x / amax) * (x.x / amax) + (x.y / amax) * (x.y / amax);
    }
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double xs2 = red[0];
  const double2 alpha = vs[0];
  double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
  double beta = alpha.x;
  if (xs2 > 0.0 || alpha.y != 0.0) {
    const double ar = alpha.x / amax, ai = alpha.y / amax;
    beta = -copysign(amax * sqrt(ar * ar + ai * ai + xs2), alpha.x);
    tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    // scale = 1 / (alpha - beta) by Smith's complex division
    const double dr = alpha.x - beta, di = alpha.y;
    if (fabs(dr) >= fabs(di)) {
      const double r = di / dr, t = 1.0 / (dr + di * r);
      scale = make_double2(t, -r * t);
    } else {
      const double r = dr / di, t = 1.0 / (di + dr * r);
      scale = make_double2(r * t, -t);
    }
  }
  const bool ident = tau.x == 0.0 && tau.y == 0.0;
  __syncthreads();  // vs[0] read by everyone
  for (int j = tid; j < m; j += 256)
    vs[j] = j == 0 ? make_double2(1.0, 0.0) : (ident ? make_double2(0.0, 0.0) : cmul(vs[j], scale));
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  double2 part = make_double2(0.0, 0.0);
  for (int rr = 0; rr < HV_ROWS / 4; ++rr) {
    const int i = lc.b * HV_ROWS + wave * (HV_ROWS / 4) + rr;
    if (i >= m) break;
    double2 yi = make_double2(0.0, 0.0);
    if (!ident) {
      const double2* arow = d.A + (int64_t)(k + 1 + i) * ld + (k + 1);
      double ax = 0.0, ay = 0.0;
      for (int j = lane; j < m; j += 64) {
        const double2 a = arow[j], v = vs[j];
        ax += a.x * v.x - a.y * v.y;
        ay += a.x * v.y + a.y * v.x;
      }
      for (int off = 32; off > 0; off >>= 1) {
        ax += __shfl_xor(ax, off);
        ay += __shfl_xor(ay, off);
      }
      yi = cmul(tau, make_double2(ax, ay));
    }
    if (lane == 0) d.y[i] = yi;
    part = cadd(part, cmulc(yi, vs[i]));
  }
  if (lane == 0) wred[wave] = part;
  __syncthreads();
  if (tid == 0) d.part[lc.b] = cadd(cadd(wred[0], wred[1]), cadd(wred[2], wred[3]));
  if (lc.b == 0) {
    for (int j = tid; j < m; j += 256) d.v[j] = vs[j];
    if (tid == 0) {
      d.tau[k] = tau;
      d.e[k] = beta;
      d.d[k] = d.A[(int64_t)k * ld + k].x;
    }
  }
}

// G22 -= v w^H + w v^H with w = y - (tau/2)(y^H v) v, on 64 x 64 tiles; the
// first tile row also stores v in row k (columns k+1 ...) for the
// back-transformation.
__global__ __launch_bounds__(256) void trd_her2_kernel(const HtdDesc* __restrict__ ds, int np, int k) {
  __shared__ double2 vr[64], wr[64], vc[64], wc[64];
  __shared__ double2 red[256];
  const Loc lc = locate(ds, np, blockIdx.x, [k](int n) { return htd_her2_blocks(n, k); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), m = n - k - 1, ld = d.ld, tid = threadIdx.x;
  const int T = (m + 63) / 64, ti = lc.b / T, tj = lc.b % T;
  const double2 tau = d.tau[k];
  const bool ident = tau.x == 0.0 && tau.y == 0.0;
  const int nbp = htd_hemv_blocks(n, k);
  double2 s = make_double2(0.0, 0.0);
  for (int q = tid; q < nbp; q += 256) s = cadd(s, d.part[q]);
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = cadd(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double2 alpha = cmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), red[0]);
  if (tid < 128) {
    const int l = tid & 63;
    const int i = (tid < 64 ? ti : tj) * 64 + l;
    double2 v = make_double2(0.0, 0.0), w = make_double2(0.0, 0.0);
    if (i < m) {
      v = d.v[i];
      w = cadd(d.y[i], cmul(alpha, v));
    }
    if (tid < 64) {
      vr[l] = v;
      wr[l] = w;
    } else {
      vc[l] = v;
      wc[l] = w;
    }
  }
  __syncthreads();
  if (!ident) {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int l = e >> 6, c = e & 63;
      const int i = ti * 64 + l, j = tj * 64 + c;
      if (i < m && j < m) {
        double2* p = d.A + (int64_t)(k + 1 + i) * ld + (k + 1 + j);
        const double2 t1 = cmulc(wc[c], vr[l]);  // v_i conj(w_j)
        const double2 t2 = cmulc(vc[c], wr[l]);  // w_i conj(v_j)
        *p = csub(csub(*p, t1), t2);
      }
    }
  }
  if (ti == 0 && tid < 64) {
    const int j = tj * 64 + tid;
    if (j < m) d.A[(int64_t)k * ld + (k + 1 + j)] = vc[tid];
  }
}

__global__ void trd_finish_kernel(const HtdDesc* __restrict__ ds, int np) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const HtdDesc& d = ds[p];
  if (skipped(d)) return;
  const int n = dim_value(d.n);
  if (n < 1) return;
  d.d[n - 1] = d.A[(int64_t)(n - 1) * d.ld + (n - 1)].x;
  d.e[n - 1] = 0.0;
}

// ======================================================= divide and conquer
// Level 0: T torn at every off-diagonal entry (d_i -= |e_{i-1}| + |e_i|),
// 1 x 1 blocks with eigenvector 1.  Both eigenvector buffers start at zero:
// a merge multiplies whole rows of its node, so the quadrants outside the
// children's blocks must hold exact zeros (later levels only ever write
// inside their own node blocks).
__global__ __launch_bounds__(256) void dc_init_kernel(const HtdDesc* __restrict__ ds, int np) {
  const Loc lc = locate(ds, np, blockIdx.x, [](int n) { return n; });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), i = lc.b, ld = d.ld;
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

// Merge of node [lo, hi) at level L (children [lo, mid), [mid, hi)):
// T_node = diag(Q1, Q2) (diag(D1, D2) + rho z z^T) diag(Q1, Q2)^T with
// z = (last row of Q1, sign(e) first row of Q2) / sqrt(2), rho = 2 |e_{mid-1}|.
// Sorts the poles, deflates small z components and (after a rotation)
// close poles, and lists the non-deflated poles for the secular equation.
__global__ __launch_bounds__(1024) void dc_prep_kernel(const HtdDesc* __restrict__ ds, int np, int L) {
  __shared__ double Ds[HTD_MAX];
  __shared__ double zs[HTD_MAX];
  __shared__ int col[HTD_MAX];
  __shared__ double red[16];
  __shared__ int sh_ndef;
  const Loc lc = locate(ds, np, blockIdx.x, [L](int n) { return htd_nodes(n, L); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), s = 1 << L, tid = threadIdx.x;
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
      z = Qin[(int64_t)(mid - 1) * ld + lo + t];
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
      z = sg * Qin[(int64_t)mid * ld + mid + q];
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
  if (tid == 0) {
    int K2 = 0, ndef = 0, nrot = 0;
    if (rho * mz <= tol) {
      for (int t = 0; t < K; ++t) {
        d.dval[lo + ndef] = Ds[t];
        d.dcol[lo + ndef] = col[t];
        ++ndef;
      }
    } else {
      int pj = -1;
      for (int t = 0; t < K; ++t) {
        if (rho * fabs(zs[t]) <= tol) {
          d.dval[lo + ndef] = Ds[t];
          d.dcol[lo + ndef] = col[t];
          ++ndef;
          continue;
        }
        if (pj < 0) {
          pj = t;
          continue;
        }
        double sn = zs[pj], cs = zs[t];
        const double tau = hypot(cs, sn), tt = Ds[t] - Ds[pj];
        cs /= tau;
        sn = -sn / tau;
        if (fabs(tt * cs * sn) <= tol) {
          // rotate columns pj, t so that z_pj = 0: pj deflates
          zs[t] = tau;
          zs[pj] = 0.0;
          d.rot_a[lo + nrot] = col[pj];
          d.rot_b[lo + nrot] = col[t];
          d.rot_c[lo + nrot] = cs;
          d.rot_s[lo + nrot] = sn;
          ++nrot;
          const double t1 = Ds[pj] * cs * cs + Ds[t] * sn * sn;
          Ds[t] = Ds[pj] * sn * sn + Ds[t] * cs * cs;
          Ds[pj] = t1;
          d.dval[lo + ndef] = Ds[pj];
          d.dcol[lo + ndef] = col[pj];
          ++ndef;
        } else {
          d.dl[lo + K2] = Ds[pj];
          d.w[lo + K2] = zs[pj];
          d.ndcol[lo + K2] = col[pj];
          ++K2;
        }
        pj = t;
      }
      if (pj >= 0) {
        d.dl[lo + K2] = Ds[pj];
        d.w[lo + K2] = zs[pj];
        d.ndcol[lo + K2] = col[pj];
        ++K2;
      }
    }
    cnt[0] = K2;
    cnt[1] = ndef;
    cnt[2] = nrot;
    cnt[3] = 1;
    d.rho[lo] = rho;
    sh_ndef = ndef;
  }
  __syncthreads();
  // deflated eigenvalues ascending (bitonic sort, ties by column)
  const int ndef = sh_ndef;
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

// Root k of the secular equation 1 + rho sum_j w_j^2 / (dl_j - lambda) = 0 in
// (dl_k, dl_{k+1}) (last root: (dl_k, dl_k + rho |w|^2]).  lambda is kept as
// dl_origin + tau with the origin at the nearer pole, so every dl_j - lambda
// is formed as (dl_j - dl_origin) - tau.  Iteration: each step replaces the
// two poles' terms by the rational model of Li's middle way (value and slope
// of both sums matched at the current point) and takes the root of the
// resulting quadratic; a bracket on the sign of f guards every step and falls
// back to bisection (geometric when the bracket spans a decade or more).
__device__ void secular_root(const double* dl, const double* w, int K2, double rho, int k, int& origin,
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
    double f = 1.0;
    for (int j = 0; j < K2; ++j) f += rho * w[j] * w[j] / ((dl[j] - dl[k]) - mid);
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
    for (int j = 0; j < K2; ++j) s += w[j] * w[j];
    tlo = 0.0;
    thi = rho * s;
  }
  const double base = dl[o];
  double tau = 0.5 * (tlo + thi);
  for (int it = 0; it < 200; ++it) {
    double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
    for (int j = 0; j < K2; ++j) {
      const double del = (dl[j] - base) - tau;
      const double t = w[j] / del;
      if (j <= k) {
        psi += w[j] * t;
        dpsi += t * t;
      } else {
        phi += w[j] * t;
        dphi += t * t;
      }
    }
    psi *= rho;
    phi *= rho;
    dpsi *= rho;
    dphi *= rho;
    const double f = 1.0 + psi + phi;
    if (f == 0.0) break;
    if (f < 0.0)
      tlo = tau;
    else
      thi = tau;
    const double err = 8.0 * EPS53 * K2 * (1.0 + fabs(psi) + fabs(phi));
    if (fabs(f) <= err || thi - tlo <= 4.0 * EPS53 * fmax(fabs(tlo), fabs(thi))) break;
    const double di = (dl[k] - base) - tau;
    double eta;
    if (!last) {
      const double dj = (dl[k + 1] - base) - tau;
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

// per-row stages of a merge level (thread per row / root / pole of a node)
__global__ __launch_bounds__(256) void dc_rows_kernel(const HtdDesc* __restrict__ ds, int np, int L, int stage) {
  const Loc lc = locate(ds, np, blockIdx.x, [](int n) { return htd_rows(n); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), i = lc.b * 256 + threadIdx.x;
  if (i >= n) return;
  const int lo = (i >> L) << L, ld = d.ld;
  const int* cnt = d.cnt + 4 * lo;
  if (!cnt[3]) return;
  const int K2 = cnt[0];
  const int k = i - lo;
  const double* dl = d.dl + lo;
  const double* w = d.w + lo;
  if (stage == 0) {
    // deflation rotations on row i of the children's eigenvectors
    double* q = d.Q[(L - 1) & 1] + (int64_t)i * ld;
    const int nrot = cnt[2];
    for (int r = 0; r < nrot; ++r) {
      const int a = d.rot_a[lo + r], b = d.rot_b[lo + r];
      const double c = d.rot_c[lo + r], s = d.rot_s[lo + r];
      const double x = q[a], y = q[b];
      q[a] = c * x + s * y;
      q[b] = c * y - s * x;
    }
  } else if (stage == 1) {
    if (k >= K2) return;
    int o;
    double tau;
    secular_root(dl, w, K2, d.rho[lo], k, o, tau);
    d.origin[lo + k] = o;
    d.stau[lo + k] = tau;
    const double base = dl[o];
    for (int j = 0; j < K2; ++j) d.DeltaT[(int64_t)(lo + j) * ld + lo + k] = (dl[j] - base) - tau;
  } else if (stage == 2) {
    // zhat_j^2 = prod_k (lambda_k - dl_j) / (rho prod_{k != j} (dl_k - dl_j))
    if (k >= K2) return;
    const double* dt = d.DeltaT + (int64_t)(lo + k) * ld + lo;
    double v = -dt[k] / d.rho[lo];
    for (int q = 0; q < K2; ++q)
      if (q != k) v *= (-dt[q]) / (dl[q] - dl[k]);
    d.zhat[lo + k] = copysign(sqrt(fmax(v, 0.0)), w[k]);
  } else {
    // eigenvector of root k: u_j = zhat_j / (dl_j - lambda_k), normalised
    if (k >= K2) return;
    const double* zh = d.zhat + lo;
    double s2 = 0.0;
    for (int j = 0; j < K2; ++j) {
      const double u = zh[j] / d.DeltaT[(int64_t)(lo + j) * ld + lo + k];
      s2 += u * u;
    }
    const double inv = 1.0 / sqrt(s2);
    for (int j = 0; j < K2; ++j) {
      const int64_t e = (int64_t)(lo + j) * ld + lo + k;
      d.U[e] = zh[j] / d.DeltaT[e] * inv;
    }
  }
}

// Orders the node's eigenvalues (roots and deflated values), writes them to
// the next level's list, copies the deflated eigenvectors and records where
// the GEMM writes each root's eigenvector.  Nodes without a right child are
// carried over unchanged.
__global__ __launch_bounds__(1024) void dc_place_kernel(const HtdDesc* __restrict__ ds, int np, int L) {
  __shared__ double lamv[HTD_MAX];
  __shared__ double dv[HTD_MAX];
  __shared__ int pdef[HTD_MAX];
  const Loc lc = locate(ds, np, blockIdx.x, [L](int n) { return htd_nodes(n, L); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), s = 1 << L, tid = threadIdx.x, ld = d.ld;
  const int lo = lc.b * s, hi = min(lo + s, n), K = hi - lo;
  const double* Din = d.D[(L - 1) & 1];
  const double* Qin = d.Q[(L - 1) & 1];
  double* Dout = d.D[L & 1];
  double* Qout = d.Q[L & 1];
  const int* cnt = d.cnt + 4 * lo;
  if (!cnt[3]) {
    for (int e = tid; e < K * K; e += 1024) {
      const int r = e / K, c = e % K;
      Qout[(int64_t)(lo + r) * ld + lo + c] = Qin[(int64_t)(lo + r) * ld + lo + c];
    }
    for (int c = tid; c < K; c += 1024) Dout[lo + c] = Din[lo + c];
    return;
  }
  const int K2 = cnt[0], ndef = cnt[1];
  for (int k = tid; k < K2; k += 1024) lamv[k] = d.dl[lo + d.origin[lo + k]] + d.stau[lo + k];
  for (int q = tid; q < ndef; q += 1024) dv[q] = d.dval[lo + q];
  __syncthreads();
  for (int k = tid; k < K2; k += 1024) {
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
  for (int q = tid; q < ndef; q += 1024) {
    const double x = dv[q];
    int a = 0, b = K2;  // roots at or below x
    while (a < b) {
      const int mm = (a + b) >> 1;
      if (lamv[mm] <= x)
        a = mm + 1;
      else
        b = mm;
    }
    pdef[q] = q + a;
    Dout[lo + q + a] = x;
  }
  __syncthreads();
  for (int e = tid; e < ndef * K; e += 1024) {
    const int q = e / K, r = e % K;
    Qout[(int64_t)(lo + r) * ld + lo + pdef[q]] = Qin[(int64_t)(lo + r) * ld + d.dcol[lo + q]];
  }
}

// Q_out[:, pos_k] = Q_in[:, ndcol] U[:, k] for the node's rows, on the matrix
// cores (f64 16x16x4); each of the four wavefronts owns a 32 x 32 quadrant of
// the 64 x 64 tile.
__global__ __launch_bounds__(256) void dc_gemm_kernel(const HtdDesc* __restrict__ ds, int np, int L) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const Loc lc = locate(ds, np, blockIdx.x, [L](int n) { return htd_gemm_tiles(n, L); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), s = 1 << L, ld = d.ld;
  const int T = (s + 63) / 64, per = T * T;
  const int node = lc.b / per, t = lc.b % per, ti = t / T, tj = t % T;
  const int lo = node * s, hi = min(lo + s, n), K = hi - lo;
  const int* cnt = d.cnt + 4 * lo;
  if (!cnt[3]) return;
  const int K2 = cnt[0];
  const int r0 = ti * 64, k0 = tj * 64;
  if (r0 >= K || k0 >= K2) return;
  const double* Qin = d.Q[(L - 1) & 1];
  double* Qout = d.Q[L & 1];
  const int* ndc = d.ndcol + lo;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<double>::zero();
  for (int j0 = 0; j0 < K2; j0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      const int c = e >> 4, kk = e & 15;  // A: row c of the tile, pole j0 + kk
      const int j = j0 + kk, r = r0 + c;
      As[kk][c] = (j < K2 && r < K) ? Qin[(int64_t)(lo + r) * ld + ndc[j]] : 0.0;
      const int kk2 = e >> 6, c2 = e & 63;  // B: pole j0 + kk2, root k0 + c2
      const int j2 = j0 + kk2, kc = k0 + c2;
      Bs[kk2][c2] = (j2 < K2 && kc < K2) ? d.U[(int64_t)(lo + j2) * ld + lo + kc] : 0.0;
    }
    __syncthreads();
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
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wm * 32 + bi * 16 + Mfma<double>::row(lane, r);
        const int kc = k0 + wn * 32 + bj * 16 + (lane & 15);
        if (row < K && kc < K2) Qout[(int64_t)(lo + row) * ld + lo + d.pos_nd[lo + kc]] = acc[bi][bj][r];
      }
}

// ======================================================= back-transformation
// V = Z (real eigenvectors of T, last level's buffer), lam = its eigenvalues.
__global__ __launch_bounds__(256) void bt_init_kernel(const HtdDesc* __restrict__ ds, int np, int Lmax) {
  const Loc lc = locate(ds, np, blockIdx.x, [](int n) { return n; });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), j = lc.b, ld = d.ld;
  const double* z = d.Q[Lmax & 1] + (int64_t)j * ld;
  double2* v = d.V + (int64_t)j * ld;
  for (int c = threadIdx.x; c < n; c += 256) v[c] = make_double2(z[c], 0.0);
  if (threadIdx.x == 0) d.lam[j] = d.D[Lmax & 1][j];
}

// reflector i of block b (k = HTD_NB b + i) at row j: 0 for j <= k, else row k of A
__device__ __forceinline__ double2 refl(const HtdDesc& d, int k, int j) {
  return j > k ? d.A[(int64_t)k * d.ld + j] : make_double2(0.0, 0.0);
}

// T of each block: H_k0 ... H_k0+nb-1 = I - V_b T V_b^H (upper triangular T,
// T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] V_b[:, 0:i]^H v_i).
__global__ __launch_bounds__(256) void bt_larft_kernel(const HtdDesc* __restrict__ ds, int np) {
  __shared__ double2 S[HTD_NB][HTD_NB];
  __shared__ double2 Ts[HTD_NB][HTD_NB];
  __shared__ double2 tv[HTD_NB];
  const Loc lc = locate(ds, np, blockIdx.x, [](int n) { return htd_nblk(n); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), b = lc.b, k0 = HTD_NB * b, tid = threadIdx.x;
  const int nb = min(HTD_NB, (n - 1) - k0);
  const int wave = tid >> 6, lane = tid & 63;
  // S[a][i] = v_a^H v_i for a < i (v_i vanishes above row k0 + i + 1)
  for (int pr = wave; pr < HTD_NB * HTD_NB; pr += 4) {
    const int a = pr / HTD_NB, i = pr % HTD_NB;
    if (a >= i || i >= nb) continue;
    double sx = 0.0, sy = 0.0;
    const double2* va = d.A + (int64_t)(k0 + a) * d.ld;
    const double2* vi = d.A + (int64_t)(k0 + i) * d.ld;
    for (int j = k0 + i + 1 + lane; j < n; j += 64) {
      const double2 x = va[j], y = vi[j];
      sx += x.x * y.x + x.y * y.y;
      sy += x.x * y.y - x.y * y.x;
    }
    for (int off = 32; off > 0; off >>= 1) {
      sx += __shfl_xor(sx, off);
      sy += __shfl_xor(sy, off);
    }
    if (lane == 0) S[a][i] = make_double2(sx, sy);
  }
  for (int e = tid; e < HTD_NB * HTD_NB; e += 256) Ts[e / HTD_NB][e % HTD_NB] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const double2 ti = d.tau[k0 + i];
    if (tid < i) {
      const double2 t = cmul(ti, S[tid][i]);
      tv[tid] = make_double2(-t.x, -t.y);
    }
    __syncthreads();
    if (tid < i) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = tid; l < i; ++l) acc = cadd(acc, cmul(Ts[tid][l], tv[l]));
      Ts[tid][i] = acc;
    }
    if (tid == 0) Ts[i][i] = ti;
    __syncthreads();
  }
  double2* out = d.T + (int64_t)b * HTD_NB * HTD_NB;
  for (int e = tid; e < HTD_NB * HTD_NB; e += 256) out[e] = Ts[e / HTD_NB][e % HTD_NB];
}

// partial W = V_b^H V over a chunk of BT_CH rows (rows from k0 + 1), 64 columns
__global__ __launch_bounds__(256) void bt_wpart_kernel(const HtdDesc* __restrict__ ds, int np, int b) {
  __shared__ double2 Vs[32][64];
  __shared__ double2 Rs[HTD_NB][32];
  const Loc lc = locate(ds, np, blockIdx.x, [b](int n) { return htd_wpart_blocks(n, b); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), ld = d.ld, tid = threadIdx.x, k0 = HTD_NB * b;
  const int nb = min(HTD_NB, (n - 1) - k0);
  const int ct = (n + 63) / 64, ch = lc.b / ct, c0 = (lc.b % ct) * 64;
  const int rbeg = k0 + 1 + ch * BT_CH, rend = min(n, rbeg + BT_CH);
  const int i = tid >> 3, c8 = (tid & 7) * 8;
  double2 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int j0 = rbeg; j0 < rend; j0 += 32) {
    for (int e = tid; e < 32 * 64; e += 256) {
      const int jj = e >> 6, c = e & 63, j = j0 + jj;
      Vs[jj][c] = (j < rend && c0 + c < n) ? d.V[(int64_t)j * ld + c0 + c] : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < HTD_NB * 32; e += 256) {
      const int ii = e >> 5, jj = e & 31, j = j0 + jj;
      Rs[ii][jj] = (ii < nb && j < rend) ? refl(d, k0 + ii, j) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int jj = 0; jj < 32; ++jj) {
      const double2 a = Rs[i][jj];  // conj(a) * V
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = cadd(acc[q], cmulc(a, Vs[jj][c8 + q]));
    }
    __syncthreads();
  }
  double2* out = d.Wp + ((int64_t)ch * HTD_NB + i) * ld + c0 + c8;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (c0 + c8 + q < n) out[q] = acc[q];
}

// W = T (sum of the partials) for 64 columns
__global__ __launch_bounds__(256) void bt_wred_kernel(const HtdDesc* __restrict__ ds, int np, int b) {
  __shared__ double2 Ws[HTD_NB][64];
  __shared__ double2 Ts[HTD_NB][HTD_NB];
  const Loc lc = locate(ds, np, blockIdx.x, [b](int n) { return htd_wred_blocks(n, b); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), ld = d.ld, tid = threadIdx.x, c0 = lc.b * 64;
  const int nch = (htd_bt_rows(n, b) + BT_CH - 1) / BT_CH;
  const double2* Tb = d.T + (int64_t)b * HTD_NB * HTD_NB;
  for (int e = tid; e < HTD_NB * HTD_NB; e += 256) Ts[e / HTD_NB][e % HTD_NB] = Tb[e];
  for (int e = tid; e < HTD_NB * 64; e += 256) {
    const int i = e >> 6, c = e & 63;
    double2 s = make_double2(0.0, 0.0);
    if (c0 + c < n)
      for (int ch = 0; ch < nch; ++ch) s = cadd(s, d.Wp[((int64_t)ch * HTD_NB + i) * ld + c0 + c]);
    Ws[i][c] = s;
  }
  __syncthreads();
  for (int e = tid; e < HTD_NB * 64; e += 256) {
    const int i = e >> 6, c = e & 63;
    if (c0 + c >= n) continue;
    double2 s = make_double2(0.0, 0.0);
    for (int l = i; l < HTD_NB; ++l) s = cadd(s, cmul(Ts[i][l], Ws[l][c]));
    d.W[(int64_t)i * ld + c0 + c] = s;
  }
}

// V[j][c] -= sum_i v_i[j] W[i][c] on 64 x 64 tiles of rows k0 + 1 ...
__global__ __launch_bounds__(256) void bt_update_kernel(const HtdDesc* __restrict__ ds, int np, int b) {
  __shared__ double2 Rs[16][64];
  __shared__ double2 Ws[16][64];
  const Loc lc = locate(ds, np, blockIdx.x, [b](int n) { return htd_update_blocks(n, b); });
  if (lc.p < 0) return;
  const HtdDesc& d = ds[lc.p];
  if (skipped(d)) return;
  const int n = dim_value(d.n), ld = d.ld, tid = threadIdx.x, k0 = HTD_NB * b;
  const int nb = min(HTD_NB, (n - 1) - k0);
  const int ct = (n + 63) / 64, rt = lc.b / ct, c0 = (lc.b % ct) * 64;
  const int j0 = k0 + 1 + rt * 64;
  const int l = tid >> 2, c16 = (tid & 3) * 16;
  double2 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < HTD_NB; i0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int ii = e >> 6, x = e & 63;
      const int j = j0 + x;
      Rs[ii][x] = (i0 + ii < nb && j < n) ? refl(d, k0 + i0 + ii, j) : make_double2(0.0, 0.0);
      Ws[ii][x] = (i0 + ii < nb && c0 + x < n) ? d.W[(int64_t)(i0 + ii) * ld + c0 + x] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int ii = 0; ii < 16; ++ii) {
      const double2 a = Rs[ii][l];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = cadd(acc[q], cmul(a, Ws[ii][c16 + q]));
    }
    __syncthreads();
  }
  const int j = j0 + l;
  if (j < n) {
    double2* row = d.V + (int64_t)j * ld + c0 + c16;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (c0 + c16 + q < n) row[q] = csub(row[q], acc[q]);
  }
}

}  // namespace

hipError_t launch_trd_hemv(const HtdDesc* d, int np, int k, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  trd_hemv_kernel<<<blocks, 256, 0, s>>>(d, np, k);
  return hipGetLastError();
}
hipError_t launch_trd_her2(const HtdDesc* d, int np, int k, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  trd_her2_kernel<<<blocks, 256, 0, s>>>(d, np, k);
  return hipGetLastError();
}
hipError_t launch_trd_finish(const HtdDesc* d, int np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  trd_finish_kernel<<<(np + 63) / 64, 64, 0, s>>>(d, np);
  return hipGetLastError();
}
hipError_t launch_dc_init(const HtdDesc* d, int np, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  dc_init_kernel<<<blocks, 256, 0, s>>>(d, np);
  return hipGetLastError();
}
hipError_t launch_dc_prep(const HtdDesc* d, int np, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  dc_prep_kernel<<<blocks, 1024, 0, s>>>(d, np, L);
  return hipGetLastError();
}
hipError_t launch_dc_rows(int stage, const HtdDesc* d, int np, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  dc_rows_kernel<<<blocks, 256, 0, s>>>(d, np, L, stage);
  return hipGetLastError();
}
hipError_t launch_dc_place(const HtdDesc* d, int np, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  dc_place_kernel<<<blocks, 1024, 0, s>>>(d, np, L);
  return hipGetLastError();
}
hipError_t launch_dc_gemm(const HtdDesc* d, int np, int L, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  dc_gemm_kernel<<<blocks, 256, 0, s>>>(d, np, L);
  return hipGetLastError();
}
hipError_t launch_bt_init(const HtdDesc* d, int np, int Lmax, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  bt_init_kernel<<<blocks, 256, 0, s>>>(d, np, Lmax);
  return hipGetLastError();
}
hipError_t launch_bt_larft(const HtdDesc* d, int np, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  bt_larft_kernel<<<blocks, 256, 0, s>>>(d, np);
  return hipGetLastError();
}
hipError_t launch_bt_wpart(const HtdDesc* d, int np, int b, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  bt_wpart_kernel<<<blocks, 256, 0, s>>>(d, np, b);
  return hipGetLastError();
}
hipError_t launch_bt_wred(const HtdDesc* d, int np, int b, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  bt_wred_kernel<<<blocks, 256, 0, s>>>(d, np, b);
  return hipGetLastError();
}
hipError_t launch_bt_update(const HtdDesc* d, int np, int b, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  bt_update_kernel<<<blocks, 256, 0, s>>>(d, np, b);
  return hipGetLastError();
}

}  // namespace ctebd
