// FP64 Hermitian eigen-solver for the Gram matrices of the split sweep
// (G = X^H D^2 X, whose eigenpairs give the singular values and right singular
// vectors of D X used by every truncated SVD of arXiv:2502.19289, Sec. II.B).
//
// Method: two-sided cyclic block Jacobi.  The padded matrix is cut into nb
// blocks of JB = 32 rows/columns; a round pairs the blocks (circle method, nb-1
// rounds per sweep) and every pair (P, Q) diagonalises its 64x64 subproblem
// G[P u Q, P u Q] with scalar cyclic Jacobi in LDS (eig_pairs, one workgroup per
// pair), producing a unitary J_PQ.  The round's rotations are then applied to
// the whole matrix, G <- J^H G J and V <- V J, as 64x64 tile products on the
// FP64 matrix cores (eig_update).  A sweep in which no subproblem needed a
// rotation ends the iteration for that matrix.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace ctebd {

namespace {

constexpr double kTolIn = 1e-15;   // inner rotation threshold (relative)
constexpr double kAbsFloor = 8.7e-19;  // 2^-60 times the trace of G

__device__ __forceinline__ int nblocks_of(int n) {
  int nb = (n + JB - 1) / JB;
  if (nb < 2) nb = 2;
  return nb + (nb & 1);
}

__device__ __forceinline__ void pair_of(int nb, int t, int s, int& P, int& Q) {
  if (s == 0) {
    P = t;
    Q = nb - 1;
  } else {
    P = (t + s) % (nb - 1);
    Q = (t - s + nb - 1) % (nb - 1);
  }
}

// slot s of round t among 64 indices (circle method)
__device__ __forceinline__ void pair64(int t, int s, int& p, int& q) {
  if (s == 0) {
    p = t;
    q = 63;
  } else {
    p = (t + s) % 63;
    q = (t - s + 63) % 63;
  }
}

__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ init --
__global__ __launch_bounds__(256) void eig_init_kernel(const EigDesc* __restrict__ descs) {
  const EigDesc& d = descs[blockIdx.y];
  const int n = dim_value(d.n);
  const int npad = nblocks_of(n) * JB;
  const int ld = d.ld;
  for (int row = blockIdx.x; row < npad; row += gridDim.x) {
    for (int c = threadIdx.x; c < npad; c += blockDim.x) {
      d.V[(int64_t)row * ld + c] = make_double2(row == c ? 1.0 : 0.0, 0.0);
      if (row >= n || c >= n) d.G[(int64_t)row * ld + c] = make_double2(0.0, 0.0);
    }
  }
  if (blockIdx.x == 0) {
    __shared__ double red[256];
    double s = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += d.G[(int64_t)i * ld + i].x;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      *d.scale = red[0];
      d.flags[0] = 0;
      d.flags[1] = 0;
    }
  }
}

// ------------------------------------------------- subproblem rotations --
__global__ __launch_bounds__(256) void eig_pairs_kernel(const EigDesc* __restrict__ descs,
                                                        const int* __restrict__ base, int nprob,
                                                        int round) {
  __shared__ double2 S[JP][JP + 1];
  __shared__ double2 Jm[JP][JP + 1];
  __shared__ double2 rot[JP / 2][4];
  __shared__ int rp[JP / 2], rq[JP / 2];
  __shared__ int need;

  const int p = find_problem(base, nprob, blockIdx.x);
  const EigDesc& d = descs[p];
  const int slot = blockIdx.x - base[p];
  const int tid = threadIdx.x;
  const int n = dim_value(d.n);
  const int nb = nblocks_of(n);
  if (d.flags[0] || 2 * slot >= nb || round >= nb - 1) {
    if (tid == 0) d.pair_rot[slot] = 0;
    return;
  }
  int P, Q;
  pair_of(nb, round, slot, P, Q);
  const int ld = d.ld;
  const double floor_abs = kAbsFloor * (*d.scale);
  const double tol_out = d.tol;

  for (int e = tid; e < JP * JP; e += 256) {
    const int i = e / JP, j = e % JP;
    const int gi = i < JB ? P * JB + i : Q * JB + (i - JB);
    const int gj = j < JB ? P * JB + j : Q * JB + (j - JB);
    S[i][j] = d.G[(int64_t)gi * ld + gj];
    Jm[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) need = 0;
  __syncthreads();
  {
    int mine = 0;
    for (int e = tid; e < JP * JP; e += 256) {
      const int i = e / JP, j = e % JP;
      if (i < j) {
        const double a2 = cabs2(S[i][j]);
        const double dd = fabs(S[i][i].x * S[j][j].x);
        if (a2 > tol_out * tol_out * dd && a2 > floor_abs * floor_abs) mine = 1;
      }
    }
    if (mine) need = 1;
  }
  __syncthreads();
  if (!need) {
    if (tid == 0) d.pair_rot[slot] = 0;
    return;
  }

  for (int sweep = 0; sweep < 12; ++sweep) {
    if (sweep > 0) {
      __syncthreads();
      if (tid == 0) need = 0;
      __syncthreads();
      int mine = 0;
      for (int e = tid; e < JP * JP; e += 256) {
        const int i = e / JP, j = e % JP;
        if (i < j) {
          const double a2 = cabs2(S[i][j]);
          const double dd = fabs(S[i][i].x * S[j][j].x);
          if (a2 > kTolIn * kTolIn * dd && a2 > floor_abs * floor_abs) mine = 1;
        }
      }
      if (mine) need = 1;
      __syncthreads();
      if (!need) break;
    }
    for (int r = 0; r < JP - 1; ++r) {
      if (tid < JP / 2) {
        int a, b;
        pair64(r, tid, a, b);
        rp[tid] = a;
        rq[tid] = b;
        const double sa = S[a][a].x, sd = S[b][b].x;
        const double2 c = S[a][b];
        const double g = sqrt(cabs2(c));
        double2 j00 = make_double2(1, 0), j01 = make_double2(0, 0), j10 = make_double2(0, 0),
                j11 = make_double2(1, 0);
        if (g > floor_abs && g * g > kTolIn * kTolIn * fabs(sa * sd)) {
          // J2 = diag(e, 1) [[cs, sn], [-sn, cs]] with e = c/|c| zeroes S_ab
          const double ex = c.x / g, ey = c.y / g;
          const double zeta = (sd - sa) / (2.0 * g);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
          j00 = make_double2(ex * cs, ey * cs);
          j01 = make_double2(ex * sn, ey * sn);
          j10 = make_double2(-sn, 0.0);
          j11 = make_double2(cs, 0.0);
        }
        rot[tid][0] = j00;
        rot[tid][1] = j01;
        rot[tid][2] = j10;
        rot[tid][3] = j11;
      }
      __syncthreads();
      // S <- J^H S J on 2x2 blocks (row slot ra, column slot cb), one owner each
      for (int blk = tid; blk < (JP / 2) * (JP / 2); blk += 256) {
        const int ra = blk / (JP / 2), cb = blk % (JP / 2);
        const int pa = rp[ra], qa = rq[ra], pb = rp[cb], qb = rq[cb];
        const double2 m00 = S[pa][pb], m01 = S[pa][qb], m10 = S[qa][pb], m11 = S[qa][qb];
        const double2 c00 = rot[cb][0], c01 = rot[cb][1], c10 = rot[cb][2], c11 = rot[cb][3];
        // T = M * Jc
        const double2 t00 = cadd(cmul(m00, c00), cmul(m01, c10));
        const double2 t01 = cadd(cmul(m00, c01), cmul(m01, c11));
        const double2 t10 = cadd(cmul(m10, c00), cmul(m11, c10));
        const double2 t11 = cadd(cmul(m10, c01), cmul(m11, c11));
        const double2 r00 = rot[ra][0], r01 = rot[ra][1], r10 = rot[ra][2], r11 = rot[ra][3];
        // M' = Jr^H T
        double2 n00 = cadd(cmulc(r00, t00), cmulc(r10, t10));
        double2 n01 = cadd(cmulc(r00, t01), cmulc(r10, t11));
        double2 n10 = cadd(cmulc(r01, t00), cmulc(r11, t10));
        double2 n11 = cadd(cmulc(r01, t01), cmulc(r11, t11));
        if (ra == cb) {
          n00.y = 0.0;
          n11.y = 0.0;
          n01 = make_double2(0.0, 0.0);
          n10 = make_double2(0.0, 0.0);
        }
        S[pa][pb] = n00;
        S[pa][qb] = n01;
        S[qa][pb] = n10;
        S[qa][qb] = n11;
      }
      // Jm <- Jm * J (columns pb, qb of every row)
      for (int e = tid; e < JP * (JP / 2); e += 256) {
        const int row = e / (JP / 2), cb = e % (JP / 2);
        const int pb = rp[cb], qb = rq[cb];
        const double2 x = Jm[row][pb], y = Jm[row][qb];
        Jm[row][pb] = cadd(cmul(x, rot[cb][0]), cmul(y, rot[cb][2]));
        Jm[row][qb] = cadd(cmul(x, rot[cb][1]), cmul(y, rot[cb][3]));
      }
      __syncthreads();
    }
  }
  double2* Jout = d.J + (int64_t)slot * JP * JP;
  for (int e = tid; e < JP * JP; e += 256) Jout[e] = Jm[e / JP][e % JP];
  if (tid == 0) {
    d.pair_rot[slot] = 1;
    d.flags[1] = 1;
  }
}

// ------------------------------------------------------ apply rotations --
// Tile products on the FP64 matrix cores: each of the four wavefronts owns a
// 32x32 quadrant of the 64x64 output (2x2 MFMA blocks of 16x16).
struct TileAcc {
  CAcc<double> a[2][2];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) a[i][j].clear();
  }
};

// acc += As * Bs over a k-slice of 16 (As[k][m], Bs[k][n] in LDS)
__device__ __forceinline__ void tile_mma16(TileAcc& acc, double2 (*As)[JP], double2 (*Bs)[JP],
                                           int lane, int wm, int wn) {
#pragma unroll
  for (int ks = 0; ks < 16; ks += 4) {
    const int kr = ks + (lane >> 4), cl = lane & 15;
    const double2 a0 = As[kr][wm * 32 + cl], a1 = As[kr][wm * 32 + 16 + cl];
    const double2 b0 = Bs[kr][wn * 32 + cl], b1 = Bs[kr][wn * 32 + 16 + cl];
    acc.a[0][0].mac(a0.x, a0.y, b0.x, b0.y);
    acc.a[0][1].mac(a0.x, a0.y, b1.x, b1.y);
    acc.a[1][0].mac(a1.x, a1.y, b0.x, b0.y);
    acc.a[1][1].mac(a1.x, a1.y, b1.x, b1.y);
  }
}

__global__ __launch_bounds__(256) void eig_update_kernel(const EigDesc* __restrict__ descs,
                                                         const int* __restrict__ base, int nprob,
                                                         int round) {
  __shared__ double2 As[16][JP];
  __shared__ double2 Bs[16][JP];
  __shared__ double2 Tt[JP][JP + 1];

  const int p = find_problem(base, nprob, blockIdx.x);
  const EigDesc& d = descs[p];
  if (d.flags[0]) return;
  const int n = dim_value(d.n);
  const int nb = nblocks_of(n);
  const int npair = nb / 2, npair_max = d.nb_max / 2;
  int t = blockIdx.x - base[p];
  const int ld = d.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;

  bool is_g;
  int ti, tj, rb = 0;
  if (t < npair_max * npair_max) {
    is_g = true;
    ti = t / npair_max;
    tj = t % npair_max;
    if (ti >= npair || tj >= npair || ti > tj) return;
  } else {
    t -= npair_max * npair_max;
    is_g = false;
    rb = t / npair_max;
    tj = t % npair_max;
    ti = 0;
    if (rb >= npair || tj >= npair) return;
  }
  const bool roti = is_g && d.pair_rot[ti];
  const bool rotj = d.pair_rot[tj];
  if (!roti && !rotj) return;

  int Pi = 0, Qi = 0, Pj, Qj;
  pair_of(nb, round, tj, Pj, Qj);
  if (is_g) pair_of(nb, round, ti, Pi, Qi);
  auto gidx = [](int P, int Q, int i) { return i < JB ? P * JB + i : Q * JB + (i - JB); };
  const double2* Ji = d.J + (int64_t)ti * JP * JP;
  const double2* Jj = d.J + (int64_t)tj * JP * JP;
  double2* Mat = is_g ? d.G : d.V;

  // ---- step 1: T = M_tile * Jj  (or M_tile when Jj = I)
  TileAcc acc;
  acc.clear();
  if (rotj) {
    for (int k0 = 0; k0 < JP; k0 += 16) {
      {
        const int m = tid >> 2, k4 = (tid & 3) * 4;
        const int grow = is_g ? gidx(Pi, Qi, m) : rb * JP + m;
#pragma unroll
        for (int i = 0; i < 4; ++i) As[k4 + i][m] = Mat[(int64_t)grow * ld + gidx(Pj, Qj, k0 + k4 + i)];
        const int kk = tid >> 4, n4 = (tid & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) Bs[kk][n4 + i] = Jj[(k0 + kk) * JP + n4 + i];
      }
      __syncthreads();
      tile_mma16(acc, As, Bs, lane, wm, wn);
      __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = wm * 32 + bi * 16 + Mfma<double>::row(lane, r);
          const int c = wn * 32 + bj * 16 + (lane & 15);
          Tt[m][c] = make_double2(acc.a[bi][bj].re[r], acc.a[bi][bj].im[r]);
        }
  } else {
    for (int e = tid; e < JP * JP; e += 256) {
      const int m = e / JP, c = e % JP;
      const int grow = is_g ? gidx(Pi, Qi, m) : rb * JP + m;
      Tt[m][c] = Mat[(int64_t)grow * ld + gidx(Pj, Qj, c)];
    }
  }
  __syncthreads();

  if (!is_g) {
    for (int e = tid; e < JP * JP; e += 256) {
      const int m = e / JP, c = e % JP;
      d.V[(int64_t)(rb * JP + m) * ld + gidx(Pj, Qj, c)] = Tt[m][c];
    }
    return;
  }

  // ---- step 2: out = Ji^H * T
  if (roti) {
    acc.clear();
    for (int k0 = 0; k0 < JP; k0 += 16) {
      {
        const int kk = tid >> 4, m4 = (tid & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double2 v = Ji[(k0 + kk) * JP + m4 + i];  // (Ji^H)[m][k] = conj(Ji[k][m])
          As[kk][m4 + i] = make_double2(v.x, -v.y);
          Bs[kk][m4 + i] = Tt[k0 + kk][m4 + i];
        }
      }
      __syncthreads();
      tile_mma16(acc, As, Bs, lane, wm, wn);
      __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = wm * 32 + bi * 16 + Mfma<double>::row(lane, r);
          const int c = wn * 32 + bj * 16 + (lane & 15);
          Tt[m][c] = make_double2(acc.a[bi][bj].re[r], acc.a[bi][bj].im[r]);
        }
    __syncthreads();
  }
  for (int e = tid; e < JP * JP; e += 256) {
    const int m = e / JP, c = e % JP;
    const int gr = gidx(Pi, Qi, m), gc = gidx(Pj, Qj, c);
    const double2 v = Tt[m][c];
    d.G[(int64_t)gr * ld + gc] = v;
    if (ti != tj) d.G[(int64_t)gc * ld + gr] = make_double2(v.x, -v.y);
  }
}

__global__ void eig_sweep_end_kernel(const EigDesc* __restrict__ descs, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const EigDesc& d = descs[p];
  if (!d.flags[0]) {
    d.flags[0] = d.flags[1] ? 0 : 1;
    d.flags[1] = 0;
  }
}

}  // namespace

hipError_t launch_eig_init(const EigDesc* d, int nprob, int ld_max, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  dim3 grid(min(ld_max, 256), nprob);
  eig_init_kernel<<<grid, 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_eig_pairs(const EigDesc* d, const int* d_base, int nprob, int blocks, int round,
                            hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  eig_pairs_kernel<<<blocks, 256, 0, s>>>(d, d_base, nprob, round);
  return hipGetLastError();
}

hipError_t launch_eig_update(const EigDesc* d, const int* d_base, int nprob, int blocks, int round,
                             hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  eig_update_kernel<<<blocks, 256, 0, s>>>(d, d_base, nprob, round);
  return hipGetLastError();
}

hipError_t launch_eig_sweep_end(const EigDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  eig_sweep_end_kernel<<<(nprob + 63) / 64, 64, 0, s>>>(d, nprob);
  return hipGetLastError();
}

}  // namespace ctebd
