// Hermitian eigen-solver for the Gram matrices of the split sweep
// (G = X^H D^2 X, whose eigenpairs give the singular values and right singular
// vectors of D X used by every truncated SVD of arXiv:2502.19289, Sec. II.B).
//
// Method: two-sided cyclic block Jacobi.  The padded matrix is cut into nb
// blocks of JB = 32 rows/columns; a round pairs the blocks (circle method, nb-1
// rounds per sweep) and every pair (P, Q) runs one cyclic sweep of scalar
// Jacobi rotations on its 64x64 subproblem G[P u Q, P u Q] in LDS (eig_pairs,
// one workgroup per pair; a matrix of at most 64 rows is solved completely),
// giving a unitary J_PQ.  The round's rotations are then applied to the whole
// matrix, G <- J^H G J and V <- V J, as 64x64 tile products on the matrix cores
// (eig_update).  A sweep in which no subproblem needed a rotation ends the
// iteration for that matrix.
//
// FP64 throughout (the kernels are written over the real type T and built for
// T = double): the eigenvalues decide the truncation and f_i.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace ctebd {

namespace {

template <typename T>
struct JacobiTol;
template <>
struct JacobiTol<double> {
  static constexpr double inner = 1e-14;     // inner rotation threshold (relative)
  static constexpr double floor = 8.9e-16;   // 2^-50: absolute floor, times trace(G)
};

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

// slot s of round t among the JP indices of a subproblem (circle method)
__device__ __forceinline__ void pair_in(int t, int s, int& p, int& q) {
  if (s == 0) {
    p = t;
    q = JP - 1;
  } else {
    p = (t + s) % (JP - 1);
    q = (t - s + JP - 1) % (JP - 1);
  }
}

template <typename C>
__device__ __forceinline__ C mkc(typename real_of<C>::type x, typename real_of<C>::type y) {
  C r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename C>
__device__ __forceinline__ C tmul(C a, C b) {
  return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__device__ __forceinline__ C tmulc(C a, C b) {  // conj(a) * b
  return mkc<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C>
__device__ __forceinline__ C tadd(C a, C b) {
  return mkc<C>(a.x + b.x, a.y + b.y);
}
template <typename C>
__device__ __forceinline__ typename real_of<C>::type tabs2(C a) {
  return a.x * a.x + a.y * a.y;
}

// ------------------------------------------------------------------ init --
template <typename T>
__global__ __launch_bounds__(256) void eig_init_kernel(const EigDesc* __restrict__ descs) {
  using C = typename cpx_of<T>::type;
  const EigDesc& d = descs[blockIdx.y];
  const int n = dim_value(d.n);
  const int npad = nblocks_of(n) * JB;
  const int ld = d.ld;
  C* Gw = (C*)d.Gw;
  C* Vw = (C*)d.Vw;
  for (int row = blockIdx.x; row < npad; row += gridDim.x) {
    for (int c = threadIdx.x; c < npad; c += blockDim.x) {
      const int64_t e = (int64_t)row * ld + c;
      Vw[e] = mkc<C>(row == c ? (T)1 : (T)0, (T)0);
      if (row >= n || c >= n)
        Gw[e] = mkc<C>((T)0, (T)0);
      else if (sizeof(T) == 4)
        Gw[e] = mkc<C>((T)d.G[e].x, (T)d.G[e].y);
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
// one wavefront per 32x32 subproblem (8 wavefronts for 64x64)
constexpr int EP_THREADS = JP == 32 ? 64 : 512;

template <typename T>
__global__ __launch_bounds__(EP_THREADS) void eig_pairs_kernel(const EigDesc* __restrict__ descs,
                                                               const int* __restrict__ base, int nprob,
                                                               int round) {
  using C = typename cpx_of<T>::type;
  __shared__ C S[JP][JP + 1];
  __shared__ C Jm[JP][JP + 1];
  __shared__ C rot[JP / 2][4];
  __shared__ int rp[JP / 2], rq[JP / 2];
  __shared__ int need;
  __shared__ int act[JP / 2];
  __shared__ int nact[2];

  const int p = find_problem(base, nprob, blockIdx.x);
  const EigDesc& d = descs[p];
  const int slot = blockIdx.x - base[p];
  const int tid = threadIdx.x;
  const int n = dim_value(d.n);
  const int nb = nblocks_of(n);
  if (tid == 0) nact[0] = 0;
  if (d.flags[0] || 2 * slot >= nb || round >= nb - 1) {
    if (tid == 0) d.pair_rot[slot] = 0;
    return;
  }
  int P, Q;
  pair_of(nb, round, slot, P, Q);
  const int ld = d.ld;
  const C* Gw = (const C*)d.Gw;
  // off-diagonal entries below the floor are rounding noise of the Gram matrix
  // itself (its eigenvalues are only accurate to that absolute level)
  const T floor_abs = (T)(JacobiTol<T>::floor * (*d.scale));
  const T tol_out = (T)d.tol;
  const T tol_in = JacobiTol<T>::inner;
  // a single pair covers the whole matrix: solve it completely here
  const int max_inner = (nb == 2) ? 30 : 1;

  for (int e = tid; e < JP * JP; e += EP_THREADS) {
    const int i = e / JP, j = e % JP;
    const int gi = i < JB ? P * JB + i : Q * JB + (i - JB);
    const int gj = j < JB ? P * JB + j : Q * JB + (j - JB);
    S[i][j] = Gw[(int64_t)gi * ld + gj];
    Jm[i][j] = mkc<C>(i == j ? (T)1 : (T)0, (T)0);
  }
  int rotated = 0;
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    if (tid == 0) need = 0;
    __syncthreads();
    {
      const T tl = sweep == 0 ? tol_out : tol_in;
      int mine = 0;
      for (int e = tid; e < JP * JP; e += EP_THREADS) {
        const int i = e / JP, j = e % JP;
        if (i < j) {
          const T a2 = tabs2(S[i][j]);
          const T dd = fabs(S[i][i].x * S[j][j].x);
          if (a2 > tl * tl * dd && a2 > floor_abs * floor_abs) mine = 1;
        }
      }
      if (mine) need = 1;
    }
    __syncthreads();
    if (!need) break;
    rotated = 1;
    // real flops of one inner sweep: 63 rounds of 1024 two-sided 2x2 updates
    // (112 flops each) and 2048 column-pair updates of Jm (28 flops each)
    int rounds_done = 0;
    for (int r = 0; r < JP - 1; ++r) {
      if (tid == 0) nact[(r + 1) & 1] = 0;
      if (tid < JP / 2) {
        int a, b;
        pair_in(r, tid, a, b);
        rp[tid] = a;
        rq[tid] = b;
        const T sa = S[a][a].x, sd = S[b][b].x;
        const C c = S[a][b];
        const T g = sqrt(tabs2(c));
        C j00 = mkc<C>(1, 0), j01 = mkc<C>(0, 0), j10 = mkc<C>(0, 0), j11 = mkc<C>(1, 0);
        const bool on = g > floor_abs && g * g > tol_in * tol_in * fabs(sa * sd);
        act[tid] = on ? 1 : 0;
        if (on) atomicAdd(&nact[r & 1], 1);
        if (on) {
          // J2 = diag(e, 1) [[cs, sn], [-sn, cs]] with e = c/|c| zeroes S_ab
          const T ex = c.x / g, ey = c.y / g;
          const T zeta = (sd - sa) / ((T)2 * g);
          const T t = (zeta >= 0 ? (T)1 : (T)-1) / (fabs(zeta) + sqrt((T)1 + zeta * zeta));
          const T cs = (T)1 / sqrt((T)1 + t * t), sn = t * cs;
          j00 = mkc<C>(ex * cs, ey * cs);
          j01 = mkc<C>(ex * sn, ey * sn);
          j10 = mkc<C>(-sn, 0);
          j11 = mkc<C>(cs, 0);
        }
        rot[tid][0] = j00;
        rot[tid][1] = j01;
        rot[tid][2] = j10;
        rot[tid][3] = j11;
      }
      __syncthreads();
      if (nact[r & 1] == 0) continue;  // every rotation of this round is the identity
      ++rounds_done;
      // S <- J^H S J on 2x2 blocks (row slot ra, column slot cb), one owner each
      for (int blk = tid; blk < (JP / 2) * (JP / 2); blk += EP_THREADS) {
        const int ra = blk / (JP / 2), cb = blk % (JP / 2);
        if (!act[ra] && !act[cb]) continue;
        const int pa = rp[ra], qa = rq[ra], pb = rp[cb], qb = rq[cb];
        const C m00 = S[pa][pb], m01 = S[pa][qb], m10 = S[qa][pb], m11 = S[qa][qb];
        const C c00 = rot[cb][0], c01 = rot[cb][1], c10 = rot[cb][2], c11 = rot[cb][3];
        const C t00 = tadd(tmul(m00, c00), tmul(m01, c10));
        const C t01 = tadd(tmul(m00, c01), tmul(m01, c11));
        const C t10 = tadd(tmul(m10, c00), tmul(m11, c10));
        const C t11 = tadd(tmul(m10, c01), tmul(m11, c11));
        const C r00 = rot[ra][0], r01 = rot[ra][1], r10 = rot[ra][2], r11 = rot[ra][3];
        C n00 = tadd(tmulc(r00, t00), tmulc(r10, t10));
        C n01 = tadd(tmulc(r00, t01), tmulc(r10, t11));
        C n10 = tadd(tmulc(r01, t00), tmulc(r11, t10));
        C n11 = tadd(tmulc(r01, t01), tmulc(r11, t11));
        if (ra == cb) {
          n00.y = 0;
          n11.y = 0;
          n01 = mkc<C>(0, 0);
          n10 = mkc<C>(0, 0);
        }
        S[pa][pb] = n00;
        S[pa][qb] = n01;
        S[qa][pb] = n10;
        S[qa][qb] = n11;
      }
      // Jm <- Jm * J (columns pb, qb of every row)
      for (int e = tid; e < JP * (JP / 2); e += EP_THREADS) {
        const int row = e / (JP / 2), cb = e % (JP / 2);
        if (!act[cb]) continue;
        const int pb = rp[cb], qb = rq[cb];
        const C x = Jm[row][pb], y = Jm[row][qb];
        Jm[row][pb] = tadd(tmul(x, rot[cb][0]), tmul(y, rot[cb][2]));
        Jm[row][qb] = tadd(tmul(x, rot[cb][1]), tmul(y, rot[cb][3]));
      }
      __syncthreads();
    }
    if (tid == 0 && d.work)  // real flops: per executed round at most 1024 two-sided
      atomicAdd(d.work + 1, (unsigned long long)rounds_done *
                                ((JP / 2) * (JP / 2) * 112 + JP * (JP / 2) * 28));  // + the Jm updates
  }
  if (!rotated) {
    if (tid == 0) d.pair_rot[slot] = 0;
    return;
  }
  C* Jout = (C*)d.J + (int64_t)slot * JP * JP;
  for (int e = tid; e < JP * JP; e += EP_THREADS) Jout[e] = Jm[e / JP][e % JP];
  if (tid == 0) {
    d.pair_rot[slot] = 1;
    d.flags[1] = 1;
  }
}

// ------------------------------------------------------ apply rotations --
// Tile products on the matrix cores: each wavefront owns a 32x32 quadrant of
// the JP x JP output (2x2 MFMA blocks of 16x16), so a 32x32 tile is one
// wavefront and a 64x64 tile four.  K = JP advances in slices of 16; the next
// slice is fetched into registers while the current one is multiplied.
constexpr int UP_WD = JP / 32;               // wavefronts per tile dimension
constexpr int UP_THREADS = 64 * UP_WD * UP_WD;
constexpr int UP_EPT = 16 * JP / UP_THREADS;  // staged elements per thread and slice
static_assert(JP == 32 || JP == 64, "update tiles are built from 32x32 wavefront quadrants");
template <typename T>
struct TileAcc {
  CAcc<T> a[2][2];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) a[i][j].clear();
  }
};

template <typename T, typename C>
__device__ __forceinline__ void tile_mma16(TileAcc<T>& acc, C (*As)[JP], C (*Bs)[JP], int lane, int wm,
                                           int wn) {
#pragma unroll
  for (int ks = 0; ks < 16; ks += 4) {
    const int kr = ks + (lane >> 4), cl = lane & 15;
    const C a0 = As[kr][wm * 32 + cl], a1 = As[kr][wm * 32 + 16 + cl];
    const C b0 = Bs[kr][wn * 32 + cl], b1 = Bs[kr][wn * 32 + 16 + cl];
    acc.a[0][0].mac(a0.x, a0.y, b0.x, b0.y);
    acc.a[0][1].mac(a0.x, a0.y, b1.x, b1.y);
    acc.a[1][0].mac(a1.x, a1.y, b0.x, b0.y);
    acc.a[1][1].mac(a1.x, a1.y, b1.x, b1.y);
  }
}

template <typename T, typename C>
__device__ __forceinline__ void acc_to_lds(const TileAcc<T>& acc, C (*Tt)[JP + 1], int lane, int wm, int wn) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = wm * 32 + bi * 16 + Mfma<T>::row(lane, r);
        const int c = wn * 32 + bj * 16 + (lane & 15);
        Tt[m][c] = mkc<C>(acc.a[bi][bj].re[r], acc.a[bi][bj].im[r]);
      }
}

template <typename T>
__global__ __launch_bounds__(UP_THREADS) void eig_update_kernel(const EigDesc* __restrict__ descs,
                                                         const int* __restrict__ base, int nprob,
                                                         int round) {
  using C = typename cpx_of<T>::type;
  __shared__ C As[16][JP];
  __shared__ C Bs[16][JP];
  __shared__ C Tt[JP][JP + 1];

  const int p = find_problem(base, nprob, blockIdx.x);
  const EigDesc& d = descs[p];
  if (d.flags[0]) return;
  const int n = dim_value(d.n);
  const int nb = nblocks_of(n);
  const int npair = nb / 2, npair_max = d.nb_max / 2;
  int t = blockIdx.x - base[p];
  const int ld = d.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave / UP_WD, wn = wave % UP_WD;

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
  if (tid == 0 && d.work)  // executed complex MACs of this tile, for the roofline
    atomicAdd(d.work, (unsigned long long)((is_g ? (int)roti + (int)rotj : 1) * JP * JP * JP));

  int Pi = 0, Qi = 0, Pj, Qj;
  pair_of(nb, round, tj, Pj, Qj);
  if (is_g) pair_of(nb, round, ti, Pi, Qi);
  auto gidx = [](int P, int Q, int i) { return i < JB ? P * JB + i : Q * JB + (i - JB); };
  const C* Ji = (const C*)d.J + (int64_t)ti * JP * JP;
  const C* Jj = (const C*)d.J + (int64_t)tj * JP * JP;
  C* Mat = is_g ? (C*)d.Gw : (C*)d.Vw;

  // ---- step 1: T = M_tile * Jj  (or M_tile when Jj = I)
  TileAcc<T> acc;
  acc.clear();
  if (rotj) {
    // A slice: row m of the tile, UP_EPT consecutive k; B slice: row kk of Jj
    const int m = tid / (16 / UP_EPT), k4 = (tid % (16 / UP_EPT)) * UP_EPT;
    const int kk = tid / (JP / UP_EPT), n4 = (tid % (JP / UP_EPT)) * UP_EPT;
    const int64_t grow = (int64_t)(is_g ? gidx(Pi, Qi, m) : rb * JP + m) * ld;
    C ra[UP_EPT], rbv[UP_EPT];
#pragma unroll
    for (int i = 0; i < UP_EPT; ++i) {
      ra[i] = Mat[grow + gidx(Pj, Qj, k4 + i)];
      rbv[i] = Jj[kk * JP + n4 + i];
    }
    for (int k0 = 0; k0 < JP; k0 += 16) {
#pragma unroll
      for (int i = 0; i < UP_EPT; ++i) {
        As[k4 + i][m] = ra[i];
        Bs[kk][n4 + i] = rbv[i];
      }
      __syncthreads();
      if (k0 + 16 < JP) {
#pragma unroll
        for (int i = 0; i < UP_EPT; ++i) {
          ra[i] = Mat[grow + gidx(Pj, Qj, k0 + 16 + k4 + i)];
          rbv[i] = Jj[(k0 + 16 + kk) * JP + n4 + i];
        }
      }
      tile_mma16<T, C>(acc, As, Bs, lane, wm, wn);
      __syncthreads();
    }
    acc_to_lds<T, C>(acc, Tt, lane, wm, wn);
  } else {
    for (int e = tid; e < JP * JP; e += UP_THREADS) {
      const int mm = e / JP, c = e % JP;
      const int grow = is_g ? gidx(Pi, Qi, mm) : rb * JP + mm;
      Tt[mm][c] = Mat[(int64_t)grow * ld + gidx(Pj, Qj, c)];
    }
  }
  __syncthreads();

  if (!is_g) {
    for (int e = tid; e < JP * JP; e += UP_THREADS) {
      const int mm = e / JP, c = e % JP;
      Mat[(int64_t)(rb * JP + mm) * ld + gidx(Pj, Qj, c)] = Tt[mm][c];
    }
    return;
  }

  // ---- step 2: out = Ji^H * T
  if (roti) {
    acc.clear();
    const int kk = tid / (JP / UP_EPT), m4 = (tid % (JP / UP_EPT)) * UP_EPT;
    C rj[UP_EPT];
#pragma unroll
    for (int i = 0; i < UP_EPT; ++i) rj[i] = Ji[kk * JP + m4 + i];
    for (int k0 = 0; k0 < JP; k0 += 16) {
#pragma unroll
      for (int i = 0; i < UP_EPT; ++i) {
        As[kk][m4 + i] = mkc<C>(rj[i].x, -rj[i].y);  // (Ji^H)[m][k] = conj(Ji[k][m])
        Bs[kk][m4 + i] = Tt[k0 + kk][m4 + i];
      }
      __syncthreads();
      if (k0 + 16 < JP) {
#pragma unroll
        for (int i = 0; i < UP_EPT; ++i) rj[i] = Ji[(k0 + 16 + kk) * JP + m4 + i];
      }
      tile_mma16<T, C>(acc, As, Bs, lane, wm, wn);
      __syncthreads();
    }
    acc_to_lds<T, C>(acc, Tt, lane, wm, wn);
    __syncthreads();
  }
  for (int e = tid; e < JP * JP; e += UP_THREADS) {
    const int mm = e / JP, c = e % JP;
    const int gr = gidx(Pi, Qi, mm), gc = gidx(Pj, Qj, c);
    const C v = Tt[mm][c];
    Mat[(int64_t)gr * ld + gc] = v;
    if (ti != tj) Mat[(int64_t)gc * ld + gr] = mkc<C>(v.x, -v.y);
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
  launch(eig_init_kernel<double>, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_eig_pairs(const EigDesc* d, const int* d_base, int nprob, int blocks, int round, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(eig_pairs_kernel<double>, dim3(blocks), dim3(EP_THREADS), 0, s, d, d_base, nprob, round);
  return hipGetLastError();
}

hipError_t launch_eig_update(const EigDesc* d, const int* d_base, int nprob, int blocks, int round, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  launch(eig_update_kernel<double>, dim3(blocks), dim3(UP_THREADS), 0, s, d, d_base, nprob, round);
  return hipGetLastError();
}

hipError_t launch_eig_sweep_end(const EigDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  launch(eig_sweep_end_kernel, dim3((nprob + 63) / 64), dim3(64), 0, s, d, nprob);
  return hipGetLastError();
}

}  // namespace ctebd
