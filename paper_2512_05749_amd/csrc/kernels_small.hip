// Small (r x r, r <= 512) FP64 kernels: blocked Cholesky with the inverse of
// the factor, and the Rayleigh-Ritz SVD by block one-sided Jacobi.  The
// matrices live in global memory (L2-resident at these sizes) and are worked
// on in 64 x 64 tiles staged in LDS; tile products use the FP64 MFMA.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int TS = 64;        // tile size
constexpr int TP = TS + 1;    // padded LDS row (doubles)
constexpr int NTH = 1024;     // threads per workgroup (16 waves)

// ---- 64 x 64 tile helpers for a 1024-thread workgroup -----------------------

__device__ __forceinline__ void tile_load(double (*T)[TP], const double* __restrict__ M, int ld, int bi, int bj) {
  for (int e = threadIdx.x; e < TS * TS; e += NTH) {
    const int i = e >> 6, j = e & 63;
    T[i][j] = M[(int64_t)(bi * TS + i) * ld + bj * TS + j];
  }
}

__device__ __forceinline__ void tile_store(double* __restrict__ M, int ld, int bi, int bj, const double (*T)[TP],
                                           double scale = 1.0) {
  for (int e = threadIdx.x; e < TS * TS; e += NTH) {
    const int i = e >> 6, j = e & 63;
    M[(int64_t)(bi * TS + i) * ld + bj * TS + j] = scale * T[i][j];
  }
}

__device__ __forceinline__ void tile_fill(double* __restrict__ M, int ld, int bi, int bj, double diag, double off) {
  for (int e = threadIdx.x; e < TS * TS; e += NTH) {
    const int i = e >> 6, j = e & 63;
    M[(int64_t)(bi * TS + i) * ld + bj * TS + j] = (i == j) ? diag : off;
  }
}

// acc += op(A) * B for the 16 x 16 output block of this wave (block (w/4, w%4)).
// TN: sum_k A[k][i] B[k][j];  NN: sum_k A[i][k] B[k][j].
template <bool TN>
__device__ __forceinline__ f64x4 tile_mma(f64x4 acc, const double (*A)[TP], const double (*B)[TP]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int bi = w >> 2, bj = w & 3, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < TS / 4; ++kk) {
    const int k = kk * 4 + lk;
    const double a = TN ? A[k][bi * 16 + li] : A[bi * 16 + li][k];
    const double b = B[k][bj * 16 + li];
    acc = mfma16x16x4d(a, b, acc);
  }
  return acc;
}

__device__ __forceinline__ void acc_to_tile(double (*T)[TP], f64x4 acc, double scale) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int bi = w >> 2, bj = w & 3, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) T[bi * 16 + 4 * v + lk][bj * 16 + li] = scale * acc[v];
}

__device__ __forceinline__ f64x4 tile_to_acc(const double (*T)[TP]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int bi = w >> 2, bj = w & 3, li = lane & 15, lk = lane >> 4;
  f64x4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = T[bi * 16 + 4 * v + lk][bj * 16 + li];
  return acc;
}
}  // namespace

// ---------------------------------------------------------------------------
// Cholesky G = R^T R (R upper, positive diagonal) and R^{-1}, both rp x rp
// row-major; rp a multiple of 64 (padding rows/columns of G are identity).
// One workgroup.  G is overwritten (trailing updates).  A pivot d_k with
// !(d_k > rp * eps * G_kk) is a breakdown (NaN: non-finite input).
//
// Blocked right-looking over 64-wide block columns.  Each 64 x 64 diagonal
// tile is factored by a single wavefront (lane j owns column j; no workgroup
// barriers inside), its triangular inverse is formed one column per
// wavefront (lanes = rows), and the panel and trailing updates are 64 x 64 x 64
// tile products on the FP64 MFMA by all 16 wavefronts.
//
// mode 0 (first CholeskyQR round) also computes the condition bound
// kappa_F = ||R D^-1||_F ||D R^-1||_F with D = diag(G)^(1/2), an upper bound
// on the 2-norm condition number of the column-equilibrated input, and sets
// st->round2 = (kappa_F > kappa_round2): one round leaves an orthogonality
// error of order eps * kappa^2, so a second round is run only when that is
// not negligible.  mode 1 (the gated second round) writes identity factors
// when st->round2 is 0.  mode 2 is a plain factorisation.
// Dynamic LDS: 4 tiles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTH) void k_cholinv(double* __restrict__ G, int rp, int r, double* __restrict__ R,
                                                 double* __restrict__ Ri, DevStatus* st, int mode,
                                                 double kappa_round2) {
  if (failed(st)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (mode == 1 && *reinterpret_cast<volatile int*>(&st->round2) == 0) {
    for (int64_t e = tid; e < (int64_t)rp * rp; e += NTH) {
      const double v = ((e / rp) == (e % rp)) ? 1.0 : 0.0;
      R[e] = v;
      Ri[e] = v;
    }
    return;
  }
  extern __shared__ double smem[];
  double(*T0)[TP] = reinterpret_cast<double(*)[TP]>(smem);
  double(*T1)[TP] = reinterpret_cast<double(*)[TP]>(smem + TS * TP);
  double(*T2)[TP] = reinterpret_cast<double(*)[TP]>(smem + 2 * TS * TP);
  double(*T3)[TP] = reinterpret_cast<double(*)[TP]>(smem + 3 * TS * TP);
  __shared__ double dorig[512];
  __shared__ double invd[TS];
  __shared__ int err;
  __shared__ double minrel;
  __shared__ double red[2][NTH / 64];
  const int nt = rp / TS;
  const double tiny = (double)rp * 2.220446049250313e-16;
  for (int i = tid; i < rp; i += NTH) dorig[i] = G[(int64_t)i * rp + i];
  if (tid == 0) {
    err = 0;
    minrel = 1.0;
  }
  for (int bi = 1; bi < nt; ++bi)
    for (int bj = 0; bj < bi; ++bj) {
      tile_fill(R, rp, bi, bj, 0.0, 0.0);
      tile_fill(Ri, rp, bi, bj, 0.0, 0.0);
    }
  __syncthreads();

  for (int kb = 0; kb < nt; ++kb) {
    tile_load(T0, G, rp, kb, kb);
    __syncthreads();
    if (wv == 0) {
      // right-looking factorisation of the diagonal tile, lane j = column j
      const int j = lane;
      double mrel = 1.0;
      int bad = 0;
      for (int k = 0; k < TS; ++k) {
        const double d = T0[k][k];
        const double d0 = dorig[kb * TS + k];
        if (!(d > tiny * d0)) {
          bad = isnan(d) ? ST_NONFINITE : ST_BREAKDOWN;
          break;
        }
        const double piv = sqrt(d);
        mrel = fmin(mrel, sqrt(d / d0));
        const double rkj = (j > k) ? T0[k][j] / piv : piv;
        __builtin_amdgcn_wave_barrier();
        if (j >= k) T0[k][j] = rkj;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (j > k)
          for (int i = k + 1; i <= j; ++i) T0[i][j] -= T0[k][i] * rkj;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      if (lane == 0) {
        if (bad) err = bad;
        if (mrel < minrel) minrel = mrel;
      }
    }
    __syncthreads();
    if (err) break;
    for (int e = tid; e < TS * TS; e += NTH) {
      const int i = e >> 6, j = e & 63;
      if (i > j) T0[i][j] = 0.0;
    }
    if (tid < TS) invd[tid] = 1.0 / T0[tid][tid];
    __syncthreads();
    // inverse of the triangular tile: column j by back substitution, one
    // wavefront per column (lanes = rows)
    for (int j = wv; j < TS; j += NTH / 64) {
      double b = (lane == j) ? 1.0 : 0.0, x = 0.0;
      for (int l = j; l >= 0; --l) {
        const double xl = __shfl(b, l, 64) * invd[l];
        if (lane == l) x = xl;
        if (lane < l) b -= T0[lane][l] * xl;
      }
      T1[lane][j] = (lane <= j) ? x : 0.0;
    }
    __syncthreads();
    tile_store(R, rp, kb, kb, T0);
    tile_store(Ri, rp, kb, kb, T1);
    // panel: R[kb][j] = R_kk^{-T} G[kb][j]
    for (int j = kb + 1; j < nt; ++j) {
      tile_load(T2, G, rp, kb, j);
      __syncthreads();
      f64x4 acc = tile_mma<true>(f64x4{0}, T1, T2);
      acc_to_tile(T3, acc, 1.0);
      __syncthreads();
      tile_store(R, rp, kb, j, T3);
      __syncthreads();
    }
    __syncthreads();
    // trailing update: G[i][j] -= R[kb][i]^T R[kb][j], kb < i <= j
    for (int i = kb + 1; i < nt; ++i) {
      tile_load(T2, R, rp, kb, i);
      for (int j = i; j < nt; ++j) {
        if (j != i) tile_load(T3, R, rp, kb, j);
        tile_load(T0, G, rp, i, j);
        __syncthreads();
        f64x4 acc = tile_to_acc(T0);
        acc = tile_mma<true>(-acc, T2, j == i ? T2 : T3);
        __syncthreads();
        acc_to_tile(T0, acc, -1.0);
        __syncthreads();
        tile_store(G, rp, i, j, T0);
        __syncthreads();
      }
    }
    __syncthreads();
  }
  if (err) {
    if (tid == 0) raise_error(st, err);
    return;
  }
  // off-diagonal tiles of R^{-1}: Ri[i][j] = -Ri[i][i] * sum_{k=i+1..j} R[i][k] Ri[k][j]
  for (int j = 1; j < nt; ++j) {
    for (int i = j - 1; i >= 0; --i) {
      f64x4 acc = f64x4{0};
      for (int k = i + 1; k <= j; ++k) {
        tile_load(T0, R, rp, i, k);
        tile_load(T1, Ri, rp, k, j);
        __syncthreads();
        acc = tile_mma<false>(acc, T0, T1);
        __syncthreads();
      }
      acc_to_tile(T2, acc, 1.0);
      tile_load(T0, Ri, rp, i, i);
      __syncthreads();
      f64x4 acc2 = tile_mma<false>(f64x4{0}, T0, T2);
      acc_to_tile(T3, acc2, -1.0);
      __syncthreads();
      tile_store(Ri, rp, i, j, T3);
      __syncthreads();
    }
  }
  if (mode == 0) {
    // kappa_F over the real r x r block
    double s1 = 0.0, s2 = 0.0;
    for (int64_t e = tid; e < (int64_t)rp * rp; e += NTH) {
      const int i = (int)(e / rp), j = (int)(e % rp);
      if (i <= j && j < r) {
        const double a = R[e] / sqrt(dorig[j]);
        const double b = Ri[e] * sqrt(dorig[i]);
        s1 += a * a;
        s2 += b * b;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s1 += __shfl_xor(s1, o, 64);
      s2 += __shfl_xor(s2, o, 64);
    }
    if (lane == 0) {
      red[0][wv] = s1;
      red[1][wv] = s2;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NTH / 64; ++w) {
        a += red[0][w];
        b += red[1][w];
      }
      const double kap = sqrt(a * b);
      const int need = !(kap <= kappa_round2);
      st->round2 = need;
      if (need) st->round2_count += 1;
      if (kap > st->kappa_max) st->kappa_max = kap;
    }
  }
  if (tid == 0) {
    st->chol_count += 1;
    if (minrel < st->min_rel_pivot) st->min_rel_pivot = minrel;
  }
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz SVD of C (r x r) by block one-sided Jacobi.
//   prep: Bc (column-major C, i.e. column j contiguous) <- C with zero padding,
//         Pc <- I, scal[0] <- ||C||_F^2.  C is given as its transpose Ct
//         (rp x rp row-major, so row j of Ct is column j of C).
//   round: nb/2 workgroups; workgroup t takes the block pair of round `rd` of
//         the round-robin over nb = rp/32 column blocks, forms the 64 x 64
//         Gram of those columns, diagonalises it by cyclic Jacobi in LDS and
//         rotates the 64 columns of Bc and Pc by the result.
//   check: after every sweep; marks convergence when no pair rotated.  A pair
//         counts as orthogonal when its cosine is <= tol or its Gram entry is
//         <= 64 eps ||C||_F^2.
//   final: sigma_j = ||c_j||, sorted descending (stable), P permuted to match.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTH) void k_jacobi_prep(const double* __restrict__ Ct, int rp, int r,
                                                     double* __restrict__ Bc, double* __restrict__ Pc,
                                                     double* __restrict__ scal, DevStatus* st) {
  if (failed(st)) return;
  __shared__ double red[NTH];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)rp * rp; e += NTH) {
    const int j = (int)(e / rp), i = (int)(e % rp);
    const double v = (j < r && i < r) ? Ct[e] : 0.0;
    Bc[e] = v;
    Pc[e] = (i == j) ? 1.0 : 0.0;
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NTH / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[0] = red[0];
    st->jacobi_done = 0;
    st->jacobi_sweeps = 0;
    st->jacobi_cosine = 0;
  }
}

__global__ __launch_bounds__(NTH) void k_jacobi_round(double* __restrict__ Bc, double* __restrict__ Pc, int rp,
                                                      int rd, double tol, const double* __restrict__ scal,
                                                      double* __restrict__ cosbuf, DevStatus* st) {
  if (failed(st) || *reinterpret_cast<volatile int*>(&st->jacobi_done)) return;
  extern __shared__ double smem[];
  double(*Hs)[TP] = reinterpret_cast<double(*)[TP]>(smem);
  double(*Js)[TP] = reinterpret_cast<double(*)[TP]>(smem + TS * TP);
  double(*Xs)[TP] = reinterpret_cast<double(*)[TP]>(smem + 2 * TS * TP);
  __shared__ int colidx[TS];
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ int rotated;
  __shared__ double red[NTH / 64];
  const int tid = threadIdx.x;
  const int nb = rp / 32;
  int bI, bJ;
  rr_pair(nb, rd, blockIdx.x, bI, bJ);
  if (tid < TS) colidx[tid] = (tid < 32) ? bI * 32 + tid : bJ * 32 + (tid - 32);
  const double floor = 4.93e-32 * scal[0];  // (eps * ||C||_F)^2
  // off-diagonal Gram entries below 64 eps ||C||_F^2 are at the rounding level
  // of the Gram itself and are not rotated (absolute part of the criterion)
  const double absfloor = 64.0 * 2.220446049250313e-16 * scal[0];
  __syncthreads();

  // H = X^T X over the rows of the 64 selected columns
  f64x4 acc = f64x4{0};
  for (int k0 = 0; k0 < rp; k0 += TS) {
    for (int e = tid; e < TS * TS; e += NTH) {
      const int c = e >> 6, k = e & 63;
      Xs[k][c] = Bc[(int64_t)colidx[c] * rp + k0 + k];
    }
    __syncthreads();
    acc = tile_mma<true>(acc, Xs, Xs);
    __syncthreads();
  }
  acc_to_tile(Hs, acc, 1.0);
  for (int e = tid; e < TS * TS; e += NTH) Js[e >> 6][e & 63] = ((e >> 6) == (e & 63)) ? 1.0 : 0.0;
  __syncthreads();

  // largest cosine between any two of the 64 columns (both blocks and across)
  double cmax = 0.0;
  for (int e = tid; e < TS * TS; e += NTH) {
    const int p = e >> 6, q = e & 63;
    if (p < q) {
      const double a = Hs[p][p], d = Hs[q][q];
      if (a > floor && d > floor && fabs(Hs[p][q]) > absfloor) cmax = fmax(cmax, fabs(Hs[p][q]) / sqrt(a * d));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = cmax;
  __syncthreads();
  if (tid == 0) {
    double c = 0.0;
    for (int i = 0; i < NTH / 64; ++i) c = fmax(c, red[i]);
    cosbuf[blockIdx.x] = c;
    red[0] = c;
  }
  __syncthreads();
  if (!(red[0] > tol)) return;

  // cyclic Jacobi on the 64 x 64 Gram, accumulating the rotation in Js.  Per
  // round: the 32 rotation parameters, then every thread transforms one 2 x 2
  // block (row pair a, column pair b) of H and two entries of J.
  for (int sweep = 0; sweep < 16; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int ird = 0; ird < TS - 1; ++ird) {
      if (tid < 32) {
        int p, q;
        rr_pair(TS, ird, tid, p, q);
        const double a = Hs[p][p], d = Hs[q][q], b = Hs[p][q];
        double c = 1.0, s = 0.0;
        if (a > floor && d > floor && fabs(b) > absfloor && fabs(b) > tol * sqrt(a * d)) {
          const double zeta = (d - a) / (2.0 * b);
          const double az = fabs(zeta);
          const double tt = az > 1e100 ? 0.5 / zeta : (zeta >= 0.0 ? 1.0 : -1.0) / (az + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = c * tt;
          rotated = 1;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      {
        const int a = tid >> 5, b = tid & 31;
        const double sa = sn[a], sb = sn[b];
        if (sa != 0.0 || sb != 0.0) {
          const double ca = cs[a], cb = cs[b];
          const int pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
          const double x11 = Hs[pa][pb], x12 = Hs[pa][qb], x21 = Hs[qa][pb], x22 = Hs[qa][qb];
          const double y11 = ca * x11 - sa * x21, y12 = ca * x12 - sa * x22;
          const double y21 = sa * x11 + ca * x21, y22 = sa * x12 + ca * x22;
          double z11 = cb * y11 - sb * y12, z12 = sb * y11 + cb * y12;
          double z21 = cb * y21 - sb * y22, z22 = sb * y21 + cb * y22;
          if (a == b && sa != 0.0) z12 = z21 = 0.0;
          Hs[pa][pb] = z11;
          Hs[pa][qb] = z12;
          Hs[qa][pb] = z21;
          Hs[qa][qb] = z22;
        }
        for (int e = tid; e < 32 * TS; e += NTH) {
          const int k = e >> 6, row = e & 63;
          const double sk = sn[k];
          if (sk != 0.0) {
            const double ck = cs[k];
            const double xp = Js[row][pp[k]], xq = Js[row][qq[k]];
            Js[row][pp[k]] = ck * xp - sk * xq;
            Js[row][qq[k]] = sk * xp + ck * xq;
          }
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }

  // order the 64 rotated columns by decreasing norm (eigenvalue of the Gram):
  // larger columns move to block I, smaller to block J, which speeds up the
  // block iteration; the permuted rotation goes to Hs.
  __shared__ int rnk[TS];
  if (tid < TS) {
    const double ev = Hs[tid][tid];
    int k = 0;
    for (int c = 0; c < TS; ++c) {
      const double e2 = Hs[c][c];
      k += (e2 > ev) || (e2 == ev && c < tid);
    }
    rnk[tid] = k;
  }
  __syncthreads();
  for (int e = tid; e < TS * TS; e += NTH) {
    const int row = e >> 6, c = e & 63;
    Hs[row][rnk[c]] = Js[row][c];
  }
  __syncthreads();

  // rotate the 64 columns of Bc and of Pc: X <- X J, 64 rows at a time
  for (int which = 0; which < 2; ++which) {
    double* M = which ? Pc : Bc;
    for (int k0 = 0; k0 < rp; k0 += TS) {
      for (int e = tid; e < TS * TS; e += NTH) {
        const int c = e >> 6, k = e & 63;
        Xs[k][c] = M[(int64_t)colidx[c] * rp + k0 + k];
      }
      __syncthreads();
      f64x4 y = tile_mma<false>(f64x4{0}, Xs, Hs);
      const int lane = tid & 63, w = tid >> 6;
      const int bi = w >> 2, bj = w & 3, li = lane & 15, lk = lane >> 4;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = bi * 16 + 4 * v + lk, c = bj * 16 + li;
        M[(int64_t)colidx[c] * rp + k0 + k] = y[v];
      }
      __syncthreads();
    }
  }
}

// After a sweep: converged when the largest cosine seen in the sweep is <= tol.
__global__ void k_jacobi_check(const double* __restrict__ cosbuf, int n, double tol, DevStatus* st) {
  if (failed(st) || st->jacobi_done) return;
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c = fmax(c, cosbuf[i]);
    st->jacobi_sweeps += 1.0;
    st->jacobi_cosine = c;
    if (!(c > tol)) st->jacobi_done = 1;
  }
}

// sigma_j = ||c_j|| sorted descending (ties keep index order); Ps (rp x rp
// row-major) holds the matching columns of P.  One workgroup.
__global__ __launch_bounds__(NTH) void k_jacobi_final(const double* __restrict__ Bc, const double* __restrict__ Pc,
                                                      int rp, int r, double* __restrict__ sig,
                                                      double* __restrict__ Ps, DevStatus* st) {
  if (failed(st)) return;
  __shared__ double nrm[512];
  __shared__ int rank[512];
  const int tid = threadIdx.x;
  for (int j = tid; j < rp; j += NTH) {
    double s = 0.0;
    for (int i = 0; i < rp; ++i) {
      const double v = Bc[(int64_t)j * rp + i];
      s += v * v;
    }
    nrm[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < rp; j += NTH) {
    int k = 0;
    const double sj = nrm[j];
    for (int i = 0; i < rp; ++i) {
      const double si = nrm[i];
      k += (si > sj) || (si == sj && i < j);
    }
    rank[j] = k;
    sig[k] = sj;
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)rp * rp; e += NTH) {
    const int j = (int)(e / rp), i = (int)(e % rp);   // P[i][j] = Pc[j][i]
    Ps[(int64_t)i * rp + rank[j]] = Pc[e];
  }
  if (tid == 0 && st->code == 0 && !st->jacobi_done) st->code = ST_WARN_NOT_CONVERGED;
}

// Ct (rp x rp row-major) = C^T with zero padding; C is r x r row-major.
__global__ void k_transpose_pad(const double* __restrict__ C, int r, int rp, double* __restrict__ Ct) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rp * rp) return;
  const int j = (int)(e / rp), i = (int)(e % rp);
  Ct[e] = (i < r && j < r) ? C[(int64_t)i * r + j] : 0.0;
}

}  // namespace wssr
