// Small (r x r, r <= 512) FP64 kernels: blocked Cholesky with the inverse of
// the factor, and the set-up and read-out of the Rayleigh-Ritz SVD.  The
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
// Reciprocal and reciprocal square root from the hardware estimates refined
// by two Newton steps (full FP64 accuracy).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}
// x of lane l (l uniform across the wavefront)
__device__ __forceinline__ double bcast_lane(double x, int l) {
  const long long v = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R (R upper, positive diagonal), rp x rp row-major; rp a
// multiple of 64 (padding rows/columns of G are identity).  One workgroup of
// 1024 threads; G is overwritten (trailing updates).  Writes R and its
// transpose Rt (so that columns of R can be read contiguously) and the
// reciprocals of its diagonal (invdiag).  A pivot d_k with
// !(d_k > rp * eps * G_kk) means column k of the input depends on the columns
// before it (NaN: non-finite input).  In a first round (gated = false) such a
// pivot, when G_kk > 0, is replaced by rp * eps * max_j G_jj (j < r: the
// scale of the whole input, so that R^{-1} stays below about
// 1 / sqrt(rp eps) of it and X R^{-1} keeps its accuracy) and counted
// (st->rank_def; st->repl forces the second round): the factor still
// satisfies X = Q1 R with Q1 = X R^{-1} by construction, and the second round
// orthonormalises Q1, whose column k is the rounding residual of x_k scaled
// up -- a direction outside the span of the other columns.  So Q R = X still
// holds exactly, with an orthonormal Q whose extra column completes the basis
// of a rank-deficient X (k_complete first gives that column a direction of
// its own where the data supply none: repeated samples).  In a second round,
// and for a zero or non-finite column, it is a breakdown.  repcol[k] is set to
// 1 for a replaced pivot of a first round (0 otherwise).
//
// Blocked right-looking over 64-wide block columns.  The 64 x 64 diagonal
// tile is factored in LDS in four sub-blocks of 16 rows (one wavefront per
// sub-block, then a workgroup-wide trailing update: two barriers per 16
// columns); its triangular inverse (needed for the panel) is formed one
// column per wavefront by back substitution; the panel and trailing updates
// are 64 x 64 x 64 tile products on the FP64 MFMA.
//
// gated: a second CholeskyQR round; when st->round2 is 0 the kernel does
// nothing (the gated consumers of R and Rt then take the identity instead).
// Dynamic LDS: 4 tiles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTH) void k_chol(double* __restrict__ G, int rp, int r, double* __restrict__ R,
                                              double* __restrict__ Rt, double* __restrict__ gdiag,
                                              double* __restrict__ invdiag, int* __restrict__ repcol, DevStatus* st,
                                              bool gated) {
  if (failed(st)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (gated && *reinterpret_cast<volatile int*>(&st->round2) == 0) return;
  extern __shared__ double smem[];
  double(*T0)[TP] = reinterpret_cast<double(*)[TP]>(smem);
  double(*T1)[TP] = reinterpret_cast<double(*)[TP]>(smem + TS * TP);
  double(*T2)[TP] = reinterpret_cast<double(*)[TP]>(smem + 2 * TS * TP);
  double(*T3)[TP] = reinterpret_cast<double(*)[TP]>(smem + 3 * TS * TP);
  __shared__ double dorig[512];
  __shared__ double invd[TS];
  __shared__ int err, nrep;
  __shared__ double minrel, dmax;
  const int nt = rp / TS;
  const double tiny = (double)rp * 2.220446049250313e-16;
  for (int i = tid; i < rp; i += NTH) {
    dorig[i] = G[(int64_t)i * rp + i];
    gdiag[i] = dorig[i];
    if (!gated) repcol[i] = 0;
  }
  if (tid == 0) {
    err = 0;
    nrep = 0;
    minrel = 1.0;
  }
  __syncthreads();
  // the largest diagonal entry of the r columns of the input: the scale of a
  // replaced pivot
  if (tid < 64) {
    double mx = 0.0;
    for (int i = tid; i < r; i += 64) mx = fmax(mx, G[(int64_t)i * rp + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (tid == 0) dmax = mx;
  }
  for (int bi = 1; bi < nt; ++bi)
    for (int bj = 0; bj < bi; ++bj) {
      tile_fill(R, rp, bi, bj, 0.0, 0.0);
      tile_fill(Rt, rp, bj, bi, 0.0, 0.0);
    }
  __syncthreads();

  for (int kb = 0; kb < nt; ++kb) {
    tile_load(T0, G, rp, kb, kb);
    __syncthreads();
    // factor the diagonal tile in four sub-blocks of 16 rows.  For each,
    // wavefront 0 alone runs the 16 right-looking steps over those rows with
    // lane j holding column j (rows s0..s0+15) in registers; pivots and row
    // entries are broadcast by readlane, so the steps need no barrier.  Then
    // all threads apply the sub-block's 16 rows to the trailing part of the
    // tile.
    for (int s0 = 0; s0 < TS; s0 += 16) {
      if (wv == 0) {
        const int j = lane;
        double col[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) col[i] = T0[s0 + i][j];
        int bad = 0, rep = 0;
        double mr = 1.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          double d = bcast_lane(col[k], s0 + k);
          const double d0 = dorig[kb * TS + s0 + k];
          // a failed pivot is replaced (first round) or recorded and the
          // steps run on (uniform: every lane sees the same d); after a
          // recorded failure the kernel stops after the sub-block
          if (!(d > tiny * d0) && !bad) {
            if (!gated && !isnan(d) && d0 > 0.0 && d0 < INFINITY) {
              d = tiny * dmax;
              ++rep;
              if (j == 0) repcol[kb * TS + s0 + k] = 1;
            } else {
              bad = isnan(d) ? ST_NONFINITE : ST_BREAKDOWN;
            }
          }
          const double ipiv = rsq_nr(d);   // 1/sqrt(d)
          mr = fmin(mr, d / d0);
          col[k] = (j > s0 + k) ? col[k] * ipiv : (j == s0 + k ? d * ipiv : col[k]);
#pragma unroll
          for (int i = k + 1; i < 16; ++i) col[i] -= bcast_lane(col[k], s0 + i) * col[k];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (j >= s0 + i) T0[s0 + i][j] = col[i];
        if (lane == 0) {
          if (bad) err = bad;
          nrep += rep;
          minrel = fmin(minrel, mr);
        }
      }
      __syncthreads();
      if (err) break;
    const int s1 = s0 + 16, w = TS - s1;
      for (int e = tid; e < w * w; e += NTH) {
        const int i = s1 + e / w, j = s1 + e % w;
        if (i <= j) {
          double acc = T0[i][j];
#pragma unroll
          for (int l = 0; l < 16; ++l) acc -= T0[s0 + l][i] * T0[s0 + l][j];
          T0[i][j] = acc;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    if (err) break;
    for (int e = tid; e < TS * TS; e += NTH) {
      const int a = e >> 6, b = e & 63;
      if (a > b) T0[a][b] = 0.0;
    }
    if (tid < TS) {
      invd[tid] = rcp_nr(T0[tid][tid]);
      invdiag[kb * TS + tid] = invd[tid];
    }
    __syncthreads();
    // inverse X of the diagonal tile in 16 x 16 blocks: wavefront w inverts
    // the diagonal block w by back substitution (lane c holds column c in
    // registers), then the blocks at distance d = 1, 2, 3 above the diagonal
    // follow from X_ab = -X_aa sum_{c=a+1..b} T_ac X_cb on the FP64 MFMA,
    // one block per wavefront (its partial sum staged in T2; the LDS
    // accesses of one wavefront take effect in program order).
    for (int e = tid; e < TS * TS; e += NTH) {
      const int a = e >> 6, b = e & 63;
      if ((a >> 4) > (b >> 4)) T1[a][b] = 0.0;
    }
    if (wv < 4 && lane < 16) {
      const int o = 16 * wv, c = lane;
      double x[16];
#pragma unroll
      for (int i = 15; i >= 0; --i) {
        double sacc = (i == c) ? 1.0 : 0.0;
#pragma unroll
        for (int l = i + 1; l < 16; ++l) sacc -= T0[o + i][o + l] * x[l];
        x[i] = sacc * invd[o + i];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) T1[o + i][o + c] = x[i];
    }
    __syncthreads();
    for (int d = 1; d < 4; ++d) {
      if (wv < 4 - d) {
        const int ba = wv, bb = wv + d;
        const int li = lane & 15, lk = lane >> 4;
        f64x4 acc = f64x4{0};
        for (int c = ba + 1; c <= bb; ++c) {
#pragma unroll
          for (int k0 = 0; k0 < 16; k0 += 4)
            acc = mfma16x16x4d(T0[16 * ba + li][16 * c + k0 + lk], T1[16 * c + k0 + lk][16 * bb + li], acc);
        }
        double(*tmp)[TP] = T2 + 16 * wv;   // rows 16 wv .. 16 wv + 15 of T2: this wavefront's scratch
#pragma unroll
        for (int v = 0; v < 4; ++v) tmp[4 * v + lk][li] = acc[v];
        f64x4 out = f64x4{0};
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4)
          out = mfma16x16x4d(T1[16 * ba + li][16 * ba + k0 + lk], tmp[k0 + lk][li], out);
#pragma unroll
        for (int v = 0; v < 4; ++v) T1[16 * ba + 4 * v + lk][16 * bb + li] = -out[v];
      }
      __syncthreads();
    }
    tile_store(R, rp, kb, kb, T0);
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
  // Rt = R^T (upper tiles of R -> lower tiles of Rt)
  for (int bi = 0; bi < nt; ++bi)
    for (int bj = bi; bj < nt; ++bj) {
      tile_load(T0, R, rp, bi, bj);
      __syncthreads();
      for (int e = tid; e < TS * TS; e += NTH) {
        const int a = e >> 6, b = e & 63;
        Rt[(int64_t)(bj * TS + a) * rp + bi * TS + b] = T0[b][a];
      }
      __syncthreads();
    }
  if (tid == 0) {
    st->chol_count += 1;
    const double mr = sqrt(minrel);
    if (mr < st->min_rel_pivot) st->min_rel_pivot = mr;
    if (nrep) {
      st->rank_def += nrep;
      st->repl = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Ri = R^{-1} for the upper triangular R (rp x rp), column-parallel: one
// wavefront per column j solves R x = e_j by back substitution, lanes = rows
// (RPL >= rp/64 rows per lane), reading column l of R as row l of Rt and
// 1 / R_ll from invdiag.  The column entries of the next 8 steps are loaded
// into registers while the current 8 are applied.
// grid: rp / 4 workgroups of 256 threads.  gated as in k_chol.
// ---------------------------------------------------------------------------
template <int RPL>
__global__ __launch_bounds__(256) void k_trinv(const double* __restrict__ Rt, int rp,
                                               const double* __restrict__ invdiag, double* __restrict__ Ri,
                                               const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  constexpr int G = 8;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= rp) return;
  double b[RPL], x[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    b[s] = (s * 64 + lane == j) ? 1.0 : 0.0;
    x[s] = 0.0;
  }
  const int jb = j >> 6;
#pragma unroll
  for (int sb = RPL - 1; sb >= 0; --sb) {
    if (sb > jb) continue;
    const int lstart = (sb == jb) ? (j & 63) : 63;
    double ca[G][RPL], cb[G][RPL], da[G], db[G];
    // entries of column l = sb*64 + ll, ll = g0, g0-1, ..., g0-G+1 (0 past
    // the end and for rows >= l, so that those steps change nothing)
    auto fetch = [&](int g0, double (&c)[G][RPL], double (&d)[G]) __attribute__((always_inline)) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int ll = g0 - g, l = sb * 64 + ll;
        const bool ok = ll >= 0;
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
          const int row = s * 64 + lane;
          c[g][s] = (s <= sb && ok && row < l) ? Rt[(int64_t)l * rp + row] : 0.0;
        }
        d[g] = ok ? invdiag[l] : 0.0;
      }
    };
    auto apply = [&](int g0, const double (&c)[G][RPL], const double (&d)[G]) __attribute__((always_inline)) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int ll = g0 - g;
        if (ll >= 0) {
          const double xl = bcast_lane(b[sb], ll) * d[g];
          if (lane == ll) x[sb] = xl;
#pragma unroll
          for (int s = 0; s < RPL; ++s)
            if (s <= sb) b[s] -= c[g][s] * xl;
        }
      }
    };
    fetch(lstart, ca, da);
    for (int g0 = lstart; g0 >= 0; g0 -= 2 * G) {
      if (g0 - G >= 0) fetch(g0 - G, cb, db);
      apply(g0, ca, da);
      if (g0 - G < 0) break;
      if (g0 - 2 * G >= 0) fetch(g0 - 2 * G, ca, da);
      apply(g0 - G, cb, db);
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s)
    if (s * 64 + lane < rp) Ri[(int64_t)(s * 64 + lane) * rp + j] = x[s];
}

// Condition bound of a first CholeskyQR round from R and R^{-1}:
// kappa_F = ||R D^-1||_F ||D R^-1||_F with D = diag(G)^(1/2) (column norms of
// the input, as saved by k_chol in gdiag), an upper bound on the 2-norm
// condition number of the column-equilibrated input.  One round leaves an
// orthogonality error of order eps * kappa^2, so
// st->round2 = (kappa_F > kappa_round2).
__global__ __launch_bounds__(1024) void k_kappa(const double* __restrict__ gdiag, const double* __restrict__ R,
                                                const double* __restrict__ Ri, int rp, int r, double kappa_round2,
                                                DevStatus* st) {
  if (failed(st)) return;
  __shared__ double red[2][1024 / 64];
  __shared__ double dsq[512], dinv[512];   // sqrt(G_jj) and its reciprocal
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < rp; i += 1024) {
    const double q = sqrt(gdiag[i]);
    dsq[i] = q;
    dinv[i] = 1.0 / q;
  }
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
  const int64_t tot = (int64_t)rp * rp;
#pragma unroll 4
  for (int64_t e = tid; e < tot; e += 1024) {
    const int i = (int)(e / rp), j = (int)(e % rp);
    const double rv = R[e], ri = Ri[e];
    if (i <= j && j < r) {
      const double a = rv * dinv[j];
      const double b = ri * dsq[i];
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
    for (int w = 0; w < 1024 / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    const double kap = sqrt(a * b);
    // a replaced pivot always takes the second round
    const int need = !(kap <= kappa_round2) || st->repl;
    st->repl = 0;
    st->round2 = need;
    if (need) st->round2_count += 1;
    if (kap > st->kappa_max) st->kappa_max = kap;
  }
}

// C = A B for rp x rp row-major FP64 matrices; one wavefront per 16 x 16
// output tile on the FP64 MFMA, operands read straight from global memory
// (L2-resident).  gated: when st->round2 is 0 the product is replaced by a
// copy of A (copy_b = false) or of B (copy_b = true), i.e. the other factor
// is taken as the identity.  grid: rp*rp/256/4 workgroups of 256 threads.
__global__ __launch_bounds__(256) void k_smallgemm(const double* __restrict__ A, const double* __restrict__ B,
                                                   int rp, double* __restrict__ C, const DevStatus* st, bool gated,
                                                   bool copy_b) {
  if (failed(st)) return;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nt16 = rp / 16;
  if (tile >= nt16 * nt16) return;
  const int row0 = (tile / nt16) * 16, col0 = (tile % nt16) * 16;
  const int li = lane & 15, lk = lane >> 4;
  if (gated && *reinterpret_cast<const volatile int*>(&st->round2) == 0) {
    const double* S = copy_b ? B : A;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t o = (int64_t)(row0 + 4 * v + lk) * rp + col0 + li;
      C[o] = S[o];
    }
    return;
  }
  f64x4 acc = f64x4{0};
  for (int k0 = 0; k0 < rp; k0 += 16) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = A[(int64_t)(row0 + li) * rp + k0 + 4 * u + lk];
      b[u] = B[(int64_t)(k0 + 4 * u + lk) * rp + col0 + li];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = mfma16x16x4d(a[u], b[u], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(int64_t)(row0 + 4 * v + lk) * rp + col0 + li] = acc[v];
}

template __global__ void k_trinv<1>(const double*, int, const double*, double*, const DevStatus*, bool);
template __global__ void k_trinv<2>(const double*, int, const double*, double*, const DevStatus*, bool);
template __global__ void k_trinv<4>(const double*, int, const double*, double*, const DevStatus*, bool);
template __global__ void k_trinv<8>(const double*, int, const double*, double*, const DevStatus*, bool);

// ---------------------------------------------------------------------------
// Rayleigh-Ritz SVD of C (r x r) by block one-sided Jacobi (the sweeps are
// k_jacobi_coop in kernels_jacobi.hip).
//   prep: Bc (column-major C, i.e. column j contiguous) <- C with zero padding,
//         Pc <- I, scal[1 + j] <- ||c_j||^2 (the sweep kernel sums them to
//         ||C||_F^2), and the grid-barrier words of the
//         sweep kernel.  C is given as its transpose Ct (rp x rp row-major, so
//         row j of Ct is column j of C).
//   A column pair counts as orthogonal when its cosine is <= tol or its Gram
//   entry is <= 64 eps ||C||_F^2.
//   final: sigma_j = ||c_j||, sorted descending (stable), P permuted to match.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_jacobi_prep(const double* __restrict__ Ct, int rp, int r,
                                                     double* __restrict__ Bc, double* __restrict__ Pc,
                                                     double* __restrict__ scal, unsigned* __restrict__ sync,
                                                     DevStatus* st) {
  // grid: rp / 4 workgroups, one column per wavefront (lanes stride the rows)
  const bool skip = failed(st);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sync[0] = 0u;
    sync[1] = 0u;
    sync[2] = skip ? 1u : 0u;
    if (!skip) {
      st->jacobi_done = 0;
      st->jacobi_sweeps = 0;
      st->jacobi_cosine = 0;
    }
  }
  if (skip) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= rp) return;
  double sq = 0.0;
  for (int i = lane; i < rp; i += 64) {
    const int64_t e = (int64_t)j * rp + i;
    const double v = (j < r && i < r) ? Ct[e] : 0.0;
    Bc[e] = v;
    Pc[e] = (i == j) ? 1.0 : 0.0;
    sq += v * v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if (lane == 0) scal[1 + j] = sq;   // column sums of squares; the sweep kernel adds them up
}

// sigma_j = ||c_j|| sorted descending (ties keep index order); Ps (rp x rp
// row-major) holds the matching columns of P.  One workgroup: the column
// norms one column per wavefront at a time (lanes stride the rows), the
// ranks one thread per column, then the permuted copy.
__global__ __launch_bounds__(NTH) void k_jacobi_final(const double* __restrict__ Bc, const double* __restrict__ Pc,
                                                      int rp, int r, double* __restrict__ sig,
                                                      double* __restrict__ Ps, DevStatus* st) {
  if (failed(st)) return;
  __shared__ double nrm[512];
  __shared__ int src[512];   // src[k] = the column of P that becomes column k of Ps
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = wv; j < rp; j += NTH / 64) {
    double s = 0.0;
    for (int i = lane; i < rp; i += 64) {
      const double v = Bc[(int64_t)j * rp + i];
      s += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) nrm[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < rp; j += NTH) {
    int k = 0;
    const double sj = nrm[j];
    for (int i = 0; i < rp; ++i) {
      const double si = nrm[i];
      k += (si > sj) || (si == sj && i < j);
    }
    src[k] = j;
    sig[k] = sj;
  }
  __syncthreads();
  // Ps[i][k] = P[i][src[k]] = Pc[src[k]][i]: consecutive threads write
  // consecutive k of a row
  for (int64_t e = tid; e < (int64_t)rp * rp; e += NTH) {
    const int i = (int)(e / rp), k = (int)(e % rp);
    Ps[e] = Pc[(int64_t)src[k] * rp + i];
  }
  if (tid == 0 && st->code == 0) {
    if (!st->jacobi_done)
      st->code = ST_WARN_NOT_CONVERGED;
    else if (st->rank_def)
      st->code = ST_WARN_RANK_DEFICIENT;
  }
}

// Completion of a rank-deficient basis, after a first-round Cholesky of
// X^T X that replaced the pivots of the columns k with repcol[k] = 1: x_k +=
// R_kk xi_k with xi_k a pseudo-random unit vector of zero sum (entries +h and
// -h on row pairs 2i, 2i+1, h uniform in [-1, 1) from an integer hash of
// (i, k), scaled by sqrt(3 / rows); a last odd row gets 0).  Then the first
// round's Q1 = X R^{-1} has column k = (old column k) + xi_k: the unit vector
// xi_k plus the rounding residual, which the second round orthonormalises
// against the others.  R stays the factor of the modified X (X = Q1 R by
// construction), so X Tq is orthonormal and R the triangular factor of the
// modified X, whose column k moved by R_kk = sqrt(rp eps) max_j |x_j|.  The
// zero sum keeps the columns of a centred basis centred.
// grid: (kCompleteBlocks, r) workgroups of 256 threads: blockIdx.y is the
// column, and a column that was not replaced leaves at once.
template <typename T>
__global__ __launch_bounds__(256) void k_complete(T* __restrict__ X, int64_t rows, int r, const double* __restrict__ R,
                                                  int rp, const int* __restrict__ repcol, const DevStatus* st) {
  if (failed(st)) return;
  const int k = blockIdx.y;
  if (!repcol[k]) return;
  const double rkk = R[(int64_t)k * rp + k];
  const double amp = sqrt(3.0 / (double)rows);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    const int64_t e = i * r + k;
    const int64_t pair = i >> 1;
    if ((rows & 1) && i == rows - 1) continue;
    // integer hash of (pair, k) (a 32-bit finaliser of multiply-xorshift steps)
    uint32_t hsh = (uint32_t)pair * 0x9E3779B1u ^ (uint32_t)(pair >> 32) * 0x85EBCA77u ^ (uint32_t)k * 0xC2B2AE3Du;
    hsh ^= hsh >> 16;
    hsh *= 0x7FEB352Du;
    hsh ^= hsh >> 15;
    hsh *= 0x846CA68Bu;
    hsh ^= hsh >> 16;
    const double h = ((double)hsh * (1.0 / 4294967296.0)) * 2.0 - 1.0;
    const double xi = ((i & 1) ? -h : h) * amp;
    X[e] = (T)((double)X[e] + rkk * xi);
  }
}
template __global__ void k_complete<float>(float*, int64_t, int, const double*, int, const int*, const DevStatus*);
template __global__ void k_complete<double>(double*, int64_t, int, const double*, int, const int*,
                                            const DevStatus*);

// Ct (rp x rp row-major) = C^T with zero padding; C is r x r row-major.
__global__ void k_transpose_pad(const double* __restrict__ C, int r, int rp, double* __restrict__ Ct) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rp * rp) return;
  const int j = (int)(e / rp), i = (int)(e % rp);
  Ct[e] = (i < r && j < r) ? C[(int64_t)i * r + j] : 0.0;
}

}  // namespace wssr
