// The comparison system of Sec. 3.2 in sample space: MinSR (eq. mT) with the
// SPRING momentum (eq. param:spring), damped.  T = A A^T (N x N) is formed on
// the FP64 MFMA from the stored O (exact products of FP32 or BF16 values,
// FP64 sums), double-centred, factored by a blocked Cholesky and solved by
// blocked triangular solves; the products with O that remain are GEMVs.
//
// Everything here is FP64: T + lambda I has a condition number of order
// ||T|| / lambda, so an FP32 T would put its rounding into delta amplified
// by that much.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int ST = 128;          // output tile of the symmetric products
constexpr int SK = 16;           // K-step
constexpr int SS = ST + 16;      // LDS row stride in doubles

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double bf16d(unsigned short u) { return (double)__uint_as_float((unsigned)u << 16); }

// Four consecutive values p[0..3] (n of them valid, the rest 0) as doubles.
// float: one 16-byte load when vec; BF16: one 8-byte load per plane when vec,
// the value is hi (+ lo at p + pstride); double: two 16-byte loads when vec.
template <int PL>
__device__ __forceinline__ f64x4 ld4(const float* __restrict__ p, int64_t, int n, bool vec) {
  if (vec && n >= 4) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(p);
    return f64x4{(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
  }
  f64x4 v = f64x4{0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (e < n) v[e] = (double)p[e];
  return v;
}
template <int PL>
__device__ __forceinline__ f64x4 ld4(const double* __restrict__ p, int64_t, int n, bool vec) {
  if (vec && n >= 4) {
    const f64x2 a = *reinterpret_cast<const f64x2*>(p), b = *reinterpret_cast<const f64x2*>(p + 2);
    return f64x4{a[0], a[1], b[0], b[1]};
  }
  f64x4 v = f64x4{0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (e < n) v[e] = p[e];
  return v;
}
template <int PL>
__device__ __forceinline__ f64x4 ld4(const unsigned short* __restrict__ p, int64_t pstride, int n, bool vec) {
  f64x4 v = f64x4{0, 0, 0, 0};
  if (vec && n >= 4) {
    const u16x4 h = *reinterpret_cast<const u16x4*>(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = bf16d(h[e]);
    if (PL == 2) {
      const u16x4 l = *reinterpret_cast<const u16x4*>(p + pstride);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += bf16d(l[e]);
    }
    return v;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (e < n) v[e] = bf16d(p[e]) + (PL == 2 ? bf16d(p[e + pstride]) : 0.0);
  return v;
}

__device__ __forceinline__ void pair_of(int pair, int ntile, int& I, int& J) {
  int rem = pair;
  I = 0;
  while (rem >= ntile - I) {
    rem -= ntile - I;
    ++I;
  }
  J = rem + I;
}

// acc += X[rowsI, k] X[rowsJ, k]^T over k in [kbeg, kend): the 128 x 128 tile
// whose rows start at iI and columns at iJ (rows beyond `rows` read as 0).
// 4 waves in 2 x 2, each 64 x 64 = 4 x 4 FP64 MFMA tiles; each K-step
// stages 16 values of the 128 rows of each block in LDS ([k][row]) while the
// next 16 are loaded into registers.
template <typename T, int PL>
__device__ __forceinline__ void sym_tile(const T* __restrict__ X, int64_t ld, int64_t pstride, int64_t rows,
                                         int64_t iI, int64_t iJ, int64_t kbeg, int64_t kend, bool vec,
                                         double (*XI)[SS], double (*XJ)[SS], f64x4 (&acc)[4][4]) {
  const bool diag = iI == iJ;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qi = w >> 1, qj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 pi[2], pj[2];
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int rr = idx >> 2;
      const int64_t gk = k0 + (idx & 3) * 4;
      const int nk = (int)max<int64_t>(0, min<int64_t>(4, kend - gk));
      const int64_t ri = iI + rr, rj = iJ + rr;
      pi[e] = ld4<PL>(X + ri * ld + gk, pstride, ri < rows ? nk : 0, vec);
      if (!diag) pj[e] = ld4<PL>(X + rj * ld + gk, pstride, rj < rows ? nk : 0, vec);
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int rr = idx >> 2, kq = (idx & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) XI[kq + q][rr] = pi[e][q];
      if (!diag) {
#pragma unroll
        for (int q = 0; q < 4; ++q) XJ[kq + q][rr] = pj[e][q];
      }
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += SK) {
    store();
    __syncthreads();
    if (k0 + SK < kend) load(k0 + SK);
    double(*B)[SS] = diag ? XI : XJ;
#pragma unroll
    for (int kk = 0; kk < SK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = XI[k][qi * 64 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = B[k][qj * 64 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4d(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
}
}  // namespace

// ---------------------------------------------------------------------------
// G = O O^T over a K-chunk of the m columns.  grid (npairs, nch): the tile
// pair (I <= J) of 128-row blocks and the chunk.  With part == NULL (one
// chunk) the tile goes straight into G (n x n, both triangles); otherwise to
// part[(chunk * npairs + pair) * 16384 + i * 128 + j].
// ---------------------------------------------------------------------------
template <typename T, int PL>
__global__ __launch_bounds__(256, 2) void k_syrk_partial(const T* __restrict__ O, int64_t ld, int64_t pstride,
                                                         int64_t n, int64_t m, int ntile, int64_t kchunk,
                                                         double* __restrict__ part, double* __restrict__ G, bool vec,
                                                         const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double XI[SK][SS];
  __shared__ double XJ[SK][SS];
  int I, J;
  pair_of(blockIdx.x, ntile, I, J);
  const int npairs = ntile * (ntile + 1) / 2;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk, kend = min<int64_t>(m, kbeg + kchunk);
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0};
  sym_tile<T, PL>(O, ld, pstride, n, (int64_t)I * ST, (int64_t)J * ST, kbeg, kend, vec, XI, XJ, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qi = w >> 1, qj = w & 1, li = lane & 15, lk = lane >> 4;
  double* out = part ? part + ((int64_t)blockIdx.y * npairs + blockIdx.x) * (ST * ST) : nullptr;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = qi * 64 + a * 16 + 4 * v + lk;
        const int j = qj * 64 + b * 16 + li;
        if (out) {
          out[i * ST + j] = acc[a][b][v];
        } else {
          const int64_t gi = (int64_t)I * ST + i, gj = (int64_t)J * ST + j;
          if (gi < n && gj < n) {
            G[gi * n + gj] = acc[a][b][v];
            G[gj * n + gi] = acc[a][b][v];
          }
        }
      }
}

// Sum the chunks of each tile pair in chunk order into G (both triangles).
// grid (npairs, 64), one entry of the 128 x 128 tile per thread.
__global__ __launch_bounds__(256) void k_syrk_reduce(const double* __restrict__ part, int nchunk, int ntile,
                                                     int64_t n, double* __restrict__ G, const DevStatus* st) {
  if (failed(st)) return;
  int I, J;
  pair_of(blockIdx.x, ntile, I, J);
  const int npairs = ntile * (ntile + 1) / 2;
  const int e = blockIdx.y * 256 + threadIdx.x;
  const int i = e / ST, j = e % ST;
  const int64_t gi = (int64_t)I * ST + i, gj = (int64_t)J * ST + j;
  if (gi >= n || gj >= n) return;
  const double* p = part + (int64_t)blockIdx.x * (ST * ST) + e;
  const int64_t stride = (int64_t)npairs * (ST * ST);
  double a0 = 0.0, a1 = 0.0;
  int c = 0;
  for (; c + 1 < nchunk; c += 2) {
    a0 += p[c * stride];
    a1 += p[(c + 1) * stride];
  }
  if (c < nchunk) a0 += p[c * stride];
  G[gi * n + gj] = a0 + a1;
  G[gj * n + gi] = a0 + a1;
}

// rho_i = (1/n) sum_j G[i][j]: one wave per row.
__global__ __launch_bounds__(256) void k_row_mean(const double* __restrict__ G, int64_t n, double* __restrict__ rho,
                                                  const DevStatus* st) {
  if (failed(st)) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s += G[i * n + j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) rho[i] = s / (double)n;
}

// T = (G - rho 1^T - 1 rho^T + tau) * scale + lambda I, in place: the Gram of
// the centred rows (tau = mean of rho).  scale = 1/N gives A A^T.
__global__ __launch_bounds__(256) void k_dcenter(double* __restrict__ G, int64_t n, const double* __restrict__ rho,
                                                 const double* __restrict__ tau, double scale, double lambda,
                                                 const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e / n, j = e % n;
  G[e] = (G[e] - rho[i] - rho[j] + tau[0]) * scale + (i == j ? lambda : 0.0);
}

// ---------------------------------------------------------------------------
// Blocked Cholesky, lower, in place in G (n x n row-major); block nb <= 64.
// Only the lower triangle is read and written.
// ---------------------------------------------------------------------------

// Factor the diagonal block at k0 (nb x nb) in LDS.  One workgroup.
__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                    DevStatus* st) {
  if (failed(st)) return;
  __shared__ double L[64][65];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    L[i][j] = G[(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (t == 0) {
      const double d = L[k][k];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
      } else {
        L[k][k] = sqrt(d);
      }
    }
    __syncthreads();
    if (bad) break;
    const double dk = L[k][k];
    for (int i = k + 1 + t; i < nb; i += 256) L[i][k] /= dk;
    __syncthreads();
    const int w = nb - k - 1;
    for (int e = t; e < w * w; e += 256) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      if (j <= i) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) raise_error(st, ST_BREAKDOWN);
    return;
  }
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    if (j <= i) G[(k0 + i) * n + k0 + j] = L[i][j];
  }
}

// The column panel below the diagonal block: rows i >= k0 + nb solve
// x L11^T = G[i][k0:k0+nb] (forward substitution over the nb columns).  Each
// workgroup takes 64 rows, staged with L11 in LDS; one thread per row.
__global__ __launch_bounds__(256) void k_trsm_panel(double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                    const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double L[64][65];
  __shared__ double X[64][65];
  const int t = threadIdx.x;
  const int64_t r0 = k0 + nb + (int64_t)blockIdx.x * 64;
  const int nr = (int)min<int64_t>(64, n - r0);
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    L[i][j] = j <= i ? G[(k0 + i) * n + k0 + j] : 0.0;
  }
  for (int e = t; e < 64 * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    X[i][j] = i < nr ? G[(r0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  if (t < nr) {
    for (int j = 0; j < nb; ++j) {
      double s = X[t][j];
      for (int l = 0; l < j; ++l) s -= X[t][l] * L[j][l];
      X[t][j] = s / L[j][j];
    }
  }
  __syncthreads();
  for (int e = t; e < 64 * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    if (i < nr) G[(r0 + i) * n + k0 + j] = X[i][j];
  }
}

// Trailing update G[i][j] -= sum_{k in panel} G[i][k] G[j][k] for i >= j >=
// k0 + nb: lower tile pairs of 128 x 128 over the trailing rows.
__global__ __launch_bounds__(256, 2) void k_syrk_update(double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                        int ntile, bool vec, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double XI[SK][SS];
  __shared__ double XJ[SK][SS];
  int I, J;
  pair_of(blockIdx.x, ntile, I, J);   // I <= J: rows of block J, columns of block I
  const int64_t base = k0 + nb;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0};
  const int64_t rI = base + (int64_t)J * ST, cJ = base + (int64_t)I * ST;
  sym_tile<double, 1>(G, n, 0, n, rI, cJ, k0, k0 + nb, vec, XI, XJ, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qi = w >> 1, qj = w & 1, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = rI + qi * 64 + a * 16 + 4 * v + lk;
        const int64_t gj = cJ + qj * 64 + b * 16 + li;
        if (gi < n && gj <= gi) G[gi * n + gj] -= acc[a][b][v];
      }
}

// ---------------------------------------------------------------------------
// Triangular solves with the factor, one right-hand side y (in place).
// ---------------------------------------------------------------------------

// L11 y_b = y_b for the diagonal block at k0 (forward).  One wave.
__global__ __launch_bounds__(64) void k_trsv_fwd_diag(const double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                      double* __restrict__ y, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double ys[64];
  const int l = threadIdx.x;
  ys[l] = l < nb ? y[k0 + l] : 0.0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    double p = (l < j) ? G[(k0 + j) * n + k0 + l] * ys[l] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if (l == 0) ys[j] = (ys[j] - p) / G[(k0 + j) * n + k0 + j];
    __syncthreads();
  }
  if (l < nb) y[k0 + l] = ys[l];
}

// y_i -= sum_{l in block} G[i][l] y_l for rows i >= k0 + nb: one wave per row.
__global__ __launch_bounds__(256) void k_trsv_fwd_update(const double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                         double* __restrict__ y, const DevStatus* st) {
  if (failed(st)) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = k0 + nb + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double p = lane < nb ? G[i * n + k0 + lane] * y[k0 + lane] : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
  if (lane == 0) y[i] -= p;
}

// L11^T x_b = y_b for the diagonal block at k0 (backward).  One wave.
__global__ __launch_bounds__(64) void k_trsv_bwd_diag(const double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                      double* __restrict__ y, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double xs[64];
  const int l = threadIdx.x;
  xs[l] = l < nb ? y[k0 + l] : 0.0;
  __syncthreads();
  for (int j = nb - 1; j >= 0; --j) {
    double p = (l > j && l < nb) ? G[(k0 + l) * n + k0 + j] * xs[l] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if (l == 0) xs[j] = (xs[j] - p) / G[(k0 + j) * n + k0 + j];
    __syncthreads();
  }
  if (l < nb) y[k0 + l] = xs[l];
}

// y_i -= sum_{l in block} G[l][i] x_l for i < k0: one thread per i (the
// block's rows read across threads).
__global__ __launch_bounds__(256) void k_trsv_bwd_update(const double* __restrict__ G, int64_t n, int64_t k0, int nb,
                                                         double* __restrict__ y, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double xs[64];
  const int t = threadIdx.x;
  if (t < 64) xs[t] = t < nb ? y[k0 + t] : 0.0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  if (i >= k0) return;
  double s = 0.0;
  for (int l = 0; l < nb; ++l) s += G[(k0 + l) * n + i] * xs[l];
  y[i] -= s;
}

// ---------------------------------------------------------------------------
// u = O x (one wave per row; x FP64), and the SPRING right-hand side
// b = a_eps eps - a_u (u - mean(u)).
// ---------------------------------------------------------------------------
template <typename T, int PL>
__global__ __launch_bounds__(256) void k_gemv_rows(const T* __restrict__ O, int64_t ld, int64_t pstride, int64_t n,
                                                   int64_t m, const double* __restrict__ x, double* __restrict__ u,
                                                   const DevStatus* st) {
  if (failed(st)) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const T* row = O + i * ld;
  double s = 0.0;
  for (int64_t k = lane; k < m; k += 64) {
    double v;
    if constexpr (sizeof(T) == 4) {
      v = (double)row[k];
    } else {
      v = bf16d(row[k]) + (PL == 2 ? bf16d(row[k + pstride]) : 0.0);
    }
    s += v * x[k];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) u[i] = s;
}

__global__ __launch_bounds__(256) void k_spring_rhs(const double* __restrict__ eps, const double* __restrict__ u,
                                                    const double* __restrict__ ubar, int64_t n, double a_eps,
                                                    double a_u, double* __restrict__ b, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  b[i] = a_eps * eps[i] - (u ? a_u * (u[i] - ubar[0]) : 0.0);
}

// dtheta = a delta + b dtheta
__global__ __launch_bounds__(256) void k_axpby(const double* __restrict__ delta, int64_t m, double a, double b,
                                               double* __restrict__ dtheta, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) dtheta[i] = a * delta[i] + b * dtheta[i];
}

template __global__ void k_syrk_partial<float, 1>(const float*, int64_t, int64_t, int64_t, int64_t, int, int64_t,
                                                  double*, double*, bool, const DevStatus*);
template __global__ void k_syrk_partial<unsigned short, 1>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                           int, int64_t, double*, double*, bool, const DevStatus*);
template __global__ void k_syrk_partial<unsigned short, 2>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                           int, int64_t, double*, double*, bool, const DevStatus*);
template __global__ void k_gemv_rows<float, 1>(const float*, int64_t, int64_t, int64_t, int64_t, const double*,
                                               double*, const DevStatus*);
template __global__ void k_gemv_rows<unsigned short, 1>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                        const double*, double*, const DevStatus*);
template __global__ void k_gemv_rows<unsigned short, 2>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                        const double*, double*, const DevStatus*);

}  // namespace wssr
