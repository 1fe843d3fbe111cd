// FP64 kernels on the 16x16x4 FP64 MFMA for the orthonormalisation of the
// tall blocks (CholeskyQR): the Gram matrix X^T X and the apply X T with a
// small square T.  Inputs may be float or double; products and sums are FP64.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int GT = 64;     // output tile
constexpr int GK = 32;     // K step
constexpr int GP = 1;      // LDS row pad (doubles)
}  // namespace

// ---------------------------------------------------------------------------
// Gram partials.  X is rows x r row-major.  grid.x enumerates the tile pairs
// (I <= J) of the rp x rp output (rp = r padded to 64), grid.y the row chunks.
// 4 waves, each a 32 x 32 quadrant = 2 x 2 MFMA tiles of 16 x 16.
// part[(chunk * npairs + pair) * 4096 + i * 64 + j].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gram_partial(const T* __restrict__ X, int64_t rows, int r, int ntile,
                                                      int64_t rows_per_chunk, double* __restrict__ part,
                                                      const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  __shared__ double XI[GK][GT + GP];
  __shared__ double XJ[GK][GT + GP];
  // decode pair index -> (I, J), I <= J, row-major over the upper triangle
  int pair = blockIdx.x, I = 0;
  {
    int rem = pair;
    while (rem >= ntile - I) {
      rem -= ntile - I;
      ++I;
    }
    pair = rem + I;  // J
  }
  const int J = pair;
  const int npairs = ntile * (ntile + 1) / 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qi = w >> 1, qj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t rend = min(rows, rbeg + rows_per_chunk);

  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0};

  for (int64_t k0 = rbeg; k0 < rend; k0 += GK) {
    // load 32 rows x 64 columns for tile I and tile J: 2048 elements each, 8 per thread
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;
      const int kr = idx >> 6, c = idx & 63;
      const int64_t gr = k0 + kr;
      const int ci = I * GT + c, cj = J * GT + c;
      XI[kr][c] = (gr < rend && ci < r) ? (double)X[gr * r + ci] : 0.0;
      XJ[kr][c] = (gr < rend && cj < r) ? (double)X[gr * r + cj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = XI[k][qi * 32 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = XJ[k][qj * 32 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x4d(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)blockIdx.y * npairs + blockIdx.x) * (GT * GT);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = qi * 32 + a * 16 + 4 * v + lk;
        const int j = qj * 32 + b * 16 + li;
        out[i * GT + j] = acc[a][b][v];
      }
}

// Sum the partials in chunk order and write the symmetric rp x rp Gram matrix,
// identity on the padding (rows/columns >= r).  grid (npairs, 16): block y
// covers 256 of the 4096 entries of its tile, one entry per thread.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int nchunk, int ntile, int r,
                                                     double* __restrict__ G, const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  int pair = blockIdx.x, I = 0;
  {
    int rem = pair;
    while (rem >= ntile - I) {
      rem -= ntile - I;
      ++I;
    }
    pair = rem + I;
  }
  const int J = pair;
  const int npairs = ntile * (ntile + 1) / 2;
  const int rp = ntile * GT;
  const int e = blockIdx.y * 256 + threadIdx.x;
  const int i = e >> 6, j = e & 63;
  const int gi = I * GT + i, gj = J * GT + j;
  double s;
  if (gi < r && gj < r) {
    const double* p = part + (int64_t)blockIdx.x * (GT * GT) + e;
    const int64_t stride = (int64_t)npairs * (GT * GT);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int c = 0;
    for (; c + 3 < nchunk; c += 4) {
      a0 += p[(c + 0) * stride];
      a1 += p[(c + 1) * stride];
      a2 += p[(c + 2) * stride];
      a3 += p[(c + 3) * stride];
    }
    for (; c < nchunk; ++c) a0 += p[c * stride];
    s = (a0 + a1) + (a2 + a3);
  } else {
    s = (gi == gj) ? 1.0 : 0.0;
  }
  G[(int64_t)gi * rp + gj] = s;
  G[(int64_t)gj * rp + gi] = s;
}

// ---------------------------------------------------------------------------
// Apply: Out[rows x ldo] = X[rows x ldx] * Tm[0:kdim, 0:ncol] (Tm rp x rp row-major,
// FP64).  grid (row tiles of 64, column tiles of 64).  When `upper`, Tm is upper
// triangular and K-steps below the column tile are skipped.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_apply(const Tin* __restrict__ X, int64_t rows, int ldx, int kdim,
                                               const double* __restrict__ Tm, int rp, int ncol,
                                               Tout* __restrict__ Out, int ldo, bool upper, const DevStatus* st,
                                               bool gated) {
  if (skipped(st, gated)) return;
  __shared__ double Xs[GK][GT + GP];   // [k][row]
  __shared__ double Ts[GK][GT + GP];   // [k][col]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qi = w >> 1, qj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * GT;
  const int col0 = blockIdx.y * GT;
  const int kend = upper ? min(kdim, col0 + GT) : kdim;

  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0};

  for (int k0 = 0; k0 < kend; k0 += GK) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;
      // X tile: 64 rows x 32 k, read along k (8 threads per row... 32 k per row)
      const int rr = idx >> 5, kk = idx & 31;
      const int64_t gr = row0 + rr;
      const int gk = k0 + kk;
      Xs[kk][rr] = (gr < rows && gk < kdim) ? (double)X[gr * ldx + gk] : 0.0;
      // T tile: 32 k x 64 cols
      const int tk = idx >> 6, tc = idx & 63;
      const int gtk = k0 + tk, gtc = col0 + tc;
      Ts[tk][tc] = (gtk < kdim && gtc < ncol) ? Tm[(int64_t)gtk * rp + gtc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Xs[k][qi * 32 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Ts[k][qj * 32 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x4d(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = row0 + qi * 32 + a * 16 + 4 * v + lk;
        const int j = col0 + qj * 32 + b * 16 + li;
        if (i < rows && j < ncol) Out[i * ldo + j] = (Tout)acc[a][b][v];
      }
}

// explicit instantiations used by the host runtime
template __global__ void k_gram_partial<float>(const float*, int64_t, int, int, int64_t, double*, const DevStatus*,
                                               bool);
template __global__ void k_gram_partial<double>(const double*, int64_t, int, int, int64_t, double*, const DevStatus*,
                                                bool);
template __global__ void k_apply<float, float>(const float*, int64_t, int, int, const double*, int, int, float*, int,
                                               bool, const DevStatus*, bool);
template __global__ void k_apply<double, float>(const double*, int64_t, int, int, const double*, int, int, float*,
                                                int, bool, const DevStatus*, bool);
template __global__ void k_apply<double, double>(const double*, int64_t, int, int, const double*, int, int, double*,
                                                 int, bool, const DevStatus*, bool);

}  // namespace wssr
