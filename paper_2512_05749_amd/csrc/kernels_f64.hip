// Kernels for the orthonormalisation of the tall blocks (CholeskyQR): the
// Gram matrix X^T X and the apply X T with a small square T.  Inputs may be
// float or double.  The FP64 kernels multiply and sum in FP64 on the 16x16x4
// FP64 MFMA.  The fast ones serve the parameter-side block, whose FP32 values
// are all there is: k_gram32_partial and k_apply32 on the FP32 MFMA at twice
// the FP64 rate, k_gram16_partial on the BF16 MFMA (two-plane split, four
// products).  The fast Grams' FP32 sums are flushed into FP64 every 256 rows,
// so their entries carry about 1e-7 (FP32) and 3e-7 (BF16 split) relative
// error; the apply's sums run over at most r terms.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int GT = 128;         // output tile (rows and columns)
constexpr int GK = 16;          // K step
constexpr int GS = GT + 16;     // LDS row stride in doubles: the four K-rows of one
                                // MFMA operand read fall into two halves of the banks

typedef double f64x2 __attribute__((ext_vector_type(2)));

// The FP64 and FP32 16x16x4 MFMAs take A[i][k] from lane i + 16 k and
// B[k][j] from lane j + 16 k alike, but place D differently: the FP64 one
// holds D[4 v + l/16][l%16] in register v of lane l, the FP32 one
// D[4 (l/16) + v][l%16] (checked on the device).  These give the D row of
// register v for lk = l/16.
__device__ __forceinline__ int drow_f64(int v, int lk) { return 4 * v + lk; }
__device__ __forceinline__ int drow_f32(int v, int lk) { return 4 * lk + v; }

// four consecutive elements p[0..3] as doubles; n of them valid (the rest 0)
__device__ __forceinline__ f64x4 load4d(const float* __restrict__ p, int n, bool vec) {
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
__device__ __forceinline__ f64x4 load4d(const double* __restrict__ p, int n, bool vec) {
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

// decode a pair index to (I, J), I <= J, row-major over the upper triangle of
// ntile x ntile tiles
__device__ __forceinline__ void tile_pair(int pair, int ntile, int& I, int& J) {
  int rem = pair;
  I = 0;
  while (rem >= ntile - I) {
    rem -= ntile - I;
    ++I;
  }
  J = rem + I;
}
}  // namespace

// ---------------------------------------------------------------------------
// FP64 Gram partials.  X is rows x r row-major (row stride r).  grid.x enumerates
// the tile pairs (I <= J) of 128 x 128 tiles of the Gram matrix, grid.y the
// row chunks.  4 waves in a 2 x 2 arrangement, each a 64 x 64 quadrant =
// 4 x 4 MFMA tiles of 16 x 16; a diagonal pair (I = J) stages its one column
// block once.  Each K-step stages 16 rows of the two column blocks in LDS as
// FP64 while the next 16 rows are being loaded into registers.
// part[(chunk * npairs + pair) * 16384 + i * 128 + j].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gram_partial(const T* __restrict__ X, int64_t rows, int r, int64_t ldx,
                                                         int ntile, int64_t rows_per_chunk, double* __restrict__ part,
                                                         bool vec, const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  __shared__ double XI[GK][GS];
  __shared__ double XJ[GK][GS];
  int I, J;
  tile_pair(blockIdx.x, ntile, I, J);
  const bool diag = I == J;
  const int npairs = ntile * (ntile + 1) / 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qi = w >> 1, qj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t rend = min(rows, rbeg + rows_per_chunk);

  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0, 0, 0, 0};

  // thread -> (K-row, 4 columns) of a 16 x 128 block, two units per thread
  f64x4 pi[2], pj[2];
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int64_t gr = k0 + (idx >> 5);
      const int c4 = (idx & 31) * 4;
      const int ci = I * GT + c4, cj = J * GT + c4;
      const bool row_ok = gr < rend;
      pi[e] = load4d(X + gr * ldx + ci, row_ok ? min(4, r - ci) : 0, vec);
      if (!diag) pj[e] = load4d(X + gr * ldx + cj, row_ok ? min(4, r - cj) : 0, vec);
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int kr = idx >> 5, c4 = (idx & 31) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) XI[kr][c4 + q] = pi[e][q];
      if (!diag) {
#pragma unroll
        for (int q = 0; q < 4; ++q) XJ[kr][c4 + q] = pj[e][q];
      }
    }
  };
  if (rbeg < rend) load(rbeg);
  for (int64_t k0 = rbeg; k0 < rend; k0 += GK) {
    store();
    __syncthreads();
    if (k0 + GK < rend) load(k0 + GK);
    const double(*B)[GS] = diag ? XI : XJ;
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
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
  double* out = part + ((int64_t)blockIdx.y * npairs + blockIdx.x) * (GT * GT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = qi * 64 + a * 16 + drow_f64(v, lk);
        const int j = qj * 64 + b * 16 + li;
        out[i * GT + j] = acc[a][b][v];
      }
}

// ---------------------------------------------------------------------------
// FP32-MFMA Gram partials of a float block, tuned for tall blocks: the
// 128 x 128 tile pairs, 2 x 2 wave layout and partial layout of
// k_gram_partial (k_gram_reduce sums them), on the FP32 16x16x4 MFMA with
// the FP32 sums flushed into FP64 every 256 rows, and
// - 16-row K-steps staged through float registers into a double-buffered LDS
//   tile (one barrier per step; the loads of step s + 1 are in flight during
//   the MFMAs of step s);
// - a one-dimensional grid of npairs x nchunk workgroups in which, when the
//   total is a multiple of 8, the tile pairs of one row chunk are consecutive
//   workgroups of one XCD (workgroups are dealt to the 8 XCDs in turn), so
//   the column blocks of a chunk that several pairs read are fetched into
//   that XCD's L2 once.
// ---------------------------------------------------------------------------
namespace {
constexpr int G32K = 16;                      // K step (rows)
constexpr int G32Flush = 256 / G32K;          // steps between FP64 flushes
}  // namespace

__global__ __launch_bounds__(256, 2) void k_gram32_partial(const float* __restrict__ X, int64_t rows, int r,
                                                           int64_t ldx, int ntile, int nchunk,
                                                           int64_t rows_per_chunk, double* __restrict__ part,
                                                           bool vec, const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  __shared__ float XI[2][G32K][GS];
  __shared__ float XJ[2][G32K][GS];
  const int npairs = ntile * (ntile + 1) / 2;
  const int total = npairs * nchunk;
  int w = blockIdx.x;
  if (total % 8 == 0) w = (w % 8) * (total / 8) + w / 8;
  const int pair = w % npairs, chunk = w / npairs;
  int I, J;
  tile_pair(pair, ntile, I, J);
  const bool diag = I == J;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int qi = wv >> 1, qj = wv & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t rbeg = (int64_t)chunk * rows_per_chunk;
  const int64_t rend = min(rows, rbeg + rows_per_chunk);

  f32x4 acc[4][4];
  f64x4 acc64[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc[a][b] = f32x4{0, 0, 0, 0};
      acc64[a][b] = f64x4{0, 0, 0, 0};
    }

  // thread -> (K-row, 4 columns) of a G32K x 128 block, G32K / 8 units per thread;
  // 32 consecutive threads read one 512-byte row piece
  f32x4 pi[G32K / 8], pj[G32K / 8];
  auto ld4 = [&](const float* p, int n) __attribute__((always_inline)) {
    if (vec && n >= 4) return *reinterpret_cast<const f32x4*>(p);
    f32x4 v = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e < n) v[e] = p[e];
    return v;
  };
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < G32K / 8; ++e) {
      const int idx = t + 256 * e;
      const int64_t gr = k0 + (idx >> 5);
      const int c4 = (idx & 31) * 4;
      const int ci = I * GT + c4, cj = J * GT + c4;
      const bool row_ok = gr < rend;
      pi[e] = ld4(X + gr * ldx + ci, row_ok ? min(4, r - ci) : 0);
      if (!diag) pj[e] = ld4(X + gr * ldx + cj, row_ok ? min(4, r - cj) : 0);
    }
  };
  auto store = [&](int b) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < G32K / 8; ++e) {
      const int idx = t + 256 * e;
      const int kr = idx >> 5, c4 = (idx & 31) * 4;
      *reinterpret_cast<f32x4*>(&XI[b][kr][c4]) = pi[e];
      if (!diag) *reinterpret_cast<f32x4*>(&XJ[b][kr][c4]) = pj[e];
    }
  };

  if (rbeg < rend) {
    load(rbeg);
    store(0);
  }
  __syncthreads();
  int since = 0, cur = 0;
  for (int64_t k0 = rbeg; k0 < rend; k0 += G32K) {
    const bool more = k0 + G32K < rend;
    if (more) load(k0 + G32K);
    const float(*A)[GS] = XI[cur];
    const float(*B)[GS] = diag ? XI[cur] : XJ[cur];
#pragma unroll
    for (int kk = 0; kk < G32K / 4; ++kk) {
      const int k = kk * 4 + lk;
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = A[k][qi * 64 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = B[k][qj * 64 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (++since == G32Flush) {
      since = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[a][b][v] += (double)acc[a][b][v];
          acc[a][b] = f32x4{0, 0, 0, 0};
        }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  double* out = part + ((int64_t)chunk * npairs + pair) * (GT * GT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = qi * 64 + a * 16 + drow_f32(v, lk);
        const int j = qj * 64 + b * 16 + li;
        out[i * GT + j] = acc64[a][b][v] + (double)acc[a][b][v];
      }
}

// ---------------------------------------------------------------------------
// Gram partials of a float block on the BF16 MFMA.  Each element is split on
// load into two RNE BF16 planes, z = h + l + e with |e| <= 2^-16 |z|, and
// the four products (h + l)^T (h + l) run on v_mfma_f32_32x32x16_bf16, whose
// BF16 products are exact in FP32.  The FP32 sums are flushed into FP64 every
// 256 rows, as in k_gram32_partial, so the entries carry the same FP32
// accumulation error; the split residual adds at most 2^-15 relative to
// sqrt(G_ii G_jj) (about 2^-16 / sqrt(rows) for rounding errors of random
// sign).  Tile pairs, row chunks, the one-dimensional XCD-grouped grid and
// the partial layout are those of k_gram32_partial.
// 512 threads = 8 waves in a 4 x 2 arrangement, each a 32 x 64 part of the
// 128 x 128 tile pair (two MFMA tiles of 32 x 32), one workgroup per compute
// unit and two waves per SIMD.  K-steps of G16K = 64 rows: each thread loads
// 16 rows of one column of each column block (coalesced across the 128
// threads of a row quarter), splits them and writes them as 16-byte LDS
// stores of 8 K-values per plane into a [plane][column][k] tile with a
// column stride of 72 elements (144 bytes, an odd multiple of 16, so the
// 16-byte fragment reads are conflict-free); double-buffered (144 KB), one
// barrier per step, the next step's loads in flight during the step's 32
// MFMAs per wave.
// ---------------------------------------------------------------------------
namespace {
typedef __bf16 g16x8 __attribute__((ext_vector_type(8)));
typedef unsigned g16u4 __attribute__((ext_vector_type(4)));
constexpr int G16K = 64;             // rows per K-step
constexpr int G16S = G16K + 8;       // LDS column stride (BF16 elements)
constexpr int G16Flush = 256 / G16K; // steps between FP64 flushes

__device__ __forceinline__ unsigned short g16_bits(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ __forceinline__ float g16_val(unsigned short b) { return (float)__builtin_bit_cast(__bf16, b); }
}  // namespace

__global__ __launch_bounds__(512, 1) void k_gram16_partial(const float* __restrict__ X, int64_t rows, int r,
                                                           int64_t ldx, int ntile, int nchunk,
                                                           int64_t rows_per_chunk, double* __restrict__ part,
                                                           const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  // [buffer][block I, J][plane hi, lo][column][k]
  __shared__ __attribute__((aligned(16))) unsigned short S[2][2][2][GT][G16S];
  const int npairs = ntile * (ntile + 1) / 2;
  const int total = npairs * nchunk;
  int w = blockIdx.x;
  if (total % 8 == 0) w = (w % 8) * (total / 8) + w / 8;
  const int pair = w % npairs, chunk = w / npairs;
  int I, J;
  tile_pair(pair, ntile, I, J);
  const bool diag = I == J;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int qi = wv >> 1, qj = wv & 1;
  const int x = lane & 31, hh = lane >> 5;
  const int64_t rbeg = (int64_t)chunk * rows_per_chunk;
  const int64_t rend = min(rows, rbeg + rows_per_chunk);

  f32x16 acc[2];
  f64x4 acc64[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    acc[b] = f32x16{0};
#pragma unroll
    for (int q = 0; q < 4; ++q) acc64[b][q] = f64x4{0, 0, 0, 0};
  }

  // thread -> rows RT h .. RT h + RT - 1 of the step, column c of each block
  constexpr int RT = G16K / 4;
  const int h4 = t >> 7, c = t & 127;
  const int ci = I * GT + c, cj = J * GT + c;
  float pi[RT], pj[RT];
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < RT; ++e) {
      const int64_t gr = k0 + RT * h4 + e;
      const bool ok = gr < rend;
      pi[e] = ok && ci < r ? X[gr * ldx + ci] : 0.0f;
      if (!diag) pj[e] = ok && cj < r ? X[gr * ldx + cj] : 0.0f;
    }
  };
  auto put = [&](int b, int blk, const float* v) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < RT / 8; ++h) {
      unsigned short hi[8], lo[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        hi[e] = g16_bits(v[8 * h + e]);
        lo[e] = g16_bits(v[8 * h + e] - g16_val(hi[e]));
      }
      g16u4 vh, vl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        vh[q] = (unsigned)hi[2 * q] | ((unsigned)hi[2 * q + 1] << 16);
        vl[q] = (unsigned)lo[2 * q] | ((unsigned)lo[2 * q + 1] << 16);
      }
      *reinterpret_cast<g16u4*>(&S[b][blk][0][c][RT * h4 + 8 * h]) = vh;
      *reinterpret_cast<g16u4*>(&S[b][blk][1][c][RT * h4 + 8 * h]) = vl;
    }
  };
  auto store = [&](int b) __attribute__((always_inline)) {
    put(b, 0, pi);
    if (!diag) put(b, 1, pj);
  };

  if (rbeg < rend) {
    load(rbeg);
    store(0);
  }
  __syncthreads();
  int since = 0, cur = 0;
  const int bj = diag ? 0 : 1;
  for (int64_t k0 = rbeg; k0 < rend; k0 += G16K) {
    const bool more = k0 + G16K < rend;
    if (more) load(k0 + G16K);
#pragma unroll
    for (int kb = 0; kb < G16K / 16; ++kb) {
      g16u4 af[2], bf[2][2];   // [plane], [tile][plane]
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        af[p] = *reinterpret_cast<const g16u4*>(&S[cur][0][p][qi * 32 + x][16 * kb + 8 * hh]);
#pragma unroll
        for (int b = 0; b < 2; ++b)
          bf[b][p] = *reinterpret_cast<const g16u4*>(&S[cur][bj][p][qj * 64 + b * 32 + x][16 * kb + 8 * hh]);
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(g16x8, af[p]),
                                                             __builtin_bit_cast(g16x8, bf[b][q]), acc[b], 0, 0, 0);
    }
    if (++since == G16Flush) {
      since = 0;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc64[b][v >> 2][v & 3] += (double)acc[b][v];
        acc[b] = f32x16{0};
      }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // D of the 32 x 32 MFMA: register v of lane l holds row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
  double* out = part + ((int64_t)chunk * npairs + pair) * (GT * GT);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = qi * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
      const int j = qj * 64 + b * 32 + x;
      out[i * GT + j] = acc64[b][v >> 2][v & 3] + (double)acc[b][v];
    }
}

// Sum the partials in chunk order and write the symmetric rp x rp Gram matrix
// (rp = r padded to 64), identity on the padding (rows/columns >= r).  grid
// (npairs, 64): block y covers 256 of the 16384 entries of its tile pair, one
// entry per thread; in a diagonal pair only the upper triangle is summed and
// mirrored.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int nchunk, int ntile, int r,
                                                     int rp, double* __restrict__ G, const DevStatus* st,
                                                     bool gated) {
  if (skipped(st, gated)) return;
  int I, J;
  tile_pair(blockIdx.x, ntile, I, J);
  const int npairs = ntile * (ntile + 1) / 2;
  const int e = blockIdx.y * 256 + threadIdx.x;
  const int i = e / GT, j = e % GT;
  const int gi = I * GT + i, gj = J * GT + j;
  if (gi >= rp || gj >= rp || (I == J && i > j)) return;
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
// Apply: Out[rows x ldo] = X[rows x ldx] * Tm[0:kdim, 0:ncol] (Tm rp x rp
// row-major, FP64), or Out += X * Tm when `acc`.  grid (row tiles of 128,
// column tiles of 128); 4 waves of 64 x 64 as in the Gram kernel.  When
// `upper`, Tm is upper triangular and K-steps below the column tile are
// skipped.  The next K-step's tiles are loaded into registers while the
// current ones are multiplied.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256, 2) void k_apply(const Tin* __restrict__ X, int64_t rows, int ldx, int kdim,
                                                  const double* __restrict__ Tm, int rp, int ncol,
                                                  Tout* __restrict__ Out, int ldo, bool upper, bool vec,
                                                  bool acc, const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  __shared__ double Xs[GK][GS];   // [k][row]
  __shared__ double Ts[GK][GS];   // [k][col]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qi = w >> 1, qj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * GT;
  const int col0 = blockIdx.y * GT;
  const int kend = upper ? min(kdim, col0 + GT) : kdim;

  f64x4 acc_v[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc_v[a][b] = f64x4{0, 0, 0, 0};

  // X: thread -> (row, 4 K-values), two units; T: thread -> (K-row, 2 columns), four units
  f64x4 px[2];
  f64x2 pt[4];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int64_t gr = row0 + (idx >> 2);
      const int gk = k0 + (idx & 3) * 4;
      px[e] = load4d(X + gr * ldx + gk, gr < rows ? min(4, kdim - gk) : 0, vec);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + 256 * e;
      const int gtk = k0 + (idx >> 6), gtc = col0 + (idx & 63) * 2;
      f64x2 v = f64x2{0, 0};
      if (gtk < kdim) {
        const double* src = Tm + (int64_t)gtk * rp + gtc;
        if (gtc + 1 < ncol)
          v = *reinterpret_cast<const f64x2*>(src);
        else if (gtc < ncol)
          v[0] = src[0];
      }
      pt[e] = v;
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int rr = idx >> 2, kq = (idx & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Xs[kq + q][rr] = px[e][q];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + 256 * e;
      Ts[idx >> 6][(idx & 63) * 2] = pt[e][0];
      Ts[idx >> 6][(idx & 63) * 2 + 1] = pt[e][1];
    }
  };
  if (kend > 0) load(0);
  for (int k0 = 0; k0 < kend; k0 += GK) {
    store();
    __syncthreads();
    if (k0 + GK < kend) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = Xs[k][qi * 64 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ts[k][qj * 64 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc_v[a][b] = mfma16x16x4d(av[a], bv[b], acc_v[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = row0 + qi * 64 + a * 16 + drow_f64(v, lk);
        const int j = col0 + qj * 64 + b * 16 + li;
        if (i < rows && j < ncol)
          Out[i * ldo + j] = acc ? (Tout)((double)acc_v[a][b][v] + (double)Out[i * ldo + j])
                                 : (Tout)acc_v[a][b][v];
      }
}

// ---------------------------------------------------------------------------
// FP32-MFMA apply Out = X Tf (X rows x kdim float, row stride ldx; Tf the
// FP64 factor rounded to float, rp x rp row-major, columns 0 .. ncol-1),
// for the blocks whose FP32 apply is taken (sums over at most kdim terms).
// 128 x 128 output tiles, 4 waves of 64 x 64 on the 16x16x4 FP32 MFMA as in
// k_apply.  16-row K-steps staged through registers into a double-buffered
// LDS tile (one barrier per step); X stays [row][k] in LDS with a row stride
// of 20 floats (the 16 rows x 4 K-values of an MFMA operand read fall into
// distinct banks) and is stored with 16-byte writes.  One-dimensional grid:
// the column tiles of one row tile are consecutive workgroups of one XCD
// when the total is a multiple of 8, so each row slab of X is fetched into
// that XCD's L2 once.  When `upper`, K-steps below the column tile are
// skipped (Tf upper triangular); with acc_out, Out += X Tf (in FP32).
// ---------------------------------------------------------------------------
namespace {
constexpr int A32S = 20;   // LDS row stride (floats) of the X tile
}  // namespace

__global__ __launch_bounds__(256, 4) void k_apply32(const float* __restrict__ X, int64_t rows, int ldx, int kdim,
                                                    const float* __restrict__ Tf, int rp, int ncol,
                                                    float* __restrict__ Out, int ldo, bool upper, bool vec,
                                                    bool acc_out, const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  __shared__ float Xs[2][GT][A32S];   // [row][k]
  __shared__ float Ts[2][GK][GS];     // [k][col]
  const int ctiles = (ncol + GT - 1) / GT;
  const int total = (int)((rows + GT - 1) / GT) * ctiles;
  int w = blockIdx.x;
  if (total % 8 == 0) w = (w % 8) * (total / 8) + w / 8;
  const int64_t row0 = (int64_t)(w / ctiles) * GT;
  const int col0 = (w % ctiles) * GT;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int qi = wv >> 1, qj = wv & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int kend = upper ? min(kdim, col0 + GT) : kdim;

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0, 0, 0, 0};

  // X: thread -> (row, 4 K-values), two units; Tf: thread -> (K-row, 4 columns), two units
  f32x4 px[2], pt[2];
  auto ld4 = [&](const float* p, int n, bool v4) __attribute__((always_inline)) {
    if (v4 && n >= 4) return *reinterpret_cast<const f32x4*>(p);
    f32x4 v = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e < n) v[e] = p[e];
    return v;
  };
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int64_t gr = row0 + (idx >> 2);
      const int gk = k0 + (idx & 3) * 4;
      px[e] = ld4(X + gr * ldx + gk, gr < rows ? min(4, kdim - gk) : 0, vec);
      const int tk = k0 + (idx >> 5), tc = col0 + (idx & 31) * 4;
      pt[e] = ld4(Tf + (int64_t)tk * rp + tc, tk < kdim ? min(4, ncol - tc) : 0, true);
    }
  };
  auto store = [&](int b) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      *reinterpret_cast<f32x4*>(&Xs[b][idx >> 2][(idx & 3) * 4]) = px[e];
      *reinterpret_cast<f32x4*>(&Ts[b][idx >> 5][(idx & 31) * 4]) = pt[e];
    }
  };

  if (kend > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < kend; k0 += GK) {
    const bool more = k0 + GK < kend;
    if (more) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int k = kk * 4 + lk;
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = Xs[cur][qi * 64 + a * 16 + li][k];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ts[cur][k][qj * 64 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = row0 + qi * 64 + a * 16 + drow_f32(v, lk);
        const int j = col0 + qj * 64 + b * 16 + li;
        if (i < rows && j < ncol) Out[i * ldo + j] = acc_out ? Out[i * ldo + j] + acc[a][b][v] : acc[a][b][v];
      }
}

// Round an FP64 array to float (the factor of k_apply32); skipped with the apply.
__global__ __launch_bounds__(256) void k_round_f32(const double* __restrict__ src, int64_t n, float* __restrict__ dst,
                                                   const DevStatus* st, bool gated) {
  if (skipped(st, gated)) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// ---------------------------------------------------------------------------
// Cross products H = X^T W of two tall blocks (rows x r, row stride r each,
// X and W of possibly different element types), as partials over row chunks:
// grid.x enumerates all ntile x ntile tiles of 128 x 128 (I, J), grid.y the
// row chunks; the waves, K-steps and staging are those of the Gram kernel.
// part[(chunk * ntile^2 + I * ntile + J) * 16384 + i * 128 + j].
// ---------------------------------------------------------------------------
template <typename TX, typename TW>
__global__ __launch_bounds__(256, 2) void k_cross_partial(const TX* __restrict__ X, const TW* __restrict__ W,
                                                          int64_t rows, int r, int ntile, int64_t rows_per_chunk,
                                                          double* __restrict__ part, bool vec, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double XI[GK][GS];
  __shared__ double WJ[GK][GS];
  const int I = blockIdx.x / ntile, J = blockIdx.x % ntile;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qi = w >> 1, qj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t rend = min(rows, rbeg + rows_per_chunk);

  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0};

  f64x4 pi[2], pj[2];
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int64_t gr = k0 + (idx >> 5);
      const int c4 = (idx & 31) * 4;
      const int ci = I * GT + c4, cj = J * GT + c4;
      const bool row_ok = gr < rend;
      pi[e] = load4d(X + gr * r + ci, row_ok ? min(4, r - ci) : 0, vec);
      pj[e] = load4d(W + gr * r + cj, row_ok ? min(4, r - cj) : 0, vec);
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = t + 256 * e;
      const int kr = idx >> 5, c4 = (idx & 31) * 4;
      *reinterpret_cast<f64x2*>(&XI[kr][c4]) = f64x2{pi[e][0], pi[e][1]};
      *reinterpret_cast<f64x2*>(&XI[kr][c4 + 2]) = f64x2{pi[e][2], pi[e][3]};
      *reinterpret_cast<f64x2*>(&WJ[kr][c4]) = f64x2{pj[e][0], pj[e][1]};
      *reinterpret_cast<f64x2*>(&WJ[kr][c4 + 2]) = f64x2{pj[e][2], pj[e][3]};
    }
  };
  if (rbeg < rend) load(rbeg);
  for (int64_t k0 = rbeg; k0 < rend; k0 += GK) {
    store();
    __syncthreads();
    if (k0 + GK < rend) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int k = kk * 4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = XI[k][qi * 64 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = WJ[k][qj * 64 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4d(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)blockIdx.y * ntile * ntile + blockIdx.x) * (GT * GT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = qi * 64 + a * 16 + 4 * v + lk;
        const int j = qj * 64 + b * 16 + li;
        out[i * GT + j] = acc[a][b][v];
      }
}

// Sum the cross partials in chunk order into H (rp x rp row-major, zero
// outside r x r).  grid (ntile^2, 64), one entry per thread.
__global__ __launch_bounds__(256) void k_cross_reduce(const double* __restrict__ part, int nchunk, int ntile, int r,
                                                      int rp, double* __restrict__ H, const DevStatus* st) {
  if (failed(st)) return;
  const int I = blockIdx.x / ntile, J = blockIdx.x % ntile;
  const int e = blockIdx.y * 256 + threadIdx.x;
  const int i = e / GT, j = e % GT;
  const int gi = I * GT + i, gj = J * GT + j;
  if (gi >= rp || gj >= rp) return;
  double s = 0.0;
  if (gi < r && gj < r) {
    const double* p = part + (int64_t)blockIdx.x * (GT * GT) + e;
    const int64_t stride = (int64_t)ntile * ntile * (GT * GT);
    double a0 = 0.0, a1 = 0.0;
    int c = 0;
    for (; c + 1 < nchunk; c += 2) {
      a0 += p[(c + 0) * stride];
      a1 += p[(c + 1) * stride];
    }
    if (c < nchunk) a0 += p[c * stride];
    s = a0 + a1;
  }
  H[(int64_t)gi * rp + gj] = s;
}

// explicit instantiations used by the host runtime
template __global__ void k_gram_partial<float>(const float*, int64_t, int, int64_t, int, int64_t, double*, bool,
                                               const DevStatus*, bool);
template __global__ void k_gram_partial<double>(const double*, int64_t, int, int64_t, int, int64_t, double*, bool,
                                                const DevStatus*, bool);
template __global__ void k_cross_partial<double, float>(const double*, const float*, int64_t, int, int, int64_t,
                                                        double*, bool, const DevStatus*);
template __global__ void k_apply<float, float>(const float*, int64_t, int, int, const double*, int, int, float*, int,
                                               bool, bool, bool, const DevStatus*, bool);
template __global__ void k_apply<double, float>(const double*, int64_t, int, int, const double*, int, int, float*,
                                                int, bool, bool, bool, const DevStatus*, bool);
template __global__ void k_apply<double, double>(const double*, int64_t, int, int, const double*, int, int, double*,
                                                 int, bool, bool, bool, const DevStatus*, bool);

}  // namespace wssr
