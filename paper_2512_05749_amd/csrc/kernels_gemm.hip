// The two tall-skinny products of each subspace-iteration pass (Alg. 1), in
// FP32 on the 32x32x2 FP32 MFMA with LDS-staged, double-buffered tiles.
//
//   sample side   Ypart[s] = O[:, Ks] V[Ks, :]     (N x r, K = M split into S ranges)
//   parameter side Z = O^T Q / sqrt(N)              (M x r, K = N)
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement, 128 x 128 output
// tile, each wave a 64 x 64 block = 2 x 2 MFMA tiles of 32 x 32.  K advances
// in steps of 32.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int BM = 128, BN = 128, BK = 32;
constexpr int APAD = 4, BPAD = 4;
}  // namespace

// ---------------------------------------------------------------------------
// Sample-side product.  O is N x M row-major (K contiguous), V is M x r
// row-major.  The contraction index inside a K-step is permuted so that each
// lane reads 4 consecutive K values of its O row with one 16-byte LDS read:
// lane (x, h) = (l%32, l/32) feeds k = h*16 + s to MFMA step s, for both
// operands.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void k_gemm_sample_side(const float* __restrict__ O, int64_t ld, int64_t n,
                                                             int64_t m, const float* __restrict__ V, int r,
                                                             float* __restrict__ ypart, int64_t kchunk,
                                                             bool vec_o, bool vec_v, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ __attribute__((aligned(16))) float As[2][BM][BK + APAD];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK][BN + BPAD];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int x = lane & 31, h = lane >> 5;
  const int64_t n0 = (int64_t)blockIdx.x * BM;
  const int j0 = blockIdx.y * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = min(m, kb + kchunk);
  float* out = ypart + (int64_t)blockIdx.z * n * r;

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{0};

  // global -> register staging: A tile 128 x 32 (4 float4 per thread),
  // B tile 32 x 128 (4 float4 per thread)
  f32x4 ra[4], rb[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = (t >> 3) + 32 * i;
      const int kq = (t & 7) * 4;
      const int64_t gi = n0 + row;
      ra[i] = (gi < n) ? load4(O + gi * ld, k0 + kq, ke, vec_o) : f32x4{0};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int krow = (t >> 5) + 8 * i;
      const int jq = (t & 31) * 4;
      const int64_t gk = k0 + krow;
      rb[i] = (gk < ke) ? load4(V + gk * r, j0 + jq, r, vec_v) : f32x4{0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = (t >> 3) + 32 * i;
      const int kq = (t & 7) * 4;
      *reinterpret_cast<f32x4*>(&As[buf][row][kq]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int krow = (t >> 5) + 8 * i;
      const int jq = (t & 31) * 4;
      *reinterpret_cast<f32x4*>(&Bs[buf][krow][jq]) = rb[i];
    }
  };

  const int64_t nk = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kb);
    sstore(0);
  }
  __syncthreads();
  for (int64_t it = 0; it < nk; ++it) {
    const int buf = (int)(it & 1);
    if (it + 1 < nk) gload(kb + (it + 1) * BK);
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
      f32x4 av[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const f32x4*>(&As[buf][wm * 64 + a * 32 + x][h * 16 + q4 * 4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = h * 16 + q4 * 4 + e;
        float bv[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs[buf][kk][wn * 64 + b * 32 + x];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = mfma32x32x2(av[a][e], bv[b], acc[a][b]);
      }
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = j0 + wn * 64 + b * 32 + x;
      if (col >= r) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = n0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < n) out[row * r + col] = acc[a][b][v];
      }
    }
}

// ---------------------------------------------------------------------------
// Parameter-side product Z = O^T Q * scale.  O is N x M row-major, Q is N x r
// row-major; both tiles are staged K-major ([k][column]) so every lane reads
// consecutive addresses.  The MFMA computes the transposed block Z^T:
// A[i][k] = Q[k][j0+i], B[k][jj] = O[k][m0+jj].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void k_gemm_param_side(const float* __restrict__ O, int64_t ld, int64_t n,
                                                            int64_t m, const float* __restrict__ Q, int r,
                                                            float scale, float* __restrict__ Z, bool vec_o,
                                                            bool vec_q, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ __attribute__((aligned(16))) float Os[2][BK][BM + BPAD];
  __shared__ __attribute__((aligned(16))) float Qs[2][BK][BN + BPAD];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wj = w & 1;
  const int x = lane & 31, h = lane >> 5;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int j0 = blockIdx.y * BN;

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{0};

  f32x4 ro[4], rq[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int krow = (t >> 5) + 8 * i;
      const int cq = (t & 31) * 4;
      const int64_t gk = k0 + krow;
      ro[i] = (gk < n) ? load4(O + gk * ld, m0 + cq, m, vec_o) : f32x4{0};
      rq[i] = (gk < n) ? load4(Q + gk * r, j0 + cq, r, vec_q) : f32x4{0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int krow = (t >> 5) + 8 * i;
      const int cq = (t & 31) * 4;
      *reinterpret_cast<f32x4*>(&Os[buf][krow][cq]) = ro[i];
      *reinterpret_cast<f32x4*>(&Qs[buf][krow][cq]) = rq[i];
    }
  };

  const int64_t nk = (n + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t it = 0; it < nk; ++it) {
    const int buf = (int)(it & 1);
    if (it + 1 < nk) gload((it + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int kk = h * 16 + s;
      float av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Qs[buf][kk][wj * 64 + a * 32 + x];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Os[buf][kk][wm * 64 + b * 32 + x];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma32x32x2(av[a], bv[b], acc[a][b]);
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // acc[a][b] holds Z^T rows (j) a-block, columns (m) b-block
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t row = m0 + wm * 64 + b * 32 + x;
      if (row >= m) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int jb = j0 + wj * 64 + a * 32 + 8 * g + 4 * h;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (jb + e < r) Z[row * r + jb + e] = acc[a][b][4 * g + e] * scale;
      }
    }
}

}  // namespace wssr
