// The two tall-skinny products of each subspace-iteration pass (Alg. 1) with O
// stored in BF16: BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.
//
//   sample side    Ypart[s] = O[:, Ks] S[Ks, :]      (N x r, K = M split into ranges)
//   parameter side Z = O^T S * scale                  (M x r, K = N)
//
// S (V or Q_Y) arrives in FP32.  k_split_skinny rounds it once per product,
// S = S_hi + S_lo with S_hi = RNE(S), S_lo = RNE(S - S_hi), into BF16 planes
// laid out K-blocked, [k / 16][column][k % 16], so that one K-step's tile of
// S is a contiguous block copied into LDS with 16-byte loads.  O has PA planes
// (1: O itself; 2: O_hi and O_lo = RNE(O_fp32 - O_hi), the split form) and S
// is used with PB planes.  The products summed are
//   O_hi S_hi                      always
//   O_hi S_lo                      when PB = 2
//   O_lo S_hi                      when PA = 2
// (the O_lo S_lo term is below FP32 rounding of the sum and is left out).
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement; output tile
// 128 rows x BN columns, each wave 64 x BN/2 = 2 x (BN/64) MFMA tiles of
// 32 x 32.  Both operand tiles are staged K-contiguous in LDS ([row][k], row
// stride BK + 8 elements, an odd multiple of 16 bytes, so the 16-byte
// fragment reads are conflict-free); a lane's MFMA fragment is one 16-byte
// read.  O on the parameter side, whose global rows are the K index, is
// loaded as 8 K-rows x 2 parameters per thread and transposed in registers,
// so its LDS stores are 16-byte stores too.  The next K-step's
// global loads are in flight during the current MFMAs (double-buffered LDS).
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int BM = 128;

__device__ __forceinline__ f32x16 mfma_bf16(const u32x4& a, const u32x4& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

__device__ __forceinline__ u16 bf16_bits(float x) { return __builtin_bit_cast(u16, (__bf16)x); }
__device__ __forceinline__ float bf16_val(u16 b) { return (float)__builtin_bit_cast(__bf16, b); }

// round x to BF16 (hi) and the rounded remainder (lo)
__device__ __forceinline__ void split_bf16(float x, u16& hi, u16& lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - bf16_val(hi));
}

__device__ __forceinline__ unsigned pack2(u16 a, u16 b) { return (unsigned)a | ((unsigned)b << 16); }

// Tile geometry shared by the kernels.  ATR: the A tile is kept as it lies
// in memory, [k][row] with row stride LDM (the parameter side, where O's rows
// are the K index), and its MFMA fragments are gathered with 2-byte reads;
// otherwise A is K-contiguous like B.
template <int BN, int BK, int PA, int PB, bool ATR>
struct Geo {
  static constexpr int LDK = BK + 8;                        // K-contiguous row stride (bf16 elements)
  static constexpr int LDM = BM + 8;                        // [k][row] row stride when ATR
  static constexpr int A_PLANE = ATR ? BK * LDM : BM * LDK; // elements per A plane
  static constexpr int B_PLANE = BN * LDK;
  static constexpr int STAGE = PA * A_PLANE + PB * B_PLANE;  // elements per stage
  static constexpr int TB = BN / 64;                        // 32-column MFMA tiles per wave
};

// MFMAs of one LDS stage: acc[a][b] += sum over products of A_p[rows] B_q[cols]^T
template <int BN, int BK, int PA, int PB, bool ATR>
__device__ __forceinline__ void mma_stage(f32x16 (&acc)[2][BN / 64], const u16* __restrict__ S, int wm, int wn,
                                          int lane) {
  using G = Geo<BN, BK, PA, PB, ATR>;
  const int x = lane & 31, h = lane >> 5;
#pragma unroll
  for (int kc = 0; kc < BK / 16; ++kc) {
    u32x4 av[PA][2], bv[PB][G::TB];
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if constexpr (ATR) {
          const u16* col = S + p * G::A_PLANE + (kc * 16 + 8 * h) * G::LDM + wm * 64 + a * 32 + x;
          u16 e[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) e[i] = col[i * G::LDM];
          av[p][a] = u32x4{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
        } else {
          av[p][a] = *reinterpret_cast<const u32x4*>(S + p * G::A_PLANE + (wm * 64 + a * 32 + x) * G::LDK +
                                                     kc * 16 + 8 * h);
        }
      }
#pragma unroll
    for (int q = 0; q < PB; ++q)
#pragma unroll
      for (int b = 0; b < G::TB; ++b)
        bv[q][b] = *reinterpret_cast<const u32x4*>(S + PA * G::A_PLANE + q * G::B_PLANE +
                                                   (wn * (BN / 2) + b * 32 + x) * G::LDK + kc * 16 + 8 * h);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) {
        acc[a][b] = mfma_bf16(av[0][a], bv[0][b], acc[a][b]);
        if constexpr (PB == 2) acc[a][b] = mfma_bf16(av[0][a], bv[1][b], acc[a][b]);
        if constexpr (PA == 2) acc[a][b] = mfma_bf16(av[1][a], bv[0][b], acc[a][b]);
      }
  }
}

// ---- S loader: BN columns x BK K-values of each split plane, copied from the
// K-blocked layout (16-byte units: column j, 8 K-values) into LDS rows.
template <int BN, int BK>
struct SUnit {
  static constexpr int UNITS = BN * (BK / 8);
  static constexpr int PER_T = (UNITS + 255) / 256;
};

template <int BN, int BK, int PB, int PT>
__device__ __forceinline__ void s_load(u32x4 (&rs)[PB][PT], const u16* __restrict__ Ss, int64_t pstride, int sw,
                                       int64_t kblocks, int j0, int64_t k0, bool fast, int t) {
#pragma unroll
  for (int q = 0; q < PB; ++q)
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int unit = t + 256 * u;
      if (unit >= SUnit<BN, BK>::UNITS) break;
      // unit -> (K-block of the stage kb, column c, half h8): consecutive
      // threads read consecutive 16-byte pieces of one K-block
      const int kb = unit / (2 * BN), c = (unit % (2 * BN)) >> 1, h8 = unit & 1;
      const int64_t blk = k0 / 16 + kb;
      const int j = j0 + c;
      const u16* src = Ss + q * pstride + (blk * sw + j) * 16 + h8 * 8;
      if (fast || blk < kblocks)
        rs[q][u] = *reinterpret_cast<const u32x4*>(src);
      else
        rs[q][u] = u32x4{0, 0, 0, 0};
    }
}

template <int BN, int BK, int PB, int PT>
__device__ __forceinline__ void s_store(const u32x4 (&rs)[PB][PT], u16* __restrict__ Bp, int plane_elems, int ldk,
                                        int t) {
#pragma unroll
  for (int q = 0; q < PB; ++q)
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int unit = t + 256 * u;
      if (unit >= SUnit<BN, BK>::UNITS) break;
      const int kb = unit / (2 * BN), c = (unit % (2 * BN)) >> 1, h8 = unit & 1;
      *reinterpret_cast<u32x4*>(Bp + q * plane_elems + c * ldk + kb * 16 + h8 * 8) = rs[q][u];
    }
}
}  // namespace

// ---------------------------------------------------------------------------
// S (K x r FP32, row-major) -> BF16 planes hi (and lo when two planes) in the
// K-blocked layout [kb][j][k % 16] with sw >= r columns (a whole number of
// product column tiles), zero for k >= K and for j >= r, so that the product
// kernels read whole tiles of S unguarded.  One thread per (kb, j):
// 16 loads that are coalesced across threads (consecutive j), two 32-byte
// stores per plane.
// With mode given and *mode == 0, S is taken as Z diag(gd)^{-1/2} (column j
// of alt times 1/sqrt(gd[j]) in FP64, 0 where gd[j] <= 0): the column scaling
// of k_colscale, without storing the scaled block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_split_skinny(const float* __restrict__ S, int64_t K, int r, int sw,
                                                      u16* __restrict__ out, int64_t pstride, int planes,
                                                      const DevStatus* st, const float* __restrict__ alt,
                                                      const double* __restrict__ gd, const int* __restrict__ mode) {
  if (failed(st)) return;
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t kblocks = (K + 15) / 16;
  if (id >= kblocks * sw) return;
  const int64_t kb = id / sw;
  const int j = (int)(id % sw);
  const bool scaled = mode != nullptr && *mode == 0;
  const float* src = scaled ? alt : S;
  double d = 1.0;
  if (scaled && j < r) d = gd[j];
  const double inv = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  u16 hi[16], lo[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int64_t k = kb * 16 + e;
    float x = (k < K && j < r) ? src[k * r + j] : 0.0f;
    if (scaled) x = (float)((double)x * inv);
    split_bf16(x, hi[e], lo[e]);
  }
  u16* dst = out + id * 16;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    u32x4 v = {pack2(hi[8 * h], hi[8 * h + 1]), pack2(hi[8 * h + 2], hi[8 * h + 3]),
               pack2(hi[8 * h + 4], hi[8 * h + 5]), pack2(hi[8 * h + 6], hi[8 * h + 7])};
    *reinterpret_cast<u32x4*>(dst + 8 * h) = v;
  }
  if (planes == 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4 v = {pack2(lo[8 * h], lo[8 * h + 1]), pack2(lo[8 * h + 2], lo[8 * h + 3]),
                 pack2(lo[8 * h + 4], lo[8 * h + 5]), pack2(lo[8 * h + 6], lo[8 * h + 7])};
      *reinterpret_cast<u32x4*>(dst + pstride + 8 * h) = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Sample side.  O planes: N x M BF16 row-major (row stride ld, plane stride
// pstride elements), K-contiguous; S = V split into BF16 planes (Vs).  1-D grid over
// (n tile, r tile, K range) with the XCD grouping of the FP32 kernel.
// ---------------------------------------------------------------------------
template <int BN, int BK, int PA, int PB>
__global__ __launch_bounds__(256, 1) void k_gemm16_sample_side(const u16* __restrict__ O, int64_t ld,
                                                               int64_t pstride, int64_t n, int64_t m,
                                                               const u16* __restrict__ Vs, int64_t vstride, int r,
                                                               float* __restrict__ ypart, int64_t kchunk,
                                                               bool vec_o, const DevStatus* st, int tn, int tj,
                                                               bool xcd_groups) {
  if (failed(st)) return;
  using G = Geo<BN, BK, PA, PB, false>;
  const int sw = tj * BN;                         // column width of the split planes of V
  constexpr int AU = BM * BK / 8;                 // 16-byte A units per plane
  constexpr int APT = (AU + 255) / 256;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem16[];
  u16* lds = reinterpret_cast<u16*>(smem16);

  int bx, by, bz;
  {
    const int id = blockIdx.x;
    int grp, i;
    if (xcd_groups) {
      const int xcd = id & 7, local = id >> 3;
      grp = (local / tn) * 8 + xcd;
      i = local % tn;
    } else {
      grp = id / tn;
      i = id % tn;
    }
    bx = i;
    by = grp % tj;
    bz = grp / tj;
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t n0 = (int64_t)bx * BM;
  const int j0 = by * BN;
  const int64_t kb = (int64_t)bz * kchunk;
  const int64_t ke = min(m, kb + kchunk);
  float* out = ypart + (int64_t)bz * n * r;

  f32x16 acc[2][G::TB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < G::TB; ++b) acc[a][b] = f32x16{0};

  u32x4 ra[PA][APT];
  constexpr int SPT = SUnit<BN, BK>::PER_T;
  u32x4 rs[PB][SPT];
  const int64_t kblocks = (m + 15) / 16;
  const bool inner = vec_o && (n0 + BM <= n);
  auto gload = [&](int64_t k0) __attribute__((always_inline)) {
    const bool fast = inner && k0 + BK <= ke;
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int u = 0; u < APT; ++u) {
        const int idx = t + 256 * u;
        if (idx >= AU) break;
        const int row = idx / (BK / 8), kq = (idx % (BK / 8)) * 8;
        const u16* src = O + p * pstride + (n0 + row) * ld + k0 + kq;
        if (fast) {
          ra[p][u] = *reinterpret_cast<const u32x4*>(src);
        } else {
          u16 e8[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) e8[e] = (n0 + row < n && k0 + kq + e < ke) ? src[e] : (u16)0;
          ra[p][u] = u32x4{pack2(e8[0], e8[1]), pack2(e8[2], e8[3]), pack2(e8[4], e8[5]), pack2(e8[6], e8[7])};
        }
      }
    s_load<BN, BK, PB, SPT>(rs, Vs, vstride, sw, kblocks, j0, k0, fast, t);
  };
  auto sstore = [&](int buf) __attribute__((always_inline)) {
    u16* S = lds + buf * G::STAGE;
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int u = 0; u < APT; ++u) {
        const int idx = t + 256 * u;
        if (idx >= AU) break;
        const int row = idx / (BK / 8), kq = (idx % (BK / 8)) * 8;
        *reinterpret_cast<u32x4*>(S + p * G::A_PLANE + row * G::LDK + kq) = ra[p][u];
      }
    s_store<BN, BK, PB, SPT>(rs, S + PA * G::A_PLANE, G::B_PLANE, G::LDK, t);
  };

  const int64_t nk = (ke - kb + BK - 1) / BK;
  gload(kb);
  sstore(0);
  __syncthreads();
  for (int64_t it = 0; it < nk; ++it) {
    const int buf = (int)(it & 1);
    if (it + 1 < nk) gload(kb + (it + 1) * BK);
    mma_stage<BN, BK, PA, PB, false>(acc, lds + buf * G::STAGE, wm, wn, lane);
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  const int x = lane & 31, h = lane >> 5;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < G::TB; ++b) {
      const int col = j0 + wn * (BN / 2) + b * 32 + x;
      if (col >= r) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = n0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < n) out[row * r + col] = acc[a][b][v];
      }
    }
}

// ---------------------------------------------------------------------------
// Parameter side Z = O^T S * scale.  O planes: N x M BF16 row-major (the K
// index is the row); S = Q_Y split into BF16 planes (Qs).  A unit of the O tile is 8 K-rows x 2
// parameters (8 four-byte loads, transposed into two 16-byte LDS rows).
// Scheduling as in the FP32 kernel: whole tiles for every full round of
// resident workgroups, the leftover tiles' K-steps shared out stream-K style
// (partials summed by k_streamk_fixup<BN>).
// ---------------------------------------------------------------------------
template <int BN, int BK, int PA, int PB>
__global__ __launch_bounds__(256, 1) void k_gemm16_param_side(const u16* __restrict__ O, int64_t ld, int64_t pstride,
                                                              int64_t n, int64_t m, const u16* __restrict__ Qs,
                                                              int64_t qstride, int r, float scale,
                                                              float* __restrict__ Z, bool vec_o, const DevStatus* st,
                                                              int tiles_j, int full_tiles, int64_t sk_units,
                                                              int sk_wgs, float* __restrict__ part) {
  if (failed(st)) return;
  using G = Geo<BN, BK, PA, PB, true>;
  const int sw = tiles_j * BN;                    // column width of the split planes of Q
  constexpr int AU = BK * (BM / 8);                // 16-byte units (8 parameters of one K-row) per plane
  constexpr int APT = (AU + 255) / 256;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem16[];
  u16* lds = reinterpret_cast<u16*>(smem16);

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  int64_t m0 = 0;
  int j0 = 0;
  bool inner = false;

  f32x16 acc[2][G::TB];
  u32x4 ro[PA][APT];
  constexpr int SPT = SUnit<BN, BK>::PER_T;
  u32x4 rs[PB][SPT];
  const int64_t kblocks = (n + 15) / 16;
  auto gload = [&](int64_t k0) __attribute__((always_inline)) {
    const bool fast = inner && k0 + BK <= n;
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int u = 0; u < APT; ++u) {
        const int unit = t + 256 * u;
        if (unit >= AU) break;
        const int kr = unit / (BM / 8), mq = (unit % (BM / 8)) * 8;
        const int64_t k = k0 + kr;
        const u16* src = O + p * pstride + k * ld + m0 + mq;
        if (fast) {
          ro[p][u] = *reinterpret_cast<const u32x4*>(src);
        } else {
          u16 e8[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) e8[e] = (k < n && m0 + mq + e < m) ? src[e] : (u16)0;
          ro[p][u] = u32x4{pack2(e8[0], e8[1]), pack2(e8[2], e8[3]), pack2(e8[4], e8[5]), pack2(e8[6], e8[7])};
        }
      }
    s_load<BN, BK, PB, SPT>(rs, Qs, qstride, sw, kblocks, j0, k0, fast, t);
  };
  auto sstore = [&](int buf) __attribute__((always_inline)) {
    u16* S = lds + buf * G::STAGE;
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int u = 0; u < APT; ++u) {
        const int unit = t + 256 * u;
        if (unit >= AU) break;
        const int kr = unit / (BM / 8), mq = (unit % (BM / 8)) * 8;
        *reinterpret_cast<u32x4*>(S + p * G::A_PLANE + kr * G::LDM + mq) = ro[p][u];
      }
    s_store<BN, BK, PB, SPT>(rs, S + PA * G::A_PLANE, G::B_PLANE, G::LDK, t);
  };
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) __attribute__((always_inline)) {
    m0 = (tile / tiles_j) * BM;
    j0 = (int)(tile % tiles_j) * BN;
    inner = vec_o && (m0 + BM <= m);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) acc[a][b] = f32x16{0};
    gload(kb * BK);
    sstore(0);
    __syncthreads();
    for (int64_t it = kb; it < ke; ++it) {
      const int buf = (int)((it - kb) & 1);
      if (it + 1 < ke) gload((it + 1) * BK);
      mma_stage<BN, BK, PA, PB, true>(acc, lds + buf * G::STAGE, wm, wn, lane);
      if (it + 1 < ke) sstore(buf ^ 1);
      __syncthreads();
    }
  };

  const int x = lane & 31, h = lane >> 5;
  const int64_t nk = (n + BK - 1) / BK;
  if ((int)blockIdx.x < full_tiles) {
    run(blockIdx.x, 0, nk);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) {
        const int col = j0 + wn * (BN / 2) + b * 32 + x;
        if (col >= r) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = m0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          if (row < m) Z[row * r + col] = acc[a][b][v] * scale;
        }
      }
    return;
  }
  // stream-K: this workgroup's range of K-steps touches at most two tiles
  // (it is never longer than one tile's nk steps); written out without a
  // loop, so that no epilogue address is hoisted over the K-loop
  const int64_t wg = (int64_t)blockIdx.x - full_tiles;
  int64_t u = wg * sk_units / sk_wgs;
  const int64_t uend = (wg + 1) * sk_units / sk_wgs;
  auto segment = [&](int seg) __attribute__((always_inline)) {
    const int64_t tl = u / nk, kb = u - tl * nk, ke = min(nk, kb + (uend - u));
    run(full_tiles + tl, kb, ke);
    float* outp = part + (wg * 2 + seg) * (int64_t)(BM * BN);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) {
        const int col = wn * (BN / 2) + b * 32 + x;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          outp[row * BN + col] = acc[a][b][v];
        }
      }
    u += ke - kb;
  };
  if (u < uend) segment(0);
  if (u < uend) segment(1);
}

// ---------------------------------------------------------------------------
// Direct-to-LDS forms of the BF16 products (used when the rows of O are
// 16-byte aligned and M is a multiple of 8).  As in the FP32 products,
// global_load_lds_dwordx4 fills a ring of three K-steps in LDS without
// passing through registers; a step's copies are waited for with an explicit
// vmcnt and published by a bare s_barrier.
//
// LDS layouts of one ring slot (per plane):
//   S (split skinny operand): the K-blocked global layout [k-block][j][16]
//     of the tile's columns, copied as is; a B fragment (8 K-values of one
//     column) is one 16-byte read, 32 bytes apart across lanes.
//   sample-side O (rows K-contiguous): CPR = BK/8 chunks of 16 bytes per row,
//     chunk c of row i at slot CPR*i + (c ^ swz(i)), swz(i) = (i >> 2) & 3
//     when CPR = 4; an A fragment is one 16-byte read.
//   parameter-side O (rows are the K index): four K-rows of 128 parameters
//     per copy instruction; chunk c (8 parameters) of the instruction's row
//     rho at slot 16 rho + (c ^ 2 rho).  An A fragment (8 K-values of one
//     parameter) is two ds_read_b64_tr_b16: in a group of 16 lanes, lane
//     4 rho + q points at parameters 4q..4q+3 of K-row rho, and lane j gets
//     K-rows 0..3 of parameter j (the swizzle keeps the group's four rows
//     in different banks).
// ---------------------------------------------------------------------------
namespace {
#define WSSR_LDS16(p) ((__attribute__((address_space(3))) void*)(p))
typedef short v4i16 __attribute__((ext_vector_type(4)));
constexpr int kStages16 = 3;

template <int BN, int BK, int PA, int PB, bool PARAM>
struct G16 {
  static constexpr int TB = BN / 64;                  // 32-column MFMA tiles per wave
  static constexpr int KB = BK / 16;                  // MFMA K-blocks per step
  static constexpr int A_PLANE = BM * BK * 2;         // bytes
  static constexpr int S_PLANE = BN * BK * 2;
  static constexpr int STAGE = PA * A_PLANE + PB * S_PLANE;
  static constexpr int A_INSTR = A_PLANE / 1024;      // copy instructions per plane and step
  static constexpr int S_INSTR = S_PLANE / 1024;
  static constexpr int PER_STEP = (PA * A_INSTR + PB * S_INSTR) / 4;   // per wave
  static_assert((PA * A_INSTR) % 4 == 0 && (PB * S_INSTR) % 4 == 0, "copies split evenly over four waves");
};

template <int N>
__device__ __forceinline__ void wait_vmcnt16() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// copies of one step of the split skinny operand: k-blocks kb0.. of columns
// j0..j0+BN of each plane (plane stride pstride elements, sw columns)
template <int BN, int BK, int PB>
__device__ __forceinline__ void dma16_s(const u16* __restrict__ Ss, int64_t pstride, int sw, int64_t kblocks,
                                        int64_t kb0, int j0, const u16* __restrict__ zeros, unsigned char* dst,
                                        int w, int lane) {
  constexpr int PER_KB = BN * 32 / 1024;   // instructions per k-block and plane
  constexpr int TOT = PB * (BK / 16) * PER_KB;
#pragma unroll
  for (int q = 0; q < TOT / 4; ++q) {
    const int ins = w * (TOT / 4) + q;
    const int pl = ins / ((BK / 16) * PER_KB), rem = ins % ((BK / 16) * PER_KB);
    const int kb = rem / PER_KB, part = rem % PER_KB;
    const int64_t blk = kb0 + kb;
    const int64_t e = (blk * sw + j0) * 16 + (int64_t)part * 512 + lane * 8;   // 8 elements per lane
    const u16* src = blk < kblocks ? Ss + pl * pstride + e : zeros;
    __builtin_amdgcn_global_load_lds((const void*)src,
                                     WSSR_LDS16(dst + pl * (BN * BK * 2) + kb * (BN * 32) + part * 1024), 16, 0, 0);
  }
}

// MFMAs of one ring slot: acc[a][b] += sum over products of A_p B_q.
// On the parameter side the fragments of K-block kb + 1 are read from LDS
// before the MFMAs of K-block kb are issued, so that the latency of their
// transposing reads hides behind those MFMAs (on the sample side a second set
// of fragment registers measured no gain; the 256-column tile with two O
// planes has no registers for it, and the 512-column tiles take one K-block
// per step).
// mid() runs once, right after the first K-block's MFMAs are issued: the
// copies for a later ring slot go out while those MFMAs execute instead of
// ahead of them.
template <int BN, int BK, int PA, int PB, bool PARAM, class Mid>
__device__ __forceinline__ void mma16_slot(f32x16 (&acc)[2][BN / 64], const unsigned char* S, int wm, int wn,
                                           int lane, Mid&& mid) {
  using G = G16<BN, BK, PA, PB, PARAM>;
  const int x = lane & 31, hh = lane >> 5;
  auto frags = [&](int kb, u32x4 (&av)[PA][2], u32x4 (&bv)[PB][G::TB]) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const unsigned char* A = S + p * G::A_PLANE;
        if constexpr (!PARAM) {
          constexpr int CPR = BK / 8;
          const int row = wm * 64 + a * 32 + x;
          const int c = 2 * kb + hh;
          const int swz = CPR == 4 ? ((row >> 2) & 3) : 0;
          av[p][a] = *reinterpret_cast<const u32x4*>(A + (row * CPR + (c ^ swz)) * 16);
        } else {
          // group g = lane / 16: parameters mbase..mbase+15, K-rows kbase.. (+4s)
          const int g = lane >> 4, i = lane & 15;
          const int rho = i >> 2, q = i & 3;
          const int mbase = wm * 64 + a * 32 + 16 * (g & 1);
          const int c = (mbase >> 3) + (q >> 1);
          v4i16 part[2];
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int k = 16 * kb + 8 * (g >> 1) + 4 * s2 + rho;   // this lane's K-row
            const unsigned char* src = A + (k >> 2) * 1024 + rho * 256 + ((c ^ (2 * rho)) * 16) + (q & 1) * 8;
            part[s2] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) v4i16*)src);
          }
          const unsigned lo0 = (unsigned)(unsigned short)part[0][0] | ((unsigned)(unsigned short)part[0][1] << 16);
          const unsigned lo1 = (unsigned)(unsigned short)part[0][2] | ((unsigned)(unsigned short)part[0][3] << 16);
          const unsigned hi0 = (unsigned)(unsigned short)part[1][0] | ((unsigned)(unsigned short)part[1][1] << 16);
          const unsigned hi1 = (unsigned)(unsigned short)part[1][2] | ((unsigned)(unsigned short)part[1][3] << 16);
          av[p][a] = u32x4{lo0, lo1, hi0, hi1};
        }
      }
#pragma unroll
    for (int q = 0; q < PB; ++q)
#pragma unroll
      for (int b = 0; b < G::TB; ++b)
        bv[q][b] = *reinterpret_cast<const u32x4*>(S + PA * G::A_PLANE + q * G::S_PLANE + kb * (BN * 32) +
                                                   (wn * (BN / 2) + b * 32 + x) * 32 + hh * 16);
  };
  constexpr bool PF = PARAM && BN <= 256 && !(BN == 256 && PA == 2);
  u32x4 av[2][PA][2], bv[2][PB][G::TB];
  if constexpr (PF) frags(0, av[0], bv[0]);
#pragma unroll
  for (int kb = 0; kb < G::KB; ++kb) {
    if constexpr (PF) {
      if (kb + 1 < G::KB) frags(kb + 1, av[(kb + 1) & 1], bv[(kb + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
    } else {
      frags(kb, av[kb & 1], bv[kb & 1]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) {
        acc[a][b] = mfma_bf16(av[kb & 1][0][a], bv[kb & 1][0][b], acc[a][b]);
        if constexpr (PB == 2) acc[a][b] = mfma_bf16(av[kb & 1][0][a], bv[kb & 1][1][b], acc[a][b]);
        if constexpr (PA == 2) acc[a][b] = mfma_bf16(av[kb & 1][1][a], bv[kb & 1][0][b], acc[a][b]);
      }
    if (kb == 0) mid();
  }
}
}  // namespace

// Sample side, direct-to-LDS form (arguments as k_gemm16_sample_side, plus a
// zero buffer of at least 16 bytes).
template <int BN, int BK, int PA, int PB>
__global__ __launch_bounds__(256, 1) void k_gemm16_sample_side_dma(const u16* __restrict__ O, int64_t ld,
                                                                   int64_t pstride, int64_t n, int64_t m,
                                                                   const u16* __restrict__ Vs, int64_t vstride, int r,
                                                                   float* __restrict__ ypart, int64_t kchunk,
                                                                   const u16* __restrict__ zeros,
                                                                   const DevStatus* st, int tn, int tj,
                                                                   bool xcd_groups) {
  if (failed(st)) return;
  using G = G16<BN, BK, PA, PB, false>;
  constexpr int CPR = BK / 8;
  extern __shared__ __attribute__((aligned(16))) unsigned char sm16[];
  const int sw = tj * BN;
  int bx, by, bz;
  {
    const int id = blockIdx.x;
    int grp, i;
    if (xcd_groups) {
      const int xcd = id & 7, local = id >> 3;
      grp = (local / tn) * 8 + xcd;
      i = local % tn;
    } else {
      grp = id / tn;
      i = id % tn;
    }
    bx = i;
    by = grp % tj;
    bz = grp / tj;
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int x = lane & 31, hh = lane >> 5;
  const int64_t n0 = (int64_t)bx * BM;
  const int j0 = by * BN;
  const int64_t kb = (int64_t)bz * kchunk;
  const int64_t ke = min(m, kb + kchunk);
  const int64_t kblocks = (m + 15) / 16;
  float* out = ypart + (int64_t)bz * n * r;

  f32x16 acc[2][G::TB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < G::TB; ++b) acc[a][b] = f32x16{0};

  auto issue = [&](int64_t k0, int slot) __attribute__((always_inline)) {
    unsigned char* base = sm16 + slot * G::STAGE;
#pragma unroll
    for (int q = 0; q < PA * G::A_INSTR / 4; ++q) {
      const int ins = w * (PA * G::A_INSTR / 4) + q;
      const int pl = ins / G::A_INSTR, pi = ins % G::A_INSTR;
      const int slotid = pi * 64 + lane;                // 16-byte slot of the plane
      const int row = slotid / CPR;
      const int c = (slotid % CPR) ^ (CPR == 4 ? ((row >> 2) & 3) : 0);
      const int64_t gr = min(n0 + row, n - 1);
      const int64_t gk = k0 + 8 * c;
      const u16* src = gk < ke ? O + pl * pstride + gr * ld + gk : zeros;
      __builtin_amdgcn_global_load_lds((const void*)src, WSSR_LDS16(base + pl * G::A_PLANE + pi * 1024), 16, 0, 0);
    }
    dma16_s<BN, BK, PB>(Vs, vstride, sw, kblocks, k0 / 16, j0, zeros, base + PA * G::A_PLANE, w, lane);
  };

  const int64_t ns = (ke - kb + BK - 1) / BK;
  if (ns > 0) issue(kb, 0);
  if (ns > 1) issue(kb + BK, 1);
  int slot = 0;
  for (int64_t it = 0; it < ns; ++it) {
    if (it + 1 < ns)
      wait_vmcnt16<G::PER_STEP>();
    else
      wait_vmcnt16<0>();
    __builtin_amdgcn_s_barrier();
    mma16_slot<BN, BK, PA, PB, false>(acc, sm16 + slot * G::STAGE, wm, wn, lane, [&] {
      if (it + 2 < ns) issue(kb + (it + 2) * BK, slot == 0 ? 2 : slot - 1);
    });
    slot = slot == 2 ? 0 : slot + 1;
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < G::TB; ++b) {
      const int col = j0 + wn * (BN / 2) + b * 32 + x;
      if (col >= r) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = n0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
        if (row < n) out[row * r + col] = acc[a][b][v];
      }
    }
}

// Parameter side, direct-to-LDS form (arguments as k_gemm16_param_side, plus
// a zero buffer of at least 16 bytes).  Below 512 columns the register budget
// is held to two waves per SIMD (two workgroups per compute unit where LDS
// allows); at one wave per SIMD the 256-column form waited on its copies
// most of the time.
template <int BN, int BK, int PA, int PB>
__global__ __launch_bounds__(256, BN == 512 ? 1 : 2) void k_gemm16_param_side_dma(const u16* __restrict__ O, int64_t ld,
                                                                  int64_t pstride, int64_t n, int64_t m,
                                                                  const u16* __restrict__ Qs, int64_t qstride, int r,
                                                                  float scale, float* __restrict__ Z,
                                                                  const u16* __restrict__ zeros, const DevStatus* st,
                                                                  int tiles_j, int full_tiles, int64_t sk_units,
                                                                  int sk_wgs, float* __restrict__ part) {
  if (failed(st)) return;
  using G = G16<BN, BK, PA, PB, true>;
  extern __shared__ __attribute__((aligned(16))) unsigned char sm16[];
  const int sw = tiles_j * BN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int x = lane & 31, hh = lane >> 5;
  const int64_t kblocks = (n + 15) / 16;
  const int64_t mlast = ((m - 1) / 8) * 8;   // first parameter of the last 16-byte chunk of a row
  int64_t m0 = 0;
  int j0 = 0;
  f32x16 acc[2][G::TB];

  auto issue = [&](int64_t ks, int slot) __attribute__((always_inline)) {
    unsigned char* base = sm16 + slot * G::STAGE;
    const int64_t k0 = ks * BK;
#pragma unroll
    for (int q = 0; q < PA * G::A_INSTR / 4; ++q) {
      const int ins = w * (PA * G::A_INSTR / 4) + q;
      const int pl = ins / G::A_INSTR, pi = ins % G::A_INSTR;   // K-rows 4 pi .. 4 pi + 3
      const int rho = lane >> 4, c = (lane & 15) ^ (2 * rho);
      const int64_t k = min(k0 + 4 * pi + rho, n - 1);
      const int64_t mm = min(m0 + 8 * c, mlast);
      __builtin_amdgcn_global_load_lds((const void*)(O + pl * pstride + k * ld + mm),
                                       WSSR_LDS16(base + pl * G::A_PLANE + pi * 1024), 16, 0, 0);
    }
    dma16_s<BN, BK, PB>(Qs, qstride, sw, kblocks, k0 / 16, j0, zeros, base + PA * G::A_PLANE, w, lane);
  };
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) __attribute__((always_inline)) {
    m0 = (tile / tiles_j) * BM;
    j0 = (int)(tile % tiles_j) * BN;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) acc[a][b] = f32x16{0};
    const int64_t ns = ke - kb;
    wait_vmcnt16<0>();
    if (ns > 0) issue(kb, 0);
    if (ns > 1) issue(kb + 1, 1);
    int slot = 0;
    for (int64_t it = 0; it < ns; ++it) {
      if (it + 1 < ns)
        wait_vmcnt16<G::PER_STEP>();
      else
        wait_vmcnt16<0>();
      __builtin_amdgcn_s_barrier();
      mma16_slot<BN, BK, PA, PB, true>(acc, sm16 + slot * G::STAGE, wm, wn, lane, [&] {
        if (it + 2 < ns) issue(kb + it + 2, slot == 0 ? 2 : slot - 1);
      });
      slot = slot == 2 ? 0 : slot + 1;
    }
    __syncthreads();
  };

  const int64_t nk = (n + BK - 1) / BK;
  if ((int)blockIdx.x < full_tiles) {
    run(blockIdx.x, 0, nk);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) {
        const int col = j0 + wn * (BN / 2) + b * 32 + x;
        if (col >= r) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = m0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
          if (row < m) Z[row * r + col] = acc[a][b][v] * scale;
        }
      }
    return;
  }
  const int64_t wg = (int64_t)blockIdx.x - full_tiles;
  int64_t u = wg * sk_units / sk_wgs;
  const int64_t uend = (wg + 1) * sk_units / sk_wgs;
  auto segment = [&](int seg) __attribute__((always_inline)) {
    const int64_t tl = u / nk, kb = u - tl * nk, ke = min(nk, kb + (uend - u));
    run(full_tiles + tl, kb, ke);
    float* outp = part + (wg * 2 + seg) * (int64_t)(BM * BN);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < G::TB; ++b) {
        const int col = wn * (BN / 2) + b * 32 + x;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
          outp[row * BN + col] = acc[a][b][v];
        }
      }
    u += ke - kb;
  };
  if (u < uend) segment(0);
  if (u < uend) segment(1);
}

// dynamic LDS bytes of a direct-to-LDS BF16 product kernel
size_t gemm16_dma_lds(int bn, int bk, int pa, int pb) {
  return (size_t)kStages16 * ((size_t)pa * BM * bk * 2 + (size_t)pb * bn * bk * 2);
}

#define WSSR_GEMM16_DMA_INST(BN, BK, PA, PB)                                                                         \
  template __global__ void k_gemm16_sample_side_dma<BN, BK, PA, PB>(                                                \
      const u16*, int64_t, int64_t, int64_t, int64_t, const u16*, int64_t, int, float*, int64_t, const u16*,        \
      const DevStatus*, int, int, bool);                                                                            \
  template __global__ void k_gemm16_param_side_dma<BN, BK, PA, PB>(                                                 \
      const u16*, int64_t, int64_t, int64_t, int64_t, const u16*, int64_t, int, float, float*, const u16*,          \
      const DevStatus*, int, int, int64_t, int, float*);
WSSR_GEMM16_DMA_INST(64, 32, 1, 1)
WSSR_GEMM16_DMA_INST(64, 32, 1, 2)
WSSR_GEMM16_DMA_INST(64, 32, 2, 2)
WSSR_GEMM16_DMA_INST(128, 32, 1, 1)
WSSR_GEMM16_DMA_INST(128, 32, 1, 2)
WSSR_GEMM16_DMA_INST(128, 32, 2, 2)
WSSR_GEMM16_DMA_INST(256, 32, 1, 1)
WSSR_GEMM16_DMA_INST(256, 32, 1, 2)
WSSR_GEMM16_DMA_INST(256, 32, 2, 2)
WSSR_GEMM16_DMA_INST(512, 32, 1, 1)
WSSR_GEMM16_DMA_INST(512, 16, 1, 2)
WSSR_GEMM16_DMA_INST(512, 16, 2, 2)

// dynamic LDS bytes of a BF16 product kernel
size_t gemm16_lds(int bn, int bk, int pa, int pb) {
  const size_t a_k = (size_t)BM * (bk + 8), a_t = (size_t)bk * (BM + 8);
  return 2 * (pa * (a_k > a_t ? a_k : a_t) + (size_t)pb * bn * (bk + 8)) * sizeof(u16);
}

#define WSSR_GEMM16_INST(BN, BK, PA, PB)                                                                             \
  template __global__ void k_gemm16_sample_side<BN, BK, PA, PB>(const u16*, int64_t, int64_t, int64_t, int64_t,     \
                                                                const u16*, int64_t, int, float*, int64_t, bool,    \
                                                                const DevStatus*, int, int, bool);                  \
  template __global__ void k_gemm16_param_side<BN, BK, PA, PB>(const u16*, int64_t, int64_t, int64_t, int64_t,      \
                                                               const u16*, int64_t, int, float, float*, bool,       \
                                                               const DevStatus*, int, int, int64_t, int, float*);
WSSR_GEMM16_INST(128, 32, 1, 1)
WSSR_GEMM16_INST(128, 32, 1, 2)
WSSR_GEMM16_INST(128, 32, 2, 2)
WSSR_GEMM16_INST(256, 32, 1, 1)
WSSR_GEMM16_INST(256, 32, 1, 2)
WSSR_GEMM16_INST(256, 32, 2, 2)
WSSR_GEMM16_INST(512, 16, 1, 1)
WSSR_GEMM16_INST(512, 16, 1, 2)
WSSR_GEMM16_INST(512, 16, 2, 2)

}  // namespace wssr
