// The two tall-skinny products of each subspace-iteration pass (Alg. 1) with O
// stored in BF16: BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.
//
//   sample side    Ypart[s] = O[:, Ks] S[Ks, :]      (N x r, K = M split into ranges)
//   parameter side Z = O^T S * scale                  (M x r, K = N)
//
// S (V or Q_Y) arrives in FP32 and is rounded to BF16 on its way into LDS:
// S = S_hi + S_lo with S_hi = RNE(S), S_lo = RNE(S - S_hi).  O has PA planes
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
// read.  Operands whose global rows are the K index (O on the parameter side,
// S on both sides) are loaded as 8 K-rows per thread and transposed in
// registers, so their LDS stores are 16-byte stores too.  The next K-step's
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

// Tile geometry shared by the kernels.
template <int BN, int BK, int PA, int PB>
struct Geo {
  static constexpr int LDK = BK + 8;                        // LDS row stride (bf16 elements)
  static constexpr int A_PLANE = BM * LDK;                  // elements per A plane
  static constexpr int B_PLANE = BN * LDK;
  static constexpr int STAGE = PA * A_PLANE + PB * B_PLANE;  // elements per stage
  static constexpr int TB = BN / 64;                        // 32-column MFMA tiles per wave
};

// MFMAs of one LDS stage: acc[a][b] += sum over products of A_p[rows] B_q[cols]^T
template <int BN, int BK, int PA, int PB>
__device__ __forceinline__ void mma_stage(f32x16 (&acc)[2][BN / 64], const u16* __restrict__ S, int wm, int wn,
                                          int lane) {
  using G = Geo<BN, BK, PA, PB>;
  const int x = lane & 31, h = lane >> 5;
#pragma unroll
  for (int kc = 0; kc < BK / 16; ++kc) {
    u32x4 av[PA][2], bv[PB][G::TB];
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[p][a] = *reinterpret_cast<const u32x4*>(S + p * G::A_PLANE + (wm * 64 + a * 32 + x) * G::LDK + kc * 16 +
                                                   8 * h);
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

// ---- S loader: FP32 rows k (K index) x columns j, to K-contiguous BF16 planes.
// A unit is 8 K-rows x 4 columns: 8 float4 loads, transposed into 4 columns of
// 8 BF16 (one 16-byte store per column and plane).
template <int BN, int BK>
struct SUnit {
  static constexpr int UNITS = (BK / 8) * (BN / 4);
  static constexpr int PER_T = (UNITS + 255) / 256;
};

template <int BN, int BK, int PT>
__device__ __forceinline__ void s_load(f32x4 (&rs)[PT][8], const float* __restrict__ Sm, int r, int j0, int64_t k0,
                                       int64_t kend, bool fast, int t) {
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int unit = t + 256 * u;
    if (unit >= SUnit<BN, BK>::UNITS) break;
    const int kg = unit / (BN / 4), cq = (unit % (BN / 4)) * 4;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t k = k0 + kg * 8 + s;
      const int c = j0 + cq;
      if (fast) {
        rs[u][s] = *reinterpret_cast<const f32x4*>(Sm + k * r + c);
      } else {
        f32x4 v = f32x4{0};
        if (k < kend) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (c + e < r) v[e] = Sm[k * r + c + e];
        }
        rs[u][s] = v;
      }
    }
  }
}

template <int BN, int BK, int PB, int PT>
__device__ __forceinline__ void s_store(const f32x4 (&rs)[PT][8], u16* __restrict__ Bp, int plane_elems, int ldk,
                                        int t) {
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int unit = t + 256 * u;
    if (unit >= SUnit<BN, BK>::UNITS) break;
    const int kg = unit / (BN / 4), cq = (unit % (BN / 4)) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      u16 hi[8], lo[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) split_bf16(rs[u][s][e], hi[s], lo[s]);
      u32x4 vh = {pack2(hi[0], hi[1]), pack2(hi[2], hi[3]), pack2(hi[4], hi[5]), pack2(hi[6], hi[7])};
      *reinterpret_cast<u32x4*>(Bp + (cq + e) * ldk + kg * 8) = vh;
      if constexpr (PB == 2) {
        u32x4 vl = {pack2(lo[0], lo[1]), pack2(lo[2], lo[3]), pack2(lo[4], lo[5]), pack2(lo[6], lo[7])};
        *reinterpret_cast<u32x4*>(Bp + plane_elems + (cq + e) * ldk + kg * 8) = vl;
      }
    }
  }
}
}  // namespace

// ---------------------------------------------------------------------------
// Sample side.  O planes: N x M BF16 row-major (row stride ld, plane stride
// pstride elements), K-contiguous; S = V: M x r FP32.  1-D grid over
// (n tile, r tile, K range) with the XCD grouping of the FP32 kernel.
// ---------------------------------------------------------------------------
template <int BN, int BK, int PA, int PB>
__global__ __launch_bounds__(256, 1) void k_gemm16_sample_side(const u16* __restrict__ O, int64_t ld,
                                                               int64_t pstride, int64_t n, int64_t m,
                                                               const float* __restrict__ V, int r,
                                                               float* __restrict__ ypart, int64_t kchunk,
                                                               bool vec_o, bool vec_v, const DevStatus* st, int tn,
                                                               int tj, bool xcd_groups) {
  if (failed(st)) return;
  using G = Geo<BN, BK, PA, PB>;
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
  f32x4 rs[SPT][8];
  const bool inner = vec_o && vec_v && (n0 + BM <= n) && (j0 + BN <= r);
  auto gload = [&](int64_t k0) {
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
    s_load<BN, BK, SPT>(rs, V, r, j0, k0, ke, fast, t);
  };
  auto sstore = [&](int buf) {
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
    mma_stage<BN, BK, PA, PB>(acc, lds + buf * G::STAGE, wm, wn, lane);
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
// index is the row); S = Q: N x r FP32.  A unit of the O tile is 8 K-rows x 2
// parameters (8 four-byte loads, transposed into two 16-byte LDS rows).
// Scheduling as in the FP32 kernel: whole tiles for every full round of
// resident workgroups, the leftover tiles' K-steps shared out stream-K style
// (partials summed by k_streamk_fixup<BN>).
// ---------------------------------------------------------------------------
template <int BN, int BK, int PA, int PB>
__global__ __launch_bounds__(256, 1) void k_gemm16_param_side(const u16* __restrict__ O, int64_t ld, int64_t pstride,
                                                              int64_t n, int64_t m, const float* __restrict__ Q,
                                                              int r, float scale, float* __restrict__ Z, bool vec_o,
                                                              bool vec_q, const DevStatus* st, int tiles_j,
                                                              int full_tiles, int64_t sk_units, int sk_wgs,
                                                              float* __restrict__ part) {
  if (failed(st)) return;
  using G = Geo<BN, BK, PA, PB>;
  constexpr int AU = (BK / 8) * (BM / 2);          // 8 x 2 units per plane
  constexpr int APT = (AU + 255) / 256;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem16[];
  u16* lds = reinterpret_cast<u16*>(smem16);

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  int64_t m0 = 0;
  int j0 = 0;
  bool inner = false;

  f32x16 acc[2][G::TB];
  unsigned ro[PA][APT][8];
  constexpr int SPT = SUnit<BN, BK>::PER_T;
  f32x4 rs[SPT][8];
  auto gload = [&](int64_t k0) {
    const bool fast = inner && k0 + BK <= n;
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int u = 0; u < APT; ++u) {
        const int unit = t + 256 * u;
        if (unit >= AU) break;
        const int kg = unit / (BM / 2), mp = (unit % (BM / 2)) * 2;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int64_t k = k0 + kg * 8 + s;
          const u16* src = O + p * pstride + k * ld + m0 + mp;
          if (fast) {
            ro[p][u][s] = *reinterpret_cast<const unsigned*>(src);
          } else {
            const u16 e0 = (k < n && m0 + mp < m) ? src[0] : (u16)0;
            const u16 e1 = (k < n && m0 + mp + 1 < m) ? src[1] : (u16)0;
            ro[p][u][s] = pack2(e0, e1);
          }
        }
      }
    s_load<BN, BK, SPT>(rs, Q, r, j0, k0, n, fast, t);
  };
  auto sstore = [&](int buf) {
    u16* S = lds + buf * G::STAGE;
#pragma unroll
    for (int p = 0; p < PA; ++p)
#pragma unroll
      for (int u = 0; u < APT; ++u) {
        const int unit = t + 256 * u;
        if (unit >= AU) break;
        const int kg = unit / (BM / 2), mp = (unit % (BM / 2)) * 2;
        const unsigned* d = ro[p][u];
        // even parameter: low halves of the 8 words; odd: high halves
        u32x4 ev = {__builtin_amdgcn_perm(d[1], d[0], 0x05040100u), __builtin_amdgcn_perm(d[3], d[2], 0x05040100u),
                    __builtin_amdgcn_perm(d[5], d[4], 0x05040100u), __builtin_amdgcn_perm(d[7], d[6], 0x05040100u)};
        u32x4 od = {__builtin_amdgcn_perm(d[1], d[0], 0x07060302u), __builtin_amdgcn_perm(d[3], d[2], 0x07060302u),
                    __builtin_amdgcn_perm(d[5], d[4], 0x07060302u), __builtin_amdgcn_perm(d[7], d[6], 0x07060302u)};
        *reinterpret_cast<u32x4*>(S + p * G::A_PLANE + mp * G::LDK + kg * 8) = ev;
        *reinterpret_cast<u32x4*>(S + p * G::A_PLANE + (mp + 1) * G::LDK + kg * 8) = od;
      }
    s_store<BN, BK, PB, SPT>(rs, S + PA * G::A_PLANE, G::B_PLANE, G::LDK, t);
  };
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) {
    m0 = (tile / tiles_j) * BM;
    j0 = (int)(tile % tiles_j) * BN;
    inner = vec_o && vec_q && (m0 + BM <= m) && (j0 + BN <= r);
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
      mma_stage<BN, BK, PA, PB>(acc, lds + buf * G::STAGE, wm, wn, lane);
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
  const int64_t wg = (int64_t)blockIdx.x - full_tiles;
  const int64_t ubeg = wg * sk_units / sk_wgs, uend = (wg + 1) * sk_units / sk_wgs;
  int seg = 0;
  for (int64_t u = ubeg; u < uend; ++seg) {
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
  }
}

// dynamic LDS bytes of a BF16 product kernel
size_t gemm16_lds(int bn, int bk, int pa, int pb) {
  return (size_t)2 * (pa * BM + pb * bn) * (bk + 8) * sizeof(u16);
}

#define WSSR_GEMM16_INST(BN, BK, PA, PB)                                                                             \
  template __global__ void k_gemm16_sample_side<BN, BK, PA, PB>(const u16*, int64_t, int64_t, int64_t, int64_t,     \
                                                                const float*, int, float*, int64_t, bool, bool,     \
                                                                const DevStatus*, int, int, bool);                  \
  template __global__ void k_gemm16_param_side<BN, BK, PA, PB>(const u16*, int64_t, int64_t, int64_t, int64_t,      \
                                                               const float*, int, float, float*, bool, bool,        \
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
