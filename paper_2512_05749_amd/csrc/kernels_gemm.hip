// The two tall-skinny products of each subspace-iteration pass (Alg. 1), in
// FP32 on the 32x32x2 FP32 MFMA.
//
//   sample side    Ypart[s] = O[:, Ks] V[Ks, :]     (N x r, K = M split into S ranges)
//   parameter side Z = O^T Q * scale                 (M x r, K = N)
//
// Three forms, chosen by the host:
//   - register-staged (k_gemm_*_side<BN>, described first below): any
//     alignment of O and of the skinny operand;
//   - direct-to-LDS (k_gemm_*_side_dma<BN>): 16-byte aligned rows, a
//     three-slot LDS ring filled by global_load_lds; BN = 32 (sample side,
//     r <= 32) to 256;
//   - narrow parameter side (k_gemm_param_side_narrow): aligned rows and
//     r <= 32, O staged through registers four K-steps ahead.
//
// Register-staged workgroup: 256 threads = 4 waves in a 2 x 2 arrangement; output tile
// 128 rows x BN columns (BN = 64, 128 or 256 over the rank dimension); each
// wave owns a 64 x (BN/2) sub-tile = 2 x (BN/64) MFMA tiles of 32 x 32, i.e.
// 8 FP32 accumulator tiles at BN = 256.  K advances 16 at a time with one barrier per
// K-step; the next K-step's global loads are in flight during the MFMAs.
//
// Both operand tiles are kept K-contiguous in LDS ([row][k]), so a lane reads
// the four K values it needs for four MFMA steps with one 16-byte LDS read.
// Inside a K-step the contraction index is permuted: lane (x, h) = (l%32,
// l/32) feeds k = h*8 + s to MFMA step s (0 <= s < 8) for both operands.
// Operands whose global rows are not K-contiguous (V, Q and O in the
// parameter-side product) are transposed on their way into LDS; their loads
// map consecutive lanes to consecutive k so the transposed LDS writes do not
// conflict.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int BM = 128, BK = 16;
constexpr int LDK = BK + 4;   // LDS row length of a K-contiguous tile (floats)

// 32 k-steps' worth of MFMAs on one K-step of LDS tiles:
// acc[a][b] += A[a-block rows][k] * B[b-block cols][k].
template <int TA, int TB>
__device__ __forceinline__ void mma_kstep(f32x16 (&acc)[TA][TB], const float (*As)[LDK], int arow0,
                                          const float (*Bs)[LDK], int brow0, int x, int h) {
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    f32x4 av[TA], bv[TB];
#pragma unroll
    for (int a = 0; a < TA; ++a) av[a] = *reinterpret_cast<const f32x4*>(&As[arow0 + a * 32 + x][h * 8 + half * 4]);
#pragma unroll
    for (int b = 0; b < TB; ++b) bv[b] = *reinterpret_cast<const f32x4*>(&Bs[brow0 + b * 32 + x][h * 8 + half * 4]);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) acc[a][b] = mfma32x32x2(av[a][e], bv[b][e], acc[a][b]);
  }
}

// store a float4 that holds 4 consecutive columns c..c+3 of global row k into
// a K-contiguous LDS tile T[col][k]
__device__ __forceinline__ void st_transposed(float (*T)[LDK], int c, int k, f32x4 v) {
#pragma unroll
  for (int e = 0; e < 4; ++e) T[c + e][k] = v[e];
}
}  // namespace

// ---------------------------------------------------------------------------
// Sample side.  O is N x M row-major (K contiguous), V is M x r row-major.
// D[i = sample][j = rank]: A = O tile, B = V^T tile.  1-D grid of
// tn * tj * S workgroups over (n tile, r tile, K range).  The workgroups that
// read the same rows of V (same K range and r tile: one "group" of tn) are
// placed on the same XCD when the group count is a multiple of the 8 XCDs
// (workgroups are dispatched round-robin over the XCDs by linear index), so
// each V range is fetched into one L2 instead of all eight.
// ---------------------------------------------------------------------------
template <int BN>
__global__ __launch_bounds__(256, 2) void k_gemm_sample_side(const float* __restrict__ O, int64_t ld, int64_t n,
                                                             int64_t m, const float* __restrict__ V, int r,
                                                             float* __restrict__ ypart, int64_t kchunk,
                                                             bool vec_o, bool vec_v, const DevStatus* st, int tn,
                                                             int tj, bool xcd_groups) {
  if (failed(st)) return;
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
  constexpr int TB = BN / 64;                 // rank blocks per wave
  constexpr int AV = BM * BK / 4 / 256;       // float4 per thread for the O tile (2)
  constexpr int BV = BK * BN / 4 / 256;       // float4 per thread for the V tile (2 or 4)
  __shared__ __attribute__((aligned(16))) float As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN][LDK];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int x = lane & 31, h = lane >> 5;
  const int64_t n0 = (int64_t)bx * BM;
  const int j0 = by * BN;
  const int64_t kb = (int64_t)bz * kchunk;
  const int64_t ke = min(m, kb + kchunk);
  float* out = ypart + (int64_t)bz * n * r;

  f32x16 acc[2][TB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = f32x16{0};

  f32x4 ra[AV], rb[BV];
  // interior tiles (whole tile in range, 16-byte aligned rows) take plain
  // vector loads; edge tiles the guarded path
  const bool inner = vec_o && vec_v && (n0 + BM <= n) && (j0 + BN <= r);
  auto gload = [&](int64_t k0) {
    if (inner && k0 + BK <= ke) {
#pragma unroll
      for (int i = 0; i < AV; ++i) {
        const int idx = t + 256 * i;
        const int row = idx >> 2, kq = (idx & 3) * 4;
        ra[i] = *reinterpret_cast<const f32x4*>(O + (n0 + row) * ld + k0 + kq);
      }
#pragma unroll
      for (int i = 0; i < BV; ++i) {
        const int idx = t + 256 * i;
        const int krow = idx & (BK - 1), jq = (idx / BK) * 4;
        rb[i] = *reinterpret_cast<const f32x4*>(V + (k0 + krow) * r + j0 + jq);
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int idx = t + 256 * i;
      const int row = idx >> 2, kq = (idx & 3) * 4;
      const int64_t gi = n0 + row;
      ra[i] = (gi < n) ? load4(O + gi * ld, k0 + kq, ke, vec_o) : f32x4{0};
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int idx = t + 256 * i;
      const int krow = idx & (BK - 1), jq = (idx / BK) * 4;
      const int64_t gk = k0 + krow;
      rb[i] = (gk < ke) ? load4(V + gk * r, j0 + jq, r, vec_v) : f32x4{0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int idx = t + 256 * i;
      const int row = idx >> 2, kq = (idx & 3) * 4;
      *reinterpret_cast<f32x4*>(&As[buf][row][kq]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int idx = t + 256 * i;
      const int krow = idx & (BK - 1), jq = (idx / BK) * 4;
      st_transposed(Bs[buf], jq, krow, rb[i]);
    }
  };

  const int64_t nk = (ke - kb + BK - 1) / BK;
  gload(kb);
  sstore(0);
  __syncthreads();
  for (int64_t it = 0; it < nk; ++it) {
    const int buf = (int)(it & 1);
    if (it + 1 < nk) gload(kb + (it + 1) * BK);
    mma_kstep<2, TB>(acc, As[buf], wm * 64, Bs[buf], wn * (BN / 2), x, h);
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) {
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
// Parameter side Z = O^T Q * scale.  O is N x M row-major, Q is N x r
// row-major.  D[i = parameter][j = rank]: A = (O^T) tile, B = Q^T tile, both
// transposed into K-contiguous LDS rows.
//
// 1-D grid over output tiles, tile = mi * tiles_j + ji (neighbouring
// workgroups share the O tile).  Workgroups below full_tiles compute one whole
// tile each.  When sk_wgs > 0, the remaining tiles are shared out stream-K
// style: their K-steps, numbered u = t * nk + k over the leftover tiles t,
// are cut into sk_wgs equal contiguous ranges, and workgroup full_tiles + w
// accumulates range w.  A range is never longer than one tile's nk K-steps,
// so it touches at most two tiles; the partial sums go to
// part[(2 w + seg) * BM * BN] (seg = 0, 1 in tile order) and
// k_streamk_fixup adds them.  This keeps every round of the launch full when
// the tile count is not a multiple of the resident workgroup slots.
// ---------------------------------------------------------------------------
template <int BN>
__global__ __launch_bounds__(256, 2) void k_gemm_param_side(const float* __restrict__ O, int64_t ld, int64_t n,
                                                            int64_t m, const float* __restrict__ Q, int r,
                                                            float scale, float* __restrict__ Z, bool vec_o,
                                                            bool vec_q, const DevStatus* st, int tiles_j,
                                                            int full_tiles, int64_t sk_units, int sk_wgs,
                                                            float* __restrict__ part) {
  if (failed(st)) return;
  constexpr int TB = BN / 64;
  constexpr int OV = BK * BM / 4 / 256;       // float4 per thread for the O tile (2)
  constexpr int QV = BK * BN / 4 / 256;       // float4 per thread for the Q tile (2 or 4)
  __shared__ __attribute__((aligned(16))) float Os[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Qs[2][BN][LDK];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wj = w & 1;
  const int x = lane & 31, h = lane >> 5;
  int64_t m0 = 0;
  int j0 = 0;
  bool inner = false;

  f32x16 acc[2][TB];
  f32x4 ro[OV], rq[QV];
  auto gload = [&](int64_t k0) {
    if (inner && k0 + BK <= n) {
#pragma unroll
      for (int i = 0; i < OV; ++i) {
        const int idx = t + 256 * i;
        const int krow = idx & (BK - 1), cq = (idx / BK) * 4;
        ro[i] = *reinterpret_cast<const f32x4*>(O + (k0 + krow) * ld + m0 + cq);
      }
#pragma unroll
      for (int i = 0; i < QV; ++i) {
        const int idx = t + 256 * i;
        const int krow = idx & (BK - 1), cq = (idx / BK) * 4;
        rq[i] = *reinterpret_cast<const f32x4*>(Q + (k0 + krow) * r + j0 + cq);
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < OV; ++i) {
      const int idx = t + 256 * i;
      const int krow = idx & (BK - 1), cq = (idx / BK) * 4;
      const int64_t gk = k0 + krow;
      ro[i] = (gk < n) ? load4(O + gk * ld, m0 + cq, m, vec_o) : f32x4{0};
    }
#pragma unroll
    for (int i = 0; i < QV; ++i) {
      const int idx = t + 256 * i;
      const int krow = idx & (BK - 1), cq = (idx / BK) * 4;
      const int64_t gk = k0 + krow;
      rq[i] = (gk < n) ? load4(Q + gk * r, j0 + cq, r, vec_q) : f32x4{0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < OV; ++i) {
      const int idx = t + 256 * i;
      const int krow = idx & (BK - 1), cq = (idx / BK) * 4;
      st_transposed(Os[buf], cq, krow, ro[i]);
    }
#pragma unroll
    for (int i = 0; i < QV; ++i) {
      const int idx = t + 256 * i;
      const int krow = idx & (BK - 1), cq = (idx / BK) * 4;
      st_transposed(Qs[buf], cq, krow, rq[i]);
    }
  };
  // acc = the product of tile `tile` over K-steps [kb, ke)
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) {
    m0 = (tile / tiles_j) * BM;
    j0 = (int)(tile % tiles_j) * BN;
    inner = vec_o && vec_q && (m0 + BM <= m) && (j0 + BN <= r);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) acc[a][b] = f32x16{0};
    gload(kb * BK);
    sstore(0);
    __syncthreads();
    for (int64_t it = kb; it < ke; ++it) {
      const int buf = (int)((it - kb) & 1);
      if (it + 1 < ke) gload((it + 1) * BK);
      mma_kstep<2, TB>(acc, Os[buf], wm * 64, Qs[buf], wj * (BN / 2), x, h);
      if (it + 1 < ke) sstore(buf ^ 1);
      __syncthreads();
    }
  };

  const int64_t nk = (n + BK - 1) / BK;
  if ((int)blockIdx.x < full_tiles) {
    run(blockIdx.x, 0, nk);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int col = j0 + wj * (BN / 2) + b * 32 + x;
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
    float* out = part + (wg * 2 + seg) * (int64_t)(BM * BN);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int col = wj * (BN / 2) + b * 32 + x;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          out[row * BN + col] = acc[a][b][v];
        }
      }
    u += ke - kb;
  }
}

// Adds the stream-K partials of the leftover tiles in workgroup order (fixed,
// so the result is reproducible) and writes them, scaled, into Z.
// grid (leftover tiles, BM * BN / 1024), 256 threads of 4 consecutive columns.
template <int BN>
__global__ __launch_bounds__(256) void k_streamk_fixup(const float* __restrict__ part, float* __restrict__ Z,
                                                       int64_t m, int r, float scale, int tiles_j, int full_tiles,
                                                       int64_t nk, int64_t sk_units, int sk_wgs,
                                                       const DevStatus* st) {
  if (failed(st)) return;
  const int64_t tl = blockIdx.x;
  const int e0 = (blockIdx.y * 256 + threadIdx.x) * 4;
  const int row = e0 / BN, col = e0 % BN;
  const int64_t tile = full_tiles + tl;
  const int64_t m0 = (tile / tiles_j) * BM;
  const int j0 = (int)(tile % tiles_j) * BN;
  const int64_t u0 = tl * nk, u1 = u0 + nk;
  auto range_begin = [&](int64_t w) { return w * sk_units / sk_wgs; };
  // the workgroup whose range holds u0: the last w with range_begin(w) <= u0
  int64_t w = min<int64_t>(sk_wgs - 1, u0 * sk_wgs / sk_units);
  while (w > 0 && range_begin(w) > u0) --w;
  while (w + 1 < sk_wgs && range_begin(w + 1) <= u0) ++w;
  f32x4 s = f32x4{0};
  for (; w < sk_wgs && range_begin(w) < u1; ++w) {
    const int64_t a = range_begin(w), e = range_begin(w + 1);
    if (e <= a || e <= u0) continue;
    const int seg = (int)(tl - a / nk);
    s += *reinterpret_cast<const f32x4*>(part + (w * 2 + seg) * (int64_t)(BM * BN) + e0);
  }
  const int64_t grow = m0 + row;
  if (grow >= m) return;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (j0 + col + c < r) Z[grow * r + j0 + col + c] = s[c] * scale;
}

// ---------------------------------------------------------------------------
// Direct-to-LDS forms of the two products (used when O and the skinny operand
// have 16-byte aligned rows).  global_load_lds_dwordx4 copies 16 bytes per
// lane from any global address into LDS at (M0 base + 16 * lane), without
// passing through registers.  That frees the prefetch registers, so the LDS
// holds a ring of three K-steps: while the MFMAs work on step i, steps i+1
// and i+2 are in flight.  A step's copies are waited for with an explicit
// vmcnt (each wave knows how many copies it issued after them) and published
// to the other waves by a bare s_barrier; the slot a copy overwrites was read
// in the previous step, before that barrier.
//
// LDS layouts (one ring slot):
//   skinny operand S (V or Q_Y), 16 K-rows x BN: K-row major; one copy
//     instruction moves 1 KB = 256 / BN K-rows, and consecutive instructions
//     sit SP bytes apart.  Lane (x, h) of MFMA step s reads S[k][j] with
//     k = s + 8h: rows k and k + 8 then fall into opposite halves of the banks.
//   parameter side O tile, 16 K-rows x 128 parameters: K-row pairs per copy
//     instruction, pairs 1056 bytes apart (same argument).
//   sample side O tile, 128 rows x 16 K-values: 16-byte chunk c of row i sits
//     at slot 4i + (c ^ ((i >> 2) & 3)); the lane reads of one MFMA fragment
//     (one 16-byte chunk per lane) then cover distinct banks in every group
//     of eight lanes.
// Out-of-range rows and columns of the skinny operand are read from a zero
// buffer, so they add nothing; out-of-range rows of O are clamped to a valid
// row (they only meet those zeros, or feed output rows that are not stored).
// ---------------------------------------------------------------------------
namespace {
#define WSSR_LDSP(p) ((__attribute__((address_space(3))) void*)(p))
constexpr int kDmaStages = 3;
constexpr int kPairPitch = 1056;   // bytes between K-row pairs of the parameter-side O tile
constexpr int kSampleA = BM * BK * 4;   // bytes of the sample-side O tile (swizzled, no padding)

template <int BN>
struct DmaS {
  static constexpr int RPI = 256 / BN;                                  // K-rows per copy instruction
  static constexpr int PITCH = 1024 + (RPI == 1 ? 16 : RPI == 2 ? 32 : RPI == 4 ? 64 : 128);
  static constexpr int INSTR = BK / RPI;                                // copy instructions per step
  static constexpr int BYTES = INSTR * PITCH;
  // byte offset of element (k, j) of the skinny tile
  __device__ static __forceinline__ int off(int k, int j) { return (k / RPI) * PITCH + (k % RPI) * (BN * 4) + j * 4; }
};

// wave layout of a BN-column tile: WN waves across the columns, WM along the
// 128 rows; each wave owns TA x TB MFMA tiles of 32 x 32
template <int BN>
struct WaveL {
  static constexpr int WN = BN >= 64 ? 2 : 1;
  static constexpr int WM = 4 / WN;
  static constexpr int TA = BM / WM / 32;
  static constexpr int TB = BN / WN / 32;
};

// vmcnt wait with lgkmcnt / expcnt left alone
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Wait before K-step `it` of `ns` for wave w: its copies per K-step are two
// of the O tile and its share of the skinny tile (with fewer than four skinny
// instructions, the first waves take one each); all but the next step's
// copies must have landed, or all of them before the last step.
template <int BN>
__device__ __forceinline__ void wait_step(int w, bool last) {
  constexpr int I = DmaS<BN>::INSTR;
  if (last) {
    wait_vmcnt<0>();
  } else if constexpr (I >= 4) {
    wait_vmcnt<2 + I / 4>();
  } else {
    if (w < I)
      wait_vmcnt<3>();
    else
      wait_vmcnt<2>();
  }
}

// copy instructions of one K-step of the skinny tile (rows k0.., columns j0..)
// issued by wave w into `dst`
template <int BN>
__device__ __forceinline__ void dma_skinny(const float* __restrict__ S, int r, int64_t k0, int64_t kend, int j0,
                                           const float* __restrict__ zeros, unsigned char* dst, int w, int lane) {
  using D = DmaS<BN>;
  constexpr int PER_W = D::INSTR >= 4 ? D::INSTR / 4 : 1;
#pragma unroll
  for (int q = 0; q < PER_W; ++q) {
    const int ins = D::INSTR >= 4 ? w * PER_W + q : w;
    if (ins >= D::INSTR) break;
    const int kr = ins * D::RPI + (lane * 4) / BN;
    const int j = j0 + (lane * 4) % BN;
    const int64_t k = k0 + kr;
    const float* src = (k < kend && j < r) ? S + k * r + j : zeros;
    __builtin_amdgcn_global_load_lds((const void*)src, WSSR_LDSP(dst + ins * D::PITCH), 16, 0, 0);
  }
}
}  // namespace

// Sample side, direct-to-LDS form.  Arguments as k_gemm_sample_side, plus a
// zero buffer of at least 16 bytes.
template <int BN>
__global__ __launch_bounds__(256, 2) void k_gemm_sample_side_dma(const float* __restrict__ O, int64_t ld, int64_t n,
                                                                 int64_t m, const float* __restrict__ V, int r,
                                                                 float* __restrict__ ypart, int64_t kchunk,
                                                                 const float* __restrict__ zeros,
                                                                 const DevStatus* st, int tn, int tj,
                                                                 bool xcd_groups) {
  if (failed(st)) return;
  using D = DmaS<BN>;
  using L = WaveL<BN>;
  constexpr int TA = L::TA, TB = L::TB;
  constexpr int STAGE = kSampleA + D::BYTES;
  extern __shared__ __attribute__((aligned(16))) unsigned char smd[];
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
  const int wm = w / L::WN, wn = w % L::WN;
  const int x = lane & 31, h = lane >> 5;
  const int64_t n0 = (int64_t)bx * BM;
  const int j0 = by * BN;
  const int64_t kb = (int64_t)bz * kchunk;
  const int64_t ke = min(m, kb + kchunk);
  float* out = ypart + (int64_t)bz * n * r;

  f32x16 acc[TA][TB];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = f32x16{0};

  auto issue = [&](int64_t k0, int slot) __attribute__((always_inline)) {
    unsigned char* base = smd + slot * STAGE;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ins = 2 * w + q;                    // rows 16 ins .. 16 ins + 15
      const int row = 16 * ins + (lane >> 2);
      const int c = (lane & 3) ^ ((row >> 2) & 3);  // chunk held by this slot
      const int64_t gr = min(n0 + row, n - 1);
      const int64_t gk = k0 + 4 * c;
      const float* src = (gk < ke) ? O + gr * ld + gk : zeros;
      __builtin_amdgcn_global_load_lds((const void*)src, WSSR_LDSP(base + ins * 1024), 16, 0, 0);
    }
    dma_skinny<BN>(V, r, k0, ke, j0, zeros, base + kSampleA, w, lane);
  };

  const int64_t ns = (ke - kb + BK - 1) / BK;
  if (ns > 0) issue(kb, 0);
  if (ns > 1) issue(kb + BK, 1);
  int slot = 0;
  for (int64_t it = 0; it < ns; ++it) {
    wait_step<BN>(w, it + 1 >= ns);
    __builtin_amdgcn_s_barrier();
    const unsigned char* S = smd + slot * STAGE;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      // the copies for step it + 2 go out once the first half's MFMAs are
      // issued, so that they overlap MFMA work instead of preceding it
      if (half == 1 && it + 2 < ns) issue(kb + (it + 2) * BK, slot == 0 ? 2 : slot - 1);
      f32x4 av[TA];
#pragma unroll
      for (int a = 0; a < TA; ++a) {
        const int row = wm * (BM / L::WM) + a * 32 + x;
        const int c = 2 * h + half;
        av[a] = *reinterpret_cast<const f32x4*>(S + (row * 4 + (c ^ ((row >> 2) & 3))) * 16);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 8 * h + 4 * half + e;
        float bv[TB];
#pragma unroll
        for (int b = 0; b < TB; ++b)
          bv[b] = *reinterpret_cast<const float*>(S + kSampleA + D::off(k, wn * (BN / L::WN) + b * 32 + x));
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) acc[a][b] = mfma32x32x2(av[a][e], bv[b], acc[a][b]);
      }
    }
    slot = slot == 2 ? 0 : slot + 1;
  }

#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const int col = j0 + wn * (BN / L::WN) + b * 32 + x;
      if (col >= r) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = n0 + wm * (BM / L::WM) + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < n) out[row * r + col] = acc[a][b][v];
      }
    }
}

// Parameter side, direct-to-LDS form.  Arguments as k_gemm_param_side, plus a
// zero buffer of at least 16 bytes.
template <int BN>
__global__ __launch_bounds__(256, 2) void k_gemm_param_side_dma(const float* __restrict__ O, int64_t ld, int64_t n,
                                                                int64_t m, const float* __restrict__ Q, int r,
                                                                float scale, float* __restrict__ Z,
                                                                const float* __restrict__ zeros, const DevStatus* st,
                                                                int tiles_j, int full_tiles, int64_t sk_units,
                                                                int sk_wgs, float* __restrict__ part) {
  if (failed(st)) return;
  using D = DmaS<BN>;
  using L = WaveL<BN>;
  constexpr int TA = L::TA, TB = L::TB;
  constexpr int SO = 8 * kPairPitch;
  constexpr int STAGE = SO + D::BYTES;
  extern __shared__ __attribute__((aligned(16))) unsigned char smd[];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w / L::WN, wj = w % L::WN;
  const int x = lane & 31, h = lane >> 5;
  int64_t m0 = 0;
  int j0 = 0;
  f32x16 acc[TA][TB];
  const int64_t mlast = ((m - 1) / 4) * 4;      // last 16-byte chunk of a row of O

  auto issue = [&](int64_t ks, int slot) __attribute__((always_inline)) {
    unsigned char* base = smd + slot * STAGE;
    const int64_t k0 = ks * BK;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = 2 * w + q;                      // K-rows 2p, 2p + 1
      const int64_t k = min(k0 + 2 * p + (lane >> 5), n - 1);
      const int64_t mm = min(m0 + (lane & 31) * 4, mlast);
      __builtin_amdgcn_global_load_lds((const void*)(O + k * ld + mm), WSSR_LDSP(base + p * kPairPitch), 16, 0, 0);
    }
    dma_skinny<BN>(Q, r, k0, n, j0, zeros, base + SO, w, lane);
  };
  // acc = the product of tile `tile` over K-steps [kb, ke)
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) __attribute__((always_inline)) {
    m0 = (tile / tiles_j) * BM;
    j0 = (int)(tile % tiles_j) * BN;
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) acc[a][b] = f32x16{0};
    const int64_t ns = ke - kb;
    wait_vmcnt<0>();        // no older stores in the count
    if (ns > 0) issue(kb, 0);
    if (ns > 1) issue(kb + 1, 1);
    int slot = 0;
    for (int64_t it = 0; it < ns; ++it) {
      wait_step<BN>(w, it + 1 >= ns);
      __builtin_amdgcn_s_barrier();
      const unsigned char* S = smd + slot * STAGE;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        // copies for step it + 2 after the first half of the MFMAs
        if (s == 4 && it + 2 < ns) issue(kb + it + 2, slot == 0 ? 2 : slot - 1);
        const int k = s + 8 * h;
        float av[TA], bv[TB];
#pragma unroll
        for (int a = 0; a < TA; ++a)
          av[a] = *reinterpret_cast<const float*>(S + (k >> 1) * kPairPitch + (k & 1) * 512 +
                                                  (wm * (BM / L::WM) + a * 32 + x) * 4);
#pragma unroll
        for (int b = 0; b < TB; ++b)
          bv[b] = *reinterpret_cast<const float*>(S + SO + D::off(k, wj * (BN / L::WN) + b * 32 + x));
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) acc[a][b] = mfma32x32x2(av[a], bv[b], acc[a][b]);
      }
      slot = slot == 2 ? 0 : slot + 1;
    }
    __syncthreads();        // every wave is done with the ring before it is refilled
  };

  const int64_t nk = (n + BK - 1) / BK;
  if ((int)blockIdx.x < full_tiles) {
    run(blockIdx.x, 0, nk);
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int col = j0 + wj * (BN / L::WN) + b * 32 + x;
        if (col >= r) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = m0 + wm * (BM / L::WM) + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          if (row < m) Z[row * r + col] = acc[a][b][v] * scale;
        }
      }
    return;
  }
  // stream-K: at most two tiles per workgroup, written out without a loop
  const int64_t wg = (int64_t)blockIdx.x - full_tiles;
  int64_t u = wg * sk_units / sk_wgs;
  const int64_t uend = (wg + 1) * sk_units / sk_wgs;
  auto segment = [&](int seg) __attribute__((always_inline)) {
    const int64_t tl = u / nk, kb = u - tl * nk, ke = min(nk, kb + (uend - u));
    run(full_tiles + tl, kb, ke);
    float* outp = part + (wg * 2 + seg) * (int64_t)(BM * BN);
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int col = wj * (BN / L::WN) + b * 32 + x;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * (BM / L::WM) + a * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          outp[row * BN + col] = acc[a][b][v];
        }
      }
    u += ke - kb;
  };
  if (u < uend) segment(0);
  if (u < uend) segment(1);
}

// ---------------------------------------------------------------------------
// Narrow form of the FP32 parameter-side product (r <= 32: one 32-column
// tile).  At that width the product does 2r flops per 4-byte element of O and
// is bound by HBM, so what sets its speed is how many bytes of O each compute
// unit keeps in flight.  A direct-to-LDS copy holds a slot of LDS for every
// byte in flight; here O and the skinny tile go through registers instead,
// kAhead K-steps ahead of the MFMAs, and LDS holds only the two stages the
// MFMAs alternate between (written at step s, read after the barrier of step
// s; stage s & 1 is rewritten at step s + 2, after every wave has passed the
// barrier of step s + 1 and so finished step s).  The LDS layouts are those
// of the direct-to-LDS kernel, so the MFMA side is the same.  (The sample
// side reads 64-byte pieces of 128 rows per K-step; staged through registers
// it ran slower than its direct-to-LDS 32-column form, which it keeps.)
namespace {
constexpr int kAhead = 4;     // K-steps in flight (even: step s uses stage s & 1 = d & 1)
using NS = DmaS<32>;

// LDS waits for this wave's LDS writes only (vmcnt left at its maximum)
__device__ __forceinline__ void wait_lgkm0() {
  __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4) | (0 << 8));
}
}  // namespace

// Parameter side, narrow form.  Arguments as k_gemm_param_side_dma.
__global__ __launch_bounds__(256, 4) void k_gemm_param_side_narrow(const float* __restrict__ O, int64_t ld, int64_t n,
                                                                int64_t m, const float* __restrict__ Q, int r,
                                                                float scale, float* __restrict__ Z,
                                                                const float* __restrict__ zeros, const DevStatus* st,
                                                                int tiles_j, int full_tiles, int64_t sk_units,
                                                                int sk_wgs, float* __restrict__ part) {
  if (failed(st)) return;
  constexpr int SO = 8 * kPairPitch;
  constexpr int STAGE = SO + NS::BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char sm[2 * STAGE];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int x = lane & 31, h = lane >> 5;
  const int64_t mlast = ((m - 1) / 4) * 4;      // last 16-byte chunk of a row of O

  // this thread's share of a K-step: the 16-byte chunk at column mc of
  // K-rows kr[q] (pairs 2w, 2w + 1), two values of row ks of Q
  const int mc = (lane & 31) * 4;
  int kr[2], aoff[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int p = 2 * w + q;
    kr[q] = 2 * p + h;
    aoff[q] = p * kPairPitch + h * 512 + (lane & 31) * 16;
  }
  const int ks = t >> 4, js = (t & 15) * 2;
  const int qoff = SO + NS::off(ks, js);

  int64_t m0 = 0;
  int j0 = 0;
  f32x16 acc;
  f32x4 ra[kAhead][2];
  f32x2 rv[kAhead];
  auto load = [&](int64_t kstep, f32x4* a, f32x2& v) __attribute__((always_inline)) {
    const int64_t k0 = kstep * BK;
    const int64_t mm = min(m0 + mc, mlast);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t k = min(k0 + kr[q], n - 1);
      a[q] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(O + k * ld + mm));
    }
    const int64_t kk = k0 + ks;
    v = *reinterpret_cast<const f32x2*>((kk < n && j0 + js < r) ? Q + kk * r + j0 + js : zeros);
  };
  // acc = the product of tile `tile` over K-steps [kb, ke)
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) __attribute__((always_inline)) {
    m0 = (tile / tiles_j) * BM;
    j0 = (int)(tile % tiles_j) * 32;
    acc = f32x16{0};
    auto step = [&](int d, bool refill, int64_t next) __attribute__((always_inline)) {
      unsigned char* S = sm + (d & 1) * STAGE;
#pragma unroll
      for (int q = 0; q < 2; ++q) *reinterpret_cast<f32x4*>(S + aoff[q]) = ra[d][q];
      *reinterpret_cast<f32x2*>(S + qoff) = rv[d];
      if (refill) load(next, ra[d], rv[d]);
      wait_lgkm0();
      __builtin_amdgcn_s_barrier();
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        const int k = s8 + 8 * h;
        const float av =
            *reinterpret_cast<const float*>(S + (k >> 1) * kPairPitch + (k & 1) * 512 + (w * 32 + x) * 4);
        const float bv = *reinterpret_cast<const float*>(S + SO + NS::off(k, x));
        acc = mfma32x32x2(av, bv, acc);
      }
    };
    // loads past the K range read clamped rows and the zero buffer (never
    // used), so every group of kAhead steps issues the same loads
    const int64_t ns = ke - kb;
#pragma unroll
    for (int d = 0; d < kAhead; ++d) load(kb + d, ra[d], rv[d]);
    int64_t it = 0;
    for (; it + kAhead <= ns; it += kAhead) {
#pragma unroll
      for (int d = 0; d < kAhead; ++d) step(d, true, kb + it + d + kAhead);
    }
#pragma unroll
    for (int d = 0; d < kAhead - 1; ++d)
      if (it + d < ns) step(d, false, 0);
    __syncthreads();        // every wave is done with both stages before they are rewritten
  };

  const int64_t nk = (n + BK - 1) / BK;
  if ((int)blockIdx.x < full_tiles) {
    run(blockIdx.x, 0, nk);
    const int col = j0 + x;
    if (col < r) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + w * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < m) Z[row * r + col] = acc[v] * scale;
      }
    }
    return;
  }
  // stream-K: at most two tiles per workgroup, written out without a loop
  const int64_t wg = (int64_t)blockIdx.x - full_tiles;
  int64_t u = wg * sk_units / sk_wgs;
  const int64_t uend = (wg + 1) * sk_units / sk_wgs;
  auto segment = [&](int seg) __attribute__((always_inline)) {
    const int64_t tl = u / nk, kb = u - tl * nk, ke = min(nk, kb + (uend - u));
    run(full_tiles + tl, kb, ke);
    float* outp = part + (wg * 2 + seg) * (int64_t)(BM * 32);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = w * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
      outp[row * 32 + x] = acc[v];
    }
    u += ke - kb;
  };
  if (u < uend) segment(0);
  if (u < uend) segment(1);
}

size_t gemm_dma_lds(bool param_side, int bn) {
  const size_t a = param_side ? (size_t)8 * kPairPitch : (size_t)kSampleA;
  const size_t b = bn == 256   ? DmaS<256>::BYTES
                   : bn == 128 ? DmaS<128>::BYTES
                   : bn == 64  ? DmaS<64>::BYTES
                               : DmaS<32>::BYTES;
  return kDmaStages * (a + b);
}

#define WSSR_GEMM_DMA_INST(BN)                                                                                       \
  template __global__ void k_gemm_sample_side_dma<BN>(const float*, int64_t, int64_t, int64_t, const float*, int,   \
                                                      float*, int64_t, const float*, const DevStatus*, int, int,    \
                                                      bool);                                                        \
  template __global__ void k_gemm_param_side_dma<BN>(const float*, int64_t, int64_t, int64_t, const float*, int,    \
                                                     float, float*, const float*, const DevStatus*, int, int,       \
                                                     int64_t, int, float*);
template __global__ void k_gemm_sample_side_dma<32>(const float*, int64_t, int64_t, int64_t, const float*, int, float*,
                                                    int64_t, const float*, const DevStatus*, int, int, bool);
WSSR_GEMM_DMA_INST(64)
WSSR_GEMM_DMA_INST(128)
WSSR_GEMM_DMA_INST(256)

template __global__ void k_gemm_sample_side<64>(const float*, int64_t, int64_t, int64_t, const float*, int, float*,
                                                int64_t, bool, bool, const DevStatus*, int, int, bool);
template __global__ void k_gemm_sample_side<128>(const float*, int64_t, int64_t, int64_t, const float*, int, float*,
                                                 int64_t, bool, bool, const DevStatus*, int, int, bool);
template __global__ void k_gemm_sample_side<256>(const float*, int64_t, int64_t, int64_t, const float*, int, float*,
                                                 int64_t, bool, bool, const DevStatus*, int, int, bool);
template __global__ void k_gemm_param_side<64>(const float*, int64_t, int64_t, int64_t, const float*, int, float,
                                               float*, bool, bool, const DevStatus*, int, int, int64_t, int, float*);
template __global__ void k_gemm_param_side<128>(const float*, int64_t, int64_t, int64_t, const float*, int, float,
                                                float*, bool, bool, const DevStatus*, int, int, int64_t, int, float*);
template __global__ void k_gemm_param_side<256>(const float*, int64_t, int64_t, int64_t, const float*, int, float,
                                                float*, bool, bool, const DevStatus*, int, int, int64_t, int, float*);
template __global__ void k_streamk_fixup<32>(const float*, float*, int64_t, int, float, int, int, int64_t, int64_t,
                                             int, const DevStatus*);
template __global__ void k_streamk_fixup<64>(const float*, float*, int64_t, int, float, int, int, int64_t, int64_t,
                                             int, const DevStatus*);
template __global__ void k_streamk_fixup<128>(const float*, float*, int64_t, int, float, int, int, int64_t, int64_t,
                                              int, const DevStatus*);
template __global__ void k_streamk_fixup<256>(const float*, float*, int64_t, int, float, int, int, int64_t, int64_t,
                                              int, const DevStatus*);
template __global__ void k_streamk_fixup<512>(const float*, float*, int64_t, int, float, int, int, int64_t, int64_t,
                                              int, const DevStatus*);

}  // namespace wssr
