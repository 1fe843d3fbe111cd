// BF16 products for wide column tiles, with the skinny operand streamed from
// global memory straight into the MFMA's registers.  Sample side:
//
//   Ypart[s] = O[:, Ks] S[Ks, :]      (N x r, K = M split into ranges)
//
// with O one BF16 plane and S = V split by k_split_skinny into PB BF16 planes
// laid out [k / 16][column][k % 16].  In that layout the B fragment of
// v_mfma_f32_32x32x16_bf16 for one 32-column tile and one 16-deep K-block
// (lane l: column l % 32, K-values 8 (l / 32) .. + 7) is one contiguous
// 1 KB block, so each lane fetches its fragment with one 16-byte load and a
// wave's loads are fully coalesced.  Only O goes through LDS.
//
// Why: with a 128 x 512 output tile the skinny operand is 8 times the O data
// of every K-step.  Staged through LDS it costs a copy into LDS plus, with
// two waves sharing each column, two reads back out: about 110 KB of LDS
// traffic per 1024 MFMA cycles, close to the LDS bandwidth.  Here each wave
// owns all 128 rows and BN / 4 columns, so no skinny fragment is read twice;
// the LDS carries one 4 KB O tile per step (written once, read by the four
// waves).
//
// Pipeline: the skinny fragments of step i + DB are loaded into a ring of
// DB + 1 register sets and the O tile of step i + DB + 1 into a ring of
// DB + 1 LDS slots while step i is multiplied, and the O fragments of step
// i + 1 are read from LDS ahead of step i's MFMAs, so that those MFMAs need
// nothing that arrives after the barrier.  Per step: wait until the O tile of
// step i + 1 and the skinny fragments of step i have landed (the
// vector-memory counter may keep DB - 1 later steps' loads in flight; within
// a step the skinny loads go out before the O copy), barrier (publishes that
// tile; every wave has read step i's fragments, so its slot is free), issue
// the next loads, read step i + 1's O fragments, multiply step i.  Every step
// issues the same loads -- past the K range the O copy reads a zero buffer
// and the skinny loads re-read the last K-block -- so the counts are exact.
// The loop runs whole trips of its unrolled body; steps past the K range
// multiply zero O tiles.  The ring is drained before the kernel ends.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int RBM = 128;   // output rows per workgroup
#define RS_LDS(p) ((__attribute__((address_space(3))) void*)(p))

__device__ __forceinline__ f32x16 mfma_bf16_rs(const u32x4& a, const u32x4& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

template <int N>
__device__ __forceinline__ void wait_vm_rs() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

constexpr int gcd_rs(int a, int b) { return b == 0 ? a : gcd_rs(b, a % b); }

// wait until this wave's LDS stores have completed
__device__ __forceinline__ void wait_lgkm0_rs() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt left at their maximum
}

#ifndef WSSR_RS_BARMASK
#define WSSR_RS_BARMASK 1
#endif
// workgroup barrier that no memory instruction is moved across; with mask 1
// ALU work (the MFMAs) may still be scheduled across it
__device__ __forceinline__ void barrier_rs() {
  __builtin_amdgcn_sched_barrier(WSSR_RS_BARMASK);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(WSSR_RS_BARMASK);
}

template <int V>
struct IC {
  static constexpr int value = V;
};

// f(IC<0>), ..., f(IC<N-1>) in order
template <int I, int N, class F>
__device__ __forceinline__ void unroll_ic(F&& f) {
  if constexpr (I < N) {
    f(IC<I>{});
    unroll_ic<I + 1, N>(f);
  }
}
}  // namespace

// Arguments as k_gemm16_sample_side_dma with one O plane.  BN: output
// columns per workgroup (a multiple of 128; each wave BN / 4); PB: planes of
// the skinny operand; DB: K-steps in flight of the skinny operand (O: DB + 1).
// Requires whole 16-byte chunks of O's rows (m % 8 == 0, ld % 8 == 0,
// 16-byte aligned O) and kchunk a multiple of 16.
template <int BN, int PB, int DB>
__global__ __launch_bounds__(256, 1) void k_gemm16_sample_side_rs(const u16* __restrict__ O, int64_t ld, int64_t n,
                                                                  int64_t m, const u16* __restrict__ Vs,
                                                                  int64_t vstride, int r, float* __restrict__ ypart,
                                                                  int64_t kchunk, const u16* __restrict__ zeros,
                                                                  const DevStatus* st, int tn, int tj,
                                                                  bool xcd_groups) {
  if (failed(st)) return;
  constexpr int CT = BN / 128;          // 32-column MFMA tiles per wave
  constexpr int DO = DB + 1;            // K-steps of O in flight
  constexpr int SB = DB + 1;            // register sets of the skinny operand
  constexpr int SO = DO;                // LDS slots of O: steps i + 1 .. i + DO
  constexpr int U = 2 * SB / gcd_rs(2, SB);   // steps per loop trip: every slot index fixed
  constexpr int TILE = RBM * 16 * 2;    // bytes of one K-step of O
  constexpr int LB = CT * PB;           // skinny loads per wave and step
  constexpr int WAITN = (DB - 1) * (LB + 1);
  static_assert(BN % 128 == 0 && DB >= 1 && DB * (LB + 1) < 64, "tile and ring");
  __shared__ __attribute__((aligned(16))) unsigned char sm[SO * TILE];

  int bx, by, bz;
  {
    const int id = blockIdx.x;
    int grp, i;
    if (xcd_groups) {
      // workgroups that read the same K range of the skinny operand share an XCD
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
  const int x = lane & 31, hh = lane >> 5;
  const int64_t n0 = (int64_t)bx * RBM;
  const int j0 = by * BN;
  const int sw = tj * BN;
  const int64_t kb = (int64_t)bz * kchunk;
  const int64_t ke = min(m, kb + kchunk);
  const int64_t ns = (ke - kb + 15) / 16;
  float* out = ypart + (int64_t)bz * n * r;

  f32x16 acc[4][CT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = f32x16{0};

  if (ns > 0) {
    // this thread's share of an O tile: row t / 2, K-values 8 cc .. + 7,
    // landing at byte 16 t of the tile (row-major, 32 bytes per row); rows
    // past n are clamped (they feed output rows that are not stored)
    // The two 16-byte halves of rows 8..15 (mod 16) are stored swapped, so
    // that the 16 lanes of a fragment read that cover 16 consecutive rows hit
    // disjoint banks.
    const int cc = (t & 1) ^ (((t >> 1) >> 3) & 1);
    const u16* osrc = O + min(n0 + (t >> 1), n - 1) * ld + cc * 8;
    // this lane's skinny fragment: column j0 + w BN/4 + 32 c + x, K-values 8 hh ..
    const int voff = (j0 + w * (BN / 4) + x) * 16 + 8 * hh;
    const int64_t kblk0 = kb / 16;
    u32x4 bq[SB][PB][CT];
    u32x4 av[2][4];

    auto issue_b = [&](int64_t i, auto slotc) __attribute__((always_inline)) {
      constexpr int s = decltype(slotc)::value;
      const u16* base = Vs + (kblk0 + min(i, ns - 1)) * (int64_t)sw * 16 + voff;
#pragma unroll
      for (int p = 0; p < PB; ++p)
#pragma unroll
        for (int c = 0; c < CT; ++c) bq[s][p][c] = *reinterpret_cast<const u32x4*>(base + p * vstride + c * 512);
    };
    auto issue_o = [&](int64_t i, auto slotc) __attribute__((always_inline)) {
      constexpr int s = decltype(slotc)::value;
      const int64_t k0 = kb + i * 16;
      const u16* src = (i < ns && k0 + cc * 8 < ke) ? osrc + k0 : zeros;
      __builtin_amdgcn_global_load_lds((const void*)src, RS_LDS(sm + s * TILE + w * 1024), 16, 0, 0);
    };
    auto read_a = [&](auto oslotc, auto aslotc) __attribute__((always_inline)) {
      constexpr int so = decltype(oslotc)::value, sa = decltype(aslotc)::value;
      const unsigned char* A = sm + so * TILE;
#pragma unroll
      for (int a = 0; a < 4; ++a)
        av[sa][a] = *reinterpret_cast<const u32x4*>(A + (32 * a + x) * 32 + (hh ^ ((x >> 3) & 1)) * 16);
    };
    auto mfmas = [&](auto aslotc, auto bslotc) __attribute__((always_inline)) {
      constexpr int sa = decltype(aslotc)::value, sb = decltype(bslotc)::value;
#pragma unroll
      for (int p = 0; p < PB; ++p)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[a][c] = mfma_bf16_rs(av[sa][a], bq[sb][p][c], acc[a][c]);
    };

    // prologue: the O tile of step 0, then the loads the trips before step 0
    // would have issued (skinny step j, O step j + 1, for j < DB)
    issue_o(0, IC<0>{});
    unroll_ic<0, DB>([&](auto sc) {
      constexpr int j = decltype(sc)::value;
      __builtin_amdgcn_sched_barrier(0);
      issue_b(j, IC<j>{});
      __builtin_amdgcn_sched_barrier(0);
      issue_o(j + 1, IC<(j + 1) % SO>{});
    });
    wait_vm_rs<DB*(LB + 1)>();
    barrier_rs();
    read_a(IC<0>{}, IC<0>{});
    for (int64_t base = 0; base < ns; base += U) {
      unroll_ic<0, U>([&](auto sc) {
        constexpr int u = decltype(sc)::value;
        const int64_t i = base + u;
        wait_vm_rs<WAITN>();
        barrier_rs();
        issue_b(i + DB, IC<(u + DB) % SB>{});
        __builtin_amdgcn_sched_barrier(0);
        issue_o(i + DO, IC<(u + DO) % SO>{});
        __builtin_amdgcn_sched_barrier(0);
        read_a(IC<(u + 1) % SO>{}, IC<(u + 1) % 2>{});
        mfmas(IC<u % 2>{}, IC<u % SB>{});
      });
    }
    // no copy into LDS may still be in flight when the workgroup ends
    wait_vm_rs<0>();
  }

#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int col = j0 + w * (BN / 4) + c * 32 + x;
      if (col >= r) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = n0 + a * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
        if (row < n) out[row * r + col] = acc[a][c][v];
      }
    }
}

// ---------------------------------------------------------------------------
// Parameter side, the same scheme for the skinny operand:
//
//   Z = O^T S * scale      (M x r, K = N; S = Q_Y split into PB BF16 planes)
//
// The A operand is O^T: a K-step's O tile is 16 sample rows x 128 parameters
// (each K-row 256 contiguous bytes of O), kept in LDS as it lies in memory
// ([k][parameter], the 16-byte chunks of K-row k at slot c ^ 2 (k % 4) within
// their 1 KB group of four rows) and read with transposing LDS reads
// (ds_read_b64_tr_b16: in a group of 16 lanes, lane 4 rho + q points at
// parameters 4 q .. 4 q + 3 of K-row rho, and lane j receives K-rows 0 .. 3
// of parameter j).  The O tile is staged through registers (one 16-byte load
// and one 16-byte LDS store per thread and step) rather than copied straight
// into LDS: the compiler cannot tell the transposing reads apart from copies
// into LDS still in flight and would wait for all of them before every read.
// Rows of O past n are clamped (they meet zero rows of S); parameters past m
// are clamped to the last whole chunk (they feed rows of Z that are not
// stored); steps past a range's K-steps load a zero buffer.
//
// Per step i: store the O tile of step i + 1 (loaded DO steps earlier) into
// LDS, wait for the stores, barrier, issue the loads of step i + DO (O) and
// i + DB (skinny), read step i + 1's fragments, multiply step i.  Two LDS
// slots suffice: the slot written at step i was last read at step i - 2.
//
// Schedule (as the other parameter-side products): workgroups below
// full_tiles own one 128 x BN tile each, over all of K; the sk_wgs workgroups
// after them share the sk_units K-steps of the remaining tiles evenly (a range
// touches at most two tiles) and write their partial tiles to `part`, which
// k_streamk_fixup adds into Z.
// ---------------------------------------------------------------------------
template <int BN, int PB, int DB>
__global__ __launch_bounds__(256, 1) void k_gemm16_param_side_rs(const u16* __restrict__ O, int64_t ld, int64_t n,
                                                                 int64_t m, const u16* __restrict__ Qs,
                                                                 int64_t qstride, int r, float scale,
                                                                 float* __restrict__ Z, const u16* __restrict__ zeros,
                                                                 const DevStatus* st, int tiles_j, int full_tiles,
                                                                 int64_t sk_units, int sk_wgs,
                                                                 float* __restrict__ part) {
  if (failed(st)) return;
  constexpr int CT = BN / 128;          // 32-column MFMA tiles per wave
  constexpr int DO = DB + 1;            // K-steps of O in flight (registers)
  constexpr int SB = DB + 1;            // register sets of the skinny operand
  constexpr int SR = DO;                // register sets of O
  constexpr int U = SB * SR / gcd_rs(SB, SR) * 2 / gcd_rs(2, SB * SR / gcd_rs(SB, SR));
  constexpr int TILE = 16 * RBM * 2;    // bytes of one K-step of O (16 K-rows x 128 parameters)
  static_assert(BN % 128 == 0 && DB >= 1, "tile and ring");
  typedef short v4i16 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) unsigned char sm[2 * TILE];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int x = lane & 31, hh = lane >> 5;
  const int sw = tiles_j * BN;
  const int64_t nk = (n + 15) / 16;
  const int64_t mlast = ((m - 1) / 8) * 8;   // first parameter of the last 16-byte chunk of a row
  // this thread's share of an O tile: K-row 4 w + rho of the step (wave w
  // covers rows 4 w .. 4 w + 3, 1 KB), chunk (t % 16) ^ 2 rho, stored at byte
  // 16 t of the tile
  const int rho = (lane >> 4), cch = (lane & 15) ^ (2 * rho);
  const int krow = 4 * w + rho;
  const int voff = (w * (BN / 4) + x) * 16 + 8 * hh;
  f32x16 acc[4][CT];
  int64_t m0 = 0;
  int j0 = 0;

  // one tile's K-steps kb .. ke - 1 into acc (zeroed first); nothing is in
  // flight before or after
  auto run = [&](int64_t tile, int64_t kb, int64_t ke) __attribute__((always_inline)) {
    m0 = (tile / tiles_j) * RBM;
    j0 = (int)(tile % tiles_j) * BN;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[a][c] = f32x16{0};
    const int64_t ns = ke - kb;
    if (ns <= 0) return;
    const u16* obase = O + min(m0 + 8 * cch, mlast);
    const u16* qbase = Qs + j0 * 16 + voff;
    u32x4 bq[SB][PB][CT];
    u32x4 ro[SR];
    u32x4 av[2][4];

    auto issue_b = [&](int64_t i, auto slotc) __attribute__((always_inline)) {
      constexpr int s = decltype(slotc)::value;
      const u16* base = qbase + (kb + min(i, ns - 1)) * (int64_t)sw * 16;
#pragma unroll
      for (int p = 0; p < PB; ++p)
#pragma unroll
        for (int c = 0; c < CT; ++c) bq[s][p][c] = *reinterpret_cast<const u32x4*>(base + p * qstride + c * 512);
    };
    auto issue_o = [&](int64_t i, auto slotc) __attribute__((always_inline)) {
      constexpr int s = decltype(slotc)::value;
      const int64_t k = min((kb + i) * 16 + krow, n - 1);
      const u16* src = i < ns ? obase + k * ld : zeros;
      ro[s] = *reinterpret_cast<const u32x4*>(src);
    };
    auto store_o = [&](auto rslotc, auto lslotc) __attribute__((always_inline)) {
      constexpr int sr = decltype(rslotc)::value, sl = decltype(lslotc)::value;
      *reinterpret_cast<u32x4*>(sm + sl * TILE + t * 16) = ro[sr];
    };
    auto read_a = [&](auto lslotc, auto aslotc) __attribute__((always_inline)) {
      constexpr int sl = decltype(lslotc)::value, sa = decltype(aslotc)::value;
      const unsigned char* A = sm + sl * TILE;
      const int g = lane >> 4, i = lane & 15;
      const int rr = i >> 2, q = i & 3;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int mbase = a * 32 + 16 * (g & 1);
        const int c = (mbase >> 3) + (q >> 1);
        v4i16 pt[2];
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const int k = 8 * (g >> 1) + 4 * s2 + rr;   // this lane's K-row
          const unsigned char* src = A + (k >> 2) * 1024 + rr * 256 + ((c ^ (2 * rr)) * 16) + (q & 1) * 8;
          pt[s2] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) v4i16*)src);
        }
        const unsigned lo0 = (unsigned)(unsigned short)pt[0][0] | ((unsigned)(unsigned short)pt[0][1] << 16);
        const unsigned lo1 = (unsigned)(unsigned short)pt[0][2] | ((unsigned)(unsigned short)pt[0][3] << 16);
        const unsigned hi0 = (unsigned)(unsigned short)pt[1][0] | ((unsigned)(unsigned short)pt[1][1] << 16);
        const unsigned hi1 = (unsigned)(unsigned short)pt[1][2] | ((unsigned)(unsigned short)pt[1][3] << 16);
        av[sa][a] = u32x4{lo0, lo1, hi0, hi1};
      }
    };
    auto mfmas = [&](auto aslotc, auto bslotc) __attribute__((always_inline)) {
      constexpr int sa = decltype(aslotc)::value, sb = decltype(bslotc)::value;
#pragma unroll
      for (int p = 0; p < PB; ++p)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[a][c] = mfma_bf16_rs(av[sa][a], bq[sb][p][c], acc[a][c]);
    };

    // prologue: O of steps 0 .. DO - 1 and the skinny operand of steps
    // 0 .. DB - 1 in flight; step 0's tile stored and its fragments read
    unroll_ic<0, DO>([&](auto sc) {
      constexpr int j = decltype(sc)::value;
      issue_o(j, IC<j % SR>{});
      if constexpr (j < DB) issue_b(j, IC<j>{});
    });
    // every wave has finished reading the LDS of the previous range
    barrier_rs();
    store_o(IC<0>{}, IC<0>{});
    wait_lgkm0_rs();
    barrier_rs();
    read_a(IC<0>{}, IC<0>{});
    for (int64_t base = 0; base < ns; base += U) {
      unroll_ic<0, U>([&](auto sc) {
        constexpr int u = decltype(sc)::value;
        const int64_t i = base + u;
        store_o(IC<(u + 1) % SR>{}, IC<(u + 1) % 2>{});
        wait_lgkm0_rs();
        barrier_rs();
        issue_o(i + DO, IC<(u + DO) % SR>{});
        __builtin_amdgcn_sched_barrier(0);
        issue_b(i + DB, IC<(u + DB) % SB>{});
        __builtin_amdgcn_sched_barrier(0);
        read_a(IC<(u + 1) % 2>{}, IC<(u + 1) % 2>{});
        mfmas(IC<u % 2>{}, IC<u % SB>{});
      });
    }
    // no load may still be in flight past the range
    wait_vm_rs<0>();
  };

  if ((int)blockIdx.x < full_tiles) {
    run(blockIdx.x, 0, nk);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = j0 + w * (BN / 4) + c * 32 + x;
        if (col >= r) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = m0 + a * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
          if (row < m) Z[row * r + col] = acc[a][c][v] * scale;
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
    float* outp = part + (wg * 2 + seg) * (int64_t)(RBM * BN);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = w * (BN / 4) + c * 32 + x;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = a * 32 + 8 * (v >> 2) + 4 * hh + (v & 3);
          outp[row * BN + col] = acc[a][c][v];
        }
      }
    u += ke - kb;
  };
  if (u < uend) segment(0);
  if (u < uend) segment(1);
}

#define WSSR_RS_INST(PB, DB)                                                                                        \
  template __global__ void k_gemm16_sample_side_rs<512, PB, DB>(const u16*, int64_t, int64_t, int64_t, const u16*, \
                                                                    int64_t, int, float*, int64_t, const u16*,       \
                                                                    const DevStatus*, int, int, bool);
WSSR_RS_INST(1, WSSR_RS1_DB)
WSSR_RS_INST(2, WSSR_RS2_DB)
#define WSSR_RSP_INST(PB, DB)                                                                                       \
  template __global__ void k_gemm16_param_side_rs<512, PB, DB>(const u16*, int64_t, int64_t, int64_t, const u16*,  \
                                                               int64_t, int, float, float*, const u16*,             \
                                                               const DevStatus*, int, int, int64_t, int, float*);
WSSR_RSP_INST(1, WSSR_RS1_DB)
WSSR_RSP_INST(2, WSSR_RS2_DB)
}  // namespace wssr
