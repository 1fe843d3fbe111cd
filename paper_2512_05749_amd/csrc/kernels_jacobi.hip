// Rayleigh-Ritz SVD of the small matrix C (r x r, FP64) by block one-sided
// Jacobi, all sweeps in one cooperative launch.
//
// Columns of B = C P (P orthogonal, accumulated alongside) are rotated until
// every pair is orthogonal: then sigma_j = ||b_j|| and P holds the right
// singular vectors.  The rp columns (rp = r padded to 64; padding columns are
// zero and never rotated) form nb = rp/16 blocks of 16.  One outer round
// pairs the blocks by the round-robin tournament, nb/2 workgroups taking one
// block pair (32 columns) each; nb - 1 rounds make a sweep, in which every
// pair of columns meets once.  A workgroup
//   1. fetches the rows of P it will update into registers (their latency
//      is hidden behind steps 2-4) and stages its 32 columns of B in LDS,
//   2. forms their 32 x 32 Gram matrix H on the FP64 MFMA (one 16 x 16 tile
//      per wave, four independent accumulation chains),
//   3. measures the largest column cosine of H (convergence test),
//   4. if a cosine exceeds tol: diagonalises H by cyclic Jacobi (in each
//      rotation round every thread owns one 2 x 2 block of H and of the
//      accumulated rotation J and computes the two rotations it needs from
//      the diagonal blocks; H alternates between two LDS buffers so that a
//      round needs one barrier), orders the resulting columns by decreasing
//      norm, and applies the ordered rotation to its columns of B (from LDS)
//      and of P (from registers) on the FP64 MFMA,
//   5. meets the other workgroups at a grid barrier.
// After the last round of a sweep every workgroup reads the sweep's largest
// cosine and all stop together once it is <= tol (or after max_sweeps).
//
// The grid barrier is a counter in global memory (release add, acquire
// spin).  Every wait is bounded: a workgroup that waits longer than 5 s of
// real time sets the abort word, raises ST_TIMEOUT and leaves; waiting
// workgroups see the abort word and leave too, so the grid always drains.
// The launch is cooperative (all workgroups resident together); inside a
// captured graph or a batch lane it is a plain launch of at most 16
// workgroups, which the device schedules as other work drains, and the
// bounded wait covers that.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {
constexpr int JB = 16;            // columns per block
constexpr int JC = 2 * JB;        // columns per block pair
constexpr int JT = 256;           // threads per workgroup: one per 2 x 2 block of H
constexpr uint64_t kWaitTicks = 500000000ull;     // 5 s of the 100 MHz real-time counter

__device__ __forceinline__ double rsq_nr_j(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
}  // namespace

// sync: [0] barrier counter, [1] abort word, [2] skip (the step had already
// failed when the SVD started); zeroed / set by k_jacobi_prep.
// NPU = rp / 64: row blocks of 16 per wave in the apply.
template <int NPU>
__global__ __launch_bounds__(JT) void k_jacobi_coop(double* __restrict__ Bc, double* __restrict__ Pc, int rp,
                                                    double tol, const double* __restrict__ scal,
                                                    double* __restrict__ cosbuf, unsigned* __restrict__ sync,
                                                    DevStatus* st, int max_sweeps, int inner_sweeps) {
  if (__hip_atomic_load((int*)&sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  extern __shared__ double jsm[];
  const int LX = rp + 1;                       // LDS column stride (odd: conflict-free column reads)
  double* Xb = jsm;                            // [JC][LX] columns of B
  __shared__ double H0[JC][JC + 1], H1[JC][JC + 1], J[JC][JC + 1];
  __shared__ double wmax[4];
  __shared__ int colidx[JC], rnk[JC];
  __shared__ unsigned char ptab[JC - 1][JB][2];   // pairs (p, q) of each rotation round
  __shared__ int proceed;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = rp / JB, nwg = nb / 2, wg = blockIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  // ||C||_F^2 from the column sums of squares k_jacobi_prep left in scal[1..rp]
  __shared__ double fro2;
  if (tid < 64) {
    double s2 = 0.0;
    for (int j = tid; j < rp; j += 64) s2 += scal[1 + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if (tid == 0) fro2 = s2;
  }
  __syncthreads();
  const double floor = 4.93e-32 * fro2;                    // (eps ||C||_F)^2
  const double absfloor = 64.0 * 2.220446049250313e-16 * fro2;
  unsigned bars = 0;
  double last_cos = 0.0;
  int sweeps_done = 0, converged = 0;

  for (int e = tid; e < (JC - 1) * JB; e += JT) {
    int p, q;
    rr_pair(JC, e / JB, e % JB, p, q);
    ptab[e / JB][e % JB][0] = (unsigned char)p;
    ptab[e / JB][e % JB][1] = (unsigned char)q;
  }

  // grid barrier; false when the grid is aborting
  auto grid_barrier = [&]() -> bool {
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      ++bars;
      const unsigned target = bars * (unsigned)nwg;
      __hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      int ok = 1;
      const uint64_t t0 = wall_clock64();
      for (;;) {
        if (__hip_atomic_load(&sync[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
        if (__hip_atomic_load((int*)&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > kWaitTicks) {
          __hip_atomic_store((int*)&sync[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          raise_error(st, ST_TIMEOUT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      proceed = ok;
    }
    __syncthreads();
    __threadfence();
    return proceed != 0;
  };

  // rotation of the pair (p, q) of H, with a = H[p][p], d = H[q][q],
  // b = H[p][q], that zeroes H[p][q]; c = 1, s = 0 and false when the pair is
  // already orthogonal (cosine <= tol or entries at rounding level).  The
  // angle comes from hardware reciprocal and square-root estimates (a rough
  // angle only slows the iteration; what it leaves is measured and removed
  // later); c and s satisfy c^2 + s^2 = 1 to FP64 rounding.  Branch-free:
  // the formula runs on every pair and a select keeps (1, 0) where it does
  // not apply (it may produce NaN there, which the select drops), so that
  // both rotations of a thread and all of its LDS reads overlap.
  auto rot = [&](double a, double d, double b, double& c, double& s) -> bool {
    const bool act = a > floor && d > floor && fabs(b) > absfloor && b * b > tol * tol * (a * d);
    const double dm = d - a;
    const double h2 = dm * dm + 4.0 * b * b;
    const double hy = h2 * __builtin_amdgcn_rsq(h2);
    const double sg = ((dm >= 0.0) == (b >= 0.0)) ? 2.0 : -2.0;
    const double t = sg * fabs(b) * __builtin_amdgcn_rcp(fabs(dm) + hy);
    const double cc = rsq_nr_j(1.0 + t * t);
    c = act ? cc : 1.0;
    s = act ? cc * t : 0.0;
    return act;
  };

  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    double sweep_cos = 0.0;
    for (int rd = 0; rd < nb - 1; ++rd) {
      int bI, bJ;
      rr_pair(nb, rd, wg, bI, bJ);
      if (tid < JC) colidx[tid] = (tid < JB) ? bI * JB + tid : bJ * JB + (tid - JB);
      __syncthreads();
      // rows of P this wave updates (row blocks wv + 4j), in the MFMA A layout
      double pv[NPU][JC / 4];
#pragma unroll
      for (int j = 0; j < NPU; ++j)
#pragma unroll
        for (int k4 = 0; k4 < JC / 4; ++k4)
          pv[j][k4] = Pc[(int64_t)colidx[k4 * 4 + lk] * rp + (wv + 4 * j) * 16 + li];
      {
        const int nld = JC * rp / 2;             // double2 per column set
#pragma unroll 8
        for (int e = tid; e < nld; e += JT) {
          const int c = e / (rp / 2), k2 = e % (rp / 2);
          const double2 v = *reinterpret_cast<const double2*>(Bc + (int64_t)colidx[c] * rp + 2 * k2);
          Xb[c * LX + 2 * k2] = v.x;
          Xb[c * LX + 2 * k2 + 1] = v.y;
        }
      }
      __syncthreads();
      // H = X^T X: wave wv forms the 16 x 16 tile (wv / 2, wv % 2)
      {
        const int ti = (wv >> 1) * 16, tj = (wv & 1) * 16;
        f64x4 a4[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) a4[c] = f64x4{0};
        const double* xa = Xb + (ti + li) * LX + lk;
        const double* xb = Xb + (tj + li) * LX + lk;
        for (int k = 0; k < rp; k += 16) {
#pragma unroll
          for (int c = 0; c < 4; ++c) a4[c] = mfma16x16x4d(xa[k + 4 * c], xb[k + 4 * c], a4[c]);
        }
        const f64x4 acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          H0[ti + 4 * v + lk][tj + li] = acc[v];
          J[ti + 4 * v + lk][tj + li] = (ti + 4 * v + lk == tj + li) ? 1.0 : 0.0;
        }
      }
      __syncthreads();
      // largest cosine of the pair's columns
      double cmax = 0.0;
      for (int e = tid; e < JC * JC; e += JT) {
        const int p = e >> 5, q = e & 31;
        if (p < q) {
          const double a = H0[p][p], d = H0[q][q], b = H0[p][q];
          if (a > floor && d > floor && fabs(b) > absfloor) cmax = fmax(cmax, fabs(b) * rsq_nr_j(a * d));
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
      if (lane == 0) wmax[wv] = cmax;
      __syncthreads();
      cmax = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
      sweep_cos = fmax(sweep_cos, cmax);
      if (cmax > tol) {
        // cyclic Jacobi on H: thread (ra, rb) owns the 2 x 2 blocks of H and
        // of J at row pair ra and column pair rb of the rotation round.  H is
        // read from one buffer and written to the other; J is touched only
        // by the owner of each block.
        const int ra = tid >> 4, rb = tid & 15;
        int cur = 0;
        // this thread's pairs in rotation round 0; each round reads the next
        // round's from the (constant) table while its own reads are in flight
        int pa = ptab[0][ra][0], qa = ptab[0][ra][1];
        int pb = ptab[0][rb][0], qb = ptab[0][rb][1];
        for (int isw = 0; isw < inner_sweeps; ++isw) {
          int myrot = 0;
          for (int ird = 0; ird < JC - 1; ++ird) {
            const double(*Hc)[JC + 1] = cur ? H1 : H0;
            double(*Hn)[JC + 1] = cur ? H0 : H1;
            const double aa = Hc[pa][pa], da = Hc[qa][qa], ba = Hc[pa][qa];
            const double ab = Hc[pb][pb], db = Hc[qb][qb], bb = Hc[pb][qb];
            const double x11 = Hc[pa][pb], x12 = Hc[pa][qb], x21 = Hc[qa][pb], x22 = Hc[qa][qb];
            const double j11 = J[pa][pb], j12 = J[pa][qb], j21 = J[qa][pb], j22 = J[qa][qb];
            const int nr = ird + 1 < JC - 1 ? ird + 1 : 0;
            const int pa2 = ptab[nr][ra][0], qa2 = ptab[nr][ra][1];
            const int pb2 = ptab[nr][rb][0], qb2 = ptab[nr][rb][1];
            double ca, sa, cb, sb;
            myrot |= (int)rot(aa, da, ba, ca, sa);
            rot(ab, db, bb, cb, sb);
            // H <- R_a^T H R_b on the block; J <- J R_b on the block (the
            // identity where the pair b does not rotate)
            const double y11 = ca * x11 - sa * x21, y12 = ca * x12 - sa * x22;
            const double y21 = sa * x11 + ca * x21, y22 = sa * x12 + ca * x22;
            const double z11 = cb * y11 - sb * y12, z22 = sb * y21 + cb * y22;
            const bool zero_off = ra == rb && sa != 0.0;
            const double z12 = zero_off ? 0.0 : sb * y11 + cb * y12;
            const double z21 = zero_off ? 0.0 : cb * y21 - sb * y22;
            Hn[pa][pb] = z11;
            Hn[pa][qb] = z12;
            Hn[qa][pb] = z21;
            Hn[qa][qb] = z22;
            J[pa][pb] = cb * j11 - sb * j12;
            J[pa][qb] = sb * j11 + cb * j12;
            J[qa][pb] = cb * j21 - sb * j22;
            J[qa][qb] = sb * j21 + cb * j22;
            cur ^= 1;
            pa = pa2, qa = qa2, pb = pb2, qb = qb2;
            __syncthreads();
          }
          if (!__syncthreads_or(myrot)) break;
        }
        // order the rotated columns by decreasing norm: larger ones go to
        // the first block of the pair; the ordered rotation Jp takes the
        // buffer H does not end in
        const double(*Hf)[JC + 1] = cur ? H1 : H0;
        double(*Jp)[JC + 1] = cur ? H0 : H1;
        if (tid < JC) {
          const double ev = Hf[tid][tid];
          int k = 0;
          for (int c = 0; c < JC; ++c) {
            const double e2 = Hf[c][c];
            k += (e2 > ev) || (e2 == ev && c < tid);
          }
          rnk[tid] = k;
        }
        __syncthreads();
        for (int e = tid; e < JC * JC; e += JT) Jp[e >> 5][rnk[e & 31]] = J[e >> 5][e & 31];
        __syncthreads();
        // B <- B Jp (B from LDS) and P <- P Jp (P from registers), 16 rows at
        // a time: four independent MFMA chains
#pragma unroll
        for (int j = 0; j < NPU; ++j) {
          const int i0 = (wv + 4 * j) * 16;
          f64x4 b0 = f64x4{0}, b1 = f64x4{0}, p0 = f64x4{0}, p1 = f64x4{0};
#pragma unroll
          for (int k4 = 0; k4 < JC / 4; ++k4) {
            const int k = k4 * 4 + lk;
            const double jl = Jp[k][li], jh = Jp[k][16 + li];
            const double xa = Xb[k * LX + i0 + li];
            b0 = mfma16x16x4d(xa, jl, b0);
            b1 = mfma16x16x4d(xa, jh, b1);
            p0 = mfma16x16x4d(pv[j][k4], jl, p0);
            p1 = mfma16x16x4d(pv[j][k4], jh, p1);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = i0 + 4 * v + lk;
            Bc[(int64_t)colidx[li] * rp + row] = b0[v];
            Bc[(int64_t)colidx[16 + li] * rp + row] = b1[v];
            Pc[(int64_t)colidx[li] * rp + row] = p0[v];
            Pc[(int64_t)colidx[16 + li] * rp + row] = p1[v];
          }
        }
      }
      // the sweep's largest cosine is published before its last barrier
      if (rd == nb - 2 && tid == 0) cosbuf[wg] = sweep_cos;
      if (!grid_barrier()) return;
    }
    double c = 0.0;
    for (int w = 0; w < nwg; ++w) c = fmax(c, cosbuf[w]);
    last_cos = c;
    ++sweeps_done;
    converged = !(c > tol);
  }
  if (wg == 0 && tid == 0) {
    st->jacobi_sweeps = sweeps_done;
    st->jacobi_cosine = last_cos;
    st->jacobi_done = converged;
  }
}

#define WSSR_JACOBI_INST(NPU)                                                                                        \
  template __global__ void k_jacobi_coop<NPU>(double*, double*, int, double, const double*, double*, unsigned*,   \
                                              DevStatus*, int, int);
WSSR_JACOBI_INST(1)
WSSR_JACOBI_INST(2)
WSSR_JACOBI_INST(3)
WSSR_JACOBI_INST(4)
WSSR_JACOBI_INST(5)
WSSR_JACOBI_INST(6)
WSSR_JACOBI_INST(7)
WSSR_JACOBI_INST(8)

}  // namespace wssr
