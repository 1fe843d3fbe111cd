// Memory-bound kernels of the step: energy centring, gradient, the reduction
// and centring of the sample-side product, the output-sign rule and the
// Woodbury apply.  All reductions run in a fixed order (no float atomics), so
// a step is bitwise reproducible.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

// ---------------------------------------------------------------------------
// eps = E_L - mean(E_L)   (eq. Lbarn); one workgroup of 1024 threads.
// ---------------------------------------------------------------------------
// Fail the running step from the host side (a launch that could not be made).
__global__ void k_raise(DevStatus* st, int code) { raise_error(st, code); }

// Keep a finished step's status code (batched steps: one slot per problem).
__global__ void k_status_save(const DevStatus* st, int* out) { *out = st->code; }

__global__ __launch_bounds__(1024) void k_center_energies(const double* __restrict__ e_l, int64_t n,
                                                          double* __restrict__ eps, DevStatus* st) {
  __shared__ double red[1024];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  double s = 0.0;
  int nf = 0;
  for (int64_t i = t; i < n; i += 1024) {
    const double v = e_l[i];
    s += v;
    nf |= !isfinite(v);
  }
  red[t] = s;
  __syncthreads();
  if (nf) bad = 1;
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (bad) {
    if (t == 0) raise_error(st, ST_NONFINITE);
    return;
  }
  const double mean = red[0] / (double)n;
  for (int64_t i = t; i < n; i += 1024) eps[i] = e_l[i] - mean;
}

// ---------------------------------------------------------------------------
// Gradient g = O^T eps / N (eq. barg; equals O_bar^T eps / N since sum eps = 0).
// Stage 1: grid (column blocks of 1024 columns, row splits); each thread owns 4
// consecutive columns and a contiguous range of rows; FP64 accumulation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gradient_partial(const float* __restrict__ O, int64_t ld, int64_t n,
                                                          int64_t m, const double* __restrict__ eps,
                                                          int64_t rows_per_split, double* __restrict__ part,
                                                          bool vec, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t c0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (c0 >= m) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = min(n, r0 + rows_per_split);
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 8
  for (int64_t i = r0; i < r1; ++i) {
    const f32x4 v = load4(O + i * ld, c0, m, vec);
    const double e = eps[i];
    a0 += (double)v[0] * e;
    a1 += (double)v[1] * e;
    a2 += (double)v[2] * e;
    a3 += (double)v[3] * e;
  }
  double* p = part + (int64_t)blockIdx.y * m;
  p[c0] = a0;
  if (c0 + 1 < m) p[c0 + 1] = a1;
  if (c0 + 2 < m) p[c0 + 2] = a2;
  if (c0 + 3 < m) p[c0 + 3] = a3;
}

// The same partial sums with O in BF16 (PL = 1) or as BF16 hi and lo planes
// (PL = 2, O = hi + lo, plane stride pstride elements).  Each thread sums CPT
// adjacent columns: 8 with 16-byte loads (rows of O 16-byte aligned) or 4
// with 8-byte loads (8-byte aligned); vec says which alignment holds.  Other
// threads, and the ragged last columns, load element by element.
template <int PL, int CPT>
__global__ __launch_bounds__(256) void k_gradient16_partial(const unsigned short* __restrict__ O, int64_t ld,
                                                            int64_t pstride, int64_t n, int64_t m,
                                                            const double* __restrict__ eps, int64_t rows_per_split,
                                                            double* __restrict__ part, bool vec, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t c0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * CPT;
  if (c0 >= m) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = min(n, r0 + rows_per_split);
  // a BF16 value is the upper half of an FP32 one
  auto lo = [](unsigned w) { return (double)__builtin_bit_cast(float, w << 16); };
  auto hi = [](unsigned w) { return (double)__builtin_bit_cast(float, w & 0xffff0000u); };
  double a[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) a[q] = 0.0;
  if (vec && c0 + CPT <= m) {
#pragma unroll 8
    for (int64_t i = r0; i < r1; ++i) {
      const double e = eps[i];
#pragma unroll
      for (int p = 0; p < PL; ++p) {
        const unsigned short* row = O + p * pstride + i * ld + c0;
        unsigned w[CPT / 2];
        if constexpr (CPT == 8) {
          const uint4 v = *reinterpret_cast<const uint4*>(row);
          w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
        } else {
          const uint2 v = *reinterpret_cast<const uint2*>(row);
          w[0] = v.x, w[1] = v.y;
        }
#pragma unroll
        for (int q = 0; q < CPT / 2; ++q) {
          a[2 * q] += lo(w[q]) * e;
          a[2 * q + 1] += hi(w[q]) * e;
        }
      }
    }
  } else {
    for (int64_t i = r0; i < r1; ++i) {
      const double e = eps[i];
#pragma unroll
      for (int p = 0; p < PL; ++p) {
        const unsigned short* row = O + p * pstride + i * ld + c0;
#pragma unroll
        for (int q = 0; q < CPT; ++q)
          if (c0 + q < m) a[q] += lo(row[q]) * e;
      }
    }
  }
  double* pp = part + (int64_t)blockIdx.y * m;
#pragma unroll
  for (int q = 0; q < CPT; ++q)
    if (c0 + q < m) pp[c0 + q] = a[q];
}
template __global__ void k_gradient16_partial<1, 4>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                    const double*, int64_t, double*, bool, const DevStatus*);
template __global__ void k_gradient16_partial<1, 8>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                    const double*, int64_t, double*, bool, const DevStatus*);
template __global__ void k_gradient16_partial<2, 4>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                    const double*, int64_t, double*, bool, const DevStatus*);
template __global__ void k_gradient16_partial<2, 8>(const unsigned short*, int64_t, int64_t, int64_t, int64_t,
                                                    const double*, int64_t, double*, bool, const DevStatus*);

__global__ __launch_bounds__(256) void k_gradient_reduce(const double* __restrict__ part, int nsplit, int64_t m,
                                                         double inv_n, double* __restrict__ g,
                                                         const DevStatus* st) {
  if (failed(st)) return;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * m + c];
  g[c] = s * inv_n;
}

// ---------------------------------------------------------------------------
// Sample side: y = sum_s ypart[s] (split-K partial products, fixed order), then
// centre the columns and scale: y <- (y - 1 mean^T) / sqrt(N).  This is the
// implicit centring of O: O_bar V = O V - 1 (mu^T V), and mu^T V is the
// column mean of O V.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ysum(const float* __restrict__ ypart, int nsplit, int64_t total,
                                              double* __restrict__ y, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  double v = 0.0;
  for (int s = 0; s < nsplit; ++s) v += (double)ypart[s * total + e];
  y[e] = v;
}

// Column sums over row blocks: grid (row blocks of `rows` rows, column blocks of 256).
__global__ __launch_bounds__(256) void k_colsum_partial(const double* __restrict__ y, int64_t n, int r, int rows,
                                                        double* __restrict__ colpart, const DevStatus* st) {
  if (failed(st)) return;
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= r) return;
  const int64_t i0 = (int64_t)blockIdx.x * rows;
  const int64_t i1 = min(n, i0 + rows);
  double a0 = 0.0, a1 = 0.0;
  int64_t i = i0;
  for (; i + 1 < i1; i += 2) {
    a0 += y[i * r + j];
    a1 += y[(i + 1) * r + j];
  }
  if (i < i1) a0 += y[i * r + j];
  colpart[(int64_t)blockIdx.x * r + j] = a0 + a1;
}

// Column reduction of partials part[c][j] over c (fixed order): one block of
// 256 threads per column, tree sum; out[j] = scale * sum.
__global__ __launch_bounds__(256) void k_colreduce(const double* __restrict__ part, int nchunk, int r, double scale,
                                                   double* __restrict__ out, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double red[256];
  const int j = blockIdx.x, t = threadIdx.x;
  double a = 0.0;
  for (int c = t; c < nchunk; c += 256) a += part[(int64_t)c * r + j];
  red[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[j] = scale * red[0];
}

__global__ __launch_bounds__(256) void k_ycenter(double* __restrict__ y, const double* __restrict__ mean,
                                                 int64_t total, int r, double inv_sqrt_n, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  y[e] = (y[e] - mean[e % r]) * inv_sqrt_n;
}

// ---------------------------------------------------------------------------
// Output signs.  Stage 1 (grid: row chunks x column blocks of 256): per column
// the partial inner product <vnew_j, vin_j> and the entry of largest magnitude
// (lowest row on ties) of vnew_j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sign_partial(const float* __restrict__ vnew, const float* __restrict__ vin,
                                                      int64_t m, int r, int64_t rows_per_chunk,
                                                      double* __restrict__ dots, float* __restrict__ maxval,
                                                      int64_t* __restrict__ maxrow, const DevStatus* st) {
  if (failed(st)) return;
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= r) return;
  const int64_t i0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t i1 = min(m, i0 + rows_per_chunk);
  double d = 0.0;
  float best = -1.0f, bestv = 0.0f;
  int64_t bestrow = -1;
  for (int64_t i = i0; i < i1; ++i) {
    const float a = vnew[i * r + j];
    if (vin) d += (double)a * (double)vin[i * r + j];
    if (fabsf(a) > best) {
      best = fabsf(a);
      bestv = a;
      bestrow = i;
    }
  }
  const int64_t o = (int64_t)blockIdx.x * r + j;
  dots[o] = d;
  maxval[o] = bestv;
  maxrow[o] = bestrow;
}

// Stage 2 (one block of 256 threads per column): sign_j from the partials.
__global__ __launch_bounds__(256) void k_sign_final(const double* __restrict__ dots, const float* __restrict__ maxval,
                                                    const int64_t* __restrict__ maxrow, int nchunk, int r,
                                                    float* __restrict__ sgn, const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double rd[256];
  __shared__ float rv[256];
  __shared__ int64_t rr[256];
  const int j = blockIdx.x, t = threadIdx.x;
  double d = 0.0;
  float bv = 0.0f;
  int64_t brow = -1;
  for (int c = t; c < nchunk; c += 256) {
    const int64_t o = (int64_t)c * r + j;
    d += dots[o];
    const float v = maxval[o];
    const int64_t row = maxrow[o];
    if (row >= 0 && (brow < 0 || fabsf(v) > fabsf(bv) || (fabsf(v) == fabsf(bv) && row < brow))) {
      bv = v;
      brow = row;
    }
  }
  rd[t] = d;
  rv[t] = bv;
  rr[t] = brow;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      rd[t] += rd[t + w];
      const float v = rv[t + w];
      const int64_t row = rr[t + w];
      if (row >= 0 && (rr[t] < 0 || fabsf(v) > fabsf(rv[t]) || (fabsf(v) == fabsf(rv[t]) && row < rr[t]))) {
        rv[t] = v;
        rr[t] = row;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const double dd = rd[0];
    sgn[j] = (fabs(dd) >= 1e-8) ? (dd >= 0.0 ? 1.0f : -1.0f) : (rv[0] >= 0.0f ? 1.0f : -1.0f);
  }
}

// Stage 3: v[i][j] = sgn[j] * vnew[i][j] (elementwise over m x r).
// grid-stride, four consecutive elements per thread and step (one 16-byte
// access each way when r % 4 == 0 and the rows are 16-byte aligned)
__global__ __launch_bounds__(256) void k_sign_apply(const float* __restrict__ vnew, const float* __restrict__ sgn,
                                                    int64_t total, int r, float* __restrict__ v,
                                                    const DevStatus* st) {
  if (failed(st)) return;
  const bool vec = (r % 4 == 0) && ((uintptr_t)vnew % 16 == 0) && ((uintptr_t)v % 16 == 0);
  const int64_t stride = (int64_t)gridDim.x * 256 * 4;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4; e < total; e += stride) {
    const int c = (int)(e % r);
    if (vec) {
      f32x4 x = *reinterpret_cast<const f32x4*>(vnew + e);
      x[0] *= sgn[c];
      x[1] *= sgn[c + 1];
      x[2] *= sgn[c + 2];
      x[3] *= sgn[c + 3];
      *reinterpret_cast<f32x4*>(v + e) = x;
    } else {
      for (int q = 0; q < 4 && e + q < total; ++q) v[e + q] = sgn[(e + q) % r] * vnew[e + q];
    }
  }
}

// ---------------------------------------------------------------------------
// Woodbury apply.  delta = (g - V diag(w) V^T g) / lambda, with
//   damped: w_j = sigma_j^2 / (sigma_j^2 + lambda)     ((V S^2 V^T + lambda I)^{-1} g)
//   floor:  w_j = 1 - lambda / sigma_j^2  (0 where sigma_j = 0)   (eq. updated_sr_1)
// Stage 1: partial c = V^T g over row chunks (grid: chunks x column blocks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vtg_partial(const float* __restrict__ v, const double* __restrict__ g,
                                                     int64_t m, int r, int64_t rows_per_chunk,
                                                     double* __restrict__ part, const DevStatus* st) {
  if (failed(st)) return;
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= r) return;
  const int64_t i0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t i1 = min(m, i0 + rows_per_chunk);
  // four rows per trip, their loads issued together; four partial sums
  // added in a fixed order at the end
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  int64_t i = i0;
  for (; i + 3 < i1; i += 4) {
    const float x0 = v[i * r + j], x1 = v[(i + 1) * r + j], x2 = v[(i + 2) * r + j], x3 = v[(i + 3) * r + j];
    d0 += (double)x0 * g[i];
    d1 += (double)x1 * g[i + 1];
    d2 += (double)x2 * g[i + 2];
    d3 += (double)x3 * g[i + 3];
  }
  for (; i < i1; ++i) d0 += (double)v[i * r + j] * g[i];
  part[(int64_t)blockIdx.x * r + j] = (d0 + d1) + (d2 + d3);
}

// Stage 2 (one block of 256 threads per column): cw_j = w_j * c_j; also
// writes sigma to the caller.  With r_reg > 0 only the columns with
// sigma_j^2 >= r_reg sigma_0^2 enter (the rank of eq. ruler); block 0 records
// that rank and whether the last column passed in the status word.
__global__ __launch_bounds__(256) void k_vtg_final(const double* __restrict__ part, int nchunk, int r,
                                                   const double* __restrict__ sig_sorted, double lambda, int floor_form,
                                                   double r_reg, double* __restrict__ cw,
                                                   double* __restrict__ sigma_out, DevStatus* st) {
  if (failed(st)) return;
  __shared__ double red[256];
  const int j = blockIdx.x, t = threadIdx.x;
  double a = 0.0;
  for (int c = t; c < nchunk; c += 256) a += part[(int64_t)c * r + j];
  red[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double s = sig_sorted[j];
    const double s2 = s * s;
    const double s0 = sig_sorted[0];
    const bool keep = s2 >= r_reg * (s0 * s0);
    const double w = !keep ? 0.0 : floor_form ? (s2 > 0.0 ? 1.0 - lambda / s2 : 0.0) : s2 / (s2 + lambda);
    cw[j] = w * red[0];
    sigma_out[j] = s;
    if (j == 0) {
      int k = 0;
      for (int i = 0; i < r; ++i) k += sig_sorted[i] * sig_sorted[i] >= r_reg * (s0 * s0);
      st->r_eff = k;
      st->grow = sig_sorted[r - 1] * sig_sorted[r - 1] >= r_reg * (s0 * s0);
    }
  }
}

// Stage 3: one wavefront per row: delta_i = (g_i - sum_j V[i][j] cw[j]) / lambda.
__global__ __launch_bounds__(256) void k_delta(const float* __restrict__ v, const double* __restrict__ g,
                                               const double* __restrict__ cw, int64_t m, int r, double inv_lambda,
                                               double* __restrict__ delta, const DevStatus* st) {
  if (failed(st)) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  double d = 0.0;
  const float* row = v + i * r;
  if ((r % 4) == 0 && ((uintptr_t)v % 16) == 0) {
    // 16-byte loads, two in flight per lane before their sums
    int j = 4 * lane;
    for (; j + 256 < r; j += 512) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(row + j);
      const f32x4 b = *reinterpret_cast<const f32x4*>(row + j + 256);
#pragma unroll
      for (int q = 0; q < 4; ++q) d += (double)a[q] * cw[j + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) d += (double)b[q] * cw[j + 256 + q];
    }
    if (j < r) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(row + j);
#pragma unroll
      for (int q = 0; q < 4; ++q) d += (double)a[q] * cw[j + q];
    }
  } else {
    for (int j = lane; j < r; j += 64) d += (double)row[j] * cw[j];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
  if (lane == 0) delta[i] = (g[i] - d) * inv_lambda;
}

}  // namespace wssr

namespace wssr {
__global__ void k_status_init(DevStatus* st) {
  if (threadIdx.x == 0) {
    st->code = 0;
    st->chol_count = 0;
    st->min_rel_pivot = 1.0;
    st->jacobi_sweeps = 0.0;
    st->jacobi_cosine = 0.0;
    st->jacobi_done = 0;
    st->round2 = 0;
    st->kappa_max = 0.0;
    st->round2_count = 0;
    st->rank_def = 0;
    st->r_eff = 0;
    st->grow = 0;
    st->repl = 0;
  }
}
}  // namespace wssr
