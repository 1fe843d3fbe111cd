// Ingest of O: one pass over a block of rows of the FP32 matrix O that writes
// the block in the handle's storage form (FP32, one BF16 plane, or BF16 hi and
// lo planes) and accumulates, from the unrounded values, the gradient sums
// O^T eps (eq. barg) and the column sums of O (the means of eq. Osr).
//
// Rounding to BF16 is round-to-nearest-even on the FP32 bit pattern.  The lo
// plane holds RNE(x - hi), and x - hi is exact in FP32.  With a mean vector
// the stored values are those of x - mu (explicit centring before rounding);
// the sums always use the unshifted x.
//
// The sums are FP64 partials per row split, reduced in a fixed order, so the
// result does not depend on scheduling.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

namespace {

// FP32 -> BF16, round to nearest, ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const unsigned b = __builtin_bit_cast(unsigned, x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((b >> 16) | 0x40u);
  return (unsigned short)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __builtin_bit_cast(float, (unsigned)h << 16);
}

}  // namespace

// grid (column blocks of 256 * 8 columns, row splits); each thread owns 8
// adjacent columns and a contiguous range of rows of the block.
//   O32 (rows x m, stride ld32): the block's FP32 values
//   eps: centred energies of the block's rows (eps[0] is the block's first row)
//   mu (nullable, FP64 [m]): subtracted before the values are stored
//   out (nullable): first stored row; PL planes, plane stride pstride elements,
//   row stride ld_out; OUT_F32 stores FP32 (PL = 1) instead of BF16
//   gpart, cpart: [split][m] FP64 partial sums of x * eps and of x
// vec: 16-byte loads of O32 (ld32 % 4 == 0, 16-byte aligned base); vec_out:
// 16-byte stores of 8 BF16 values (ld_out % 8 == 0, 16-byte aligned base).
template <int PL, bool OUT_F32>
__global__ __launch_bounds__(256) void k_ingest_partial(const float* __restrict__ O32, int64_t ld32, int64_t rows,
                                                        int64_t m, const double* __restrict__ eps,
                                                        const double* __restrict__ mu, void* __restrict__ out,
                                                        int64_t ld_out, int64_t pstride, int64_t rows_per_split,
                                                        double* __restrict__ gpart, double* __restrict__ cpart,
                                                        bool vec, bool vec_out, DevStatus* st) {
  const int64_t c0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
  if (c0 >= m) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = min(rows, r0 + rows_per_split);
  const bool full = c0 + 8 <= m;
  float shift[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) shift[q] = (mu && c0 + q < m) ? (float)mu[c0 + q] : 0.0f;
  double ga[8], ca[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) ga[q] = ca[q] = 0.0;
  bool finite = true;
#pragma unroll 4
  for (int64_t i = r0; i < r1; ++i) {
    const float* src = O32 + i * ld32 + c0;
    float x[8];
    if (vec && full) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(src);
      const f32x4 b = *reinterpret_cast<const f32x4*>(src + 4);
      x[0] = a[0], x[1] = a[1], x[2] = a[2], x[3] = a[3];
      x[4] = b[0], x[5] = b[1], x[6] = b[2], x[7] = b[3];
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = c0 + q < m ? src[q] : 0.0f;
    }
    const double e = eps[i];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      ga[q] += (double)x[q] * e;
      ca[q] += (double)x[q];
      finite = finite && isfinite(x[q]);
    }
    if (!out) continue;
    float y[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) y[q] = x[q] - shift[q];
    if constexpr (OUT_F32) {
      float* dst = static_cast<float*>(out) + i * ld_out + c0;
      if (vec_out && full) {
        *reinterpret_cast<f32x4*>(dst) = f32x4{y[0], y[1], y[2], y[3]};
        *reinterpret_cast<f32x4*>(dst + 4) = f32x4{y[4], y[5], y[6], y[7]};
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (c0 + q < m) dst[q] = y[q];
      }
    } else {
      unsigned short h[8], l[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        h[q] = bf16_rne(y[q]);
        l[q] = PL == 2 ? bf16_rne(y[q] - bf16_to_f32(h[q])) : (unsigned short)0;
      }
      unsigned short* dst = static_cast<unsigned short*>(out) + i * ld_out + c0;
#pragma unroll
      for (int p = 0; p < PL; ++p) {
        const unsigned short* v = p == 0 ? h : l;
        unsigned short* d = dst + p * pstride;
        if (vec_out && full) {
          uint4 w;
          w.x = v[0] | ((unsigned)v[1] << 16);
          w.y = v[2] | ((unsigned)v[3] << 16);
          w.z = v[4] | ((unsigned)v[5] << 16);
          w.w = v[6] | ((unsigned)v[7] << 16);
          *reinterpret_cast<uint4*>(d) = w;
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (c0 + q < m) d[q] = v[q];
        }
      }
    }
  }
  if (!finite) raise_error(st, ST_NONFINITE);
  double* gp = gpart + (int64_t)blockIdx.y * m;
  double* cp = cpart + (int64_t)blockIdx.y * m;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (c0 + q < m) {
      gp[c0 + q] = ga[q];
      cp[c0 + q] = ca[q];
    }
}

// g (+)= inv_n * sum_s gpart[s], mu (+)= inv_n * sum_s cpart[s], in split
// order; `first` overwrites instead of adding.  Either output may be NULL.
__global__ __launch_bounds__(256) void k_ingest_reduce(const double* __restrict__ gpart,
                                                       const double* __restrict__ cpart, int nsplit, int64_t m,
                                                       double inv_n, bool first, double* __restrict__ g,
                                                       double* __restrict__ mu) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  double a = 0.0, b = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    a += gpart[(int64_t)s * m + c];
    b += cpart[(int64_t)s * m + c];
  }
  if (g) g[c] = (first ? 0.0 : g[c]) + a * inv_n;
  if (mu) mu[c] = (first ? 0.0 : mu[c]) + b * inv_n;
}

template __global__ void k_ingest_partial<1, true>(const float*, int64_t, int64_t, int64_t, const double*,
                                                   const double*, void*, int64_t, int64_t, int64_t, double*, double*,
                                                   bool, bool, DevStatus*);
template __global__ void k_ingest_partial<1, false>(const float*, int64_t, int64_t, int64_t, const double*,
                                                    const double*, void*, int64_t, int64_t, int64_t, double*, double*,
                                                    bool, bool, DevStatus*);
template __global__ void k_ingest_partial<2, false>(const float*, int64_t, int64_t, int64_t, const double*,
                                                    const double*, void*, int64_t, int64_t, int64_t, double*, double*,
                                                    bool, bool, DevStatus*);

}  // namespace wssr
