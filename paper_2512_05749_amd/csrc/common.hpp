// Shared definitions of the libwssr kernels (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace wssr {

// Device-side status of the running step.  code: 0 ok, < 0 error (first error
// sticks), > 0 warning.  The remaining fields are diagnostics.
struct DevStatus {
  int code;
  int chol_count;
  double min_rel_pivot;   // smallest sqrt(pivot / original diagonal) seen
  double jacobi_sweeps;
  double jacobi_cosine;   // largest column cosine left after the Rayleigh-Ritz Jacobi
  int jacobi_done;        // set once a Jacobi sweep found every column pair orthogonal
  int round2;             // set by a first-round Cholesky when a second CholeskyQR round is needed
  double kappa_max;       // largest condition bound ||R D^-1||_F ||D R^-1||_F seen
  int round2_count;       // second rounds actually run
  int rank_def;           // pivots of first-round Cholesky factorizations replaced in this step
  int repl;               // set by a first-round Cholesky that replaced a pivot; forces its second round
  int r_eff;              // rank kept by the truncation ratio (eq. ruler) in the last step's direction
  int grow;               // the last computed value passed the ratio (the condition for growing r_max)
};

enum : int {
  ST_OK = 0,
  ST_WARN_RANK_DEFICIENT = 1,
  ST_WARN_NOT_CONVERGED = 2,
  ST_NONFINITE = -5,
  ST_BREAKDOWN = -6,
  ST_TIMEOUT = -7,
  ST_SKIP = -1000          // a shadow status word whose kernels are not to run
};

__device__ __forceinline__ void raise_error(DevStatus* st, int code) {
  atomicCAS(&st->code, 0, code);
}

__device__ __forceinline__ bool failed(const DevStatus* st) {
  return *reinterpret_cast<const volatile int*>(&st->code) < 0;
}

// Kernels of an optional second CholeskyQR round run only when the first
// round asked for it (st->round2); `gated` selects that behaviour.
__device__ __forceinline__ bool skipped(const DevStatus* st, bool gated) {
  return failed(st) || (gated && *reinterpret_cast<const volatile int*>(&st->round2) == 0);
}

// 32x32x2 FP32 MFMA.  Lane l: A[i][k] with i = l%32, k = l/32; B[k][j] with
// j = l%32, k = l/32; D[i][j] in register v: i = 8*(v/4) + 4*(l/32) + v%4, j = l%32.
__device__ __forceinline__ f32x16 mfma32x32x2(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// 16x16x4 FP64 MFMA.  Lane l: A[i][k] with i = l%16, k = l/16; B[k][j] with
// j = l%16, k = l/16; D[i][j] in register v: i = 4*v + l/16, j = l%16.
__device__ __forceinline__ f64x4 mfma16x16x4d(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Four consecutive floats p[i0..i0+3], zero beyond lim; one 16-byte load when
// vec (caller guarantees 16-byte alignment of p + i0 in that case).
__device__ __forceinline__ f32x4 load4(const float* __restrict__ p, int64_t i0, int64_t lim, bool vec) {
  if (vec && i0 + 3 < lim) return *reinterpret_cast<const f32x4*>(p + i0);
  f32x4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = (i0 + e < lim) ? p[i0 + e] : 0.0f;
  return v;
}

// Pairing of a round-robin tournament on n (even) players: in round `rd`
// (0 <= rd < n-1) slot t (0 <= t < n/2) pairs players (p, q); over the n-1
// rounds every pair meets once.  Player n-1 stays fixed, the others rotate.
__device__ __forceinline__ void rr_pair(int n, int rd, int t, int& p, int& q) {
  const int m = n - 1;
  int a, b;
  if (t == 0) {
    a = m;
    b = rd % m;
  } else {
    a = (rd + t) % m;
    b = (rd - t + m) % m;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

}  // namespace wssr
