// Small kernels of the averaged-state step (Sec. 4.1, eqs. Ohat, Lhat, Obar,
// Lbar, barg), of the randomized-sketch step (App. A) and of Alg. 1's
// diag(R) ending.  In the averaged
// step the stored matrix of the previous step, U diag(sigma), enters the
// subspace iteration as r extra rows of the sample-side block; these kernels
// build those rows and the r x r factors that carry them through the
// parameter-side product, the averaged gradient, and the new stored vector.
#include "common.hpp"
#include "kernels.hpp"

namespace wssr {

// History rows of the sample-side block: Yh[i][j] = c sigma_i H[i][j]
// (i, j < r; Yh has row stride r, H row stride ldh).  c = 0 writes zeros
// without reading H.
__global__ __launch_bounds__(256) void k_hist_rows(double* __restrict__ yh, int r, const double* __restrict__ sig,
                                                   const double* __restrict__ H, int ldh, double c,
                                                   const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e / r), j = (int)(e % r);
  yh[e] = c == 0.0 ? 0.0 : c * sig[i] * H[(int64_t)i * ldh + j];
}

// Factor of the history term of the parameter-side product:
// B[i][j] = c sigma_i Qtop[i][j] for i, j < r, zero elsewhere in rp x rp
// (Qtop: the r history rows of the orthonormal sample-side block, stride r).
__global__ __launch_bounds__(256) void k_hist_b(const float* __restrict__ qtop, int r, const double* __restrict__ sig,
                                                double c, double* __restrict__ B, int rp, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rp * rp) return;
  const int i = (int)(e / rp), j = (int)(e % rp);
  B[e] = (i < r && j < r) ? c * sig[i] * (double)qtop[(int64_t)i * r + j] : 0.0;
}

// Weights of the averaged gradient's history term: cw_j = coef sigma_j l_j.
__global__ __launch_bounds__(256) void k_gbar_w(const double* __restrict__ sig, const double* __restrict__ l, int r,
                                                double coef, double* __restrict__ cw, const DevStatus* st) {
  if (failed(st)) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < r) cw[j] = coef * sig[j] * l[j];
}

// The stacked vector of eq. Lhat in the row order of the sample-side block:
// lhat[i] = a_new eps_i (i < n), lhat[n + i] = a_old l_i (i < r).
__global__ __launch_bounds__(256) void k_lhat(const double* __restrict__ eps, int64_t n, const double* __restrict__ l,
                                              int r, double a_new, double a_old, double* __restrict__ lhat,
                                              const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n)
    lhat[e] = a_new * eps[e];
  else if (e < n + r)
    lhat[e] = a_old * l[e - n];
}

// New stored vector (eq. Lbar) and singular values.  With the Rayleigh-Ritz
// matrix C = R_Z^T = G diag(s) P^T, the sample-side singular vectors are
// Q_Y G and G^T = diag(1/s) P^T R_Z, so L = sgn * diag(1/s) P^T (R_Z t) with
// t = Q_Y^T Lhat.  A zero singular value gives L_j = 0.  The singular values
// are then scaled in place by `wscale` (those of the block the iteration ran
// on are 1/wscale times those of the stacked matrix).  One workgroup.
__global__ __launch_bounds__(512) void k_state_l(const double* __restrict__ Rz, const double* __restrict__ Ps, int rp,
                                                 int r, const double* __restrict__ t, const float* __restrict__ sgn,
                                                 double* __restrict__ sig, double wscale, double* __restrict__ l_out,
                                                 const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double ts[512], us[512];
  for (int k = threadIdx.x; k < r; k += blockDim.x) ts[k] = t[k];
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    double a = 0.0;
    for (int k = i; k < r; ++k) a += Rz[(int64_t)i * rp + k] * ts[k];
    us[i] = a;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    double a = 0.0;
    for (int k = 0; k < r; ++k) a += Ps[(int64_t)k * rp + j] * us[k];
    const double s = sig[j];
    l_out[j] = s > 0.0 ? (double)sgn[j] * a / s : 0.0;
    sig[j] = wscale * s;
  }
}

// Ct = R^T restricted to r x r (zero elsewhere in rp x rp); R is rp x rp
// row-major.
__global__ __launch_bounds__(256) void k_transpose_rp(const double* __restrict__ R, int rp, int r,
                                                      double* __restrict__ Ct, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rp * rp) return;
  const int i = (int)(e / rp), j = (int)(e % rp);
  Ct[e] = (i < r && j < r) ? R[(int64_t)j * rp + i] : 0.0;
}

// Alg. 1's diag(R) ending: sig = |diag(R)| (R rp x rp row-major, r used)
// in descending order (ties by index) and perm[j] = the column that goes to
// position j.  One workgroup; the rank of each value is counted.
__global__ __launch_bounds__(512) void k_diag_sort(const double* __restrict__ R, int rp, int r,
                                                   double* __restrict__ sig, int* __restrict__ perm,
                                                   const DevStatus* st) {
  if (failed(st)) return;
  __shared__ double d[512];
  for (int i = threadIdx.x; i < r; i += blockDim.x) d[i] = fabs(R[(int64_t)i * rp + i]);
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    int pos = 0;
    for (int k = 0; k < r; ++k) pos += d[k] > d[i] || (d[k] == d[i] && k < i);
    sig[pos] = d[i];
    perm[pos] = i;
  }
}

// dst[:, j] = src[:, perm[j]] (m x r, row stride r).
__global__ __launch_bounds__(256) void k_permute_cols(const float* __restrict__ src, int64_t m, int r,
                                                      const int* __restrict__ perm, float* __restrict__ dst,
                                                      const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * r) return;
  const int64_t i = e / r;
  const int j = (int)(e % r);
  dst[e] = src[i * r + perm[j]];
}

// The choice between the FP32 probe's factorisation and the FP64
// CholeskyQR2, from the probe (the FP32 Gram's Cholesky): mode 0 when the
// columns are already orthogonal (condition bound <= kappa_orth, every
// relative pivot >= 0.99), 1 when every relative pivot is >= piv_fast, 2
// otherwise (and on any breakdown or replaced pivot); -1 when the step has
// already failed.  The alternatives' status words start clean, or skipped
// (code ST_SKIP) when not chosen: st_m1 runs in mode 1, st_m2 in mode 2,
// st_m01 in modes 0 and 1.  When the probe's factor is used its diagnostics
// are folded into the step's status.
__global__ void k_fast_decide(const DevStatus* __restrict__ probe, double kappa_orth, double piv_fast,
                              DevStatus* __restrict__ main, DevStatus* __restrict__ st_m1, DevStatus* __restrict__ st_m2,
                              DevStatus* __restrict__ st_m01, int* __restrict__ mode) {
  if (threadIdx.x != 0) return;
  int md = 2;
  if (!failed(probe) && probe->rank_def == 0 && probe->repl == 0) {
    const double piv = probe->min_rel_pivot;
    if (probe->kappa_max <= kappa_orth && piv >= 0.99)
      md = 0;
    else if (piv >= piv_fast)
      md = 1;
  }
  if (failed(main)) md = -1;
  *mode = md;
  if (md == 0 || md == 1) {
    main->chol_count += probe->chol_count;
    if (probe->min_rel_pivot < main->min_rel_pivot) main->min_rel_pivot = probe->min_rel_pivot;
    if (probe->kappa_max > main->kappa_max) main->kappa_max = probe->kappa_max;
  }
  DevStatus* sts[3] = {st_m1, st_m2, st_m01};
  const bool run[3] = {md == 1, md == 2, md == 0 || md == 1};
  for (int k = 0; k < 3; ++k) {
    DevStatus* s = sts[k];
    s->code = run[k] ? 0 : ST_SKIP;
    s->chol_count = 0;
    s->min_rel_pivot = 1.0;
    s->jacobi_sweeps = 0.0;
    s->jacobi_cosine = 0.0;
    s->jacobi_done = 0;
    s->round2 = 0;
    s->kappa_max = 0.0;
    s->round2_count = 0;
    s->rank_def = 0;
    s->repl = 0;
    s->r_eff = 0;
    s->grow = 0;
  }
}

// The factor T of an intermediate pass's basis V = Z T (fast_orth's mode):
// 0: diag(G)^{-1/2} (0 where G_jj <= 0), 1: the probe's R^{-1}, 2: the FP64
// CholeskyQR2's Tq; rp x rp, zero outside the r x r block in mode 0 (the
// others carry the factors' identity padding).  Nothing in mode -1.
__global__ __launch_bounds__(256) void k_select_t(const int* __restrict__ mode, const double* __restrict__ gdiag,
                                                  const double* __restrict__ r1i, const double* __restrict__ tq,
                                                  int rp, int r, double* __restrict__ out) {
  const int md = *mode;
  if (md < 0) return;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)rp * rp) return;
  if (md == 0) {
    const int i = (int)(idx / rp), j = (int)(idx % rp);
    const double d = (i == j && i < r) ? gdiag[i] : 0.0;
    out[idx] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  } else {
    out[idx] = (md == 1 ? r1i : tq)[idx];
  }
}

// dst = src (count doubles) unless the status word says skip.
__global__ __launch_bounds__(256) void k_copy_st(const double* __restrict__ src, int64_t count,
                                                 double* __restrict__ dst, const DevStatus* st) {
  if (failed(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = src[e];
}

// V = Z diag(gdiag)^{-1/2} (columns scaled to unit norm) when mode == 0.
// Grid-stride, four consecutive elements per thread and step (16-byte
// accesses when r % 4 == 0 and the rows are 16-byte aligned).
__global__ __launch_bounds__(256) void k_colscale(const float* __restrict__ z, const double* __restrict__ gdiag,
                                                  int64_t m, int r, float* __restrict__ v, const int* __restrict__ mode) {
  if (*mode != 0) return;
  const int64_t total = m * r;
  const bool vec = (r % 4 == 0) && ((uintptr_t)z % 16 == 0) && ((uintptr_t)v % 16 == 0);
  const int64_t stride = (int64_t)gridDim.x * 256 * 4;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4; e < total; e += stride) {
    if (vec) {
      const int c = (int)(e % r);
      f32x4 x = *reinterpret_cast<const f32x4*>(z + e);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double d = gdiag[c + q];
        x[q] = d > 0.0 ? (float)((double)x[q] / sqrt(d)) : 0.0f;
      }
      *reinterpret_cast<f32x4*>(v + e) = x;
    } else {
      for (int q = 0; q < 4 && e + q < total; ++q) {
        const double d = gdiag[(e + q) % r];
        v[e + q] = d > 0.0 ? (float)((double)z[e + q] / sqrt(d)) : 0.0f;
      }
    }
  }
}

// Fold the FP64 alternative's outcome into the step's status: its error (if
// it ran and failed) and its diagnostics.
__global__ void k_status_merge(const DevStatus* __restrict__ from, DevStatus* __restrict__ to) {
  if (threadIdx.x != 0 || from->code == ST_SKIP) return;
  if (from->code < 0) raise_error(to, from->code);
  to->chol_count += from->chol_count;
  to->round2_count += from->round2_count;
  to->rank_def += from->rank_def;
  if (from->min_rel_pivot < to->min_rel_pivot) to->min_rel_pivot = from->min_rel_pivot;
  if (from->kappa_max > to->kappa_max) to->kappa_max = from->kappa_max;
}

}  // namespace wssr
