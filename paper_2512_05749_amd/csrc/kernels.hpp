// Kernel declarations shared by the kernel sources and the host runtime.
#pragma once
#include "common.hpp"

namespace wssr {

__global__ void k_raise(DevStatus* st, int code);
__global__ void k_status_save(const DevStatus* st, int* out);
__global__ void k_status_init(DevStatus* st);
__global__ void k_center_energies(const double* e_l, int64_t n, double* eps, DevStatus* st);
__global__ void k_gradient_partial(const float* O, int64_t ld, int64_t n, int64_t m, const double* eps,
                                   int64_t rows_per_split, double* part, bool vec, const DevStatus* st);
__global__ void k_gradient_reduce(const double* part, int nsplit, int64_t m, double inv_n, double* g,
                                  const DevStatus* st);
__global__ void k_ysum(const float* ypart, int nsplit, int64_t total, double* y, const DevStatus* st);
__global__ void k_colsum_partial(const double* y, int64_t n, int r, int rows, double* colpart, const DevStatus* st);
__global__ void k_colreduce(const double* part, int nchunk, int r, double scale, double* out, const DevStatus* st);
__global__ void k_ycenter(double* y, const double* mean, int64_t total, int r, double inv_sqrt_n,
                          const DevStatus* st);
__global__ void k_sign_partial(const float* vnew, const float* vin, int64_t m, int r, int64_t rows_per_chunk,
                               double* dots, float* maxval, int64_t* maxrow, const DevStatus* st);
__global__ void k_sign_final(const double* dots, const float* maxval, const int64_t* maxrow, int nchunk, int r,
                             float* sgn, const DevStatus* st);
__global__ void k_sign_apply(const float* vnew, const float* sgn, int64_t total, int r, float* v,
                             const DevStatus* st);
__global__ void k_vtg_partial(const float* v, const double* g, int64_t m, int r, int64_t rows_per_chunk,
                              double* part, const DevStatus* st);
__global__ void k_vtg_final(const double* part, int nchunk, int r, const double* sig_sorted, double lambda,
                            int floor_form, double r_reg, double* cw, double* sigma_out, DevStatus* st);
__global__ void k_delta(const float* v, const double* g, const double* cw, int64_t m, int r, double inv_lambda,
                        double* delta, const DevStatus* st);

template <int BN>
__global__ void k_gemm_sample_side(const float* O, int64_t ld, int64_t n, int64_t m, const float* V, int r,
                                   float* ypart, int64_t kchunk, bool vec_o, bool vec_v, const DevStatus* st,
                                   int tn, int tj, bool xcd_groups);
template <int BN>
__global__ void k_gemm_sample_side_dma(const float* O, int64_t ld, int64_t n, int64_t m, const float* V, int r,
                                       float* ypart, int64_t kchunk, const float* zeros, const DevStatus* st, int tn,
                                       int tj, bool xcd_groups);
template <int BN>
__global__ void k_gemm_param_side_dma(const float* O, int64_t ld, int64_t n, int64_t m, const float* Q, int r,
                                      float scale, float* Z, const float* zeros, const DevStatus* st, int tiles_j,
                                      int full_tiles, int64_t sk_units, int sk_wgs, float* part);
// dynamic LDS bytes of the direct-to-LDS product kernels
size_t gemm_dma_lds(bool param_side, int bn);
// narrow parameter side (one 32-column tile, O staged through registers, static LDS)
__global__ void k_gemm_param_side_narrow(const float* O, int64_t ld, int64_t n, int64_t m, const float* Q, int r,
                                         float scale, float* Z, const float* zeros, const DevStatus* st, int tiles_j,
                                         int full_tiles, int64_t sk_units, int sk_wgs, float* part);
template <int BN>
__global__ void k_gemm_param_side(const float* O, int64_t ld, int64_t n, int64_t m, const float* Q, int r,
                                  float scale, float* Z, bool vec_o, bool vec_q, const DevStatus* st, int tiles_j,
                                  int full_tiles, int64_t sk_units, int sk_wgs, float* part);
template <int BN>
__global__ void k_streamk_fixup(const float* part, float* Z, int64_t m, int r, float scale, int tiles_j,
                                int full_tiles, int64_t nk, int64_t sk_units, int sk_wgs, const DevStatus* st);

template <int PL, int CPT>
__global__ void k_gradient16_partial(const unsigned short* O, int64_t ld, int64_t pstride, int64_t n, int64_t m,
                                     const double* eps, int64_t rows_per_split, double* part, bool vec,
                                     const DevStatus* st);

// BF16 products (kernels_gemm16.hip): BN output columns per tile, BK K-step,
// PA planes of O, PB planes of the skinny operand, which k_split_skinny has
// split into BF16 planes laid out [k / 16][column][k % 16] (plane stride in
// elements).
__global__ void k_split_skinny(const float* S, int64_t K, int r, int sw, unsigned short* out, int64_t pstride,
                               int planes, const DevStatus* st, const float* alt, const double* gd, const int* mode);
template <int BN, int BK, int PA, int PB>
__global__ void k_gemm16_sample_side(const unsigned short* O, int64_t ld, int64_t pstride, int64_t n, int64_t m,
                                     const unsigned short* Vs, int64_t vstride, int r, float* ypart, int64_t kchunk,
                                     bool vec_o, const DevStatus* st, int tn, int tj, bool xcd_groups);
template <int BN, int BK, int PA, int PB>
__global__ void k_gemm16_param_side(const unsigned short* O, int64_t ld, int64_t pstride, int64_t n, int64_t m,
                                    const unsigned short* Qs, int64_t qstride, int r, float scale, float* Z,
                                    bool vec_o, const DevStatus* st, int tiles_j, int full_tiles, int64_t sk_units,
                                    int sk_wgs, float* part);
size_t gemm16_lds(int bn, int bk, int pa, int pb);
template <int BN, int BK, int PA, int PB>
__global__ void k_gemm16_sample_side_dma(const unsigned short* O, int64_t ld, int64_t pstride, int64_t n, int64_t m,
                                         const unsigned short* Vs, int64_t vstride, int r, float* ypart,
                                         int64_t kchunk, const unsigned short* zeros, const DevStatus* st, int tn,
                                         int tj, bool xcd_groups);
template <int BN, int BK, int PA, int PB>
__global__ void k_gemm16_param_side_dma(const unsigned short* O, int64_t ld, int64_t pstride, int64_t n, int64_t m,
                                        const unsigned short* Qs, int64_t qstride, int r, float scale, float* Z,
                                        const unsigned short* zeros, const DevStatus* st, int tiles_j, int full_tiles,
                                        int64_t sk_units, int sk_wgs, float* part);
// dynamic LDS bytes of the direct-to-LDS BF16 product kernels
size_t gemm16_dma_lds(int bn, int bk, int pa, int pb);
// K-steps of the skinny operand in flight in the register-streamed BF16
// sample-side product (O: one more), per plane count of the skinny operand
#ifndef WSSR_RS1_DB
#define WSSR_RS1_DB 2
#endif
#ifndef WSSR_RS2_DB
#define WSSR_RS2_DB 2
#endif
// BF16 sample side with the skinny operand streamed into registers
// (kernels_gemm16_rs.hip): one O plane, BN columns per workgroup, DB K-steps
// of the skinny operand in flight
template <int BN, int PB, int DB>
__global__ void k_gemm16_param_side_rs(const unsigned short* O, int64_t ld, int64_t n, int64_t m,
                                       const unsigned short* Qs, int64_t qstride, int r, float scale, float* Z,
                                       const unsigned short* zeros, const DevStatus* st, int tiles_j, int full_tiles,
                                       int64_t sk_units, int sk_wgs, float* part);
template <int BN, int PB, int DB>
__global__ void k_gemm16_sample_side_rs(const unsigned short* O, int64_t ld, int64_t n, int64_t m,
                                        const unsigned short* Vs, int64_t vstride, int r, float* ypart,
                                        int64_t kchunk, const unsigned short* zeros, const DevStatus* st, int tn,
                                        int tj, bool xcd_groups);

template <typename T>
__global__ void k_gram_partial(const T* X, int64_t rows, int r, int64_t ldx, int ntile, int64_t rows_per_chunk,
                               double* part, bool vec, const DevStatus* st, bool gated);
__global__ void k_gram32_partial(const float* X, int64_t rows, int r, int64_t ldx, int ntile, int nchunk,
                                 int64_t rows_per_chunk, double* part, bool vec, const DevStatus* st, bool gated);
__global__ void k_gram16_partial(const float* X, int64_t rows, int r, int64_t ldx, int ntile, int nchunk,
                                 int64_t rows_per_chunk, double* part, const DevStatus* st, bool gated);
__global__ void k_gram_reduce(const double* part, int nchunk, int ntile, int r, int rp, double* G,
                              const DevStatus* st, bool gated);
template <typename Tin, typename Tout>
__global__ void k_apply(const Tin* X, int64_t rows, int ldx, int kdim, const double* Tm, int rp, int ncol,
                        Tout* Out, int ldo, bool upper, bool vec, bool acc, const DevStatus* st, bool gated);
__global__ void k_apply32(const float* X, int64_t rows, int ldx, int kdim, const float* Tf, int rp, int ncol,
                          float* Out, int ldo, bool upper, bool vec, bool acc_out, const DevStatus* st, bool gated);
__global__ void k_round_f32(const double* src, int64_t n, float* dst, const DevStatus* st, bool gated);
template <typename TX, typename TW>
__global__ void k_cross_partial(const TX* X, const TW* W, int64_t rows, int r, int ntile, int64_t rows_per_chunk,
                                double* part, bool vec, const DevStatus* st);
__global__ void k_cross_reduce(const double* part, int nchunk, int ntile, int r, int rp, double* H,
                               const DevStatus* st);
// tile of the Gram and apply kernels, and the Gram partial-buffer budget
constexpr int kF64Tile = 128;
constexpr size_t kGramPartBytes = (size_t)64 << 20;

__global__ void k_chol(double* G, int rp, int r, double* R, double* Rt, double* gdiag, double* invdiag, int* repcol,
                       DevStatus* st, bool gated);
template <typename T>
__global__ void k_complete(T* X, int64_t rows, int r, const double* R, int rp, const int* repcol,
                           const DevStatus* st);
template <int RPL>
__global__ void k_trinv(const double* Rt, int rp, const double* invdiag, double* Ri, const DevStatus* st, bool gated);
__global__ void k_kappa(const double* gdiag, const double* R, const double* Ri, int rp, int r, double kappa_round2,
                        DevStatus* st);
__global__ void k_smallgemm(const double* A, const double* B, int rp, double* C, const DevStatus* st, bool gated,
                            bool copy_b);
__global__ void k_jacobi_prep(const double* Ct, int rp, int r, double* Bc, double* Pc, double* scal,
                              unsigned* sync, DevStatus* st);
template <int NPU>
__global__ void k_jacobi_coop(double* Bc, double* Pc, int rp, double tol, const double* scal, double* cosbuf,
                              unsigned* sync, DevStatus* st, int max_sweeps, int inner_sweeps);
__global__ void k_jacobi_final(const double* Bc, const double* Pc, int rp, int r, double* sig, double* Ps,
                               DevStatus* st);

__global__ void k_transpose_pad(const double* C, int r, int rp, double* Ct);
// ingest of O (kernels_ingest.hip): storage form plus gradient and column sums
// from the unrounded values
template <int PL, bool OUT_F32>
__global__ void k_ingest_partial(const float* O32, int64_t ld32, int64_t rows, int64_t m, const double* eps,
                                 const double* mu, void* out, int64_t ld_out, int64_t pstride,
                                 int64_t rows_per_split, double* gpart, double* cpart, bool vec, bool vec_out,
                                 DevStatus* st);
__global__ void k_ingest_reduce(const double* gpart, const double* cpart, int nsplit, int64_t m, double inv_n,
                                bool first, double* g, double* mu);

// averaged-state step (kernels_avg.hip)
__global__ void k_hist_rows(double* yh, int r, const double* sig, const double* H, int ldh, double c,
                            const DevStatus* st);
__global__ void k_hist_b(const float* qtop, int r, const double* sig, double c, double* B, int rp,
                         const DevStatus* st);
__global__ void k_gbar_w(const double* sig, const double* l, int r, double coef, double* cw, const DevStatus* st);
__global__ void k_lhat(const double* eps, int64_t n, const double* l, int r, double a_new, double a_old,
                       double* lhat, const DevStatus* st);
__global__ void k_state_l(const double* Rz, const double* Ps, int rp, int r, const double* t, const float* sgn,
                          double* sig, double wscale, double* l_out, const DevStatus* st);
__global__ void k_transpose_rp(const double* R, int rp, int r, double* Ct, const DevStatus* st);
__global__ void k_diag_sort(const double* R, int rp, int r, double* sig, int* perm, const DevStatus* st);
__global__ void k_permute_cols(const float* src, int64_t m, int r, const int* perm, float* dst, const DevStatus* st);
__global__ void k_select_t(const int* mode, const double* gdiag, const double* r1i, const double* tq, int rp, int r,
                           double* out);
__global__ void k_fast_decide(const DevStatus* probe, double kappa_orth, double piv_fast, DevStatus* main,
                              DevStatus* st_m1, DevStatus* st_m2, DevStatus* st_m01, int* mode);
__global__ void k_copy_st(const double* src, int64_t count, double* dst, const DevStatus* st);
__global__ void k_colscale(const float* z, const double* gdiag, int64_t m, int r, float* v, const int* mode);
__global__ void k_status_merge(const DevStatus* from, DevStatus* to);
// sample-space solver (kernels_minsr.hip)
template <typename T, int PL>
__global__ void k_syrk_partial(const T* O, int64_t ld, int64_t pstride, int64_t n, int64_t m, int ntile,
                               int64_t kchunk, double* part, double* G, bool vec, const DevStatus* st);
__global__ void k_syrk_reduce(const double* part, int nchunk, int ntile, int64_t n, double* G, const DevStatus* st);
__global__ void k_row_mean(const double* G, int64_t n, double* rho, const DevStatus* st);
__global__ void k_dcenter(double* G, int64_t n, const double* rho, const double* tau, double scale, double lambda,
                          const DevStatus* st);
__global__ void k_potrf_diag(double* G, int64_t n, int64_t k0, int nb, DevStatus* st);
__global__ void k_trsm_panel(double* G, int64_t n, int64_t k0, int nb, const DevStatus* st);
__global__ void k_syrk_update(double* G, int64_t n, int64_t k0, int nb, int ntile, bool vec, const DevStatus* st);
__global__ void k_trsv_fwd_diag(const double* G, int64_t n, int64_t k0, int nb, double* y, const DevStatus* st);
__global__ void k_trsv_fwd_update(const double* G, int64_t n, int64_t k0, int nb, double* y, const DevStatus* st);
__global__ void k_trsv_bwd_diag(const double* G, int64_t n, int64_t k0, int nb, double* y, const DevStatus* st);
__global__ void k_trsv_bwd_update(const double* G, int64_t n, int64_t k0, int nb, double* y, const DevStatus* st);
template <typename T, int PL>
__global__ void k_gemv_rows(const T* O, int64_t ld, int64_t pstride, int64_t n, int64_t m, const double* x,
                            double* u, const DevStatus* st);
__global__ void k_spring_rhs(const double* eps, const double* u, const double* ubar, int64_t n, double a_eps,
                             double a_u, double* b, const DevStatus* st);
__global__ void k_axpby(const double* delta, int64_t m, double a, double b, double* dtheta, const DevStatus* st);

// dynamic LDS sizes (bytes)
constexpr size_t kCholLds = 4 * 64 * 65 * sizeof(double);
// dynamic LDS of k_jacobi_coop: the 32 columns of B, stride rp + 1
inline size_t jacobi_lds(int rp) { return (size_t)32 * (rp + 1) * sizeof(double); }

}  // namespace wssr
