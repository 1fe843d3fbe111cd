// Host runtime of libwssr: handle, workspace, launch plans and the C ABI.
#include "wssr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

using namespace wssr;

namespace {

// K-step of a direct-to-LDS BF16 product kernel instantiation (wssr_ctx::bk_dma)
#define BKD(BN, PA, PB) ((BN) == 512 && ((PA) > 1 || (PB) > 1) ? 16 : 32)
constexpr int kS1Max = 32;      // split-K ranges of the sample-side product
constexpr int kGSplitMax = 16;  // row splits of the gradient
constexpr int kVecChunkMax = 1024;
constexpr int kJacobiSweeps = 30;
constexpr int kJacobiInner = 1;     // inner sweeps per block step
constexpr double kJacobiTol = 1e-8;
constexpr double kKappaRound2 = 1e4;
#ifdef WSSR_FAST_MID_OFF
constexpr bool kFastMid = false;   // intermediate passes always take the FP64 CholeskyQR2
#else
constexpr bool kFastMid = true;
#endif
constexpr int kBatchMax = 1024;     // problems per batched step
// Gram of a float block: FP64 MFMA; FP32 MFMA with FP64 flushes (entries to
// about 1e-7 relative); the BF16 MFMA on the two-plane split (about 3e-7)
enum { kGram64 = 0, kGram32 = 1, kGram16 = 2 };
constexpr int kLanesMax = 16;       // concurrent batch lanes
#ifndef WSSR_RS_ROUNDS
#define WSSR_RS_ROUNDS 4
#endif
constexpr int kRsRounds = WSSR_RS_ROUNDS;
#ifdef WSSR_RS_OFF
constexpr bool kUseRs = false;
#else
constexpr bool kUseRs = true;
#endif

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

}  // namespace

struct wssr_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  wssr_config cfg{};
  std::string err;
  int rp_max = 0;
  int64_t rows_max = 0;
  int slots = 512;               // resident product workgroups: 2 per compute unit
  unsigned* jsync = nullptr;     // grid-barrier words of the Rayleigh-Ritz sweep kernel
  bool own_stream = false;       // a batch lane: the stream was created with the context
  bool capturing = false;        // enqueueing into a graph capture (no cooperative launch, no profiling)
  bool plain_svd = false;        // batch lanes: the Jacobi grid as a plain launch (see small_svd)
  std::vector<wssr_ctx*> lanes;  // batch lanes (children with their own stream and workspace)
  std::vector<hipEvent_t> lane_done;
  int* bstat = nullptr;          // per-problem status codes of the last batch
  int active_lanes = 0;          // lanes a batch uses (0: all); set by wssr_tune_batched
  int slot_div = 1;              // product kernels size their split for slots / slot_div workgroups
  std::vector<wssr_problem> gkey;  // the batch the cached graph was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_broken = false;
  hipStream_t cstream = nullptr;   // capture origin (the caller's stream may be the null stream)
  std::string graph_why;
  hipError_t coop_err = hipSuccess;
  hipStream_t side = nullptr;    // second stream: the gradient pass runs beside the Rayleigh-Ritz SVD
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  float* skpart = nullptr;       // stream-K partial tiles of the parameter-side product
  float* zeros = nullptr;        // 4 KB of zeros: the source of out-of-range direct-to-LDS copies
  unsigned short* s16 = nullptr; // BF16 forms: split planes of the skinny operand of a product
  int64_t skpart_elems = 0;
  std::vector<void*> allocs;

  DevStatus* st = nullptr;
  double *eps = nullptr, *g = nullptr, *gpart = nullptr;
  float* ypart = nullptr;
  double *y64 = nullptr, *yq1 = nullptr, *colpart = nullptr;
  float *qy = nullptr, *z = nullptr, *q1 = nullptr, *vw = nullptr;
  double* gram_part = nullptr;
  double *G = nullptr, *R1 = nullptr, *R1i = nullptr, *R2 = nullptr, *R2i = nullptr, *Rz = nullptr;
  double *Bc = nullptr, *Pc = nullptr, *Ps = nullptr, *T = nullptr, *scal = nullptr, *sig = nullptr;
  double *cosbuf = nullptr, *cw = nullptr, *vpart = nullptr, *dots = nullptr, *ymean = nullptr, *Tq = nullptr;
  double *Rt = nullptr, *gdiag = nullptr, *invdiag = nullptr;
  int* repcol = nullptr;          // columns whose first-round pivot was replaced (rank deficiency)
  // averaged-state step: the first pass's sample-side block, the cross
  // products that carry the history rows through later passes, the factor of
  // the parameter-side history term, the averaged gradient, the stacked
  // vector Lhat and its projection
  double *y1 = nullptr, *Hc = nullptr, *Hn = nullptr, *Bm = nullptr, *gbar = nullptr, *lhat = nullptr;
  double* tvec = nullptr;
  int64_t gram_part_elems = 0;
  // sample-space solver (wssr_spring, flag WSSR_SAMPLE_SPACE): T (n_max^2),
  // its K-chunk partial tiles, and n-vectors
  double *Tn = nullptr, *tpart = nullptr, *rho = nullptr, *su = nullptr, *sb = nullptr, *sscal = nullptr;
  int64_t tpart_tiles = 0;
  double r_reg = 0.0;             // truncation ratio of eq. ruler (wssr_set_rank_ratio; 0: none)
  DevStatus* shadow = nullptr;    // status words of the factorisation probe and its alternatives (4)
  int* fmode = nullptr;           // fast_orth's choice (0 scale, 1 FP32 apply, 2 FP64 CholeskyQR)
  const float* split_alt = nullptr;  // Z for the next split_skinny to scale itself (fast_orth, mode 0)
  float* tf32 = nullptr;          // the factor of an FP32 apply, rounded to float (rp x rp)
  int* perm = nullptr;            // column order of the diag(R) ending
  float *maxval = nullptr, *sgn = nullptr;
  int64_t* maxrow = nullptr;

  // stage timing (wssr_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;

  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  // record events around `launch` when profiling is on
  template <typename F>
  void timed(int slot, F&& launch) {
    if (!prof || capturing) {
      launch();
      return;
    }
    hipEvent_t a = next_event(), b = next_event();
    if (a) (void)hipEventRecord(a, stream);
    launch();
    if (b) (void)hipEventRecord(b, stream);
    if (a && b) ev_marks.push_back({slot, {a, b}});
  }

  wssr_status fail(wssr_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }

  void release() {
    for (wssr_ctx* c : lanes) {
      c->release();
      delete c;
    }
    lanes.clear();
    for (hipEvent_t e : lane_done) (void)hipEventDestroy(e);
    lane_done.clear();
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    if (cstream) {
      (void)hipStreamSynchronize(cstream);
      (void)hipStreamDestroy(cstream);
      cstream = nullptr;
    }
    if (own_stream && stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
      stream = nullptr;
    }
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
    side = nullptr;
    ev_fork = ev_join = nullptr;
    ev_pool.clear();
    allocs.clear();
  }

  template <typename T>
  bool alloc(T*& p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    allocs.push_back(q);
    p = static_cast<T*>(q);
    return true;
  }

  // ---------------------------------------------------------------- kernels
  hipError_t last() { return hipGetLastError(); }

  // Averaged state of a step (wssr_step_avg): the stored matrix of the
  // previous step is V_in diag(sig_state) and its vector l_state.
  struct AvgArgs {
    double avg;           // averaging weight, 0 <= avg < 1
    double* sig_state;    // r: in, the stored singular values; out, the new ones
    double* l_state;      // r: in, the stored vector; out, the new one
    double* gbar_out;     // m (nullable): the averaged gradient
  };

  // Enqueue one step on this context's stream (arguments already checked).
  // g_ext (nullable): a gradient the caller formed (wssr_step_g); the step
  // then makes no gradient pass and, without averaging, does not read e_l.
  // av (nullable): the averaged-state step.  The iteration then runs on the
  // block [A ; c diag(sig_state) V_in^T] (n + r rows, c = sqrt(avg/(1-avg))),
  // which is the stacked matrix of eq. Ohat divided by sqrt(1 - avg):
  //  * pass 1's history rows are c diag(sig) V_in^T V_in (a Gram of V_in);
  //  * later passes' are c diag(sig) V_in^T V_p with V_p = Z Tq of the pass
  //    before, and V_in^T Z = Y_1^T Q_Y (Y_1 = pass 1's block, Z its product
  //    with Q_Y), so no further product over the M rows of V_in is needed;
  //  * the parameter-side product gains V_in B, B = c diag(sig) Q_Y[n:n+r];
  //  * the Rayleigh-Ritz step is unchanged (C = R_Z^T), and the singular
  //    values are scaled back by sqrt(1 - avg) at the end.
  // Continuation of another step's work (the sketch's power passes): the
  // passes start from vstart (m x r) instead of V, keep the status word, sign
  // by the largest entry instead of against V, and return the first r_out
  // columns.
  struct Cont {
    const float* vstart;
    int r_out;
  };

  wssr_status enqueue(int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l, float* V,
                      double lambda, int32_t r, int32_t q, double* delta, double* sigma,
                      const double* g_ext = nullptr, const AvgArgs* av = nullptr, const Cont* cont = nullptr) {
    wssr_ctx* h = this;
    const double* gv = g_ext ? g_ext : h->g;
    const int rp = (int)rup(r, 64);
    const int r_out = cont ? cont->r_out : r;
    const DevStatus* cst = h->st;
    hipStream_t stream = h->stream;
    h->split_alt = nullptr;
    if (!cont) hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, stream, h->st);

    const double c_hist = av ? std::sqrt(av->avg / (1.0 - av->avg)) : 0.0;
    const bool hist = av && c_hist > 0.0;          // history rows that are not all zero
    const int64_t ny = av ? n + r : n;             // rows of the sample-side block
    double* yh = h->y64 + n * r;                   // its history rows
    if (av && g_ext) hipLaunchKernelGGL(k_center_energies, dim3(1), dim3(1024), 0, stream, e_l, n, h->eps, h->st);
    // pass 1's history rows come from the Gram of V_in
    if (hist) h->gram(V, m, r, false, kGram32);

    const float* vcur = cont ? cont->vstart : V;
    // Alg. 1's own ending: the last pass stops after the QR of its
    // sample-side block, whose basis must be orthonormal (for q = 1, V_in is
    // orthonormalised first)
    const bool diag_end = (h->cfg.flags & WSSR_DIAGR_EXTRACT) && !cont && !av;
    if (diag_end && q == 1) {
      h->cholqr<float, float>(V, m, r, h->q1, nullptr);
      h->apply((const float*)V, m, r, r, h->Tq, rp, r, h->vw, r, true);
      vcur = h->vw;
    }
    for (int p = 1; p <= q; ++p) {
      // sample side: Y = A V (FP64), then its QR: Q_Y = Y Tq (float)
      h->gemm_sample_side(O, ld_o, n, m, vcur, r);
      if (diag_end && p == q) {
        // sigma = |diag(R_Y)| sorted, V = the pass's basis in that order
        h->cholqr<double, double>(h->y64, n, r, h->yq1, h->Rz);
        hipLaunchKernelGGL(k_diag_sort, dim3(1), dim3(512), 0, stream, (const double*)h->Rz, rp, r, h->sig, h->perm,
                           cst);
        hipLaunchKernelGGL(k_permute_cols, dim3(cdiv(m * r, 256)), dim3(256), 0, stream, vcur, m, r,
                           (const int*)h->perm, h->z, cst);
        if (!g_ext) h->gradient(O, ld_o, n, m, e_l, h->g, stream, false);
        return finish(n, m, h->z, V, V, r, lambda, delta, sigma, gv, nullptr, n);
      }
      if (av) {
        hipLaunchKernelGGL(k_hist_rows, dim3(cdiv((int64_t)r * r, 256)), dim3(256), 0, stream, yh, r,
                           (const double*)av->sig_state, (const double*)(p == 1 ? h->G : h->Hn), rp, c_hist, cst);
        if (hist && p == 1 && q > 1)
          (void)hipMemcpyAsync(h->y1, h->y64, sizeof(double) * ny * r, hipMemcpyDeviceToDevice, stream);
      }
      h->cholqr<double, double>(h->y64, ny, r, h->yq1, nullptr);
      h->apply((const double*)h->y64, ny, r, r, h->Tq, rp, r, h->qy, r, true);
      // parameter side: Z = A^T Q_Y (+ V_in B), then its QR: Q_Z = Z Tq, R_Z
      h->gemm_param_side(O, ld_o, n, m, h->qy, r, h->z);
      if (hist) {
        hipLaunchKernelGGL(k_hist_b, dim3(cdiv((int64_t)rp * rp, 256)), dim3(256), 0, stream,
                           (const float*)(h->qy + n * r), r, (const double*)av->sig_state, c_hist, h->Bm, rp, cst);
        h->apply((const float*)V, m, r, r, h->Bm, rp, r, h->z, r, false, false, true, true);
      }
      const bool fast = kFastMid;
      if (fast && p < q) {
        // an intermediate pass: only the span of Z is carried on
        // (in the BF16 forms the next sample side reads V only through its
        // split, which can scale Z itself; Alg. 1's ending reads V too)
        h->fast_orth(h->z, m, r, h->bf16() && !diag_end);
        if (hist) {
          // V_in^T V_{p+1} = (Y_1^T Q_Y) T with the factor T the pass took
          h->cross(h->y1, h->qy, ny, r, h->Hc);
          hipLaunchKernelGGL(k_select_t, dim3(cdiv((int64_t)rp * rp, 256)), dim3(256), 0, stream,
                             (const int*)h->fmode, (const double*)h->gdiag, (const double*)h->R1i,
                             (const double*)h->Tq, rp, r, h->T);
          h->smallgemm(h->Hc, h->T, rp, h->Hn, false, false);
        }
        vcur = h->vw;
        continue;
      }
      if (fast)
        h->fast_factor(h->z, m, r);
      else
        h->cholqr<float, float>(h->z, m, r, h->q1, p == q ? h->Rz : nullptr);
      if (p < q) {
        if (av) {
          // V_in^T V_{p+1} = (Y_1^T Q_Y) Tq for the next pass's history rows
          if (hist) {
            h->cross(h->y1, h->qy, ny, r, h->Hc);
            h->smallgemm(h->Hc, h->Tq, rp, h->Hn, false, false);
          }
        }
        h->apply((const float*)h->z, m, r, r, h->Tq, rp, r, h->vw, r, true);
        vcur = h->vw;
      } else {
        // the gradient (one HBM-bound pass over O) runs on the second stream
        // while this stream works through the few-workgroup Jacobi launches
        if (!g_ext) {
          (void)hipEventRecord(h->ev_fork, stream);
          (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
          h->gradient(O, ld_o, n, m, e_l, h->g, h->side, true);
          (void)hipEventRecord(h->ev_join, h->side);
        }
        // Rayleigh-Ritz: C = Q_Y^T A Q_Z = R_Z^T;  C = G diag(sigma) P^T
        h->small_svd(h->Rz, r);
        // V = Q_Z P = Z (Tq P)
        h->smallgemm(h->Tq, h->Ps, rp, h->T, false, false);
        if (fast && r_out == r)
          h->final_apply(h->z, m, r, h->T, h->vw);
        else
          h->apply((const float*)h->z, m, r, r, h->T, rp, r_out, h->vw, r_out, false);
      }
    }
    if (!g_ext) (void)hipStreamWaitEvent(stream, h->ev_join, 0);
    return finish(n, m, h->vw, V, cont ? nullptr : V, r_out, lambda, delta, sigma, gv, av, ny);
  }

  // Randomized-sketch step (App. A, eq. randsvd): the rank-rs sketch of A
  // from the random sample-side block omega (n x rs, row stride rs),
  // truncated to rank r; no warm start.  In this orientation the paper's
  // Y = Ohat Omega is Z = A^T Omega, its B = Q^T Ohat is the transpose of
  // W = A Q, and the SVD of B comes from W = Q_W R_W and the SVD of R_W.
  // With q > 0, q passes of the subspace iteration at rank rs follow from Q
  // (the power scheme of the randomized range finder) and end in the usual
  // Rayleigh-Ritz step.
  wssr_status enqueue_sketch(int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                             const float* omega, int rs, int32_t q, float* V, double lambda, int32_t r,
                             double* delta, double* sigma, const double* g_ext) {
    wssr_ctx* h = this;
    const double* gv = g_ext ? g_ext : h->g;
    const int rps = (int)rup(rs, 64);
    const DevStatus* cst = h->st;
    hipStream_t stream = h->stream;
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, stream, h->st);
    // Q_Omega: omega less its column means (A^T Omega does not change, since
    // the columns of A sum to zero; the parameter-side product needs 1^T X = 0)
    const int64_t tot = n * rs;
    hipLaunchKernelGGL(k_ysum, dim3(cdiv(tot, 256)), dim3(256), 0, stream, omega, 1, tot, h->y64, cst);
    h->center_y(n, rs, 1.0);
    h->cholqr<double, double>(h->y64, n, rs, h->yq1, nullptr);
    h->apply((const double*)h->y64, n, rs, rs, h->Tq, rps, rs, h->qy, rs, true);
    // Z = A^T Q_Omega and its orthonormal basis Q (into vw)
    h->gemm_param_side(O, ld_o, n, m, h->qy, rs, h->z);
    h->cholqr<float, float>(h->z, m, rs, h->q1, nullptr);
    h->apply((const float*)h->z, m, rs, rs, h->Tq, rps, rs, h->vw, rs, true);
    if (q > 0) {
      Cont cont{h->vw, r};
      return enqueue(n, m, O, ld_o, e_l, V, lambda, rs, q, delta, sigma, g_ext, nullptr, &cont);
    }
    // W = A Q, W = Q_W R_W
    h->gemm_sample_side(O, ld_o, n, m, h->vw, rs);
    if (!g_ext) {
      (void)hipEventRecord(h->ev_fork, stream);
      (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
      h->gradient(O, ld_o, n, m, e_l, h->g, h->side, true);
      (void)hipEventRecord(h->ev_join, h->side);
    }
    h->cholqr<double, double>(h->y64, n, rs, h->yq1, h->Rz);
    // right singular vectors of R_W (the small SVD takes the transpose)
    hipLaunchKernelGGL(k_transpose_rp, dim3(cdiv((int64_t)rps * rps, 256)), dim3(256), 0, stream,
                       (const double*)h->Rz, rps, rs, h->Hc, cst);
    h->small_svd(h->Hc, rs);
    // V = Q P, its first r columns (into z)
    h->apply((const float*)h->vw, m, rs, rs, h->Ps, rps, r, h->z, r, false);
    if (!g_ext) (void)hipStreamWaitEvent(stream, h->ev_join, 0);
    return finish(n, m, h->z, V, nullptr, r, lambda, delta, sigma, gv, nullptr, n);
  }

  // MinSR with the SPRING momentum in sample space (Sec. 3.2, eqs. mT and
  // param:spring, damped): T = A A^T + lambda I on the FP64 MFMA, its blocked
  // Cholesky, b = eps/sqrt(N) - momentum A dtheta, x = T^{-1} b, delta = A^T x
  // (= O^T x / sqrt(N): x sums to zero), dtheta <- -eta delta + momentum dtheta.
  wssr_status enqueue_spring(int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l, double lambda,
                             double mom, double eta, double* dtheta, double* delta) {
    wssr_ctx* h = this;
    const DevStatus* cst = h->st;
    hipStream_t stream = h->stream;
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, stream, h->st);
    hipLaunchKernelGGL(k_center_energies, dim3(1), dim3(1024), 0, stream, e_l, n, h->eps, h->st);
    const bool b16 = bf16();
    const int pl = o_planes();
    // G = O O^T
    const int nt = (int)cdiv(n, 128), npairs = nt * (nt + 1) / 2;
    int nch = 1;
    int64_t kchunk = rup(m, 16);
    if (npairs < 512) {
      nch = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(cdiv(1024, npairs), tpart_tiles / npairs),
                                                        cdiv(m, 256)));
      kchunk = rup(cdiv(m, nch), 16);
      nch = (int)cdiv(m, kchunk);
    }
    double* part = nch > 1 ? h->tpart : nullptr;
    const dim3 g1((unsigned)npairs, (unsigned)nch);
    h->timed(2, [&] {
      if (!b16) {
        const bool vec = (ld_o % 4 == 0) && ((uintptr_t)O % 16 == 0);
        hipLaunchKernelGGL((k_syrk_partial<float, 1>), g1, dim3(256), 0, stream, static_cast<const float*>(O), ld_o,
                           (int64_t)0, n, m, nt, kchunk, part, h->Tn, vec, cst);
      } else {
        const bool vec = (ld_o % 4 == 0) && ((uintptr_t)O % 8 == 0);
        const auto* o16 = static_cast<const unsigned short*>(O);
        if (pl == 2)
          hipLaunchKernelGGL((k_syrk_partial<unsigned short, 2>), g1, dim3(256), 0, stream, o16, ld_o, n * ld_o, n,
                             m, nt, kchunk, part, h->Tn, vec, cst);
        else
          hipLaunchKernelGGL((k_syrk_partial<unsigned short, 1>), g1, dim3(256), 0, stream, o16, ld_o, n * ld_o, n,
                             m, nt, kchunk, part, h->Tn, vec, cst);
      }
      if (part)
        hipLaunchKernelGGL(k_syrk_reduce, dim3(npairs, 64), dim3(256), 0, stream, (const double*)part, nch, nt, n,
                           h->Tn, cst);
    });
    // T = (G - rho 1^T - 1 rho^T + tau) / n + lambda I
    hipLaunchKernelGGL(k_row_mean, dim3(cdiv(n, 4)), dim3(256), 0, stream, (const double*)h->Tn, n, h->rho, cst);
    hipLaunchKernelGGL(k_colreduce, dim3(1), dim3(256), 0, stream, (const double*)h->rho, (int)n, 1, 1.0 / (double)n,
                       h->sscal + 1, cst);
    hipLaunchKernelGGL(k_dcenter, dim3(cdiv(n * n, 256)), dim3(256), 0, stream, h->Tn, n, (const double*)h->rho,
                       (const double*)(h->sscal + 1), 1.0 / (double)n, lambda, cst);
    // blocked Cholesky (64-column panels)
    const bool vecd = (n % 2 == 0);
    h->timed(3, [&] {
      for (int64_t k0 = 0; k0 < n; k0 += 64) {
        const int nb = (int)std::min<int64_t>(64, n - k0);
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, stream, h->Tn, n, k0, nb, h->st);
        const int64_t rest = n - k0 - nb;
        if (rest > 0) {
          hipLaunchKernelGGL(k_trsm_panel, dim3(cdiv(rest, 64)), dim3(256), 0, stream, h->Tn, n, k0, nb, cst);
          const int ntr = (int)cdiv(rest, 128);
          hipLaunchKernelGGL(k_syrk_update, dim3(ntr * (ntr + 1) / 2), dim3(256), 0, stream, h->Tn, n, k0, nb, ntr,
                             vecd, cst);
        }
      }
    });
    // right-hand side
    const double isn = 1.0 / std::sqrt((double)n);
    if (mom != 0.0) {
      if (!b16) {
        hipLaunchKernelGGL((k_gemv_rows<float, 1>), dim3(cdiv(n, 4)), dim3(256), 0, stream,
                           static_cast<const float*>(O), ld_o, (int64_t)0, n, m, (const double*)dtheta, h->su, cst);
      } else if (pl == 2) {
        hipLaunchKernelGGL((k_gemv_rows<unsigned short, 2>), dim3(cdiv(n, 4)), dim3(256), 0, stream,
                           static_cast<const unsigned short*>(O), ld_o, n * ld_o, n, m, (const double*)dtheta, h->su,
                           cst);
      } else {
        hipLaunchKernelGGL((k_gemv_rows<unsigned short, 1>), dim3(cdiv(n, 4)), dim3(256), 0, stream,
                           static_cast<const unsigned short*>(O), ld_o, n * ld_o, n, m, (const double*)dtheta, h->su,
                           cst);
      }
      hipLaunchKernelGGL(k_colreduce, dim3(1), dim3(256), 0, stream, (const double*)h->su, (int)n, 1, 1.0 / (double)n,
                         h->sscal, cst);
    }
    hipLaunchKernelGGL(k_spring_rhs, dim3(cdiv(n, 256)), dim3(256), 0, stream, (const double*)h->eps,
                       mom != 0.0 ? (const double*)h->su : nullptr, (const double*)h->sscal, n, isn, mom * isn, h->sb,
                       cst);
    // x = (L L^T)^{-1} b, in place in sb
    for (int64_t k0 = 0; k0 < n; k0 += 64) {
      const int nb = (int)std::min<int64_t>(64, n - k0);
      hipLaunchKernelGGL(k_trsv_fwd_diag, dim3(1), dim3(64), 0, stream, (const double*)h->Tn, n, k0, nb, h->sb, cst);
      const int64_t rest = n - k0 - nb;
      if (rest > 0)
        hipLaunchKernelGGL(k_trsv_fwd_update, dim3(cdiv(rest, 4)), dim3(256), 0, stream, (const double*)h->Tn, n, k0,
                           nb, h->sb, cst);
    }
    for (int64_t k0 = (n - 1) / 64 * 64; k0 >= 0; k0 -= 64) {
      const int nb = (int)std::min<int64_t>(64, n - k0);
      hipLaunchKernelGGL(k_trsv_bwd_diag, dim3(1), dim3(64), 0, stream, (const double*)h->Tn, n, k0, nb, h->sb, cst);
      if (k0 > 0)
        hipLaunchKernelGGL(k_trsv_bwd_update, dim3(cdiv(k0, 256)), dim3(256), 0, stream, (const double*)h->Tn, n, k0,
                           nb, h->sb, cst);
    }
    // delta = O^T x / sqrt(n); the momentum update
    h->otv(O, ld_o, n, m, h->sb, isn, delta, stream, false);
    if (dtheta)
      hipLaunchKernelGGL(k_axpby, dim3(cdiv(m, 256)), dim3(256), 0, stream, (const double*)delta, m, -eta, mom,
                         dtheta, cst);
    if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
    return WSSR_OK;
  }

  // The end of a step, once vnew holds the new basis (unsigned, m x r), sig
  // the sorted singular values and, for the averaged step, Rz and Ps the last
  // pass's factors: output signs (against vref, or by the largest entry when
  // vref is NULL), the averaged state, and the Woodbury direction into V and
  // delta.
  wssr_status finish(int64_t n, int64_t m, const float* vnew, float* V, const float* vref, int32_t r, double lambda,
                     double* delta, double* sigma, const double* gv, const AvgArgs* av, int64_t ny) {
    wssr_ctx* h = this;
    const int rp = (int)rup(r, 64);
    const DevStatus* cst = h->st;
    hipStream_t stream = h->stream;
    if (h->coop_err != hipSuccess)
      return h->fail(WSSR_ERR_HIP, "cooperative launch of the SVD kernel failed: %s", hipGetErrorString(h->coop_err));
    // row chunks: as many as the partial buffers hold (enough blocks to cover
    // every compute unit several times), at least 64 rows each
    const int64_t rpc = std::max<int64_t>(64, cdiv(m, kVecChunkMax));
    const int nch = (int)cdiv(m, rpc);
    if (av) {
      // averaged gradient (eq. barg): gbar = (1-avg) g + avg V_in (sig o l),
      // read before V and the state are overwritten
      const double a = av->avg;
      double* gb = av->gbar_out ? av->gbar_out : h->gbar;
      hipLaunchKernelGGL(k_gbar_w, dim3(cdiv(r, 256)), dim3(256), 0, stream, (const double*)av->sig_state,
                         (const double*)av->l_state, r, -a / (1.0 - a), h->cw, cst);
      hipLaunchKernelGGL(k_delta, dim3(cdiv(m, 4)), dim3(256), 0, stream, (const float*)V, gv, (const double*)h->cw,
                         m, r, 1.0 - a, gb, cst);
      gv = gb;
      // t = Q_Y^T Lhat (eq. Lhat in the block's row order)
      const int64_t rpy = std::max<int64_t>(64, cdiv(ny, kVecChunkMax));
      const int nchy = (int)cdiv(ny, rpy);
      hipLaunchKernelGGL(k_lhat, dim3(cdiv(ny, 256)), dim3(256), 0, stream, (const double*)h->eps, n,
                         (const double*)av->l_state, r, std::sqrt((1.0 - a) / (double)n), std::sqrt(a), h->lhat,
                         cst);
      hipLaunchKernelGGL(k_vtg_partial, dim3(nchy, cdiv(r, 256)), dim3(256), 0, stream, (const float*)h->qy,
                         (const double*)h->lhat, ny, r, rpy, h->vpart, cst);
      hipLaunchKernelGGL(k_colreduce, dim3(r), dim3(256), 0, stream, (const double*)h->vpart, nchy, r, 1.0, h->tvec,
                         cst);
    }
    // output signs, then V <- signed vw
    {
      hipLaunchKernelGGL(k_sign_partial, dim3(nch, cdiv(r, 256)), dim3(256), 0, stream, vnew, vref, m, r, rpc,
                         h->dots, h->maxval, h->maxrow, cst);
      hipLaunchKernelGGL(k_sign_final, dim3(r), dim3(256), 0, stream, (const double*)h->dots, (const float*)h->maxval,
                         (const int64_t*)h->maxrow, nch, r, h->sgn, cst);
      if (av)
        // new stored vector (eq. Lbar) with the output signs; singular values
        // of the stacked matrix
        hipLaunchKernelGGL(k_state_l, dim3(1), dim3(512), 0, stream, (const double*)h->Rz, (const double*)h->Ps, rp, r,
                           (const double*)h->tvec, (const float*)h->sgn, h->sig, std::sqrt(1.0 - av->avg),
                           av->l_state, cst);
      const int64_t tot = m * r;
      hipLaunchKernelGGL(k_sign_apply, dim3((unsigned)std::min<int64_t>(8192, cdiv(tot, 1024))), dim3(256), 0, stream,
                         vnew, (const float*)h->sgn, tot, r, V, cst);
      // Woodbury
      hipLaunchKernelGGL(k_vtg_partial, dim3(nch, cdiv(r, 256)), dim3(256), 0, stream, (const float*)V,
                         gv, m, r, rpc, h->vpart, cst);
      hipLaunchKernelGGL(k_vtg_final, dim3(r), dim3(256), 0, stream, (const double*)h->vpart, nch, r,
                         (const double*)h->sig, lambda, (h->cfg.flags & WSSR_FLOOR_PRECOND) ? 1 : 0, h->r_reg, h->cw,
                         sigma, h->st);
      hipLaunchKernelGGL(k_delta, dim3(cdiv(m, 4)), dim3(256), 0, stream, (const float*)V, gv,
                         (const double*)h->cw, m, r, 1.0 / lambda, delta, cst);
    }
    if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
    return WSSR_OK;
  }

  // dynamic-LDS limits and occupancy (resident workgroups on the whole
  // device) of the BF16 product variants
  bool setup16() {
    bool ok = true;
    int cus = std::max(1, slots / 2);
    auto one = [&](const void* fn, int bn, int bk, int pa, int pb, int& out) {
      const int lds = (int)gemm16_lds(bn, bk, pa, pb);
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) ok = false;
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, (size_t)lds) != hipSuccess || per < 1) per = 1;
      out = per * cus;
    };
    auto oned = [&](const void* fn, int bn, int bk, int pa, int pb, int& out) {
      const int lds = (int)gemm16_dma_lds(bn, bk, pa, pb);
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) ok = false;
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, (size_t)lds) != hipSuccess || per < 1) per = 1;
      out = per * cus;
    };
#define WSSR_SETUP16(BN, BK, PA, PB)                                                                                 \
  one((const void*)k_gemm16_sample_side<BN, BK, PA, PB>, BN, BK, PA, PB, slots16s[v16(BN, PA, PB)]);                 \
  one((const void*)k_gemm16_param_side<BN, BK, PA, PB>, BN, BK, PA, PB, slots16p[v16(BN, PA, PB)]);                  \
  oned((const void*)k_gemm16_sample_side_dma<BN, BKD(BN, PA, PB), PA, PB>, BN, BKD(BN, PA, PB), PA, PB,              \
       slots16sd[v16(BN, PA, PB)]);                                                                                 \
  oned((const void*)k_gemm16_param_side_dma<BN, BKD(BN, PA, PB), PA, PB>, BN, BKD(BN, PA, PB), PA, PB,               \
       slots16pd[v16(BN, PA, PB)]);
    for (int pp = 0; pp < 3; ++pp) {
      const int pa = pp == 2 ? 2 : 1, pb = pp == 0 ? 1 : 2;
      const void* fs = pp == 0   ? (const void*)k_gemm16_sample_side_dma<64, 32, 1, 1>
                       : pp == 1 ? (const void*)k_gemm16_sample_side_dma<64, 32, 1, 2>
                                 : (const void*)k_gemm16_sample_side_dma<64, 32, 2, 2>;
      const void* fp = pp == 0   ? (const void*)k_gemm16_param_side_dma<64, 32, 1, 1>
                       : pp == 1 ? (const void*)k_gemm16_param_side_dma<64, 32, 1, 2>
                                 : (const void*)k_gemm16_param_side_dma<64, 32, 2, 2>;
      oned(fs, 64, 32, pa, pb, slots16sd[v16(64, pa, pb)]);
      oned(fp, 64, 32, pa, pb, slots16pd[v16(64, pa, pb)]);
    }
    WSSR_SETUP16(128, 32, 1, 1) WSSR_SETUP16(128, 32, 1, 2) WSSR_SETUP16(128, 32, 2, 2)
    WSSR_SETUP16(256, 32, 1, 1) WSSR_SETUP16(256, 32, 1, 2) WSSR_SETUP16(256, 32, 2, 2)
    WSSR_SETUP16(512, 16, 1, 1) WSSR_SETUP16(512, 16, 1, 2) WSSR_SETUP16(512, 16, 2, 2)
#undef WSSR_SETUP16
    for (int pb = 1; pb <= 2; ++pb) {
      const void* f = pb == 1 ? (const void*)k_gemm16_sample_side_rs<512, 1, WSSR_RS1_DB>
                              : (const void*)k_gemm16_sample_side_rs<512, 2, WSSR_RS2_DB>;
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 256, 0) != hipSuccess || per < 1) per = 1;
      slots16rs[pb - 1] = per * cus;
      const void* fp = pb == 1 ? (const void*)k_gemm16_param_side_rs<512, 1, WSSR_RS1_DB>
                               : (const void*)k_gemm16_param_side_rs<512, 2, WSSR_RS2_DB>;
      per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fp, 256, 0) != hipSuccess || per < 1) per = 1;
      slots16rsp[pb - 1] = per * cus;
    }
    (void)hipGetLastError();
    return ok;
  }

  // K-step of a direct-to-LDS BF16 product: 32, or 16 where three ring
  // slots of 32 would not fit in LDS (BN = 512 with a second plane)
  static constexpr int bk_dma(int bn, int pa, int pb) { return bn == 512 && (pa > 1 || pb > 1) ? 16 : 32; }

  // ---- storage precision of O
  bool bf16() const { return cfg.o_dtype != WSSR_F32; }
  int o_planes() const { return cfg.o_dtype == WSSR_BF16X2 ? 2 : 1; }
  int s_planes() const { return cfg.o_dtype == WSSR_BF16 ? 1 : 2; }
  static int bn_for(int r, bool b16) {
    return r <= 64 && !b16 ? 64 : r <= 128 ? 128 : (r <= 256 || !b16 ? 256 : 512);
  }
  // index of a BF16 product variant: (BN, PA, PB) with BN in {64, 128, 256, 512}
  // (BN = 64 exists only in the direct-to-LDS form)
  static int v16(int bn, int pa, int pb) {
    return (bn == 64 ? 0 : bn == 128 ? 1 : bn == 256 ? 2 : 3) * 3 + (pa == 2 ? 2 : pb - 1);
  }
  int slots16s[12] = {0}, slots16p[12] = {0};   // resident workgroups per variant (sample, parameter side)
  int slots16sd[12] = {0}, slots16pd[12] = {0}; // the same for the direct-to-LDS variants
  int slots32s = 0, slots32p = 0;             // the same for the FP32 32-column kernels
  int slots16rs[2] = {0, 0};                   // register-streamed 512-column sample side, PB = 1, 2
  int slots16rsp[2] = {0, 0};                  // the same for the parameter side

  // BF16 forms: round the K x r FP32 skinny operand S into s16 (hi, and lo
  // when pb = 2), K-blocked, r padded with zero columns to the product's
  // column tiles (bn); returns the plane stride in elements.  With split_alt
  // set (by fast_orth), the device's mode decides whether S or the column-scaled
  // split_alt is rounded; split_alt is cleared.
  int64_t split_skinny(const float* S, int64_t K, int r, int pb, int bn) {
    const int sw = (int)rup(r, bn);
    const int64_t kblocks = cdiv(K, 16), ps = kblocks * 16 * sw;
    const float* alt = split_alt;
    split_alt = nullptr;
    hipLaunchKernelGGL(k_split_skinny, dim3(cdiv(kblocks * sw, 256)), dim3(256), 0, stream, S, K, r, sw, s16, ps, pb,
                       (const DevStatus*)st, alt, (const double*)(alt ? gdiag : nullptr),
                       (const int*)(alt ? fmode : nullptr));
    return ps;
  }

  // Y = A V (FP64) from the split-K partials: fixed-order sum, then centre
  // the columns and scale (the implicit centring of O)
  void y_finish(int64_t n, int r, int s1) {
    const int64_t tot = n * r;
    hipLaunchKernelGGL(k_ysum, dim3(cdiv(tot, 256)), dim3(256), 0, stream, (const float*)ypart, s1, tot, y64,
                       (const DevStatus*)st);
    center_y(n, r, 1.0 / std::sqrt((double)n));
  }

  // y64 (n x r) <- (y64 - column means) * scale
  void center_y(int64_t n, int r, double scale) {
    const int64_t tot = n * r;
    const int rows = 128, nrb = (int)cdiv(n, rows);
    hipLaunchKernelGGL(k_colsum_partial, dim3(nrb, cdiv(r, 256)), dim3(256), 0, stream, (const double*)y64, n, r,
                       rows, colpart, (const DevStatus*)st);
    hipLaunchKernelGGL(k_colreduce, dim3(r), dim3(256), 0, stream, (const double*)colpart, nrb, r, 1.0 / (double)n,
                       ymean, (const DevStatus*)st);
    hipLaunchKernelGGL(k_ycenter, dim3(cdiv(tot, 256)), dim3(256), 0, stream, y64, (const double*)ymean, tot, r,
                       scale, (const DevStatus*)st);
  }

  void gemm_sample_side(const void* Ov, int64_t ld, int64_t n, int64_t m, const float* V, int r) {
    const bool b16 = bf16();
    const bool vec_v = (r % 4 == 0) && ((uintptr_t)V % 16 == 0);
    // FP32 direct-to-LDS form: 16-byte aligned rows of O and V, whole 16-byte
    // chunks of O's rows; with it, r <= 32 takes the 32-column tile
    const bool dma = !b16 && vec_v && (ld % 4 == 0) && ((uintptr_t)Ov % 16 == 0) && (m % 4 == 0);
    // BF16 direct-to-LDS form: 16-byte aligned rows of O, whole 16-byte chunks of its rows
    const bool dma16 = b16 && (ld % 8 == 0) && ((uintptr_t)Ov % 16 == 0) && (m % 8 == 0);
    // narrow column tiles where r allows: FP32 32 (direct form), BF16 64
    const int bn = dma && r <= 32 ? 32 : dma16 && r <= 64 ? 64 : bn_for(r, b16);
    const int pa = o_planes(), pb = s_planes();
    // 512-column tiles with one O plane: the skinny operand streamed into registers
    const bool rs = kUseRs && dma16 && bn == 512 && pa == 1;
    const int64_t tn = cdiv(n, 128), tj = cdiv(r, bn);
    const int bk = !b16 ? 16 : rs ? 16 : dma16 ? bk_dma(bn, pa, pb) : (bn == 512 ? 16 : 32);
    const int sl = std::max(
        1, (rs ? slots16rs[pb - 1]
               : b16 ? (dma16 ? slots16sd : slots16s)[v16(bn, pa, pb)]
                     : bn == 32 ? slots32s : slots) / slot_div);
    // about one round of resident workgroups; split K = M into s1 ranges (the
    // register-streamed kernel: several rounds, whose later workgroups fill
    // the compute units that finish first)
    int s1 = (int)std::min<int64_t>(kS1Max, std::max<int64_t>(1, cdiv((int64_t)sl * (rs ? kRsRounds : 1), tn * tj)));
    int64_t kchunk = rup(cdiv(m, s1), bk);
    s1 = (int)cdiv(m, kchunk);
    const bool xcd = ((int64_t)s1 * tj) % 8 == 0;
    const dim3 grid((unsigned)(tn * tj * s1));
    if (!b16) {
      const float* O = static_cast<const float*>(Ov);
      const bool vec_o = (ld % 4 == 0) && ((uintptr_t)O % 16 == 0);
      const unsigned dl = (unsigned)gemm_dma_lds(false, bn);
      timed(0, [&] {
        if (bn == 32)
          hipLaunchKernelGGL(k_gemm_sample_side_dma<32>, grid, dim3(256), dl, stream, O, ld, n, m, V, r, ypart,
                             kchunk, (const float*)zeros, (const DevStatus*)st, (int)tn, (int)tj, xcd);
        else if (dma && bn == 256)
          hipLaunchKernelGGL(k_gemm_sample_side_dma<256>, grid, dim3(256), dl, stream, O, ld, n, m, V, r, ypart,
                             kchunk, (const float*)zeros, (const DevStatus*)st, (int)tn, (int)tj, xcd);
        else if (dma && bn == 128)
          hipLaunchKernelGGL(k_gemm_sample_side_dma<128>, grid, dim3(256), dl, stream, O, ld, n, m, V, r, ypart,
                             kchunk, (const float*)zeros, (const DevStatus*)st, (int)tn, (int)tj, xcd);
        else if (dma)
          hipLaunchKernelGGL(k_gemm_sample_side_dma<64>, grid, dim3(256), dl, stream, O, ld, n, m, V, r, ypart,
                             kchunk, (const float*)zeros, (const DevStatus*)st, (int)tn, (int)tj, xcd);
        else if (bn == 256)
          hipLaunchKernelGGL(k_gemm_sample_side<256>, grid, dim3(256), 0, stream, O, ld, n, m, V, r, ypart, kchunk,
                             vec_o, vec_v, (const DevStatus*)st, (int)tn, (int)tj, xcd);
        else if (bn == 128)
          hipLaunchKernelGGL(k_gemm_sample_side<128>, grid, dim3(256), 0, stream, O, ld, n, m, V, r, ypart, kchunk,
                             vec_o, vec_v, (const DevStatus*)st, (int)tn, (int)tj, xcd);
        else
          hipLaunchKernelGGL(k_gemm_sample_side<64>, grid, dim3(256), 0, stream, O, ld, n, m, V, r, ypart, kchunk,
                             vec_o, vec_v, (const DevStatus*)st, (int)tn, (int)tj, xcd);
      });
    } else {
      const auto* O = static_cast<const unsigned short*>(Ov);
      const int64_t ps = n * ld;
      const bool vec_o = (ld % 8 == 0) && ((uintptr_t)O % 16 == 0);
      const unsigned lds = (unsigned)(dma16 ? gemm16_dma_lds(bn, bk, pa, pb) : gemm16_lds(bn, bk, pa, pb));
      const int64_t vs = split_skinny(V, m, r, pb, bn);
      timed(0, [&] {
#define WSSR_S16(BN, BK, PA, PB)                                                                                     \
  if (dma16)                                                                                                         \
    hipLaunchKernelGGL((k_gemm16_sample_side_dma<BN, BKD(BN, PA, PB), PA, PB>), grid, dim3(256), lds, stream, O, ld, \
                       ps, n, m,                                                                                    \
                       (const unsigned short*)s16, vs, r, ypart, kchunk, (const unsigned short*)zeros,              \
                       (const DevStatus*)st, (int)tn, (int)tj, xcd);                                                \
  else                                                                                                               \
    hipLaunchKernelGGL((k_gemm16_sample_side<BN, BK, PA, PB>), grid, dim3(256), lds, stream, O, ld, ps, n, m,        \
                       (const unsigned short*)s16, vs, r, ypart, kchunk, vec_o, (const DevStatus*)st, (int)tn,        \
                       (int)tj, xcd)
#define WSSR_S16D(PA, PB)                                                                                            \
  hipLaunchKernelGGL((k_gemm16_sample_side_dma<64, 32, PA, PB>), grid, dim3(256), lds, stream, O, ld, ps, n, m,        \
                     (const unsigned short*)s16, vs, r, ypart, kchunk, (const unsigned short*)zeros,                  \
                     (const DevStatus*)st, (int)tn, (int)tj, xcd)
        if (rs) {
          if (pb == 1)
            hipLaunchKernelGGL((k_gemm16_sample_side_rs<512, 1, WSSR_RS1_DB>), grid, dim3(256), 0, stream, O, ld, n, m,
                               (const unsigned short*)s16, vs, r, ypart, kchunk, (const unsigned short*)zeros,
                               (const DevStatus*)st, (int)tn, (int)tj, xcd);
          else
            hipLaunchKernelGGL((k_gemm16_sample_side_rs<512, 2, WSSR_RS2_DB>), grid, dim3(256), 0, stream, O, ld, n, m,
                               (const unsigned short*)s16, vs, r, ypart, kchunk, (const unsigned short*)zeros,
                               (const DevStatus*)st, (int)tn, (int)tj, xcd);
        } else switch (v16(bn, pa, pb)) {
          case 0: WSSR_S16D(1, 1); break;
          case 1: WSSR_S16D(1, 2); break;
          case 2: WSSR_S16D(2, 2); break;
          case 3: WSSR_S16(128, 32, 1, 1); break;
          case 4: WSSR_S16(128, 32, 1, 2); break;
          case 5: WSSR_S16(128, 32, 2, 2); break;
          case 6: WSSR_S16(256, 32, 1, 1); break;
          case 7: WSSR_S16(256, 32, 1, 2); break;
          case 8: WSSR_S16(256, 32, 2, 2); break;
          case 9: WSSR_S16(512, 16, 1, 1); break;
          case 10: WSSR_S16(512, 16, 1, 2); break;
          default: WSSR_S16(512, 16, 2, 2); break;
        }
#undef WSSR_S16D
#undef WSSR_S16
      });
    }
    y_finish(n, r, s1);
  }

  void gemm_param_side(const void* Ov, int64_t ld, int64_t n, int64_t m, const float* Q, int r, float* Z) {
    const bool b16 = bf16();
    const int pa = o_planes(), pb = s_planes();
    const bool vec_q = (r % 4 == 0) && ((uintptr_t)Q % 16 == 0);
    // FP32 direct-to-LDS form: 16-byte aligned rows of O and Q; with it,
    // r <= 32 takes the 32-column tile
    const bool dma = !b16 && vec_q && (ld % 4 == 0) && ((uintptr_t)Ov % 16 == 0);
    // BF16 direct-to-LDS form: 16-byte aligned rows of O
    const bool dma16 = b16 && (ld % 8 == 0) && ((uintptr_t)Ov % 16 == 0);
    // narrow column tiles where r allows (FP32 32: the narrow kernel; BF16
    // 64); BF16 with one plane of each operand and r > 256: two 256-column
    // tiles (two workgroups per compute unit) in place of one 512-column tile
    // (one)
    // one O plane and r > 256: one 512-column tile with the skinny operand
    // streamed into registers
    const bool rs = kUseRs && dma16 && pa == 1 && r > 256;
    const int bn = dma && r <= 32                           ? 32
                   : dma16 && r <= 64                       ? 64
                   : rs                                     ? 512
                   : dma16 && pa == 1 && pb == 1 && r > 256 ? 256
                                                            : bn_for(r, b16);
    const float scale = (float)(1.0 / std::sqrt((double)n));
    const int bk = !b16 ? 16 : rs ? 16 : dma16 ? bk_dma(bn, pa, pb) : (bn == 512 ? 16 : 32);
    const int sl = std::max(
        1, (rs ? slots16rsp[pb - 1]
               : b16 ? (dma16 ? slots16pd : slots16p)[v16(bn, pa, pb)]
                     : bn == 32 ? slots32p : slots) / slot_div);
    const int64_t tj = cdiv(r, bn), tiles = cdiv(m, 128) * tj, nk = cdiv(n, bk);
    // whole tiles for every full round of resident workgroups; the leftover
    // tiles' K-steps shared evenly by one more round (stream-K) unless the
    // leftover round is nearly full anyway
    int full = (int)tiles, skw = 0;
    int64_t rem = 0, units = 0;
    if (skpart && tiles > sl && (int64_t)sl * 2 * 128 * bn <= skpart_elems) {
      rem = tiles % sl;
      if (rem != 0 && rem * 5 < (int64_t)sl * 4) {
        full = (int)(tiles - rem);
        skw = sl;
        units = rem * nk;
      }
    }
    const dim3 grid(full + skw);
    const int64_t qs = b16 ? split_skinny(Q, n, r, pb, bn) : 0;
    timed(1, [&] {
      if (!b16) {
        const float* O = static_cast<const float*>(Ov);
        const bool vec_o = (ld % 4 == 0) && ((uintptr_t)O % 16 == 0);
        const unsigned dl = (unsigned)gemm_dma_lds(true, bn);
        if (bn == 32)
          hipLaunchKernelGGL(k_gemm_param_side_narrow, grid, dim3(256), 0, stream, O, ld, n, m, Q, r, scale, Z,
                             (const float*)zeros, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        else if (dma && bn == 256)
          hipLaunchKernelGGL(k_gemm_param_side_dma<256>, grid, dim3(256), dl, stream, O, ld, n, m, Q, r, scale, Z,
                             (const float*)zeros, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        else if (dma && bn == 128)
          hipLaunchKernelGGL(k_gemm_param_side_dma<128>, grid, dim3(256), dl, stream, O, ld, n, m, Q, r, scale, Z,
                             (const float*)zeros, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        else if (dma)
          hipLaunchKernelGGL(k_gemm_param_side_dma<64>, grid, dim3(256), dl, stream, O, ld, n, m, Q, r, scale, Z,
                             (const float*)zeros, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        else if (bn == 256)
          hipLaunchKernelGGL(k_gemm_param_side<256>, grid, dim3(256), 0, stream, O, ld, n, m, Q, r, scale, Z, vec_o,
                             vec_q, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        else if (bn == 128)
          hipLaunchKernelGGL(k_gemm_param_side<128>, grid, dim3(256), 0, stream, O, ld, n, m, Q, r, scale, Z, vec_o,
                             vec_q, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        else
          hipLaunchKernelGGL(k_gemm_param_side<64>, grid, dim3(256), 0, stream, O, ld, n, m, Q, r, scale, Z, vec_o,
                             vec_q, (const DevStatus*)st, (int)tj, full, units, skw, skpart);
      } else {
        const auto* O = static_cast<const unsigned short*>(Ov);
        const int64_t ps = n * ld;
        const bool vec_o = (ld % 8 == 0) && ((uintptr_t)O % 16 == 0);
        const unsigned lds = (unsigned)(dma16 ? gemm16_dma_lds(bn, bk, pa, pb) : gemm16_lds(bn, bk, pa, pb));
#define WSSR_P16(BN, BK, PA, PB)                                                                                     \
  if (dma16)                                                                                                         \
    hipLaunchKernelGGL((k_gemm16_param_side_dma<BN, BKD(BN, PA, PB), PA, PB>), grid, dim3(256), lds, stream, O, ld,  \
                       ps, n, m,                                                                                    \
                       (const unsigned short*)s16, qs, r, scale, Z, (const unsigned short*)zeros,                   \
                       (const DevStatus*)st, (int)tj, full, units, skw, skpart);                                    \
  else                                                                                                               \
    hipLaunchKernelGGL((k_gemm16_param_side<BN, BK, PA, PB>), grid, dim3(256), lds, stream, O, ld, ps, n, m,         \
                       (const unsigned short*)s16, qs, r, scale, Z, vec_o, (const DevStatus*)st, (int)tj, full,       \
                       units, skw, skpart)
#define WSSR_P16D(PA, PB)                                                                                            \
  hipLaunchKernelGGL((k_gemm16_param_side_dma<64, 32, PA, PB>), grid, dim3(256), lds, stream, O, ld, ps, n, m,         \
                     (const unsigned short*)s16, qs, r, scale, Z, (const unsigned short*)zeros, (const DevStatus*)st, \
                     (int)tj, full, units, skw, skpart)
        if (rs) {
          if (pb == 1)
            hipLaunchKernelGGL((k_gemm16_param_side_rs<512, 1, WSSR_RS1_DB>), grid, dim3(256), 0, stream, O, ld, n, m,
                               (const unsigned short*)s16, qs, r, scale, Z, (const unsigned short*)zeros,
                               (const DevStatus*)st, (int)tj, full, units, skw, skpart);
          else
            hipLaunchKernelGGL((k_gemm16_param_side_rs<512, 2, WSSR_RS2_DB>), grid, dim3(256), 0, stream, O, ld, n, m,
                               (const unsigned short*)s16, qs, r, scale, Z, (const unsigned short*)zeros,
                               (const DevStatus*)st, (int)tj, full, units, skw, skpart);
        } else switch (v16(bn, pa, pb)) {
          case 0: WSSR_P16D(1, 1); break;
          case 1: WSSR_P16D(1, 2); break;
          case 2: WSSR_P16D(2, 2); break;
          case 3: WSSR_P16(128, 32, 1, 1); break;
          case 4: WSSR_P16(128, 32, 1, 2); break;
          case 5: WSSR_P16(128, 32, 2, 2); break;
          case 6: WSSR_P16(256, 32, 1, 1); break;
          case 7: WSSR_P16(256, 32, 1, 2); break;
          case 8: WSSR_P16(256, 32, 2, 2); break;
          case 9: WSSR_P16(512, 16, 1, 1); break;
          case 10: WSSR_P16(512, 16, 1, 2); break;
          default: WSSR_P16(512, 16, 2, 2); break;
        }
#undef WSSR_P16D
#undef WSSR_P16
      }
      if (skw) {
        const dim3 fg(rem, 128 * bn / 1024);
        if (bn == 512)
          hipLaunchKernelGGL(k_streamk_fixup<512>, fg, dim3(256), 0, stream, (const float*)skpart, Z, m, r, scale,
                             (int)tj, full, nk, units, skw, (const DevStatus*)st);
        else if (bn == 256)
          hipLaunchKernelGGL(k_streamk_fixup<256>, fg, dim3(256), 0, stream, (const float*)skpart, Z, m, r, scale,
                             (int)tj, full, nk, units, skw, (const DevStatus*)st);
        else if (bn == 128)
          hipLaunchKernelGGL(k_streamk_fixup<128>, fg, dim3(256), 0, stream, (const float*)skpart, Z, m, r, scale,
                             (int)tj, full, nk, units, skw, (const DevStatus*)st);
        else if (bn == 32)
          hipLaunchKernelGGL(k_streamk_fixup<32>, fg, dim3(256), 0, stream, (const float*)skpart, Z, m, r, scale,
                             (int)tj, full, nk, units, skw, (const DevStatus*)st);
        else
          hipLaunchKernelGGL(k_streamk_fixup<64>, fg, dim3(256), 0, stream, (const float*)skpart, Z, m, r, scale,
                             (int)tj, full, nk, units, skw, (const DevStatus*)st);
      }
    });
  }

  // lean: at most about one workgroup per compute unit, for running beside
  // other work without taking the compute units it needs
  void gradient(const void* Ov, int64_t ld, int64_t n, int64_t m, const double* e_l, double* gout,
                hipStream_t on = nullptr, bool lean = false) {
    hipStream_t stream = on ? on : this->stream;
    hipLaunchKernelGGL(k_center_energies, dim3(1), dim3(1024), 0, stream, e_l, n, eps, st);
    otv(Ov, ld, n, m, eps, 1.0 / (double)n, gout, stream, lean);
  }

  // out = scale * O^T x (x: n doubles), one HBM-bound pass over O
  void otv(const void* Ov, int64_t ld, int64_t n, int64_t m, const double* x, double scale, double* gout,
           hipStream_t stream, bool lean) {
    // BF16 rows that are whole 16-byte chunks: 8 columns per thread
    const bool vec8 = bf16() && (ld % 8 == 0) && ((uintptr_t)Ov % 16 == 0);
    const int64_t cb = cdiv(m, vec8 ? 2048 : 1024);
    const int64_t want = lean ? std::max<int64_t>(1, slots / 2 / cb) : cdiv(2048, cb);
    const int gs = (int)std::min<int64_t>(kGSplitMax, std::max<int64_t>(1, std::min<int64_t>(want, n)));
    const int64_t rows = cdiv(n, gs);
    if (!bf16()) {
      const float* O = static_cast<const float*>(Ov);
      const bool vec = (ld % 4 == 0) && ((uintptr_t)O % 16 == 0);
      hipLaunchKernelGGL(k_gradient_partial, dim3(cb, gs), dim3(256), 0, stream, O, ld, n, m, x,
                         rows, gpart, vec, (const DevStatus*)st);
    } else {
      const auto* O = static_cast<const unsigned short*>(Ov);
      const bool vec = vec8 || ((ld % 4 == 0) && ((uintptr_t)O % 8 == 0));
      const dim3 grid((unsigned)cb, (unsigned)gs);
      if (o_planes() == 2)
        hipLaunchKernelGGL((vec8 ? k_gradient16_partial<2, 8> : k_gradient16_partial<2, 4>), grid, dim3(256), 0,
                           stream, O, ld, n * ld, n, m, x, rows, gpart, vec, (const DevStatus*)st);
      else
        hipLaunchKernelGGL((vec8 ? k_gradient16_partial<1, 8> : k_gradient16_partial<1, 4>), grid, dim3(256), 0,
                           stream, O, ld, n * ld, n, m, x, rows, gpart, vec, (const DevStatus*)st);
    }
    hipLaunchKernelGGL(k_gradient_reduce, dim3(cdiv(m, 256)), dim3(256), 0, stream, (const double*)gpart, gs, m,
                       scale, gout, (const DevStatus*)st);
  }

  // Ingest of a block of rows of FP32 O (see wssr_ingest).  The first block
  // (row0 == 0) centres the energies and starts the sums.
  int64_t ingest_next = -1, ingest_n = 0, ingest_m = 0;
  void ingest(int64_t n, int64_t m, int64_t row0, int64_t rows, const float* O32, int64_t ld32,
              const double* e_l, const double* mu, void* out, int64_t ld_o, double* gout, double* mout) {
    const bool first = row0 == 0;
    if (first) {
      hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, stream, st);
      hipLaunchKernelGGL(k_center_energies, dim3(1), dim3(1024), 0, stream, e_l, n, eps, st);
    }
    const int64_t cb = cdiv(m, 2048);
    const int gs = (int)std::min<int64_t>(kGSplitMax / 2, std::max<int64_t>(1, std::min(cdiv(2048, cb), rows)));
    const int64_t rps = cdiv(rows, gs);
    const int nsplit = (int)cdiv(rows, rps);
    double* gp = gpart;
    double* cp = gpart + (int64_t)(kGSplitMax / 2) * m;
    const bool vec = (ld32 % 4 == 0) && ((uintptr_t)O32 % 16 == 0);
    const dim3 grid((unsigned)cb, (unsigned)nsplit);
    const double* e = eps + row0;
    if (!bf16()) {
      float* o = out ? static_cast<float*>(out) + row0 * ld_o : nullptr;
      const bool vo = (ld_o % 4 == 0) && ((uintptr_t)out % 16 == 0);
      hipLaunchKernelGGL((k_ingest_partial<1, true>), grid, dim3(256), 0, stream, O32, ld32, rows, m, e, mu,
                         (void*)o, ld_o, n * ld_o, rps, gp, cp, vec, vo, st);
    } else {
      unsigned short* o = out ? static_cast<unsigned short*>(out) + row0 * ld_o : nullptr;
      const bool vo = (ld_o % 8 == 0) && ((uintptr_t)out % 16 == 0);
      if (o_planes() == 2)
        hipLaunchKernelGGL((k_ingest_partial<2, false>), grid, dim3(256), 0, stream, O32, ld32, rows, m, e, mu,
                           (void*)o, ld_o, n * ld_o, rps, gp, cp, vec, vo, st);
      else
        hipLaunchKernelGGL((k_ingest_partial<1, false>), grid, dim3(256), 0, stream, O32, ld32, rows, m, e, mu,
                           (void*)o, ld_o, n * ld_o, rps, gp, cp, vec, vo, st);
    }
    hipLaunchKernelGGL(k_ingest_reduce, dim3(cdiv(m, 256)), dim3(256), 0, stream, (const double*)gp,
                       (const double*)cp, nsplit, m, 1.0 / (double)n, first, gout, mout);
  }

  // row chunks of the Gram partials: about 512 workgroups, at least 256 rows
  // each, within the partial buffer
  static int gram_chunks(int64_t rows, int npairs) {
    const int64_t per = (int64_t)npairs * kF64Tile * kF64Tile * (int64_t)sizeof(double);
    const int64_t cap = std::max<int64_t>(1, (int64_t)kGramPartBytes / per);
    return (int)std::max<int64_t>(1, std::min(std::min(cdiv(512, npairs), cdiv(rows, 256)), cap));
  }

  // kind (float X only): kGram32 the FP32-MFMA Gram, kGram16 the Gram of the
  // two-plane BF16 split on the BF16 MFMA; otherwise the FP64 one
  template <typename T>
  void gram(const T* X, int64_t rows, int r, bool gated, int kind = kGram64) {
    const int rp = (int)rup(r, 64), nt = (int)cdiv(r, kF64Tile), npairs = nt * (nt + 1) / 2;
    int nch = gram_chunks(rows, npairs);
    const int64_t rpc = std::max<int64_t>(16, rup(cdiv(rows, nch), 16));
    nch = (int)std::max<int64_t>(1, cdiv(rows, rpc));
    const bool vec = (r % 4 == 0) && ((uintptr_t)X % 16 == 0);
    const int64_t ldx = r;
    if constexpr (std::is_same<T, float>::value) {
      if (kind != kGram64) {
        // whole groups of 8 chunks, so that every XCD holds whole chunks
        int nc = gram_chunks(rows, npairs);
        if (nc >= 8) nc -= nc % 8;
        const int64_t rpc32 = std::max<int64_t>(16, rup(cdiv(rows, nc), 16));
        nch = (int)std::max<int64_t>(1, cdiv(rows, rpc32));
        if (kind == kGram16)
          hipLaunchKernelGGL(k_gram16_partial, dim3(npairs * nch), dim3(512), 0, stream, X, rows, r, ldx, nt, nch,
                             rpc32, gram_part, (const DevStatus*)st, gated);
        else
          hipLaunchKernelGGL(k_gram32_partial, dim3(npairs * nch), dim3(256), 0, stream, X, rows, r, ldx, nt, nch,
                             rpc32, gram_part, vec, (const DevStatus*)st, gated);
      } else
        hipLaunchKernelGGL((k_gram_partial<float>), dim3(npairs, nch), dim3(256), 0, stream, X, rows, r, ldx,
                           nt, rpc, gram_part, vec, (const DevStatus*)st, gated);
    } else {
      hipLaunchKernelGGL((k_gram_partial<T>), dim3(npairs, nch), dim3(256), 0, stream, X, rows, r, ldx, nt,
                         rpc, gram_part, vec, (const DevStatus*)st, gated);
    }
    hipLaunchKernelGGL(k_gram_reduce, dim3(npairs, kF64Tile * kF64Tile / 256), dim3(256), 0, stream,
                       (const double*)gram_part, nch, nt, r, rp, G, (const DevStatus*)st, gated);
  }

  // Cholesky of G into R and R^{-1}; a first round (gated = false) also sets
  // the device flag that decides the second round.
  void chol(int rp, int r, double* R, double* Ri, bool gated) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(1024), kCholLds, stream, G, rp, r, R, Rt, gdiag, invdiag, repcol, st,
                       gated);
    const dim3 g(cdiv(rp, 4));
    switch (rp / 64) {
      case 1: hipLaunchKernelGGL(k_trinv<1>, g, dim3(256), 0, stream, (const double*)Rt, rp, (const double*)invdiag, Ri, (const DevStatus*)st, gated); break;
      case 2: hipLaunchKernelGGL(k_trinv<2>, g, dim3(256), 0, stream, (const double*)Rt, rp, (const double*)invdiag, Ri, (const DevStatus*)st, gated); break;
      case 3:
      case 4: hipLaunchKernelGGL(k_trinv<4>, g, dim3(256), 0, stream, (const double*)Rt, rp, (const double*)invdiag, Ri, (const DevStatus*)st, gated); break;
      default: hipLaunchKernelGGL(k_trinv<8>, g, dim3(256), 0, stream, (const double*)Rt, rp, (const double*)invdiag, Ri, (const DevStatus*)st, gated); break;
    }
    if (!gated)
      hipLaunchKernelGGL(k_kappa, dim3(1), dim3(1024), 0, stream, (const double*)gdiag, (const double*)R,
                         (const double*)Ri, rp, r, kKappaRound2, st);
  }

  // C = A B (rp x rp); gated: C = A (copy_b = false) or B when no second round ran
  void smallgemm(const double* A, const double* B, int rp, double* C, bool gated, bool copy_b) {
    const int tiles = (rp / 16) * (rp / 16);
    hipLaunchKernelGGL(k_smallgemm, dim3(cdiv(tiles, 4)), dim3(256), 0, stream, A, B, rp, C, (const DevStatus*)st,
                       gated, copy_b);
  }

  template <typename Tin, typename Tout>
  void apply(const Tin* X, int64_t rows, int ldx, int kdim, const double* Tm, int rp, int ncol, Tout* out, int ldo,
             bool upper, bool gated = false, bool acc = false, bool f32 = false) {
    const bool vec = (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
    const dim3 grid(cdiv(rows, kF64Tile), cdiv(ncol, kF64Tile));
    if constexpr (std::is_same<Tin, float>::value && std::is_same<Tout, float>::value) {
      if (f32) {
        const int64_t cnt = (int64_t)rp * rp;
        hipLaunchKernelGGL(k_round_f32, dim3(cdiv(cnt, 256)), dim3(256), 0, stream, Tm, cnt, tf32,
                           (const DevStatus*)st, gated);
        hipLaunchKernelGGL(k_apply32, dim3((unsigned)(grid.x * grid.y)), dim3(256), 0, stream, X, rows, ldx, kdim,
                           (const float*)tf32, rp, ncol, out, ldo, upper, vec, acc, (const DevStatus*)st, gated);
        return;
      }
    }
    hipLaunchKernelGGL((k_apply<Tin, Tout>), grid, dim3(256), 0, stream, X, rows, ldx, kdim, Tm, rp, ncol, out,
                       ldo, upper, vec, acc, (const DevStatus*)st, gated);
  }

  // Probe for the orthonormalisation of the parameter-side block Z: an
  // FP32-MFMA Gram and its FP64 Cholesky (into G, R1, R1i, gdiag), then the
  // device's choice of mode (k_fast_decide) and clean shadow status words for
  // the alternatives.
  void probe_factor(float* Z, int64_t m, int r, double piv_fast, int kind) {
    const int rp = (int)rup(r, 64);
    DevStatus* main = st;
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, stream, shadow);
    st = shadow;
    gram((const float*)Z, m, r, false, kind);
    chol(rp, r, R1, R1i, false);
    st = main;
    hipLaunchKernelGGL(k_fast_decide, dim3(1), dim3(64), 0, stream, (const DevStatus*)shadow,
                       std::sqrt((double)r * (r + 8.0)), piv_fast, main, shadow + 1, shadow + 2, shadow + 3, fmode);
  }

  // An intermediate pass's parameter-side basis: any V = Z T with the span of
  // Z serves the next pass, so the exact FP64 CholeskyQR is not needed where
  // Z is well conditioned.  Mode 0 (columns already orthogonal): V = Z
  // diag(G)^{-1/2}; mode 1 (relative pivots >= 0.03): V = Z R^{-1} by the
  // FP32-MFMA apply; mode 2: the FP64 CholeskyQR2 and apply.  The
  // alternatives not taken skip through their status words; the FP64 path's
  // errors and diagnostics are merged into the step's status.  Leaves V in vw;
  // with defer_scale, mode 0 leaves vw as it is and the next split_skinny
  // (the BF16 sample side, the only reader of this V) scales Z itself.
  void fast_orth(float* Z, int64_t m, int r, bool defer_scale) {
    const int rp = (int)rup(r, 64);
    DevStatus* main = st;
    probe_factor(Z, m, r, 0.03, kGram16);
    if (defer_scale)
      split_alt = Z;
    else
      hipLaunchKernelGGL(k_colscale, dim3((unsigned)std::min<int64_t>(8192, cdiv(m * r, 1024))), dim3(256), 0,
                         stream, (const float*)Z, (const double*)gdiag, m, r, vw, (const int*)fmode);
    st = shadow + 1;
    apply((const float*)Z, m, r, r, R1i, rp, r, vw, r, true, false, false, true);
    st = shadow + 2;
    cholqr<float, float>(Z, m, r, q1, nullptr);
    apply((const float*)Z, m, r, r, Tq, rp, r, vw, r, true);
    st = main;
    hipLaunchKernelGGL(k_status_merge, dim3(1), dim3(64), 0, stream, (const DevStatus*)(shadow + 2), main);
  }

  // The last pass's factorisation Z = Q_Z R_Z (Q_Z = Z Tq): the probe's R
  // where every relative pivot is >= 0.3 (its FP32-accurate Gram then gives R
  // and R^{-1} to about 1e-6 relative), else the FP64 CholeskyQR2.  Leaves R_Z
  // in Rz and Tq; the final apply of the same step chooses its precision the
  // same way (final_apply).
  void fast_factor(float* Z, int64_t m, int r) {
    const int rp = (int)rup(r, 64);
    DevStatus* main = st;
    probe_factor(Z, m, r, 0.3, kGram32);
    const int64_t cnt = (int64_t)rp * rp;
    hipLaunchKernelGGL(k_copy_st, dim3(cdiv(cnt, 256)), dim3(256), 0, stream, (const double*)R1, cnt, Rz,
                       (const DevStatus*)(shadow + 3));
    hipLaunchKernelGGL(k_copy_st, dim3(cdiv(cnt, 256)), dim3(256), 0, stream, (const double*)R1i, cnt, Tq,
                       (const DevStatus*)(shadow + 3));
    st = shadow + 2;
    cholqr<float, float>(Z, m, r, q1, Rz);
    st = main;
    hipLaunchKernelGGL(k_status_merge, dim3(1), dim3(64), 0, stream, (const DevStatus*)(shadow + 2), main);
  }

  // V = Z T after fast_factor: the FP32-MFMA apply where the probe's factor
  // was taken, the FP64 apply otherwise.
  void final_apply(const float* Z, int64_t m, int r, const double* T, float* out) {
    const int rp = (int)rup(r, 64);
    DevStatus* main = st;
    st = shadow + 3;
    apply(Z, m, r, r, T, rp, r, out, r, false, false, false, true);
    st = shadow + 2;
    apply(Z, m, r, r, T, rp, r, out, r, false);
    st = main;
  }

  // H = X^T W (rp x rp, zero outside r x r) for two rows x r blocks
  void cross(const double* X, const float* W, int64_t rows, int r, double* H) {
    const int rp = (int)rup(r, 64), nt = (int)cdiv(r, kF64Tile), tiles = nt * nt;
    const int64_t per = (int64_t)tiles * kF64Tile * kF64Tile;
    const int64_t cap = std::max<int64_t>(1, gram_part_elems / per);
    int nch = (int)std::max<int64_t>(1, std::min(std::min<int64_t>(cdiv(512, tiles), cdiv(rows, 256)), cap));
    const int64_t rpc = std::max<int64_t>(16, rup(cdiv(rows, nch), 16));
    nch = (int)std::max<int64_t>(1, cdiv(rows, rpc));
    const bool vec = (r % 4 == 0) && ((uintptr_t)X % 16 == 0) && ((uintptr_t)W % 16 == 0);
    hipLaunchKernelGGL((k_cross_partial<double, float>), dim3(tiles, nch), dim3(256), 0, stream, X, W, rows, r, nt,
                       rpc, gram_part, vec, (const DevStatus*)st);
    hipLaunchKernelGGL(k_cross_reduce, dim3(tiles, kF64Tile * kF64Tile / 256), dim3(256), 0, stream,
                       (const double*)gram_part, nch, nt, r, rp, H, (const DevStatus*)st);
  }

  // CholeskyQR of X (rows x r) with a second round when the first round's
  // condition bound asks for it (decided on the device).  Leaves the combined
  // orthonormaliser Tq = R1^{-1} R2^{-1} (upper, rp x rp) so that Q = X Tq, and,
  // if Rout is given, the triangular factor Rout = R2 R1 (X = Q Rout).  The
  // second round's X R1^{-1} goes to `mid`.
  template <typename Tin, typename Tmid>
  void cholqr(const Tin* X, int64_t rows, int r, Tmid* mid, double* Rout) {
    const int rp = (int)rup(r, 64);
    gram(X, rows, r, false);
    chol(rp, r, R1, R1i, false);
    // a rank-deficient X: its dependent columns get directions of their own
    // (X is modified in place; X Tq and the factor R then refer to the
    // modified X)
    hipLaunchKernelGGL((k_complete<Tin>), dim3((unsigned)std::min<int64_t>(64, cdiv(rows, 256)), r), dim3(256), 0,
                       stream, const_cast<Tin*>(X), rows, r, (const double*)R1, rp, (const int*)repcol,
                       (const DevStatus*)st);
    apply(X, rows, r, r, R1i, rp, r, mid, r, true, true);
    gram((const Tmid*)mid, rows, r, true);
    chol(rp, r, R2, R2i, true);
    smallgemm(R1i, R2i, rp, Tq, true, false);
    if (Rout) smallgemm(R2, R1, rp, Rout, true, true);
  }

  // the SVD kernel instantiated for rp (row blocks of 16 per wave: rp / 64)
  static const void* jacobi_fn(int rp) {
    switch (rp / 64) {
      case 1: return (const void*)k_jacobi_coop<1>;
      case 2: return (const void*)k_jacobi_coop<2>;
      case 3: return (const void*)k_jacobi_coop<3>;
      case 4: return (const void*)k_jacobi_coop<4>;
      case 5: return (const void*)k_jacobi_coop<5>;
      case 6: return (const void*)k_jacobi_coop<6>;
      case 7: return (const void*)k_jacobi_coop<7>;
      default: return (const void*)k_jacobi_coop<8>;
    }
  }

  // SVD of the r x r matrix whose transpose is Ct (rp x rp row-major): sorted
  // singular values into sig[0..rp), right singular vectors into Ps (rp x rp).
  void small_svd(const double* Ct, int r) {
    int rp = (int)rup(r, 64);
    hipLaunchKernelGGL(k_jacobi_prep, dim3(rp / 4), dim3(256), 0, stream, Ct, rp, r, Bc, Pc, scal, jsync, st);
    // all sweeps in one cooperative launch: rp/32 workgroups, one per block
    // pair of 32 columns, meeting at grid barriers between rounds
    double tol = kJacobiTol;
    const double* scal_c = scal;
    double* cosb = cosbuf;
    unsigned* sy = jsync;
    DevStatus* stp = st;
    int sweeps = kJacobiSweeps, inner = kJacobiInner;
    void* args[] = {&Bc, &Pc, &rp, &tol, &scal_c, &cosb, &sy, &stp, &sweeps, &inner};
    const void* fn = jacobi_fn(rp);
    if (capturing || plain_svd) {
      // a graph node, or a batch lane running beside other lanes: a plain
      // launch (a cooperative launch may hold the whole device).  The grid is
      // at most 16 workgroups, which the device schedules as other work
      // drains, and its barrier waits are bounded.
      coop_err = hipLaunchKernel(fn, dim3(rp / 32), dim3(256), args, jacobi_lds(rp), stream);
    } else {
      coop_err = hipLaunchCooperativeKernel(fn, dim3(rp / 32), dim3(256), args, (unsigned)jacobi_lds(rp), stream);
    }
    if (coop_err != hipSuccess) {
      // nothing was rotated: fail the step on the device so that no later
      // kernel writes an output
      (void)hipGetLastError();
      hipLaunchKernelGGL(k_raise, dim3(1), dim3(1), 0, stream, st, (int)WSSR_ERR_HIP);
    }
    hipLaunchKernelGGL(k_jacobi_final, dim3(1), dim3(1024), 0, stream, (const double*)Bc, (const double*)Pc, rp, r, sig,
                       Ps, st);
  }

};

namespace {

bool device_ok(int* dev, std::string& why) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    why = "no HIP device visible";
    return false;
  }
  if (hipGetDevice(dev) != hipSuccess) {
    why = "hipGetDevice failed";
    return false;
  }
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, *dev) != hipSuccess) {
    why = "hipGetDeviceProperties failed";
    return false;
  }
  if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) {
    why = std::string("device is ") + p.gcnArchName + ", libwssr is built for gfx950";
    return false;
  }
  return true;
}

thread_local std::string g_create_error;

}  // namespace

extern "C" {

const char* wssr_version(void) { return "libwssr 0.1 gfx950"; }

}  // extern "C"

namespace {

// One context: workspace sized from the config, the second stream, events.
// stream == nullptr with own = true: the context creates its own stream (a
// batch lane).
wssr_status build_ctx(const wssr_config* cfg, int dev, hipStream_t stream, bool own, wssr_ctx** out,
                      std::string& why) {
  auto* h = new wssr_ctx();
  h->device = dev;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    h->slots = 2 * cus;
  h->cfg = *cfg;
  h->stream = stream;
  if (own) {
    h->own_stream = true;
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      h->stream = nullptr;
      delete h;
      why = "stream creation failed";
      return WSSR_ERR_HIP;
    }
  }
  const int64_t n = cfg->n_max, m = cfg->m_max;
  const int r = cfg->r_max;
  const int rp = (int)rup(r, 64), nt = (int)cdiv(r, kF64Tile), npairs = nt * (nt + 1) / 2;
  h->rp_max = rp;
  h->rows_max = std::max(n, m);
  const int64_t rows = h->rows_max;
  // Gram partials: the largest block is the parameter side (m rows) or the
  // averaged step's sample side (n + r rows)
  h->gram_part_elems =
      (int64_t)wssr_ctx::gram_chunks(std::max(n + r, m), npairs) * npairs * kF64Tile * kF64Tile;
  bool ok = h->alloc(h->st, 1) && h->alloc(h->eps, n) && h->alloc(h->g, m) &&
            h->alloc(h->gpart, (size_t)kGSplitMax * m) && h->alloc(h->ypart, (size_t)kS1Max * n * r) &&
            h->alloc(h->y64, (size_t)(n + r) * r) && h->alloc(h->yq1, (size_t)(n + r) * r) &&
            h->alloc(h->colpart, (size_t)cdiv(n, 128) * r) && h->alloc(h->qy, (size_t)(n + r) * r) &&
            h->alloc(h->z, (size_t)m * r) && h->alloc(h->q1, (size_t)rows * r) && h->alloc(h->vw, (size_t)m * r) &&
            h->alloc(h->gram_part, (size_t)h->gram_part_elems) &&
            h->alloc(h->y1, (size_t)(n + r) * r) && h->alloc(h->Hc, (size_t)rp * rp) &&
            h->alloc(h->Hn, (size_t)rp * rp) && h->alloc(h->Bm, (size_t)rp * rp) && h->alloc(h->gbar, m) &&
            h->alloc(h->lhat, (size_t)(n + r)) && h->alloc(h->tvec, rp) && h->alloc(h->perm, rp) &&
            h->alloc(h->shadow, 4) && h->alloc(h->fmode, 1) && h->alloc(h->tf32, (size_t)rp * rp) &&
            h->alloc(h->G, (size_t)rp * rp) &&
            h->alloc(h->R1, (size_t)rp * rp) && h->alloc(h->R1i, (size_t)rp * rp) && h->alloc(h->R2, (size_t)rp * rp) &&
            h->alloc(h->R2i, (size_t)rp * rp) && h->alloc(h->Rz, (size_t)rp * rp) && h->alloc(h->Bc, (size_t)rp * rp) &&
            h->alloc(h->Pc, (size_t)rp * rp) && h->alloc(h->Ps, (size_t)rp * rp) && h->alloc(h->T, (size_t)rp * rp) &&
            h->alloc(h->scal, (size_t)rp + 1) && h->alloc(h->sig, rp) && h->alloc(h->cosbuf, (size_t)rp * rp / 64) &&
            h->alloc(h->cw, rp) && h->alloc(h->vpart, (size_t)kVecChunkMax * r) &&
            h->alloc(h->dots, (size_t)kVecChunkMax * r) && h->alloc(h->maxval, (size_t)kVecChunkMax * r) &&
            h->alloc(h->maxrow, (size_t)kVecChunkMax * r) && h->alloc(h->sgn, rp) && h->alloc(h->ymean, rp) &&
            h->alloc(h->Tq, (size_t)rp * rp) && h->alloc(h->Rt, (size_t)rp * rp) && h->alloc(h->gdiag, rp) && h->alloc(h->invdiag, rp) && h->alloc(h->repcol, rp) &&
            h->alloc(h->jsync, 4) && h->alloc(h->bstat, kBatchMax);
  // stream-K partials (two 128 x 256 tiles per workgroup of one round), only
  // when a parameter-side product can have more tiles than one round holds
  // (capacity for 2 slots per CU at 128 x 256 or 1 slot per CU at 128 x 512)
  const int64_t ptiles = cdiv(m, 128);
  if (ok && cfg->o_dtype != WSSR_F32)
    ok = h->alloc(h->s16, (size_t)2 * cdiv(rows, 16) * 16 * rup(r, wssr_ctx::bn_for(r, true)));
  if (ok && ptiles > h->slots / 2) {
    h->skpart_elems = (int64_t)h->slots * 2 * 128 * 256;
    ok = h->alloc(h->skpart, (size_t)h->skpart_elems);
  }
  if (ok) {
    ok = h->alloc(h->zeros, 1024) && hipMemset(h->zeros, 0, 1024 * sizeof(float)) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    h->release();
    delete h;
    why = "workspace allocation failed";
    return WSSR_ERR_OOM;
  }
  bool attr_ok =
      hipFuncSetAttribute((const void*)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCholLds) == hipSuccess;
  for (int bn = 32; bn <= 256; bn *= 2) {
    const void* fs = bn == 256   ? (const void*)k_gemm_sample_side_dma<256>
                     : bn == 128 ? (const void*)k_gemm_sample_side_dma<128>
                     : bn == 64  ? (const void*)k_gemm_sample_side_dma<64>
                                 : (const void*)k_gemm_sample_side_dma<32>;
    attr_ok = attr_ok &&
              hipFuncSetAttribute(fs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_dma_lds(false, bn)) ==
                  hipSuccess;
    if (bn == 32) continue;   // the 32-column parameter side is the narrow kernel (static LDS)
    const void* fp = bn == 256   ? (const void*)k_gemm_param_side_dma<256>
                     : bn == 128 ? (const void*)k_gemm_param_side_dma<128>
                                 : (const void*)k_gemm_param_side_dma<64>;
    attr_ok = attr_ok &&
              hipFuncSetAttribute(fp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_dma_lds(true, bn)) ==
                  hipSuccess;
  }
  // the 32-column kernels hold little LDS: more of them are resident per
  // compute unit than of the wider tiles
  {
    const int cus = std::max(1, h->slots / 2);
    int ps = 0, pp = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&ps, (const void*)k_gemm_sample_side_dma<32>, 256,
                                                     gemm_dma_lds(false, 32)) != hipSuccess || ps < 1)
      ps = 2;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pp, (const void*)k_gemm_param_side_narrow, 256, 0) !=
            hipSuccess || pp < 1)
      pp = 2;
    h->slots32s = ps * cus;
    h->slots32p = pp * cus;
  }
  for (int k = 64; k <= rp; k += 64)
    attr_ok = attr_ok && hipFuncSetAttribute(wssr_ctx::jacobi_fn(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)jacobi_lds(k)) == hipSuccess;
  if (!attr_ok) {
    h->release();
    delete h;
    why = "hipFuncSetAttribute failed";
    return WSSR_ERR_HIP;
  }
  if (!h->setup16()) {
    h->release();
    delete h;
    why = "BF16 kernel set-up failed";
    return WSSR_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
    h->release();
    delete h;
    why = "stream or event creation failed";
    return WSSR_ERR_HIP;
  }
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  if (hipGetLastError() != hipSuccess) {
    h->release();
    delete h;
    why = "kernel launch failed";
    return WSSR_ERR_HIP;
  }
  *out = h;
  return WSSR_OK;
}

}  // namespace

extern "C" {

wssr_status wssr_create(const wssr_config* cfg, wssr_handle* out) {
  if (!out) return WSSR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!cfg || cfg->n_max < 2 || cfg->m_max < 1 || cfg->r_max < 1 || cfg->r_max > 512 || cfg->q_max < 1 ||
      cfg->o_dtype < WSSR_F32 || cfg->o_dtype > WSSR_BF16_SPLIT || cfg->lanes < 0 || cfg->lanes > kLanesMax) {
    g_create_error = "invalid config";
    return WSSR_ERR_INVALID_ARG;
  }
  if (cfg->flags & WSSR_GRAPH) {
    // switched off: the first device run of a captured batch ended in a host
    // segmentation fault whose cause is not found yet
    g_create_error = "WSSR_GRAPH is disabled in this build (graph capture of the batched step is switched off)";
    return WSSR_ERR_INVALID_ARG;
  }
  int dev = -1;
  std::string why;
  if (!device_ok(&dev, why)) {
    g_create_error = why;
    return WSSR_ERR_NO_DEVICE;
  }
  wssr_ctx* h = nullptr;
  wssr_status s = build_ctx(cfg, dev, static_cast<hipStream_t>(cfg->stream), false, &h, why);
  if (s != WSSR_OK) {
    g_create_error = why;
    return s;
  }
  if (cfg->flags & WSSR_SAMPLE_SPACE) {
    const int64_t n = cfg->n_max;
    const int nt = (int)cdiv(n, 128), npairs = nt * (nt + 1) / 2;
    // partial tiles only where the K range is split (fewer than 512 pairs)
    h->tpart_tiles = npairs < 512 ? 2048 : 0;
    bool ok = h->alloc(h->Tn, (size_t)n * n) && h->alloc(h->rho, n) && h->alloc(h->su, n) && h->alloc(h->sb, n) &&
              h->alloc(h->sscal, 2) && h->alloc(h->tpart, (size_t)h->tpart_tiles * 128 * 128);
    if (!ok) {
      (void)hipGetLastError();
      h->release();
      delete h;
      g_create_error = "sample-space workspace allocation failed";
      return WSSR_ERR_OOM;
    }
  }
  for (int i = 0; i < cfg->lanes; ++i) {
    wssr_ctx* c = nullptr;
    hipEvent_t e = nullptr;
    s = build_ctx(cfg, dev, nullptr, true, &c, why);
    if (s == WSSR_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      c->release();
      delete c;
      s = WSSR_ERR_HIP;
      why = "event creation failed";
    }
    if (s != WSSR_OK) {
      h->release();
      delete h;
      g_create_error = why;
      return s;
    }
    c->plain_svd = true;
    h->lanes.push_back(c);
    h->lane_done.push_back(e);
  }
  *out = h;
  return WSSR_OK;
}

wssr_status wssr_destroy(wssr_handle h) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(h->stream);
  h->release();
  delete h;
  return WSSR_OK;
}

const char* wssr_last_error(wssr_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

static wssr_status check_common(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, int32_t r) {
  if (!O) return h->fail(WSSR_ERR_INVALID_ARG, "O is NULL");
  if (n < 2 || n > h->cfg.n_max) return h->fail(WSSR_ERR_INVALID_ARG, "n=%lld outside [2, n_max]", (long long)n);
  if (m < 1 || m > h->cfg.m_max) return h->fail(WSSR_ERR_INVALID_ARG, "m=%lld outside [1, m_max]", (long long)m);
  if (ld_o < m) return h->fail(WSSR_ERR_INVALID_ARG, "ld_o < m");
  if (r < 1 || r > h->cfg.r_max) return h->fail(WSSR_ERR_INVALID_ARG, "r=%d outside [1, r_max]", r);
  return WSSR_OK;
}

static wssr_status check_step(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o,
                              const double* e_l, const float* V, double lambda, int32_t r, int32_t q,
                              const double* delta, const double* sigma) {
  wssr_status s = check_common(h, n, m, O, ld_o, r);
  if (s != WSSR_OK) return s;
  if (!e_l || !V || !delta || !sigma) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (r > std::min<int64_t>(n - 1, m)) return h->fail(WSSR_ERR_INVALID_ARG, "r=%d exceeds min(n-1, m)", r);
  if (q < 1 || q > h->cfg.q_max) return h->fail(WSSR_ERR_INVALID_ARG, "q=%d outside [1, q_max]", q);
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return h->fail(WSSR_ERR_INVALID_ARG, "lambda must be > 0 and finite");
  return WSSR_OK;
}

wssr_status wssr_step(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l, float* V,
                      double lambda, int32_t r, int32_t q, double* delta, double* sigma) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  wssr_status s = check_step(h, n, m, O, ld_o, e_l, V, lambda, r, q, delta, sigma);
  if (s != WSSR_OK) return s;
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");

  return h->enqueue(n, m, O, ld_o, e_l, V, lambda, r, q, delta, sigma);
}

wssr_status wssr_step_g(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* g,
                        float* V, double lambda, int32_t r, int32_t q, double* delta, double* sigma) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!g) return h->fail(WSSR_ERR_INVALID_ARG, "g is NULL");
  // e_l is not read: any non-null pointer passes the common check
  wssr_status s = check_step(h, n, m, O, ld_o, g, V, lambda, r, q, delta, sigma);
  if (s != WSSR_OK) return s;
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  return h->enqueue(n, m, O, ld_o, nullptr, V, lambda, r, q, delta, sigma, g);
}

wssr_status wssr_step_avg(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                          const double* g, float* V, double lambda, int32_t r, int32_t q, double avg,
                          double* sig_state, double* l_state, double* delta, double* g_bar) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  wssr_status s = check_step(h, n, m, O, ld_o, e_l, V, lambda, r, q, delta, sig_state);
  if (s != WSSR_OK) return s;
  if (!l_state) return h->fail(WSSR_ERR_INVALID_ARG, "l_state is NULL");
  if (!(avg >= 0.0 && avg < 1.0)) return h->fail(WSSR_ERR_INVALID_ARG, "avg must be in [0, 1)");
  if (h->cfg.flags & WSSR_DIAGR_EXTRACT)
    return h->fail(WSSR_ERR_INVALID_ARG, "the averaged step needs the Rayleigh-Ritz ending (no WSSR_DIAGR_EXTRACT)");
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  wssr_ctx::AvgArgs av{avg, sig_state, l_state, g_bar};
  return h->enqueue(n, m, O, ld_o, e_l, V, lambda, r, q, delta, sig_state, g, &av);
}

wssr_status wssr_step_sketch(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                             const double* g, const float* omega, int32_t p, int32_t q, float* V, double lambda,
                             int32_t r, double* delta, double* sigma) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!e_l && !g) return h->fail(WSSR_ERR_INVALID_ARG, "e_l and g are both NULL");
  if (!omega) return h->fail(WSSR_ERR_INVALID_ARG, "omega is NULL");
  if (p < 0) return h->fail(WSSR_ERR_INVALID_ARG, "p < 0");
  if (r < 1) return h->fail(WSSR_ERR_INVALID_ARG, "r < 1");
  if (q < 0 || q > h->cfg.q_max) return h->fail(WSSR_ERR_INVALID_ARG, "q=%d outside [0, q_max]", q);
  // the sketch's rank r + p takes the place of r in the common checks
  wssr_status s = check_step(h, n, m, O, ld_o, e_l ? e_l : g, V, lambda, r + p, 1, delta, sigma);
  if (s != WSSR_OK) return s;
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  return h->enqueue_sketch(n, m, O, ld_o, e_l, omega, r + p, q, V, lambda, r, delta, sigma, g);
}

wssr_status wssr_spring(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                        double lambda, double momentum, double eta, double* dtheta, double* delta) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!(h->cfg.flags & WSSR_SAMPLE_SPACE))
    return h->fail(WSSR_ERR_INVALID_ARG, "the handle was created without WSSR_SAMPLE_SPACE");
  wssr_status s = check_common(h, n, m, O, ld_o, 1);
  if (s != WSSR_OK) return s;
  if (!e_l || !delta) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return h->fail(WSSR_ERR_INVALID_ARG, "lambda must be > 0 and finite");
  if (!(momentum >= 0.0 && momentum < 1.0)) return h->fail(WSSR_ERR_INVALID_ARG, "momentum must be in [0, 1)");
  if (!std::isfinite(eta)) return h->fail(WSSR_ERR_INVALID_ARG, "eta must be finite");
  if (momentum != 0.0 && !dtheta) return h->fail(WSSR_ERR_INVALID_ARG, "dtheta is NULL with nonzero momentum");
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  return h->enqueue_spring(n, m, O, ld_o, e_l, lambda, momentum, eta, dtheta, delta);
}

wssr_status wssr_ingest(wssr_handle h, int64_t n, int64_t m, int64_t row0, int64_t rows, const float* O32,
                        int64_t ld32, const double* e_l, const double* mu, void* O_out, int64_t ld_o, double* g,
                        double* colmean) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!O32 || !e_l) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (n < 2 || n > h->cfg.n_max) return h->fail(WSSR_ERR_INVALID_ARG, "n=%lld outside [2, n_max]", (long long)n);
  if (m < 1 || m > h->cfg.m_max) return h->fail(WSSR_ERR_INVALID_ARG, "m=%lld outside [1, m_max]", (long long)m);
  if (rows < 1 || row0 < 0 || row0 + rows > n)
    return h->fail(WSSR_ERR_INVALID_ARG, "rows [%lld, %lld) outside [0, n)", (long long)row0, (long long)(row0 + rows));
  if (ld32 < m) return h->fail(WSSR_ERR_INVALID_ARG, "ld32 < m");
  if (O_out && ld_o < m) return h->fail(WSSR_ERR_INVALID_ARG, "ld_o < m");
  if (mu && mu == colmean) return h->fail(WSSR_ERR_INVALID_ARG, "colmean must not alias mu");
  if (row0 != 0 && (row0 != h->ingest_next || n != h->ingest_n || m != h->ingest_m))
    return h->fail(WSSR_ERR_INVALID_ARG,
                   "blocks must follow each other from row 0 without gaps (expected row0=%lld for n=%lld, m=%lld)",
                   (long long)h->ingest_next, (long long)h->ingest_n, (long long)h->ingest_m);
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  h->ingest(n, m, row0, rows, O32, ld32, e_l, mu, O_out, ld_o, g, colmean);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  h->ingest_n = n;
  h->ingest_m = m;
  h->ingest_next = row0 + rows == n ? -1 : row0 + rows;
  return WSSR_OK;
}

namespace {
bool same_batch(const std::vector<wssr_problem>& a, const wssr_problem* b, int32_t count) {
  return (int32_t)a.size() == count && std::memcmp(a.data(), b, sizeof(wssr_problem) * (size_t)count) == 0;
}
}  // namespace

// Enqueue a batch: problems spread over the lanes (longest first onto the
// least-loaded lane, cost ~ n m r q), each lane running its problems one
// after another on its own stream, forked from and joined back into the
// handle's stream; per-problem status codes are saved to bstat.
static wssr_status enqueue_batch(wssr_ctx* h, const wssr_problem* p, int32_t count) {
  const int avail = (int)h->lanes.size();
  const int nl = std::max(1, h->active_lanes > 0 ? std::min(h->active_lanes, avail) : avail);
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto cost = [&](int i) { return (double)p[i].n * (double)p[i].m * (double)p[i].r * (double)p[i].q; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<std::vector<int>> plan(nl);
  std::vector<double> load(nl, 0.0);
  for (int i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    plan[l].push_back(i);
    load[l] += cost(i);
  }
  if (h->lanes.empty()) {
    for (int i : plan[0]) {
      wssr_status s = h->enqueue(p[i].n, p[i].m, p[i].O, p[i].ld_o, p[i].e_l, p[i].V, p[i].lambda, p[i].r, p[i].q,
                                 p[i].delta, p[i].sigma);
      if (s != WSSR_OK) return s;
      hipLaunchKernelGGL(k_status_save, dim3(1), dim3(1), 0, h->stream, (const DevStatus*)h->st, h->bstat + i);
    }
    return hipGetLastError() == hipSuccess ? WSSR_OK : h->fail(WSSR_ERR_HIP, "kernel launch failed");
  }
  (void)hipEventRecord(h->ev_fork, h->stream);
  for (int l = 0; l < nl; ++l) {
    wssr_ctx* c = h->lanes[l];
    c->capturing = h->capturing;
    (void)hipStreamWaitEvent(c->stream, h->ev_fork, 0);
    for (int i : plan[l]) {
      wssr_status s = c->enqueue(p[i].n, p[i].m, p[i].O, p[i].ld_o, p[i].e_l, p[i].V, p[i].lambda, p[i].r, p[i].q,
                                 p[i].delta, p[i].sigma);
      if (s != WSSR_OK) return h->fail(s, "batch lane %d: %s", l, c->err.c_str());
      hipLaunchKernelGGL(k_status_save, dim3(1), dim3(1), 0, c->stream, (const DevStatus*)c->st, h->bstat + i);
    }
    (void)hipEventRecord(h->lane_done[l], c->stream);
    (void)hipStreamWaitEvent(h->stream, h->lane_done[l], 0);
  }
  return hipGetLastError() == hipSuccess ? WSSR_OK : h->fail(WSSR_ERR_HIP, "kernel launch failed");
}

wssr_status wssr_step_batched(wssr_handle h, const wssr_problem* probs, int32_t count) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!probs || count < 1 || count > kBatchMax)
    return h->fail(WSSR_ERR_INVALID_ARG, "count=%d outside [1, %d]", count, kBatchMax);
  for (int i = 0; i < count; ++i) {
    const wssr_problem& q = probs[i];
    wssr_status s = check_step(h, q.n, q.m, q.O, q.ld_o, q.e_l, q.V, q.lambda, q.r, q.q, q.delta, q.sigma);
    if (s != WSSR_OK) return h->fail(s, "problem %d: %s", i, h->err.c_str());
  }
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  if (!(h->cfg.flags & WSSR_GRAPH) || h->graph_broken) return enqueue_batch(h, probs, count);
  if (!h->gexec || !same_batch(h->gkey, probs, count)) {
    // capture the batch once; replay it while the same problems are passed
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->gkey.clear();
    (void)hipGetLastError();
    if (!h->cstream && hipStreamCreateWithFlags(&h->cstream, hipStreamNonBlocking) != hipSuccess) {
      h->cstream = nullptr;
      h->graph_broken = true;
      h->graph_why = "capture stream creation failed";
      return enqueue_batch(h, probs, count);
    }
    // capture on the private stream: the batch's fork/join hangs off it
    hipStream_t user = h->stream;
    h->stream = h->cstream;
    hipError_t e = hipStreamBeginCapture(h->cstream, hipStreamCaptureModeRelaxed);
    bool ok = e == hipSuccess;
    h->capturing = true;
    wssr_status s = ok ? enqueue_batch(h, probs, count) : WSSR_ERR_HIP;
    h->capturing = false;
    for (wssr_ctx* c : h->lanes) c->capturing = false;
    hipGraph_t g = nullptr;
    if (ok) {
      e = hipStreamEndCapture(h->cstream, &g);
      ok = e == hipSuccess && g != nullptr && s == WSSR_OK;
    }
    if (ok) {
      e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
      ok = e == hipSuccess;
    }
    h->stream = user;
    if (!ok) {
      if (g) (void)hipGraphDestroy(g);
      h->gexec = nullptr;
      (void)hipGetLastError();
      h->graph_broken = true;   // this handle runs batches without a graph from now on
      h->graph_why = std::string("graph capture failed: ") + hipGetErrorString(e) + (s != WSSR_OK ? " (enqueue)" : "");
      return enqueue_batch(h, probs, count);
    }
    h->graph = g;
    h->gkey.assign(probs, probs + count);
  }
  if (hipGraphLaunch(h->gexec, h->stream) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipGraphLaunch failed");
  return WSSR_OK;
}

wssr_status wssr_batched_status(wssr_handle h, int32_t count, int32_t* codes) {
  if (!h || !codes || count < 1 || count > kBatchMax) return WSSR_ERR_INVALID_ARG;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipStreamSynchronize failed");
  if (hipMemcpy(codes, h->bstat, sizeof(int32_t) * (size_t)count, hipMemcpyDeviceToHost) != hipSuccess)
    return h->fail(WSSR_ERR_HIP, "status copy failed");
  return WSSR_OK;
}

// Autotuner of the batched form.  Candidates: the number of lanes in use
// (1, 2, 4, ... up to the handle's lanes) and, for each, how many resident
// workgroups a product sizes its split-K and stream-K decomposition for (the
// whole device, or its share: slots / lanes).  Each candidate runs the batch
// `reps` times on scratch copies of V, delta and sigma (the caller's buffers
// are not written) and the fastest by HIP events is kept.
wssr_status wssr_tune_batched(wssr_handle h, const wssr_problem* probs, int32_t count, int32_t reps,
                              int32_t* best_lanes, int32_t* best_div, double* best_ms) {
  if (!h || !probs || count < 1 || count > kBatchMax || reps < 1) return WSSR_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    const wssr_problem& q = probs[i];
    wssr_status s = check_step(h, q.n, q.m, q.O, q.ld_o, q.e_l, q.V, q.lambda, q.r, q.q, q.delta, q.sigma);
    if (s != WSSR_OK) return h->fail(s, "problem %d: %s", i, h->err.c_str());
  }
  if (hipSetDevice(h->device) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipSetDevice failed");
  // scratch copies of the written arguments
  std::vector<wssr_problem> work(probs, probs + count);
  std::vector<void*> scratch;
  bool ok = true;
  for (auto& q : work) {
    void *v = nullptr, *d = nullptr, *sg = nullptr;
    ok = ok && hipMalloc(&v, sizeof(float) * q.m * q.r) == hipSuccess;
    ok = ok && hipMalloc(&d, sizeof(double) * q.m) == hipSuccess;
    ok = ok && hipMalloc(&sg, sizeof(double) * q.r) == hipSuccess;
    scratch.push_back(v);
    scratch.push_back(d);
    scratch.push_back(sg);
    if (!ok) break;
    (void)hipMemcpyAsync(v, q.V, sizeof(float) * q.m * q.r, hipMemcpyDeviceToDevice, h->stream);
    q.V = static_cast<float*>(v);
    q.delta = static_cast<double*>(d);
    q.sigma = static_cast<double*>(sg);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  const int saved_lanes = h->active_lanes;
  std::vector<int> saved_div;
  for (wssr_ctx* c : h->lanes) saved_div.push_back(c->slot_div);
  const int saved_div0 = h->slot_div;
  int bl = std::max(1, (int)h->lanes.size()), bd = 1;
  double bms = 1e300;
  const int avail = std::max(1, (int)h->lanes.size());
  std::vector<int> cands;
  for (int nl = 1; nl < avail; nl *= 2) cands.push_back(nl);
  cands.push_back(avail);
  for (int nl : cands) {
    for (int div : {1, nl}) {
      if (!ok) break;
      h->active_lanes = nl;
      h->slot_div = div;
      for (wssr_ctx* c : h->lanes) c->slot_div = div;
      // one untimed run (first use of the configuration), then `reps` timed
      if (enqueue_batch(h, work.data(), count) != WSSR_OK) {
        ok = false;
        break;
      }
      (void)hipEventRecord(e0, h->stream);
      for (int k = 0; k < reps && ok; ++k) ok = enqueue_batch(h, work.data(), count) == WSSR_OK;
      (void)hipEventRecord(e1, h->stream);
      if (!ok || hipEventSynchronize(e1) != hipSuccess) {
        ok = false;
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / reps;
      if (per < bms) {
        bms = per;
        bl = nl;
        bd = div;
      }
      if (nl == 1) break;   // the device share of one lane is the device
    }
    if (!ok) break;
  }
  (void)hipStreamSynchronize(h->stream);
  for (void* p : scratch) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!ok) {
    h->active_lanes = saved_lanes;
    h->slot_div = saved_div0;
    for (size_t i = 0; i < h->lanes.size(); ++i) h->lanes[i]->slot_div = saved_div[i];
    return h->fail(WSSR_ERR_HIP, "tuning run failed");
  }
  h->active_lanes = bl;
  h->slot_div = bd;
  for (wssr_ctx* c : h->lanes) c->slot_div = bd;
  if (best_lanes) *best_lanes = bl;
  if (best_div) *best_div = bd;
  if (best_ms) *best_ms = bms;
  return WSSR_OK;
}

wssr_status wssr_graph_active(wssr_handle h, int32_t* active) {
  if (!h || !active) return WSSR_ERR_INVALID_ARG;
  *active = (h->gexec != nullptr && !h->graph_broken) ? 1 : 0;
  if (!*active && !h->graph_why.empty()) h->err = h->graph_why;
  return WSSR_OK;
}

wssr_status wssr_status_sync(wssr_handle h, int32_t* numeric_status, double* diag) {
  if (!h || !numeric_status) return WSSR_ERR_INVALID_ARG;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipStreamSynchronize failed");
  DevStatus s;
  if (hipMemcpy(&s, h->st, sizeof s, hipMemcpyDeviceToHost) != hipSuccess)
    return h->fail(WSSR_ERR_HIP, "status copy failed");
  *numeric_status = s.code;
  if (diag) {
    diag[0] = s.min_rel_pivot;
    diag[1] = s.jacobi_sweeps;
    diag[2] = s.jacobi_cosine;
    diag[3] = (double)s.chol_count;
    diag[4] = s.kappa_max;
    diag[5] = (double)s.round2_count;
  }
  return WSSR_OK;
}

wssr_status wssr_set_rank_ratio(wssr_handle h, double r_reg) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!(r_reg >= 0.0 && r_reg < 1.0)) return h->fail(WSSR_ERR_INVALID_ARG, "r_reg must be in [0, 1)");
  h->r_reg = r_reg;
  for (wssr_ctx* c : h->lanes) c->r_reg = r_reg;
  return WSSR_OK;
}

wssr_status wssr_rank_info(wssr_handle h, int32_t* r_eff, int32_t* grow) {
  if (!h || !r_eff || !grow) return WSSR_ERR_INVALID_ARG;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipStreamSynchronize failed");
  DevStatus s;
  if (hipMemcpy(&s, h->st, sizeof s, hipMemcpyDeviceToHost) != hipSuccess)
    return h->fail(WSSR_ERR_HIP, "status copy failed");
  *r_eff = s.r_eff;
  *grow = s.grow;
  return WSSR_OK;
}

wssr_status wssr_profile(wssr_handle h, int32_t enable) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipStreamSynchronize failed");
  h->ev_marks.clear();
  h->ev_used = 0;
  h->prof = enable != 0;
  return WSSR_OK;
}

wssr_status wssr_profile_read(wssr_handle h, double* ms, int64_t* counts, int32_t nslots) {
  if (!h || !ms || !counts || nslots < 1 || nslots > 4) return WSSR_ERR_INVALID_ARG;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(WSSR_ERR_HIP, "hipStreamSynchronize failed");
  for (int i = 0; i < nslots; ++i) {
    ms[i] = 0.0;
    counts[i] = 0;
  }
  for (auto& mk : h->ev_marks) {
    float t = 0.0f;
    if (mk.first < nslots && hipEventElapsedTime(&t, mk.second.first, mk.second.second) == hipSuccess) {
      ms[mk.first] += t;
      counts[mk.first] += 1;
    }
  }
  return WSSR_OK;
}

// ------------------------------------------------------------ single stages

wssr_status wssr_dbg_sample_side(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const float* V,
                                 int32_t r, double* y) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  wssr_status s = check_common(h, n, m, O, ld_o, r);
  if (s != WSSR_OK) return s;
  if (!V || !y) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  h->gemm_sample_side(O, ld_o, n, m, V, r);
  (void)hipMemcpyAsync(y, h->y64, sizeof(double) * n * r, hipMemcpyDeviceToDevice, h->stream);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

wssr_status wssr_dbg_param_side(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const float* X,
                                int32_t r, float* z) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  wssr_status s = check_common(h, n, m, O, ld_o, r);
  if (s != WSSR_OK) return s;
  if (!X || !z) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  h->gemm_param_side(O, ld_o, n, m, X, r, z);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

wssr_status wssr_dbg_gradient(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                              double* g) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  wssr_status s = check_common(h, n, m, O, ld_o, 1);
  if (s != WSSR_OK) return s;
  if (!e_l || !g) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  h->gradient(O, ld_o, n, m, e_l, g);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

wssr_status wssr_dbg_cholqr2(wssr_handle h, int64_t rows, const float* X, int32_t r, float* Q, double* R) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!X || !Q || !R) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (r < 1 || r > h->cfg.r_max) return h->fail(WSSR_ERR_INVALID_ARG, "r outside [1, r_max]");
  if (rows < r || rows > h->rows_max) return h->fail(WSSR_ERR_INVALID_ARG, "rows outside [r, max(n_max, m_max)]");
  const int rp = (int)rup(r, 64);
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  // a workspace copy of X (a rank-deficient X is completed in place)
  float* xc = rows <= h->cfg.m_max ? h->vw : h->qy;
  (void)hipMemcpyAsync(xc, X, sizeof(float) * rows * r, hipMemcpyDeviceToDevice, h->stream);
  h->cholqr<float, float>(xc, rows, r, h->q1, h->Rz);
  h->apply((const float*)xc, rows, r, r, h->Tq, rp, r, Q, r, true);
  (void)hipMemcpy2DAsync(R, sizeof(double) * r, h->Rz, sizeof(double) * rp, sizeof(double) * r, r,
                         hipMemcpyDeviceToDevice, h->stream);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

wssr_status wssr_dbg_gram(wssr_handle h, int64_t rows, const float* X, int32_t r, int32_t kind, double* G) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!X || !G) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (kind < 0 || kind > 2) return h->fail(WSSR_ERR_INVALID_ARG, "kind outside 0..2");
  if (r < 1 || r > h->cfg.r_max) return h->fail(WSSR_ERR_INVALID_ARG, "r outside [1, r_max]");
  if (rows < 1 || rows > h->rows_max) return h->fail(WSSR_ERR_INVALID_ARG, "rows outside [1, max(n_max, m_max)]");
  const int rp = (int)rup(r, 64);
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  h->gram(X, rows, r, false, (int)kind);
  (void)hipMemcpy2DAsync(G, sizeof(double) * r, h->G, sizeof(double) * rp, sizeof(double) * r, r,
                         hipMemcpyDeviceToDevice, h->stream);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

wssr_status wssr_dbg_span_basis(wssr_handle h, int64_t rows, const float* X, int32_t r, float* V, int32_t* mode) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!X || !V || !mode) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (r < 1 || r > h->cfg.r_max) return h->fail(WSSR_ERR_INVALID_ARG, "r outside [1, r_max]");
  if (rows < r || rows > h->cfg.m_max) return h->fail(WSSR_ERR_INVALID_ARG, "rows outside [r, m_max]");
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  (void)hipMemcpyAsync(h->z, X, sizeof(float) * rows * r, hipMemcpyDeviceToDevice, h->stream);
  h->fast_orth(h->z, rows, r, false);
  (void)hipMemcpyAsync(V, h->vw, sizeof(float) * rows * r, hipMemcpyDeviceToDevice, h->stream);
  (void)hipMemcpyAsync(mode, h->fmode, sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

wssr_status wssr_dbg_small_svd(wssr_handle h, const double* C, int32_t r, double* s, double* P) {
  if (!h) return WSSR_ERR_INVALID_ARG;
  if (!C || !s || !P) return h->fail(WSSR_ERR_INVALID_ARG, "NULL pointer argument");
  if (r < 1 || r > h->cfg.r_max) return h->fail(WSSR_ERR_INVALID_ARG, "r outside [1, r_max]");
  const int rp = (int)rup(r, 64);
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, h->stream, h->st);
  hipLaunchKernelGGL(k_transpose_pad, dim3(cdiv((int64_t)rp * rp, 256)), dim3(256), 0, h->stream, C, r, rp, h->Rz);
  h->small_svd(h->Rz, r);
  if (h->coop_err != hipSuccess)
    return h->fail(WSSR_ERR_HIP, "cooperative launch of the SVD kernel failed: %s", hipGetErrorString(h->coop_err));
  (void)hipMemcpyAsync(s, h->sig, sizeof(double) * r, hipMemcpyDeviceToDevice, h->stream);
  (void)hipMemcpy2DAsync(P, sizeof(double) * r, h->Ps, sizeof(double) * rp, sizeof(double) * r, r,
                         hipMemcpyDeviceToDevice, h->stream);
  if (hipGetLastError() != hipSuccess) return h->fail(WSSR_ERR_HIP, "kernel launch failed");
  return WSSR_OK;
}

}  // extern "C"
