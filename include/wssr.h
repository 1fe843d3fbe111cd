/*
 * libwssr: one warm-started stochastic-reconfiguration (WSSR) step on an
 * AMD Instinct MI355X (gfx950), as a plain C ABI.
 *
 * The step (paper: Sec. 3.1 eqs. Osr/Osrn/Lbarn for the centred matrices,
 * Sec. 4.1 eq. barg for the gradient, Sec. 4.2 Alg. 1 for the warm-started
 * subspace iteration, Sec. 4.1 eq. updated_sr_1 and Sec. 3.2 for the
 * regularised low-rank preconditioner) computes, from the N x M matrix O of
 * per-sample log-derivatives (rows = samples) and the local energies E_L:
 *
 *   eps   = E_L - mean(E_L)                       (eq. Lbarn)
 *   A     = (O - 1 mu^T) / sqrt(N)                 (eqs. Osr, Osrn; mu = column means)
 *   g     = A^T eps / sqrt(N) = O_bar^T eps / N    (eq. barg at averaging weight 0, no factor 2)
 *   V, sigma <- q passes of subspace iteration on A^T A started from V_in,
 *                closed by a Rayleigh-Ritz SVD      (Alg. 1)
 *   delta = (V diag(sigma^2) V^T + lambda I)^{-1} g  (Woodbury)        [default]
 *   delta = (V diag(sigma^-2) V^T + (I - V V^T)/lambda) g               [WSSR_FLOOR_PRECOND,
 *                                                     eq. updated_sr_1 with floor lambda]
 *
 * sigma are the singular values of A (descending); sigma^2 are the
 * eigenvalues of S = A^T A.  The caller applies theta <- theta - eta * delta.
 *
 * Precision.  The products run on the MFMA in the configured dtype with FP32
 * accumulation; the sample-side block Y is kept and orthonormalised in FP64
 * (CholeskyQR2).  The parameter-side block Z (FP32) is orthonormalised from a
 * fast Gram (an FP32-MFMA one, or the BF16 MFMA on a two-plane split of Z,
 * with FP64 sums every 256 rows; entries to 1e-7 / 3e-7 of sqrt(G_ii G_jj))
 * and an FP64 Cholesky where Z is well conditioned, else by the FP64
 * CholeskyQR2; an intermediate pass carries on only the span of Z, which
 * leaves the iteration's subspace that of Alg. 1 in exact arithmetic.
 *
 * Memory.  Every data pointer passed to wssr_step and the wssr_dbg_* calls is
 * DEVICE memory on the handle's device; the caller owns it.  The library owns
 * only the workspace it allocates in wssr_create.  wssr_step never allocates.
 * Layouts are row-major.  O is read-only; V is read, then overwritten.
 *
 * Streams.  All work is enqueued on the stream given at create time (a
 * hipStream_t; NULL means the null stream); calls return without waiting.
 * Inside wssr_step, the gradient pass runs on a second, library-owned stream (beside the Rayleigh-Ritz SVD)
 * forked from and joined back into that stream with events, so the step is
 * still ordered on the caller's stream as one unit.  Results are valid once
 * that stream has been synchronised.  A handle is not thread-safe; use one
 * handle per stream.
 *
 * Errors.  Argument errors are detected on the host before anything is
 * enqueued and returned as negative codes; nothing is enqueued then.
 * Numerical errors (non-finite input, Cholesky breakdown) are recorded in a
 * device status word and read with wssr_status_sync; after such an error the
 * remaining kernels of the step leave V, delta and sigma untouched.
 */
#ifndef WSSR_H
#define WSSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wssr_ctx* wssr_handle;

typedef enum {
  WSSR_OK = 0,
  WSSR_WARN_RANK_DEFICIENT = 1,  /* a basis of the iteration lost rank (r exceeds the rank of the
                                    centred O, e.g. repeated samples); the basis was completed with
                                    directions from rounding and the extra singular values are at
                                    rounding level, so delta is unaffected; results usable */
  WSSR_WARN_NOT_CONVERGED = 2,   /* Rayleigh-Ritz Jacobi hit its sweep limit; results usable */
  WSSR_ERR_INVALID_ARG = -1,
  WSSR_ERR_NO_DEVICE = -2,
  WSSR_ERR_OOM = -3,
  WSSR_ERR_HIP = -4,
  WSSR_ERR_NONFINITE = -5,       /* NaN/Inf in E_L, or reached the Gram matrices from O or V */
  WSSR_ERR_BREAKDOWN = -6,       /* the iterated basis lost rank and could not be completed (a zero
                                    column, or a second CholeskyQR round that broke down) */
  WSSR_ERR_TIMEOUT = -7          /* internal: a bounded wait between the workgroups of the
                                    Rayleigh-Ritz SVD expired; outputs untouched */
} wssr_status;

/* Storage and multiply precision of O.  The Gram matrices, Cholesky factors,
 * the r x r SVD, the gradient sums and the Woodbury core are FP64 in every
 * form; V is FP32.  In the BF16 forms the products run on the BF16 MFMA with
 * FP32 accumulation and the skinny operand (V or the sample-side basis, FP32)
 * is rounded to BF16 on the fly: S_hi = RNE(S), S_lo = RNE(S - S_hi).
 *   WSSR_F32         O float; FP32 products.
 *   WSSR_BF16        O BF16; one product O S_hi.
 *   WSSR_BF16_SPLIT  O BF16; two products O S_hi + O S_lo (the skinny operand
 *                    kept to about 16 bits).
 *   WSSR_BF16X2      O given as two BF16 planes, O_hi = RNE(O) at O and
 *                    O_lo = RNE(O - O_hi) at O + n * ld_o elements; three
 *                    products O_hi S_hi + O_hi S_lo + O_lo S_hi.  The gradient
 *                    uses O_hi + O_lo. */
typedef enum {
  WSSR_F32 = 0,
  WSSR_BF16 = 1,
  WSSR_BF16X2 = 2,
  WSSR_BF16_SPLIT = 3
} wssr_dtype;

/* Flags (wssr_config.flags). */
#define WSSR_FLOOR_PRECOND 0x1u  /* eq. updated_sr_1 weights w_j = 1 - lambda/sigma_j^2 instead of
                                    the damped w_j = sigma_j^2/(sigma_j^2 + lambda) */
#define WSSR_DIAGR_EXTRACT 0x8u  /* Alg. 1's own ending instead of the Rayleigh-Ritz step: the last
                                    pass stops after the QR of its sample-side block A V (V
                                    orthonormal), sigma = |diag(R)| sorted, and V is that basis in
                                    the same order (one product fewer; sigma and V converge more
                                    slowly inside the top r).  wssr_step, wssr_step_g and the
                                    batched form; wssr_step_avg rejects it */
#define WSSR_SAMPLE_SPACE 0x4u   /* allocate the workspace of wssr_spring: an n_max x n_max FP64
                                    matrix (8 n_max^2 bytes) and up to 268 MB of partial tiles */
#define WSSR_GRAPH 0x2u          /* wssr_step_batched captures a batch into a HIP graph on its first
                                    call and replays the graph while the same problem array (same
                                    sizes and pointers) is passed again.  Currently disabled:
                                    wssr_create returns WSSR_ERR_INVALID_ARG for this flag. */

typedef struct {
  int64_t n_max;        /* largest N (samples) a step will be called with */
  int64_t m_max;        /* largest M (parameters) */
  int32_t r_max;        /* largest rank r, 1 <= r_max <= 512 */
  int32_t q_max;        /* largest pass count q */
  int32_t o_dtype;      /* wssr_dtype */
  uint32_t flags;
  void* stream;         /* hipStream_t */
  int32_t lanes;        /* wssr_step_batched: problems run concurrently on this many lanes, each
                           with its own stream and workspace (0 or 1: one after another on the
                           handle's stream); 0 <= lanes <= 16 */
} wssr_config;

/* One problem of a batched step: the arguments of wssr_step. */
typedef struct {
  int64_t n, m, ld_o;
  const void* O;
  const double* e_l;
  float* V;
  double lambda;
  int32_t r, q;
  double* delta;
  double* sigma;
} wssr_problem;

/* Create a handle on the current HIP device and allocate its workspace
 * (sized from n_max, m_max, r_max).  Returns WSSR_ERR_NO_DEVICE when no
 * gfx950 device is visible, WSSR_ERR_OOM when the workspace does not fit,
 * WSSR_ERR_INVALID_ARG for a bad config.  *out is NULL on failure. */
wssr_status wssr_create(const wssr_config* cfg, wssr_handle* out);

/* Release the workspace.  Waits for the handle's stream first. */
wssr_status wssr_destroy(wssr_handle h);

/* One WSSR step (see the top of this file).
 *   n, m     sample and parameter counts, 2 <= n <= n_max, 1 <= m <= m_max
 *   O        device, n x m, row stride ld_o >= m elements, in the configured dtype
 *            (WSSR_BF16X2: the lo plane follows at O + n * ld_o elements)
 *   e_l      device, double[n]
 *   V        device, float[m x r] row-major (row stride r): in: warm start whose
 *            column span seeds the iteration (orthonormality not required);
 *            out: right singular vectors of A, column j paired with sigma[j].
 *            Column signs: <v_out_j, v_in_j> >= 0; where that inner product is
 *            below 1e-8 in magnitude, the entry of largest magnitude (lowest row
 *            on ties) is positive.
 *   lambda   damping > 0 and finite
 *   r        rank, 1 <= r <= min(n - 1, m, r_max)
 *   q        passes, 1 <= q <= q_max
 *   delta    device, double[m], out
 *   sigma    device, double[r], out, descending
 * Returns WSSR_OK or an argument error; numerical status via wssr_status_sync. */
wssr_status wssr_step(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o,
                      const double* e_l, float* V, double lambda, int32_t r, int32_t q,
                      double* delta, double* sigma);

/* One WSSR step with a gradient the caller supplies: the same step as
 * wssr_step, except that g (device, double[m]) is used as the gradient of
 * eq. barg and the step makes no gradient pass over O (E_L is not needed).
 * This is how the BF16 forms use a gradient formed from the unrounded O by
 * wssr_ingest: BF16 storage of O perturbs g by about 2^-9 relative, and the
 * damping 1/lambda of the update amplifies that into delta, while the
 * subspace iteration tolerates it.  g is read only. */
wssr_status wssr_step_g(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* g,
                        float* V, double lambda, int32_t r, int32_t q, double* delta, double* sigma);

/* One WSSR step with the averaged state (Sec. 4.1: eqs. Ohat, Lhat, svd:det,
 * Obar, Lbar, barg, barS; Alg. 2).  The state of the previous step is the
 * stored matrix Obar = V_in diag(sig_state) (parameters x r) and the stored
 * vector l_state (r); the step
 *   - stacks them with the new samples, weights sqrt(avg) and sqrt(1 - avg)
 *     (eqs. Ohat, Lhat), and runs q passes of the subspace iteration on the
 *     stacked matrix (n + r rows in this library's orientation), warm-started
 *     from V_in;
 *   - returns its rank-r right singular vectors in V and its singular values
 *     in sig_state: the new Obar = V diag(sig_state) (eq. Obar);
 *   - sets l_state to the sample-side singular vectors applied to the
 *     stacked vector (eq. Lbar), signed like the columns of V;
 *   - forms the averaged gradient gbar = (1 - avg) g + avg V_in (sig o l)
 *     (eq. barg) and the direction delta = (V diag(sig^2) V^T + lambda I)^{-1}
 *     gbar (the floor form with WSSR_FLOOR_PRECOND), i.e. with Sbar of eq.
 *     barS in place of S.
 * Arguments as for wssr_step, and:
 *   e_l        device, double[n]: read always (the stacked vector needs eps)
 *   g          device, double[m] or NULL: a gradient formed by wssr_ingest; NULL:
 *              the step forms g from O and e_l
 *   V          in: the U of the previous averaged step (the state's basis and the
 *              warm start); for the first step any basis, with sig_state = 0
 *   avg        averaging weight, 0 <= avg < 1 (0: the plain step; the state is
 *              then ignored but must be finite)
 *   sig_state  device, double[r], in/out, finite; zero for the initial state
 *   l_state    device, double[r], in/out, finite; zero for the initial state
 *   g_bar      device, double[m] or NULL: out, the averaged gradient
 * The history rows are weighted by sqrt(avg / (1 - avg)) relative to the
 * samples; the cost beyond wssr_step is one Gram of V_in (m x r), one
 * accumulating apply V_in B (m x r times r x r) per pass, and r x r work. */
wssr_status wssr_step_avg(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                          const double* g, float* V, double lambda, int32_t r, int32_t q, double avg,
                          double* sig_state, double* l_state, double* delta, double* g_bar);

/* One SR step whose rank-r SVD comes from a randomized sketch (App. A, eq.
 * randsvd; the RSSR variant of the remark on randomized sketching in Sec.
 * 4.1), for a cold start or in place of the warm-started iteration: with the
 * random sample-side block Omega (n x (r + p)), Q = orth(A^T Omega) (the
 * paper's Y = Ohat Omega), the SVD of B = Q^T A^T (through A Q = Q_W R_W and
 * the SVD of R_W), V = Q U_B truncated to r columns, and the Woodbury
 * direction as in wssr_step.  Two products over O at rank r + p.  With q > 0
 * the power scheme of the same randomized range finder: q passes of the
 * subspace iteration at rank r + p start from Q and end in the Rayleigh-Ritz
 * step of wssr_step (1 + 2q products); that makes the result far less
 * sensitive to perturbations of O such as BF16 storage.
 *   e_l, g     as in wssr_step / wssr_step_g: g (device, double[m]) may be
 *              NULL, then e_l is read and g formed; e_l may be NULL when g is given
 *   omega      device, float[n x (r + p)] row-major: the random block (e.g.
 *              Gaussian), read only; its column means are removed before use,
 *              which leaves A^T Omega unchanged
 *   p          oversampling, p >= 0, with r + p <= min(n - 1, m, r_max)
 *   q          power passes, 0 <= q <= q_max (0: the scheme of App. A as printed)
 *   V          device, float[m x r], out only (no warm start).  Column signs:
 *              the entry of largest magnitude (lowest row on ties) is positive.
 *   delta, sigma as in wssr_step (sigma: the r largest of the sketch). */
wssr_status wssr_step_sketch(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                             const double* g, const float* omega, int32_t p, int32_t q, float* V, double lambda,
                             int32_t r, double* delta, double* sigma);

/* The comparison system of Sec. 3.2 on the same GPU: MinSR (eq. mT) with the
 * SPRING momentum (eq. param:spring), damped and solved in sample space.
 *   Ltilde = eps/sqrt(N) - momentum A dtheta_in
 *   delta  = A^T (A A^T + lambda I)^{-1} Ltilde          (no factor 2, as in wssr_step)
 *   dtheta = -eta delta + momentum dtheta_in             (the next theta_{k+1} - theta_k)
 * momentum = 0 is MinSR, and its delta is the damped full-rank SR direction
 * (S + lambda I)^{-1} g that wssr_step approximates at rank r.  T = A A^T is
 * formed on the FP64 MFMA (exact products of the stored values, FP64 sums;
 * N^2 M multiply-adds, half of them by symmetry), double-centred, and solved
 * by a blocked FP64 Cholesky and two blocked triangular solves.
 * Needs a handle created with WSSR_SAMPLE_SPACE (WSSR_ERR_INVALID_ARG otherwise).
 *   O, ld_o, n, m, e_l  as in wssr_step (any storage form)
 *   lambda     damping > 0
 *   momentum   0 <= momentum < 1
 *   eta        the step size of the momentum update (finite)
 *   dtheta     device, double[m], in/out, or NULL when momentum = 0 (then not written):
 *              in theta_k - theta_{k-1}, out -eta delta + momentum dtheta_in
 *   delta      device, double[m], out
 * A Cholesky pivot that is not positive raises WSSR_ERR_BREAKDOWN. */
wssr_status wssr_spring(wssr_handle h, int64_t n, int64_t m, const void* O, int64_t ld_o, const double* e_l,
                        double lambda, double momentum, double eta, double* dtheta, double* delta);

/* Ingest of O: one pass over a block of rows of the unrounded FP32 matrix
 * that writes them in the handle's storage form and forms, from the unrounded
 * values, the gradient g = O_bar^T eps / n (Sec. 4.1 eq. barg; eps = E_L -
 * mean(E_L), Sec. 3.1 eq. Lbarn) and the column means mu of O (eq. Osr).
 *   n, m      the whole matrix: n rows (samples), m columns; n <= n_max, m <= m_max
 *   row0, rows  this block: rows row0 .. row0 + rows - 1.  The block with
 *             row0 = 0 centres e_l and starts the sums (overwriting g and
 *             colmean); the following calls must continue from the next row,
 *             without gaps, with the same n and m (checked: WSSR_ERR_INVALID_ARG),
 *             and after the block that ends at row n, g and colmean hold their
 *             final values.  A block may be the whole matrix.
 *   O32, ld32 device, float, the block's rows (row i of the block at O32 + i * ld32), ld32 >= m
 *   e_l       device, double[n]: all n energies (the same array for every block)
 *   mu        device, double[m] or NULL: when given, the stored values are
 *             x - mu[j] (explicit centring before rounding, for data whose
 *             column means are large against its spread; pass the colmean of a
 *             first pass with O_out = NULL).  g and colmean always use x.
 *   O_out, ld_o  device, the whole stored matrix (row 0), row stride ld_o >= m, in
 *             the handle's dtype: float (WSSR_F32), BF16 (WSSR_BF16, WSSR_BF16_SPLIT),
 *             or the hi plane with the lo plane at O_out + n * ld_o (WSSR_BF16X2);
 *             rows row0 .. row0 + rows - 1 are written.  BF16 values are
 *             round-to-nearest-even: hi = RNE(x), lo = RNE(x - hi).  NULL: nothing
 *             is stored (a statistics pass).
 *   g         device, double[m] or NULL: out, sum_i O[i, j] eps_i / n
 *   colmean   device, double[m] or NULL: out, the column means of O; must not alias mu
 * Numerical status (a non-finite value of O or E_L: WSSR_ERR_NONFINITE) is
 * read with wssr_status_sync after the last block; the next step resets it.
 * Cost: one read of the FP32 block and one write of its stored form (HBM-bound). */
wssr_status wssr_ingest(wssr_handle h, int64_t n, int64_t m, int64_t row0, int64_t rows, const float* O32,
                        int64_t ld32, const double* e_l, const double* mu, void* O_out, int64_t ld_o, double* g,
                        double* colmean);

/* Batched form: `count` independent steps (1 <= count <= 1024), each with its
 * own sizes, lambda, r and q within the handle's capacities, in the handle's
 * dtype.  The problems are spread over the handle's lanes (longest first onto
 * the least-loaded lane; cost ~ n m r q), each lane running its share one
 * after another on its own stream; the lanes fork from and join back into the
 * handle's stream, so the batch is ordered on that stream as one unit.  With
 * WSSR_GRAPH the whole batch is one graph launch after the first call.
 * Per-problem results are those of wssr_step on the same inputs (bit for bit:
 * the same kernels in the same configuration).  Argument errors of any
 * problem are reported before anything is enqueued.  Numerical status: one
 * code per problem, read with wssr_batched_status. */
wssr_status wssr_step_batched(wssr_handle h, const wssr_problem* probs, int32_t count);

/* Synchronise the handle's stream and copy the status codes of the problems
 * of the last batch (codes[0..count)). */
wssr_status wssr_batched_status(wssr_handle h, int32_t count, int32_t* codes);

/* Autotuner of the batched form: runs the batch `reps` times under each
 * candidate configuration -- lanes in use (1, 2, 4, ... up to the handle's
 * lanes) and, per lane count, the number of resident workgroups the product
 * kernels size their split-K / stream-K decomposition for (the whole device,
 * or its share, slots / lanes) -- and keeps the fastest for later batches.
 * It works on scratch copies of V, delta and sigma (it allocates them), so the
 * caller's buffers are not written; O and e_l are only read.  Outputs
 * (nullable): the chosen lane count, the split divisor and the batch time in
 * milliseconds. */
wssr_status wssr_tune_batched(wssr_handle h, const wssr_problem* probs, int32_t count, int32_t reps,
                              int32_t* best_lanes, int32_t* best_div, double* best_ms);

/* *active = 1 when the last batch ran as a replayed or fresh graph.  When a
 * capture has failed, the handle runs its batches as direct launches from
 * then on, and wssr_last_error gives the reason after this call. */
wssr_status wssr_graph_active(wssr_handle h, int32_t* active);

/* Synchronise the handle's stream and read the numerical status of the last
 * step (a wssr_status value) into *numeric_status.  If diag is non-NULL it
 * receives 6 doubles: the smallest relative Cholesky pivot of the last step,
 * the number of Rayleigh-Ritz Jacobi sweeps, the largest column cosine seen in
 * the last sweep, the number of Cholesky factorisations performed, the
 * largest condition bound ||R D^-1||_F ||D R^-1||_F of a first CholeskyQR
 * round (D = column norms), and the number of second CholeskyQR rounds run. */
wssr_status wssr_status_sync(wssr_handle h, int32_t* numeric_status, double* diag);

/* Text of the last host-side error on this handle (never NULL). */
const char* wssr_last_error(wssr_handle h);

/* Stage timing for benchmarks.  wssr_profile(h, 1) clears the counters and
 * starts recording a pair of HIP events on the handle's stream around every
 * launch of the two data-matrix products (the sample-side product with its
 * split-K reduction excluded, and the parameter-side product); 0 stops.
 * wssr_profile_read synchronises the stream and returns, per slot, the summed
 * milliseconds and the launch count: slot 0 = sample-side product kernel,
 * slot 1 = parameter-side product kernel, slot 2 = wssr_spring's product
 * T = O O^T (with its chunk reduction), slot 3 = wssr_spring's blocked
 * Cholesky (all its launches as one interval).  nslots <= 4. */
wssr_status wssr_profile(wssr_handle h, int32_t enable);
wssr_status wssr_profile_read(wssr_handle h, double* ms, int64_t* counts, int32_t nslots);

/* Adaptive rank (Sec. 4.3, eq. ruler).  With r_reg > 0 the steps that follow
 * keep in the preconditioned direction only the columns j with
 * sigma_j^2 >= r_reg sigma_1^2 (the ratio on the eigenvalues of S): the
 * damped weights of the others are 0, and in the floor form they take the
 * floor 1/lambda (eq. updated_sr_1 with U of that rank).  V and sigma still
 * return all r columns (the warm start and the averaged state keep them).
 * 0 <= r_reg < 1; 0 (the default) keeps every column.  Applies to the
 * handle's batch lanes too. */
wssr_status wssr_set_rank_ratio(wssr_handle h, double r_reg);

/* After a step: *r_eff = the rank eq. ruler kept, *grow = 1 when the last
 * computed column passed the ratio (the paper's condition for growing r_max:
 * the caller then pads V with new columns and steps at the larger rank; any
 * full-rank basis is a valid warm start).  Synchronises the handle's stream. */
wssr_status wssr_rank_info(wssr_handle h, int32_t* r_eff, int32_t* grow);

/* Library version string, e.g. "libwssr 0.1 gfx950". */
const char* wssr_version(void);

/* ---------------------------------------------------------------------------
 * Single-kernel entry points, for checking each stage on its own.  Same
 * conventions as wssr_step (device pointers, handle stream, host-side argument
 * checks); sizes must fit the handle's capacities.
 * ------------------------------------------------------------------------- */

/* y = A V = (O - 1 mu^T) V / sqrt(n)   (Alg. 1, the product with the data
 * matrix on the parameter-side block).  V float[m x r]; y double[n x r]. */
wssr_status wssr_dbg_sample_side(wssr_handle h, int64_t n, int64_t m, const void* O,
                                 int64_t ld_o, const float* V, int32_t r, double* y);

/* z = O^T X / sqrt(n)   (Alg. 1, the product with the transposed data matrix).
 * X float[n x r]; z float[m x r].  Equals A^T X when the columns of X sum to 0. */
wssr_status wssr_dbg_param_side(wssr_handle h, int64_t n, int64_t m, const void* O,
                                int64_t ld_o, const float* X, int32_t r, float* z);

/* g = O_bar^T eps / n with eps = e_l - mean(e_l)  (eq. barg); g double[m]. */
wssr_status wssr_dbg_gradient(wssr_handle h, int64_t n, int64_t m, const void* O,
                              int64_t ld_o, const double* e_l, double* g);

/* CholeskyQR of a tall matrix X (rows x r, float): X = Q R with Q^T Q = I,
 * R upper triangular with positive diagonal (Alg. 1 "QR decomposition").  The
 * Gram matrix and the factors are FP64; a second round (CholeskyQR2) runs when
 * the first round's condition bound exceeds 1e4, as in wssr_step.  A
 * rank-deficient X is completed as in wssr_step (WSSR_WARN_RANK_DEFICIENT is
 * not raised here; Q R then equals X up to sqrt(r eps) max_j |x_j| in each
 * completed column).
 * Q float[rows x r]; R double[r x r] row-major.  rows <= max(n_max, m_max). */
wssr_status wssr_dbg_cholqr2(wssr_handle h, int64_t rows, const float* X, int32_t r,
                             float* Q, double* R);

/* Gram matrix G = X^T X (X float[rows x r] row-major, G double[r x r]) as
 * the step forms it for a parameter-side block Z: kind 0 on the FP64 MFMA
 * (exact products, FP64 sums; the CholeskyQR2); kind 1 on the FP32 MFMA,
 * FP32 sums flushed into FP64 every 256 rows (entries to about 1e-7 relative
 * to sqrt(G_ii G_jj); the last pass's probe); kind 2 on the BF16 MFMA, each
 * element split into two BF16 planes and the four products summed in FP32,
 * flushed into FP64 every 256 rows (about 3e-7; the intermediate passes'
 * probe, where only a span is carried on).  WSSR_ERR_INVALID_ARG for another
 * kind.  rows <= max(n_max, m_max). */
wssr_status wssr_dbg_gram(wssr_handle h, int64_t rows, const float* X, int32_t r, int32_t kind, double* G);

/* The basis an intermediate pass carries on from Z = X (float[rows x r]): V
 * (float[rows x r]) spans the columns of X, and *mode (device int32) says how
 * it was made: 0 the columns scaled to unit norm (they were orthogonal), 1
 * X R^{-1} from the FP32-MFMA Gram, 2 the FP64 CholeskyQR2.  rows <= m_max. */
wssr_status wssr_dbg_span_basis(wssr_handle h, int64_t rows, const float* X, int32_t r, float* V, int32_t* mode);

/* SVD of a small square matrix C (r x r, double, row-major): C = G diag(s) P^T
 * by block one-sided Jacobi.  s double[r] descending; P double[r x r] row-major. */
wssr_status wssr_dbg_small_svd(wssr_handle h, const double* C, int32_t r, double* s, double* P);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the r x r
 * SVD of wssr_dbg_small_svd without a handle and without any allocation.
 * Its working arrays live in a fixed device array of about 8.4 MB that the
 * library holds on each device it runs on until the process ends.
 *   C       device, double[r x r] row-major, read only
 *   r       1 <= r <= 512 (larger: WSSR_ERR_INVALID_ARG, nothing enqueued)
 *   s       device, double[r], out: singular values, descending
 *   P       device, double[r x r] row-major, out: right singular vectors (C = G diag(s) P^T)
 *   status  device, int32 or NULL: out, the numerical status (WSSR_OK,
 *           WSSR_WARN_NOT_CONVERGED, WSSR_ERR_NONFINITE, WSSR_ERR_TIMEOUT)
 *   stream  hipStream_t the work is enqueued on (NULL: the null stream)
 * Runs on the current HIP device.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (other streams,
 * other threads) race and must not be issued.  Returns WSSR_ERR_NO_DEVICE or
 * WSSR_ERR_HIP when the set-up (first call on a device) or a launch fails. */
wssr_status wssr_small_svd_noalloc(const double* C, int32_t r, double* s, double* P, int32_t* status,
                                   void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WSSR_H */
