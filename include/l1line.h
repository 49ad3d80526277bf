/*
 * l1line.h -- C ABI of the MI355X (gfx950) library for the sparse robust
 * l1 best-fit line of Ling & Brooks, "l1-Norm Regularized l1-Norm Best-Fit
 * Lines" (Sec. 2: LP (3), Lemma 1, Algorithm 1).
 *
 * THE METHOD
 *   X is n x m (rows = points, columns = coordinates).  For every preserved
 *   coordinate j the LP (3) separates (proof of Lemma 1, LP (4)) into m-1
 *   one-dimensional problems, one per other column k:
 *     v_k = argmin_v  sum_{i: x_ij != 0} |x_ij| |x_ik/x_ij - v| + lambda |v|
 *   -- a weighted median of the n ratios plus the point 0 with weight lambda.
 *   Algorithm 1 sets v_j = 1, scores
 *     z_j = sum_i sum_k |x_ik - v_k x_ij| + lambda sum_k |v_k|
 *   and returns the v of the smallest z_j.
 *
 * CONVENTIONS (identical in every entry point)
 *   - X is column-major: x(i,k) = X[i + k*ld], ld >= n, FP64, a DEVICE
 *     pointer.  Every other array argument is a DEVICE pointer too unless
 *     its comment says HOST.  The caller allocates and frees all of them;
 *     the library only owns the workspace inside its context.
 *   - Indices are 0-based.  Penalties lambda are FP64, finite and >= 0.
 *   - Ratios are r_i = fl(x_ik / x_ij) (IEEE division, round to nearest),
 *     -0 taken as +0, ordered by (r_i, i).
 *   - Every weight sum and every comparison of such sums with lambda is
 *     exact (128-bit fixed point per column), so v_k is the exact weighted
 *     median of the rounded ratios.  Among equal minimisers: v_k = 0 when 0
 *     is a minimiser, else the minimiser closest to 0; the reported median
 *     row is the position meeting Lemma 1's condition that lies nearest 0.
 *   - Reported sums (z_j, e_jk, column masses) use the fixed order R64:
 *     term t added to partial (t mod 64) in increasing t, then
 *     p[l] += p[l+d] for d = 32..1; residual terms |x_ik - fl(v_k x_ij)|
 *     with no fused multiply-add.  z_j = E_j + fl(lambda * P_j).
 *   - j* = the smallest index among the minimal z_j (Algorithm 1's strict
 *     "<" over ascending j).
 *   - All calls are asynchronous on `stream` (a hipStream_t; NULL = the
 *     default stream) and copy nothing back to the host.  Calls on one
 *     context must be issued on one stream (or serialised by the caller):
 *     they share the context's workspace.
 *
 * ERRORS
 *   Every entry point returns an int: 0 on success, a negative code below.
 *   Argument errors are found on the host, before anything is launched.
 *   Data-dependent conditions are found on the device and written to the
 *   optional `status` output (one int32, device memory): 0, or the first
 *   that applies of ENONFINITE, EWIDE, EINTERNAL, ERANGE.  With a nonzero
 *   status the other outputs are unspecified.  The context also keeps a
 *   sticky error: the first nonzero code an entry point returned, else the
 *   first data-dependent status any call produced (l1line_last_error).
 */
#ifndef L1LINE_H
#define L1LINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define L1LINE_OK 0
#define L1LINE_EINVAL (-1)     /* bad argument (host check)                          */
#define L1LINE_EHIP (-2)       /* a HIP runtime call failed                          */
#define L1LINE_ENONFINITE (-3) /* X holds a NaN or an infinity (device check)        */
#define L1LINE_ERANGE (-4)     /* a selected ratio overflowed to +-inf (device)      */
#define L1LINE_ENOMEM (-5)     /* workspace allocation failed                        */
#define L1LINE_EWIDE (-6)      /* a column's nonzero magnitudes span too many binades
                                  for exact 128-bit weight sums: (highest bit - lowest
                                  bit + 1) + bitlength(#nonzeros) > 124 (device)     */
#define L1LINE_ESIZE (-7)      /* n above L1LINE_MAX_N (L1LINE_BP_MAX_N for Algorithms 2 and 3), or m
                                  above L1LINE_RANKER_MAX_M for the ranker (host check) */
#define L1LINE_EINTERNAL (-8)  /* a selection exceeded its round bound (device)      */
#define L1LINE_EIO (-9)        /* a file could not be read or written, or is malformed */
#define L1LINE_ENOMODEL (-10)  /* the context holds no ranker weights                */

#define L1LINE_MAX_N 65535         /* rows per matrix: the segment lists hold 16-bit row ids, and
                                      with fewer than 2^16 nonzeros per column the 37-bit chunk
                                      sums of the exact weights stay below 2^53 */
#define L1LINE_BP_MAX_N 16384      /* rows per matrix for l1line_breakpoints and
                                      l1line_solution_path (ESIZE above)           */
#define L1LINE_MAX_LAMBDAS 128     /* penalties per call (passed by value)        */

typedef struct l1line_ctx_s *l1line_ctx;

/* Create a context on HIP device `device` (its workspace starts empty and
 * grows on demand; it owns the launch parameters and the ranker weights).
 * *ctx receives the handle.  tune_cache_path (HOST string, nullable): a
 * file holding launch parameters, read here when it exists and written by
 * l1line_autotune.  Returns EINVAL for a bad device or null ctx, EHIP if the
 * device cannot be selected. */
int l1line_create(l1line_ctx *ctx, int device, const char *tune_cache_path);

/* Free the context's workspace (synchronises its device first). */
int l1line_destroy(l1line_ctx ctx);

/* The context's sticky error, then cleared: the first nonzero code an entry
 * point returned on it since the last call, else the first data-dependent
 * status (ENONFINITE, EWIDE, EINTERNAL, ERANGE) of any call, else 0.  Reads a
 * device word synchronously: call it after the work's stream has finished. */
int l1line_last_error(l1line_ctx ctx);

/* Human-readable name of a status code (static string, never NULL). */
const char *l1line_strerror(int code);

/* Column statistics (feed the penalty scale Lambda = max_j W_j):
 *   W[j]     = R64 sum over i of |x_ij|           (m doubles, nullable)
 *   zeros[j] = #{i : x_ij == 0}                    (m int32, nullable)
 *   status   = 0 or ENONFINITE                     (nullable) */
int l1line_column_stats(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                        int64_t ld, double *W, int32_t *zeros, int32_t *status,
                        void *stream);

/* Algorithm 1 for one penalty (Sec. 2, Algorithm 1; Lemma 1 per column).
 *   lambda       HOST value, finite, >= 0
 *   v            [m]  v* with v[j*] = 1 exactly
 *   j            [1]  j* (int64)
 *   obj          [1]  z_{j*}
 *   median_row   [m]  row i whose ratio gave v*_k; -1 when v*_k = 0 and at
 *                     k = j* (nullable)
 *   z_all        [m]  z_j for every candidate j (nullable)
 *   status       [1]  device status (nullable)
 * Host errors: EINVAL (n<1, m<1, ld<n, null X/v/j/obj, bad lambda), ESIZE
 * (n > L1LINE_MAX_N), ENOMEM, EHIP. */
int l1line_fit(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
               int64_t ld, double lambda, double *v, int64_t *j, double *obj,
               int32_t *median_row, double *z_all, int32_t *status,
               void *stream);

/* For callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, arguments, outputs and errors as l1line_fit, with the
 * workspace in a fixed device array of L1LINE_NOALLOC_SCRATCH_MB MiB that the
 * library holds on every GPU it runs on until the process ends.  The call
 * allocates nothing (no hipMalloc / hipFree, no pinned staging: its metadata
 * travels as kernel arguments).  The workspace needs about 36 m^2 + 64 m
 * bytes plus a few KB, so m <= L1LINE_NOALLOC_MAX_M (n up to L1LINE_MAX_N).
 * Every call on one GPU, from any context, stream or thread, shares that
 * GPU's array and leaves its contents there; each call re-initialises what
 * it reads.  Calls that overlap in time on the same GPU race: the caller
 * must serialise them (one stream, or events).  Host errors: as l1line_fit,
 * plus ESIZE for m > L1LINE_NOALLOC_MAX_M and EHIP when the array's device
 * address could not be obtained when the context was created. */
#define L1LINE_NOALLOC_SCRATCH_MB 40
#define L1LINE_NOALLOC_MAX_M 1024
int l1line_fit_noalloc(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                       int64_t ld, double lambda, double *v, int64_t *j,
                       double *obj, int32_t *median_row, double *z_all,
                       int32_t *status, void *stream);

/* Algorithm 1 along a path of L penalties, each ratio list built once per
 * (j, k) and reused for every lambda (the solution for each lambda is the
 * one l1line_fit returns for it, bit for bit).
 *   lambdas  HOST array of L values (1 <= L <= L1LINE_MAX_LAMBDAS)
 *   V        [L*m]  row t = v*(lambda_t)
 *   J        [L]    j*(lambda_t)
 *   OBJ      [L]    z_{j*}(lambda_t)
 *   ROW      [L*m]  median rows (nullable)
 *   ZALL     [L*m]  row t = z_j(lambda_t) for every j (nullable)
 *   status   [1]    (nullable) */
int l1line_fit_path(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                    int64_t ld, const double *lambdas, int64_t L, double *V,
                    int64_t *J, double *OBJ, int32_t *ROW, double *ZALL,
                    int32_t *status, void *stream);

/* One problem of a batch.  Same conventions as l1line_fit_path. */
typedef struct {
  const double *X;        /* DEVICE, n x m column-major, leading dimension ld */
  int64_t n, m, ld;
  const double *lambdas;  /* HOST, L penalties (1 <= L <= L1LINE_MAX_LAMBDAS) */
  int64_t L;
  double *V;              /* DEVICE [L*m]  v*(lambda_t), row t              */
  int64_t *J;             /* DEVICE [L]    j*(lambda_t)                     */
  double *OBJ;            /* DEVICE [L]    z_{j*}(lambda_t)                 */
  int32_t *ROW;           /* DEVICE [L*m]  median rows (nullable)           */
  double *ZALL;           /* DEVICE [L*m]  z_j(lambda_t) (nullable)         */
  int32_t *status;        /* DEVICE [1]    device status (nullable)         */
} l1line_problem;

/* Flag of l1line_fit_batch: capture the launch sequence into a HIP graph the
 * first time a batch layout (the problems' pointers, sizes and penalties) is
 * seen, and replay it while the same layout is submitted again.  The first
 * call with a new layout waits for its metadata copy (host synchronisation). */
#define L1LINE_BATCH_GRAPH 1

/* Algorithm 1 (with a lambda path each) for B independent matrices of
 * uneven sizes in one launch sequence: a persistent segment kernel pulls
 * (matrix, j, k-range) work items, largest first, from a device counter.
 *   probs  HOST array of B problem descriptors (read during the call only)
 *   flags  0 or L1LINE_BATCH_GRAPH
 * Each problem's outputs equal those of l1line_fit_path on it, bit for bit.
 * Host errors: EINVAL (bad flags, B < 1, any problem failing the checks of
 * l1line_fit_path), ESIZE, ENOMEM, EHIP. */
int l1line_fit_batch(l1line_ctx ctx, const l1line_problem *probs, int64_t B,
                     int flags, void *stream);

/* Autotuner.  Launch parameters are kept per size class: one problem or a
 * batch, one penalty or several, and the bit lengths of the largest n, the
 * largest m and (halved) the total work sum n m^2 L.  l1line_autotune runs
 * the given problems under every candidate of a small grid (persistent
 * workgroups per compute unit {2,3,4} x fewest k per work item {8,32,128},
 * or {64,256,512} for one problem, x work items per compute unit
 * {12,24,48} for a batch), times the segment kernel with HIP events, and
 * stores the fastest as the entry of their size class: every later call
 * of that class (fit, path, batch, ranked fit, breakpoints, components,
 * solution path) launches with it; other classes keep the default.  The
 * entry also goes to the context's cache file (keyed by the device's
 * architecture name; read by l1line_create), and to params_out (HOST [3],
 * nullable).  Results never depend on the parameters.  Synchronises the
 * stream. */
int l1line_autotune(l1line_ctx ctx, const l1line_problem *probs, int64_t B,
                    void *stream, int32_t *params_out);

/* Read / set the context's default launch parameters, used for size
 * classes without a tuned entry (HOST [3]: workgroups per CU in [1, 16],
 * fewest k per item >= 1, items per CU in [1, 4096]; initially 4, 8, 24:
 * four 256-thread workgroups per CU fill the four wave slots per SIMD that
 * the segment kernel's registers allow wherever its LDS leaves room). */
int l1line_tune_get(l1line_ctx ctx, int32_t *params);
int l1line_tune_set(l1line_ctx ctx, const int32_t *params);

/* The launch parameters a call with these problems uses (HOST [3]) and
 * whether they are a tuned entry of its size class (tuned, HOST [1],
 * nullable: 1 tuned, 0 default).  EINVAL as l1line_fit_batch. */
int l1line_tune_lookup(l1line_ctx ctx, const l1line_problem *probs, int64_t B,
                       int32_t *params, int32_t *tuned);

/* ------------------------------------------------------------------------
 * Learned candidate ranker.  Exhaustive search solves every preserved
 * coordinate j (Algorithm 1); the ranker scores the columns with a small MLP
 * and solves only the K best exactly, falling back to the exhaustive search
 * when the scores do not separate the candidates from the rest.
 * ---------------------------------------------------------------------- */
#define L1LINE_FEATURES 32        /* features per column                     */
#define L1LINE_MLP_PARAMS 20865   /* FP32 parameters of the 32-128-128-1 MLP:
                                     W1[32][128], b1[128], W2[128][128],
                                     b2[128], W3[128], b3 (in this order)     */

/* Per-column features F [m][32] (FP32, DEVICE).  With D_jk = sum_i x_ij
 * sgn(x_ik) and Zr_jk = sum_i |x_ij| [x_ik == 0] (the weight balance of the
 * ratios x_ik / x_ij over all rows, Lemma 1 of Sec. 2; here as computed by
 * l1line_ranker_signsums), the segment (j, k) has v_k != 0
 * exactly when its initial slope s_jk = |D_jk| - Zr_jk - lambda is > 0, and
 * z_j = sum_k W_k - W_j + lambda - sum_k Delta_jk with Delta_jk >= 0 the
 * segment's improvement over v_k = 0.  Per column j (W = column l1 mass):
 *   A1 = sum_k s_jk, A2 = sum_k s_jk^2 / W_k, A3 = sum_k s_jk / W_k,
 *   A4 = #{k != j : s_jk > 0}, over the k with s_jk > 0; then
 *   f0 (W - mean W) / sd W        f1 (W - max W) / sd W     f2 log(W / mean W)
 *   f3 zero fraction of column j  f4 min(lambda / W, 10)     f5 A4 / (m - 1)
 *   f6, f8, f10, f12  (A_q - mean A_q) / sd A_q     (q = 1..4)
 *   f7, f9, f11, f13  (A_q - max A_q) / sd A_q
 *   f14 log1p(A1 / W)             f15 1;  f16-31 = 0
 * (mean, sd, max over the m columns; 0 where sd = 0; f2 = -30, f4 = 10 and
 * f14 = 0 for W = 0).  m <= L1LINE_RANKER_MAX_M, else ESIZE. */
#define L1LINE_RANKER_MAX_M 65536
int l1line_ranker_features(l1line_ctx ctx, const double *X, int64_t n,
                           int64_t m, int64_t ld, double lambda, float *F,
                           void *stream);

/* The sign sums behind the features: DZ [m][m][2] (FP64, DEVICE, caller
 * owned), DZ[(j m + k) 2] = D_jk, DZ[(j m + k) 2 + 1] = Zr_jk as above (the
 * weight balance of Lemma 1, Sec. 2).  They only rank the columns, so they run
 * on the BF16 matrix units: column j scaled by the power of two that brings
 * its largest magnitude into [1, 2), each value split into BF16 parts h + l
 * (|x - h - l| <= 2^-15 |x|), FP32 accumulation over the rows.  Bounds, with
 * W_j = sum_i |x_ij| and u = 2^-24:
 *   |D_jk - exact|  <= (2^-15 + 2 n u) W_j
 *   |Zr_jk - exact| <= (2^-8 + 2 n u) Zr_jk(exact)   (h alone; terms >= 0)
 * (up to magnitudes 2^-126 below the column's largest, flushed to 0).  The
 * exact solve never uses these: it computes its own in FP64.  Errors as
 * l1line_ranker_features; m <= L1LINE_RANKER_MAX_M, else ESIZE. */
int l1line_ranker_signsums(l1line_ctx ctx, const double *X, int64_t n,
                           int64_t m, int64_t ld, double *DZ, void *stream);

/* MLP forward: out[r] = MLP(F[r]) for N rows (all DEVICE).  Matrix products
 * take BF16 operands (features, weights, hidden activations rounded to
 * nearest-even BF16) on the MFMA units with FP32 accumulation:
 *   H1 = bf16(relu(F W1 + b1)), H2 = bf16(relu(H1 W2 + b2)),
 *   out = H2 . bf16(W3) + b3. */
int l1line_mlp_forward(l1line_ctx ctx, const float *params, const float *F,
                       int64_t N, float *out, void *stream);

/* Gradient of the loss mean_r (out[r] - y[r])^2 with respect to the
 * parameters (grad [L1LINE_MLP_PARAMS], loss [1], DEVICE).  Deterministic:
 * per-tile partials are added in a fixed order. */
int l1line_mlp_grad(l1line_ctx ctx, const float *params, const float *F,
                    const float *y, int64_t N, float *grad, float *loss,
                    void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * on the FP32 master parameters with moments m1, m2 (all DEVICE). */
int l1line_mlp_adam(l1line_ctx ctx, float *params, float *m1, float *m2,
                    const float *grad, int64_t step, float lr, void *stream);

/* Ranked fit with the context's ranker weights: features, MLP scores (lower
 * = better candidate), the K best columns solved exactly by Algorithm 1
 * restricted to them; if the score gap between the best column and the
 * first one left out is below margin_threshold (or K = m) the exhaustive
 * search runs instead (decided on the device, no host synchronisation; the
 * FP32 score gap is compared with the threshold in double).
 *   v, j, obj, median_row, status  as l1line_fit (DEVICE)
 *   used_fallback  [1] 1 when the exhaustive search ran (DEVICE, nullable)
 *   scores         [m] the MLP scores (DEVICE, nullable)
 * Host errors: as l1line_fit, EINVAL for K outside [1, m] or a negative or
 * non-finite threshold, ESIZE for m > L1LINE_RANKER_MAX_M, ENOMODEL when no
 * weights were loaded, set or trained. */
int l1line_fit_ranked(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                      int64_t ld, double lambda, int32_t K,
                      double margin_threshold, double *v, int64_t *j,
                      double *obj, int32_t *median_row,
                      int32_t *used_fallback, float *scores, int32_t *status,
                      void *stream);

/* Ranker weights owned by the context.
 * File format (little endian): "L1RK", u32 version 1, u32 parameter count
 * (L1LINE_MLP_PARAMS), u32 flags (bit 0: Adam state follows), i64 steps
 * taken, u64 training seed, u64 next training example; FP32 weights; with
 * bit 0 the FP32 Adam moments m1 and m2.
 * l1line_ranker_load: weights (and state) from `path` (HOST string); EIO for
 *   a missing, short or malformed file or non-finite weights.
 * l1line_ranker_save: writes the weights (and the state after training) to
 *   `path` atomically (a temporary file renamed); ENOMODEL without weights.
 * l1line_ranker_set_params / get_params: copy L1LINE_MLP_PARAMS FP32 weights
 *   from / to DEVICE memory on `stream` (set clears the Adam state). */
int l1line_ranker_load(l1line_ctx ctx, const char *path);
int l1line_ranker_save(l1line_ctx ctx, const char *path);
int l1line_ranker_set_params(l1line_ctx ctx, const float *params, void *stream);
int l1line_ranker_get_params(l1line_ctx ctx, float *params, void *stream);

/* Train the context's ranker until `steps` Adam steps have been taken in
 * total, one step per generated matrix: n ~ U{500..4000}, m ~ U{50..500}
 * (sizes from splitmix64 of (seed, example)), entries from Philox-4x32-10
 * keyed by (seed, example): x_ik = u_i l_k + Laplace(0, 0.1) noise, l_k ~
 * U[-1, 1] on 10% of the columns, 10% of the rows replaced by 20 N(0, 1),
 * 1% zeros; lambda = 0.05 x max column mass.  Labels: the exact z_j of the
 * exhaustive fit, as y_j = (z_j - min z) / (mean z - min z); loss: mean
 * squared error of the MLP; Adam (lr 1e-3).  ckpt_path (HOST string,
 * nullable): resumed from when it exists (the seed is then the file's),
 * rewritten every 1000 steps and at the end; the run is deterministic, so a
 * resumed run ends with the same weights as an uninterrupted one.
 * Synchronous (uses the default stream).  EIO for an unreadable checkpoint
 * or one without Adam state. */
int l1line_ranker_train(l1line_ctx ctx, const char *ckpt_path, int64_t steps,
                        uint64_t seed);

/* ------------------------------------------------------------------------
 * Algorithm 2 (Sec. 2): the breakpoints of every segment's solution path.
 * For preserved column j and column k (segment g = j*m + k), v_k(lambda) of
 * Algorithm 1 (tie rule as above) is piecewise constant in lambda; its
 * entries, in increasing lambda, are (lam, v, row) triples: v_k = v (median
 * row `row`) for lambda in [lam[t], lam[t+1]), starting at lam = 0, and a
 * terminal entry (lambda_max, 0, -1) from which v_k = 0.  With the points
 * sorted by (ratio, row), exact prefix weights S_p, W = sum of the weights,
 * A = weight of the negative ratios, B = A + weight of the zero ratios:
 *   negative side (2A > W): points p from the lambda = 0 minimiser up to the
 *     last negative one, lam = max(0, 2 S_{p-1} - W); lambda_max = 2A - W;
 *   positive side (W > 2B): points from the lambda = 0 minimiser down to the
 *     first positive one, lam = max(0, W - 2 S_p); lambda_max = W - 2B;
 *   otherwise the single entry (0, 0, -1).
 * These are Algorithm 2's lambda_p = sgn(r_p)(weight after p - weight before
 * p) - w_p kept where lambda_p + 2 w_p > 0, zero ratios left out (they never
 * move the minimiser off 0).  Each lam is exact and rounded once to the
 * nearest double.  Segments with j = k, and every segment of a column j
 * with a NaN, an infinity or too wide a range, have no entries.
 *   offsets     [m*m + 1] int64 (DEVICE, required): entries of segment g are
 *               [offsets[g], offsets[g+1]); offsets[m*m] = total entries
 *   lambda_max  [m*m] (DEVICE, nullable); 0 where a segment has no entries
 *   lam, v, row [capacity] (DEVICE; nullable when capacity = 0)
 *   status      as l1line_fit, and ESIZE (nothing written to lam, v, row)
 *               when the total exceeds capacity
 * Usage: a call with capacity 0 fills offsets; read offsets[m*m], size the
 * arrays, call again.  A call with capacity > 0 also keeps in the context
 * up to 1296 bytes per segment (each segment's entries of at most 128, so
 * that they are not searched for twice) when m*m*1296 bytes stay within
 * 6 GiB; where that cannot be allocated the call runs without it.  Host
 * errors: as l1line_fit; ESIZE for m > L1LINE_BP_MAX_M. */
#define L1LINE_BP_MAX_M 8192
int l1line_breakpoints(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                       int64_t ld, int64_t *offsets, double *lambda_max,
                       double *lam, double *v, int32_t *row, int64_t capacity,
                       int32_t *status, void *stream);

/* ------------------------------------------------------------------------
 * Successive components (Sec. 2, after Algorithm 3: further components come
 * from Algorithm 1 applied to the data projected onto the null space of the
 * components found so far).  With X_0 = X and the same lambda throughout:
 *   component c = Algorithm 1 on X_c  ->  V[c*m ..], J[c], OBJ[c]
 *   w_c = v_c made orthogonal to w_0 .. w_{c-1} (classical Gram-Schmidt,
 *         unnormalised: w_k = fl(w_k - fl(fl(R64(w_l . v_c) / |w_l|^2) w_lk)))
 *   X_c+1: x_ik = fl(x_ik - fl(s_i u_k)), s_i = R64_k fl(x_ik w_ck),
 *          u_k = fl(w_ck / |w_c|^2), |w|^2 = R64_k fl(w_k w_k)
 * (products rounded on their own, R64 as above).
 *   p      1 <= p <= min(m, L1LINE_MAX_COMPONENTS)
 *   work   [n*m] DEVICE scratch owned by the caller (column-major, ld = n);
 *          holds X_{p-1} on return
 *   V [p*m], J [p], OBJ [p]  DEVICE outputs; OBJ[c] is z on X_c
 *   status (nullable): the first fit status other than ERANGE in component
 *          order (ERANGE is kept if nothing else occurs), or EINVAL when a
 *          component lies in the span of the earlier ones (its projection
 *          is 0; the later outputs are then unspecified).
 * Host errors: as l1line_fit, EINVAL for a bad p or a null pointer. */
#define L1LINE_MAX_COMPONENTS 1024
int l1line_components(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                      int64_t ld, double lambda, int64_t p, double *work,
                      double *V, int64_t *J, double *OBJ, int32_t *status,
                      void *stream);

/* Algorithm 3 (Sec. 2; Table I for the worked example): the exact solution
 * path z*(lambda), v*(lambda) over every lambda >= 0, merged over the
 * preserved coordinates from the per-coordinate paths of Algorithm 2.
 *
 * For a preserved coordinate j, Algorithm 2's entries (l1line_breakpoints)
 * fix every v_k between breakpoints; entry t of segment (j, k) holds for
 * lambda >= its breakpoint (the double it reports), entries at equal lambda
 * applying in (k, t) order.  With them z_j is the line E_j + lambda P_j,
 * E_j = sum_k e_jk(v_k) (each e_jk the R64 residual Algorithm 1 reports) and
 * P_j = 1 + sum_{k != j} |v_k|, both summed EXACTLY.  The path follows the
 * lowest line (value, then slope, then the lower j) through every lambda:
 * the preserved coordinate changes where lines cross (the crossings the
 * paper's Algorithm 3 adds), each crossing compared exactly and reported
 * rounded once to the nearest double.
 *
 * Output: `count` records in lambda order (DEVICE arrays of `capacity`):
 *   lam[r]  where the change happens
 *   j[r]    the preserved coordinate from there on
 *   k[r], v[r], row[r]  coordinate k of v* becomes v (row: its median row,
 *           -1 when v is 0 and for k = j, where v = 1)
 *   E[r], P[r]  z*(lambda) = E + lambda P from there on (each rounded once)
 * The start (lambda = 0) and every change of the preserved coordinate list
 * all m coordinates k = 0..m-1 at one lambda; otherwise each record is one
 * breakpoint entry of the current j.  Replaying the records up to lambda gives
 * v*(lambda); lambda beyond the last record keeps the last line.
 *
 *   count    HOST: the number of records (always written on success)
 *   capacity records the outputs hold; 0 (outputs may be null) only counts
 *   status   nullable DEVICE int32: 0 or the error returned
 * Synchronous in part: the call waits for `stream` to learn the count; the
 * records are written asynchronously after it returns.
 * Errors (returned): EINVAL (arguments, null count), ESIZE (m above
 * L1LINE_BP_MAX_M, more than 2^32 - 1 breakpoint entries, or count above
 * a nonzero capacity: nothing is written, count holds the size needed),
 * ENONFINITE / EWIDE as l1line_fit, EWIDE also when some residual or |v| has
 * bits more than 110 places below the largest (the exact lines would not fit
 * 128 bits), ENOMEM for the workspace: about 120 bytes per breakpoint entry
 * plus 28 bytes per (tile, column) for 4096 tiles (and, when it can be had,
 * the per-segment entry lists of l1line_breakpoints). */
int l1line_solution_path(l1line_ctx ctx, const double *X, int64_t n, int64_t m,
                         int64_t ld, int64_t capacity, int64_t *count,
                         double *lam, int64_t *j, int32_t *k, double *v,
                         int32_t *row, double *E, double *P, int32_t *status,
                         void *stream);

/* Measured ceilings of the device, for roofline figures (microbenchmarks,
 * best of 3 timed runs each after a warm-up):
 *   out[0] HBM copy bandwidth, GB/s (bytes read + written; 1 GiB buffers)
 *   out[1] LDS read bandwidth, GB/s (16-byte reads, conflict-free)
 *   out[2] FP64 VALU, TFLOP/s (independent FMA chains, 2 flops each)
 *   out[3] FP64 matrix, TFLOP/s (v_mfma_f64_16x16x4f64)
 *   out[4] BF16 matrix, TFLOP/s (v_mfma_f32_16x16x32_bf16)
 * out is a HOST array of L1LINE_PEAKS doubles.  Synchronous; allocates and
 * frees 2 GiB of scratch.  Errors: EINVAL (null), ENOMEM, EHIP. */
#define L1LINE_PEAKS 5
int l1line_measure_peaks(l1line_ctx ctx, double *out);

/* Kernel timing for measurement tools.  While enabled, every kernel the
 * context launches is bracketed by HIP events on its stream.
 * l1line_profile_read waits for the recorded events, returns the summed
 * duration (ms) and launch count of the kernels whose name is `kernel`
 * ("colprep", "signsum", "zero_seg", "fit_seg", "reduce", "argmin", "features",
 * "mlp_fwd", "mlp_bwd", "bp_count", "bp_emit", "sp_resid", "sp_delta",
 * "sp_sort", "sp_bounds", "sp_sweep"; NULL = all), and with
 * reset != 0
 * forgets every record.  Outputs are HOST pointers (nullable). */
int l1line_profile(l1line_ctx ctx, int enable);
int l1line_profile_read(l1line_ctx ctx, const char *kernel, double *total_ms,
                        int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* L1LINE_H */
