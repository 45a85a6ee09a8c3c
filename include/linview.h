/*
 * linview.h -- C ABI of an MI355X (gfx950) library that keeps matrix-power
 * views P = A^k current under low-rank updates of A.
 *
 * Method (LINVIEW, Nikolic, ElSeidy, Koch, arXiv 1403.6968):
 *  - A view of A^k, k = 2^m, stores every power of the exponential model,
 *    P_1 = A, P_2, P_4, ..., P_k with P_i = P_{i/2} P_{i/2}
 *    (Table 1, "Exponential"; Sec. 5.2).  The library numbers them by level
 *    j = 0..m, level j holding A^(2^j).
 *  - An update Delta A = U V^T (Sec. 4.2, factored form) is propagated with
 *    the compact two-block factors of Sec. 4.3 / App. A (exponential model):
 *        U_{2i} = [U_i, P_i U_i + U_i (V_i^T U_i)],   V_{2i} = [P_i^T V_i, V_i]
 *    computed from the OLD powers, after which every stored power takes
 *    P_i += U_i V_i^T (the trigger of Sec. 4.4 assigns all factors first and
 *    then applies all updates).
 *  - Re-evaluation (ReevalExp, Sec. 5.2.2 "Re-evaluation") applies Delta A
 *    and recomputes the m squarings with dense products.
 *
 * Conventions for every entry point:
 *  - Matrices are dense, row-major, with a leading dimension (elements per
 *    row) ld >= n.  Element type: double in LV_FP64 mode, float in LV_FP32
 *    and LV_FP32_BF16SHADOW modes.  A, U, V and outputs use the view's
 *    element type.
 *  - Device pointers unless stated otherwise.  `stream` is a hipStream_t
 *    (NULL = the default stream).  All device work is enqueued on `stream`
 *    and is asynchronous: the caller keeps inputs unchanged and outputs
 *    unread until the stream has passed the call.
 *  - Ownership: the caller owns A, U, V, every output buffer and the device
 *    `workspace`; a view borrows its workspace for its lifetime.  The
 *    library never allocates device memory.  The lv_view handle itself is
 *    host memory owned by the library and freed by lv_view_destroy.
 *  - Errors: every call returns an lv_status; no exception crosses the ABI.
 *    On failure nothing has been enqueued unless the status is LV_EDEVICE.
 *    lv_last_error() returns a message for the last failure on the calling
 *    host thread.
 *  - A view is not thread-safe; distinct views are independent.
 */
#ifndef LINVIEW_H
#define LINVIEW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LV_OK = 0,
  LV_EINVAL = 1,  /* bad argument: k not a power of two, n or r out of range,
                     null pointer, ld < n, power not stored, ...            */
  LV_ENOMEM = 2,  /* workspace too small or misaligned                       */
  LV_EDEVICE = 3, /* a HIP runtime call or kernel launch failed              */
  LV_ESTATE = 4   /* operation not valid for this view                       */
} lv_status;

typedef enum {
  LV_FP64 = 0, /* double storage and arithmetic                           */
  LV_FP32 = 1, /* float storage and arithmetic; creation and re-anchoring
                  square in double and round once; Gram V^T U and the
                  factor assembly are accumulated in double                */
  LV_FP32_BF16SHADOW = 2
               /* float storage as LV_FP32, plus a bfloat16 copy (shadow)
                  of every stored power below the top, rewritten by the
                  pass that applies the rank update.  The tall-skinny
                  products P_j U_j and P_j^T V_j of the exponential model
                  (App. A) read the shadow and multiply on the matrix cores
                  (bfloat16 inputs, float accumulation); the rank update
                  itself, the Gram V^T U (double) and the factor assembly
                  are those of LV_FP32.  Element type at the API: float.
                  Re-evaluation (lv_reeval) does not take this mode.      */
} lv_mode;

typedef struct lv_view lv_view;

typedef struct {
  int64_t n;          /* matrix order                                      */
  int64_t n_pad;      /* padded order used on the device                   */
  int64_t ld;         /* leading dimension of the stored powers            */
  int32_t k;          /* view power                                        */
  int32_t levels;     /* m + 1 stored powers                               */
  int32_t r_max;      /* largest update rank accepted                      */
  int32_t mode;       /* lv_mode                                           */
  int64_t updates;    /* updates applied since creation                    */
  int64_t reanchors;  /* re-evaluations requested by lv_view_reanchor       */
  size_t footprint;   /* workspace bytes in use                            */
  int64_t drift_reanchors; /* re-evaluations triggered by drift checks     */
  double last_residual;    /* max_j rho_j of the last drift check          */
  int64_t drift_checks;    /* periodic drift checks run (enqueued)         */
  int64_t drift_every;     /* interval of the periodic check (0: off)      */
  double drift_tau;        /* its bound                                    */
} lv_stats;

/* Human-readable name of a status code (static string). */
const char* lv_status_str(lv_status s);

/* Message for the last failed call on this host thread ("" if none). */
const char* lv_last_error(void);

/* Exact workspace size in bytes for a view of order n, power k and largest
 * update rank r_max.  Returns 0 if the arguments are invalid (same rules as
 * lv_view_create).  The layout is: the m + 1 stored powers (padded order),
 * m + 1 factor slabs (U_j, V_j of every level), per-level reduction
 * partials, the bfloat16 shadows (LV_FP32_BF16SHADOW) and a double-precision
 * squaring scratch (both float modes). */
size_t lv_view_footprint(int64_t n, int k, int r_max, lv_mode mode);

/* Create a view of A^k (Table 1 exponential model; ReevalExp).
 *  A         n x n, leading dimension lda >= n (device).
 *  k         power of two, 1 <= k <= 1024 (the paper assumes log2 k
 *            integral, Table 1 caption).
 *  r_max     largest rank of later updates, 1 <= r_max; k * r_max, with
 *            r_max rounded up to a power of two, is the width of the top
 *            factors (App. A: the level-j factors have 2^j r columns) and
 *            must not exceed 512 for LV_FP32 and LV_FP32_BF16SHADOW views
 *            created without flags (level ranks up to 256, a rank-512 update
 *            of the top power), 256 otherwise (LV_FP64, LV_WITH_SUMS).
 *  workspace device buffer of ws_bytes >= lv_view_footprint(...), 256-byte
 *            aligned; borrowed until lv_view_destroy.
 *  out       receives the new handle (host).
 * All stored powers are computed by repeated squaring in double precision
 * on the device (MFMA) and then rounded once to the storage type. */
lv_status lv_view_create(const void* A, int64_t n, int64_t lda, int k, int r_max,
                         lv_mode mode, void* workspace, size_t ws_bytes,
                         void* stream, lv_view** out);

/* Creation flags.
 *  LV_WITH_SUMS  also maintain the sums of powers S_i = I + A + ... + A^(i-1)
 *                for i in {1, 2, 4, ..., k} (Sec. 5.2.3, Table 1, exponential
 *                model: S_1 = I, S_{2i} = P_i S_i + S_i).  Every update then
 *                also applies the factored deltas Delta S_i = Q_i W_i^T,
 *                obtained from the old powers and sums by the delta rule of
 *                Sec. 4.1:  Q_{2i} = [U_i, P_i Q_i + Q_i],
 *                W_{2i} = [S_i^T V_i + W_i (Q_i^T V_i), W_i],  Q_1 = W_1 = 0
 *                (U_i, V_i the factors of Delta P_i).  Creation and
 *                re-anchoring evaluate the sums by the recurrence in double
 *                precision and round once.  Such views are single-view only
 *                (lv_batch_create and servers reject them). */
#define LV_WITH_SUMS 1

/* lv_view_footprint / lv_view_create with creation flags (0 = as those). */
size_t lv_view_footprint_ex(int64_t n, int k, int r_max, lv_mode mode, int flags);
lv_status lv_view_create_ex(const void* A, int64_t n, int64_t lda, int k, int r_max,
                            lv_mode mode, int flags, void* workspace, size_t ws_bytes,
                            void* stream, lv_view** out);

/* Apply one update Delta A = U V^T (IncrExp, App. A exponential model; the
 * trigger of Sec. 4.4).
 *  U, V      n x r (device), leading dimensions ldu, ldv >= r.
 *  r         1 <= r <= r_max.
 * After the stream passes the call every stored power equals the
 * corresponding power of the updated A (up to rounding). */
lv_status lv_view_update(lv_view* v, const void* U, const void* V, int64_t r,
                         int64_t ldu, int64_t ldv, void* stream);

/* Apply `count` updates in order, (U_t, V_t) = (U + t*strideU, V + t*strideV)
 * for t = 0..count-1 (strides in elements).  The result equals `count`
 * calls of lv_view_update, bit for bit.  count >= 0.
 * Pipelining: for a view without sums or general form and with k >= 4,
 * level j of update t depends only on P_j after update t-1 and on the
 * factors that level j-1 of update t assembles (App. A), so the levels run
 * as up to four stages on streams of their own (stage 0 on `stream`; the
 * others are created on the first such call, on the current device) and
 * up to min(log2 k + 1, 5) successive updates are in flight, each with
 * a factor-slab pair of the workspace.  Every kernel sees the inputs of the
 * sequential order; the call returns with all stages joined into `stream`,
 * so stream order is as for one call of lv_view_update per update.  Not
 * used while kernel timing is on; a periodic drift check falling inside
 * the batch joins the stages first.  Two batches on one view must not
 * overlap (as for every call on a view). */
lv_status lv_view_update_batch(lv_view* v, const void* U, const void* V, int64_t r,
                               int64_t count, int64_t ldu, int64_t ldv,
                               int64_t strideU, int64_t strideV, void* stream);

/* Pick the view's tile rows (the same at every level) by measurement:
 * for each allowed height 256, 384, ..., 1024 times `trial_updates` zero
 * updates (U = V = 0, which leave every stored value and the update count
 * unchanged bit for bit) as lv_view_update_batch runs them, pipelined
 * (pipelined != 0) or one after the other, and keeps the fastest; *chosen
 * (may be NULL) receives it.  Blocks the host until the trials are done
 * (stream-ordered on `stream`).  The choice depends on the device's timing,
 * so two runs may choose differently; lv_view_set_tile_rows fixes a value.
 * Views without sums or general form (else LV_ESTATE); trial_updates in
 * [2, 1000]. */
lv_status lv_view_autotune(lv_view* v, int pipelined, int64_t trial_updates, void* stream, int* chosen);

/* Turn the pipelining of lv_view_update_batch on (default) or off
 * (enable = 0: every batch runs its updates one after the other on
 * `stream`; the results are the same bit for bit). */
lv_status lv_view_set_pipeline(lv_view* v, int enable);

/* Copy stored power A^power (power in {1, 2, 4, ..., k}) to out (n x n,
 * leading dimension ldo >= n, device). */
lv_status lv_view_read(const lv_view* v, int power, void* out, int64_t ldo, void* stream);

/* Copy the stored sum S_index (index in {1, 2, 4, ..., k}; S_1 = I) of a
 * view created with LV_WITH_SUMS to out (n x n, ld ldo >= n, device).
 * LV_ESTATE for a view without sums. */
lv_status lv_view_read_sum(const lv_view* v, int index, void* out, int64_t ldo, void* stream);

/* General iterative form T_{i+1} = A T_i + B (Sec. 5.3 and Table 1,
 * exponential model: T_1 = A T_0 + B, T_{2i} = P_i T_i + S_i B), T_i and B
 * n x p.  A view created here stores T_1, T_2, T_4, ..., T_k beside the
 * powers and the sums (it implies LV_WITH_SUMS) and keeps them current
 * under lv_view_update / lv_view_update_batch by hybrid evaluation
 * (Sec. 5.3.2): the change of each T_i is one dense n x p matrix D_i, taken
 * from the old values by the delta rule of Sec. 4.1 (the factored form of
 * App. B, multiplied out):
 *     D_1 = U (V^T T_0),
 *     D_{2i} = P_i D_i + U_i (V_i^T (T_i + D_i)) + Q_i (W_i^T B)
 * with Delta P_i = U_i V_i^T and Delta S_i = Q_i W_i^T.  T_0 and B are fixed.
 * With strategy LV_GENERAL_FACTORED the change of each T_i is kept
 * factored instead, Delta T_i = Y_i Z_i^T (incremental evaluation, App. B):
 *     Y_1 = U, Z_1 = T_0^T V,
 *     Y_{2i} = [U_i, P_i Y_i + U_i (V_i^T Y_i), Q_i],
 *     Z_{2i} = [T_i^T V_i, Z_i, B^T W_i]         (widths (2i - 1) r),
 * all from the old values, then T_i += Y_i Z_i^T; its cost grows with n p
 * rather than n^2 p, for large p.
 * Creation and re-anchoring evaluate every T_i by the recurrence in double
 * precision from the double powers and sums and round once.
 *  p         hybrid: 1 <= p <= 64 (padded to a power of two in the
 *            workspace); factored: 1 <= p <= 4096 (padded to a multiple of
 *            128), and k * r_max (s * r_max under the skip model below)
 *            rounded up to a power of two <= 128.
 *  T0, B     n x p (device, element type of the mode), leading dimensions
 *            ldt, ldb >= p; copied into the workspace, not retained.
 *  strategy  LV_GENERAL_HYBRID or LV_GENERAL_FACTORED.
 *  s         0 (or k): the exponential model above.  Else the skip-s model
 *            (Table 1; App. B skip model; factored deltas only): the powers
 *            and sums stop at P_s, S_s (s a power of two dividing k), and
 *            beyond T_s the view stores T_2s, T_3s, ..., T_k with
 *            T_js = P_s T_(j-1)s + S_s B, whose factored deltas are
 *            [U_s, P_s Y + U_s (V_s^T Y), Q_s] [T^T V_s, Z, B^T W_s]^T from the
 *            previous T's factors (Y, Z) and the top-level ones;
 *            (2k - 1 - 2s) * r_max rounded up must not exceed 128.
 * Other arguments, ownership and errors as lv_view_create; the footprint
 * is 0 for invalid arguments.  Such views are single-view only. */
#define LV_GENERAL_HYBRID 0
#define LV_GENERAL_FACTORED 1
size_t lv_view_footprint_general(int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy,
                                 int s);
lv_status lv_view_create_general(const void* A, int64_t n, int64_t lda, int k, int r_max,
                                 lv_mode mode, const void* T0, int64_t ldt, const void* B,
                                 int64_t ldb, int64_t p, int strategy, int s, void* workspace,
                                 size_t ws_bytes, void* stream, lv_view** out);

/* Copy stored T_index (index in {1, 2, 4, ..., k}, or {1, 2, 4, ..., s, 2s,
 * 3s, ..., k} under the skip model) of a general-form view to out (n x p,
 * leading dimension ldo >= p, device).  LV_ESTATE for a view created
 * otherwise. */
lv_status lv_view_read_general(const lv_view* v, int index, void* out, int64_t ldo, void* stream);

/* Borrowed device pointer to stored power A^power and its leading
 * dimension (written to *ld if ld is non-null); NULL if power is not
 * stored.  Valid until the next update, re-anchor or destroy. */
const void* lv_view_data(const lv_view* v, int power, int64_t* ld);

/* Recompute every stored power from the current A (= the stored P_1) by
 * repeated squaring in double precision, discarding accumulated rounding
 * (bfloat16 shadows are rewritten from the new values; stored sums and T_i
 * are re-evaluated the same way). */
lv_status lv_view_reanchor(lv_view* v, void* stream);

/* Copy out (n x n, leading dimension lds >= n, device) into stored power
 * A^power: restores a checkpoint written with lv_view_read, or lets a test
 * perturb a stored power (its bfloat16 shadow, if any, is rewritten).  The
 * caller is responsible for consistency of the chain afterwards (see
 * lv_view_drift_check); stored sums and T_i are not changed (lv_view_reanchor
 * re-evaluates powers, sums and T_i from the stored A). */
lv_status lv_view_write(lv_view* v, int power, const void* src, int64_t lds, void* stream);

/* Drift check of the stored chain (the exponential model defines
 * P_{2i} = P_i P_i, Table 1; incremental updates keep it only up to
 * accumulated rounding).  For z (n doubles, device) and every level
 * j = 0..m-1 (level j stores A^(2^j)):
 *     rho_j = max|P_{j+1} z - P_j (P_j z)| / max|P_{j+1} z|
 * with double accumulation over the stored values.  When some rho_j > tau
 * (or is not finite), every stored power is recomputed from the stored A by
 * repeated squaring in double precision (as lv_view_reanchor); the decision
 * is taken on the device, the host does not wait.  residuals (device, m
 * doubles) receives rho_j if non-null.  tau >= 0.  For k = 1 there is nothing
 * to check.  lv_view_stats reports the count of triggered re-evaluations and
 * the last max_j rho_j (it waits for the device to read them). */
lv_status lv_view_drift_check(lv_view* v, const void* z, double tau, double* residuals,
                              void* stream);

/* Periodic drift check: after every `every`-th update of the view (counted
 * as lv_stats.updates, whichever entry point applies it: lv_view_update,
 * lv_view_update_batch, batch rounds or server rounds), the check of
 * lv_view_drift_check runs on the update's stream with this view's probe
 * vector and bound, and re-anchors the chain on the device when some
 * rho_j > tau.  every = 0 turns it off (the default).
 *  tau   the bound; tau < 0 takes the mode's default: LV_DRIFT_TAU_FP64,
 *        LV_DRIFT_TAU_FP32 or LV_DRIFT_TAU_BF16SHADOW, a tenth of the
 *        maximum relative error the mode is held to against the exact
 *        powers (1e-10, 1e-4 and 5e-3): rho_j compares two ways of forming
 *        P_{j+1} z from the stored values, so it stays of the order of the
 *        storage rounding (about 20 units of 2^-24 after 1000 float updates
 *        of an n = 8192 view) until the chain drifts.
 *  z     n doubles on the device, copied into the view; NULL takes the
 *        library's probe vector (entries +1 / -1 from splitmix64, fixed seed).
 * Each check reads every stored power twice (2 m + 1 matrix-vector
 * products).  LV_EINVAL for a negative interval or a NaN bound. */
#define LV_DRIFT_TAU_FP64 1e-11
#define LV_DRIFT_TAU_FP32 1e-5
#define LV_DRIFT_TAU_BF16SHADOW 5e-4
lv_status lv_view_set_drift_check(lv_view* v, int64_t every, double tau, const void* z, void* stream);

/* Per-kernel timing of a view's updates (diagnostics).  While enabled, the
 * library brackets every level-pass launch with HIP events recorded on the
 * update's stream; lv_view_timing waits for those events, returns the
 * accumulated device time per kernel kind and clears the accumulators.
 * Enabling adds one event pair per launch to the stream. */
typedef struct {
  double fused_ms;        /* fused level passes (levels 0..m-1)            */
  int64_t fused_launches;
  double tail_ms;         /* reductions and factor assembly                */
  int64_t tail_launches;
  double top_ms;          /* update-only pass of the top stored power      */
  int64_t top_launches;
} lv_timing;

lv_status lv_view_set_timing(lv_view* v, int enable);
lv_status lv_view_timing(lv_view* v, lv_timing* out);

/* Rows per tile of the level pass of `level` (0 <= level < log2 k): the
 * height of the P_j tiles whose partial sums of P_j^T V_j are reduced by the
 * tail, so it fixes the summation order of the update.  Default 512;
 * lv_batch_create sets it by autotuning.  Allowed values: multiples of 64
 * in [256, 1024].  Two views with equal tiles, inputs and updates hold equal
 * values bit for bit whichever entry point applies the updates. */
lv_status lv_view_tile_rows(const lv_view* v, int level, int* rows);
lv_status lv_view_set_tile_rows(lv_view* v, int level, int rows);

/* Counters and shape of a view.  Reads the drift counters from the device
 * (a synchronous copy). */
lv_status lv_view_stats(const lv_view* v, lv_stats* out);

/* Release the handle (the caller frees the workspace afterwards, once the
 * stream has drained).  NULL is ignored. */
void lv_view_destroy(lv_view* v);

/* ---------------------------------------------------------------------
 * Batched rounds over many views (one update per view per round).
 *
 * A batch is built over existing views of one mode (uneven n, k and r_max
 * allowed).  Each round applies, to every view, the update staged in that
 * view's input buffers (lv_batch_inputs): U, V of n rows and r_max columns,
 * row-major with leading dimension r_max (a view without an update this
 * round stages zeros, which leaves it unchanged bit for bit).  The round is
 * one launch from the host: a HIP graph captured at lv_batch_create and
 * replayed by lv_batch_update.  Inside it, every level step of all views
 * runs as one multi-view launch per level rank (work-groups map to
 * (view, tile) through descriptor tables in the workspace), so small views
 * share the GPU instead of launching separately.  The per-view results equal
 * lv_view_update bit for bit (with the tile rows the batch chose, see
 * lv_view_tile_rows).
 *
 * Tiles are autotuned at lv_batch_create: one round with zero inputs runs
 * first (it leaves every stored power unchanged), then for each level and
 * level rank the tile heights 256, 384, ..., 1024 rows (every multiple of
 * 128) are timed over that level's launches, and the fastest is kept in the
 * views.  Choices are cached per process by device architecture, mode,
 * rank and the orders of the views concerned (rounded up to powers of two),
 * so a batch of the same shape is not timed again; lv_tune_cache_save /
 * lv_tune_cache_load keep them across processes.
 * --------------------------------------------------------------------- */
typedef struct lv_batch lv_batch;

/* Workspace bytes for a batch over `views` (count >= 1); 0 if invalid. */
size_t lv_batch_footprint(lv_view* const* views, int count);

/* Build the batch (descriptor tables, input staging, the captured round).
 * workspace: device, >= lv_batch_footprint bytes, 256-byte aligned,
 * borrowed until lv_batch_destroy.  The views must outlive the batch and
 * must not be updated through other calls while the batch is used. */
lv_status lv_batch_create(lv_view* const* views, int count, void* workspace, size_t ws_bytes,
                          void* stream, lv_batch** out);

/* Device input buffers of view i (U and V, n x r_max, leading dimension r_max). */
lv_status lv_batch_inputs(const lv_batch* b, int i, void** U, void** V, int64_t* ld);

/* Stage the next update of view i: U, V n x r (device, leading dimensions
 * ldu, ldv >= r), 0 <= r <= r_max; columns r..r_max-1 of the staging are
 * zeroed (r = 0 stages "no update"; U and V may then be NULL). */
lv_status lv_batch_stage(lv_batch* b, int i, const void* U, const void* V, int64_t r, int64_t ldu,
                         int64_t ldv, void* stream);

/* One round: every view applies its staged update (stream-ordered). */
lv_status lv_batch_update(lv_batch* b, void* stream);

/* Autotuning record of the batch: (level, rank) groups timed at creation,
 * and groups whose choice came from the process cache. */
lv_status lv_batch_tuning(const lv_batch* b, int* tuned_groups, int* cache_hits);

/* The autotuner's choices persist across processes through a JSON file: a
 * flat object mapping "arch|m<mode>|R<level rank>|n:<n bucket>:..." (the
 * device architecture, the mode, the level rank and the orders of the
 * group's views, each rounded up to a power of two) to tile rows.
 * lv_tune_cache_save writes the process cache (atomically, by rename);
 * lv_tune_cache_load merges a file into it (*entries = entries read; an
 * entry whose tile rows lv_view_set_tile_rows would refuse makes the whole
 * load fail with LV_EINVAL and changes nothing); lv_tune_cache_clear
 * empties it.  Host only; thread-safe. */
lv_status lv_tune_cache_save(const char* path);
lv_status lv_tune_cache_load(const char* path, int* entries);
void lv_tune_cache_clear(void);

/* Release the batch (after the stream has drained).  NULL is ignored. */
void lv_batch_destroy(lv_batch* b);

/* ---------------------------------------------------------------------
 * Serving loop.  Views live inside one caller-provided HBM arena: each
 * admitted view takes one block (its workspace and an input staging area)
 * from a first-fit free list, so admission is by exact footprint and
 * removing a view returns its block.  Rank-1 update requests arrive from
 * host memory and queue per view; each step coalesces up to r_coalesce
 * queued requests of a view into one rank-r update (the delta of U V^T is
 * the sum of the rank-1 deltas, Sec. 4.1-4.2) and launches one multi-view
 * round over exactly the views with pending requests, without waiting for
 * earlier rounds (continuous batching: requests that arrive meanwhile join
 * the next step).  Completion events give each request's latency from its
 * arrival time to the end of the round that applied it.  Not thread-safe.
 * --------------------------------------------------------------------- */
typedef struct lv_server lv_server;

typedef struct {
  uint64_t submitted;         /* requests accepted                             */
  uint64_t completed;         /* requests applied (their round has finished)    */
  uint64_t rounds;            /* rounds launched                                */
  uint64_t coalesced_updates; /* per-view rank-r updates launched               */
  int32_t views;              /* views admitted                                 */
  size_t arena_free;          /* free arena bytes                               */
  double latency_p50_s;       /* arrival -> completion, over completed requests */
  double latency_p99_s;
  double latency_max_s;
  int32_t views_waiting;      /* views in the admission queue                   */
  uint64_t admitted_late;     /* views admitted from the queue so far           */
} lv_server_counters;

/* arena: device, 256-byte aligned, >= 4 MiB (descriptor ring) plus the
 * views; r_coalesce in [1, 64] is every view's r_max (so k * r_coalesce,
 * rounded up, obeys the width rule of lv_view_create when views are added). */
lv_status lv_server_create(void* arena, size_t arena_bytes, lv_mode mode, int r_coalesce,
                           void* stream, lv_server** out);
/* Arena bytes one view of order n and power k takes (0 if invalid). */
size_t lv_server_view_bytes(const lv_server* s, int64_t n, int k);
/* Hold policy of the rounds (coalescing of Sec. 4.2 traded against latency):
 * a view with pending requests joins a round only once it has
 * min(min_fill, r_coalesce) requests queued or its oldest request has
 * waited max_wait_s seconds (arrival clock), so rounds carry fuller updates
 * and the busiest views get more rounds; with no round in flight every
 * view with pending requests goes, so queued work never waits on an idle
 * device.  min_fill = 1 (the default) puts every pending view in every
 * round.  LV_EINVAL for min_fill < 1 or a negative (or NaN) max_wait_s. */
lv_status lv_server_set_hold(lv_server* s, int min_fill, double max_wait_s);
/* Admit a view of A^k (A: n x n device, lda >= n).  When no free block is
 * large enough: LV_ENOMEM, unless the admission queue is on (below), in
 * which case the view waits: A is copied to pinned host memory (the call
 * returns once the copy is done), the view gets its id, requests to it are
 * accepted and queued, and it is admitted (created from the host copy) as
 * soon as a removal frees room for it.  Waiting views are admitted in the
 * order they were added, each one that fits.  LV_ENOMEM still when the view
 * is larger than the whole arena. */
lv_status lv_server_add_view(lv_server* s, const void* A, int64_t n, int64_t lda, int k,
                             int* view_id);
/* Admission queue on (enable != 0) or off (the default). */
lv_status lv_server_set_admission_queue(lv_server* s, int enable);
/* Wait for in-flight rounds, then free the view and its block, and admit
 * waiting views that now fit.  A waiting view is dropped with its queued
 * requests (they no longer count as submitted). */
lv_status lv_server_remove_view(lv_server* s, int view_id);
/* The view handle (for lv_view_read / lv_view_data); NULL if none or
 * while the view waits for admission. */
lv_view* lv_server_view(lv_server* s, int view_id);
/* Seconds on the server's clock (arrival times are on this clock). */
double lv_server_now(const lv_server* s);
/* Queue the rank-1 request u v^T (u, v: n elements of the view's type in
 * host memory, copied before return).  arrival < 0 means now. */
lv_status lv_server_submit(lv_server* s, int view_id, const void* u, const void* v, double arrival,
                           uint64_t* ticket);
/* Launch one round over the views with pending requests (non-blocking;
 * *launched = requests in the round).  At most two rounds are in flight:
 * one running and one queued behind it on the stream; while both are
 * there, step launches nothing (*launched = 0) and new requests keep
 * coalescing in the queues, so each round takes what arrived during the
 * previous one and the device never waits for the host. */
lv_status lv_server_step(lv_server* s, int* launched);
/* Retire finished rounds without waiting; *completed = total applied. */
lv_status lv_server_poll(lv_server* s, uint64_t* completed);
/* Apply every queued request of the admitted views (launching rounds as
 * room frees up), then wait for every launched round.  Requests of views
 * still waiting for admission stay queued. */
lv_status lv_server_drain(lv_server* s);
lv_status lv_server_stats(const lv_server* s, lv_server_counters* out);
/* Drain, destroy the views, release host resources (the caller frees the
 * arena).  NULL is ignored. */
void lv_server_destroy(lv_server* s);

/* Workspace bytes for lv_reeval at order n; 0 if invalid. */
size_t lv_reeval_footprint(int64_t n, int r_max, lv_mode mode);

/* Re-evaluation baseline (ReevalExp, Sec. 5.2.2): out = (A + U V^T)^k
 * computed as one rank-r update and m = log2 k dense squarings in the
 * mode's own precision (MFMA).  A: n x n (lda); U, V: n x r (ldu, ldv);
 * out: n x n (ldo).  A is not modified.  r = 0 skips the update (U, V
 * may then be NULL). */
lv_status lv_reeval(const void* A, int64_t n, int64_t lda, int k,
                    const void* U, const void* V, int64_t r, int64_t ldu, int64_t ldv,
                    lv_mode mode, void* out, int64_t ldo,
                    void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- allocation-free update
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * update Delta A = U V^T of stored powers the caller holds, exactly as
 * lv_view_update applies it to a view of the same order, power, mode and
 * rank with the default tile rows (the same kernels, so equal results bit
 * for bit).  The factor slabs and reduction partials live in a static
 * device array of the library (64 MiB per GPU, held until the process
 * ends); the call allocates nothing.  A shape needs 2 n W e bytes of
 * factor slabs (W = k r_pad, r_pad = r rounded up to a power of two, e the
 * element size) and, for each level j < m with rank R = 2^j r_pad, partials
 * of n R e (nct + n / 256) bytes (nct = n / 256 column tiles in FP32,
 * n / 128 in FP64) and 8 R^2 max(n / 256, n / 64) bytes of Gram partials,
 * each region rounded up to 256 bytes: n = 8192, k = 16, r = 1 in FP32
 * takes 31 MiB.  Calls on one GPU share that array, so calls that overlap
 * on one GPU (different streams or host threads) race and must be
 * serialised by the caller.
 *  powers   host array of m + 1 device pointers (k = 2^m): powers[j] holds
 *           A^(2^j), n x n with leading dimension ld, updated in place.
 *  n        a multiple of 256 (the kernels' padding granule), <= 65536.
 *  ld       >= n, ld * element size a multiple of 16 bytes; pointers 16-byte
 *           aligned.
 *  mode     LV_FP32 or LV_FP64 (element type float or double).
 *  U, V     n x r (device), ldu, ldv >= r; k * r rounded up to a power of
 *           two <= 256.
 * LV_EINVAL for bad arguments; LV_ENOMEM when the scratch the shape needs
 * exceeds the array.  Nothing is enqueued on failure unless the status is
 * LV_EDEVICE. */
lv_status lv_powers_update_noalloc(void* const* powers, int64_t n, int64_t ld, int k, lv_mode mode,
                                   const void* U, const void* V, int64_t r, int64_t ldu, int64_t ldv,
                                   void* stream);

/* ---------------------------------------------------------------- streaming ceiling
 *
 * Measured HBM ceiling for the level passes (diagnostics; none of the
 * method's arithmetic).  One launch streams `bytes` with the access pattern
 * of the level passes: 16-byte non-temporal loads and stores, whole 1 KiB
 * row segments per wave, work-groups of 256 threads striding over chunks of
 * depth x 4 KiB.  Kinds:
 *   LV_STREAM_RMW    dst[i] = 1 * dst[i] in place (one read and one write at
 *                    the same address, as a level pass does to P_j)
 *   LV_STREAM_COPY   dst[i] = 1 * src[i]
 *   LV_STREAM_READ   reads src; one float per thread (blocks * 1 KiB) goes
 *                    to dst so that the loads stay live
 *   LV_STREAM_WRITE  dst[i] = 0
 *  bytes      a positive multiple of depth * 4096.
 *  blocks     work-groups in the grid, 1 .. 2^20 (blocks per CU x CUs).
 *  depth      16-byte vectors per thread per iteration: 1, 2, 4, 8, 16, 32.
 *  pipelined  nonzero: the next iteration's loads are issued before the
 *             current stores (2 x depth vectors in flight per thread).
 * Buffers are device memory, 16-byte aligned, owned by the caller.  The
 * caller times the launch with events on `stream`.  LV_EINVAL for bad
 * arguments (nothing is launched). */
#define LV_STREAM_RMW 0
#define LV_STREAM_COPY 1
#define LV_STREAM_READ 2
#define LV_STREAM_WRITE 3
lv_status lv_stream_probe(int kind, void* dst, const void* src, size_t bytes, int blocks, int depth,
                          int pipelined, void* stream);

/* ---------------------------------------------------------------- models
 *
 * Matrix-power views under the other iterative models of Sec. 3.2 and
 * Table 1 (matrix-powers column), for comparing IncrLin / IncrSkip-s with
 * IncrExp (Table 2; App. A):
 *   LV_MODEL_LIN   stores P_1 .. P_k,  P_i = A P_{i-1}          (any k >= 1)
 *   LV_MODEL_EXP   stores P_1, P_2, P_4, .., P_k, P_i = P_{i/2} P_{i/2}
 *                  (k a power of two; the same model as lv_view, on this
 *                  generic engine)
 *   LV_MODEL_SKIP  the exponential model up to P_s, then
 *                  P_i = P_s P_{i-s} for i = 2s, 3s, .., k
 *                  (s a power of two dividing k)
 * An update Delta A = U V^T forms, for every product P_c = P_a P_b in
 * order and from the OLD matrices (App. A),
 *     U_c = [U_a, P_a U_b + U_a (V_a^T U_b)],   V_c = [P_b^T V_a, V_b]
 * (widths c * r), then applies P_c += U_c V_c^T to every stored matrix.
 * Modes LV_FP64 and LV_FP32 (creation in double, rounded once).  k * r_max
 * rounded up to a power of two must not exceed 128.  Workspace, streams,
 * ownership and errors as for lv_view. */
#define LV_MODEL_EXP 0
#define LV_MODEL_LIN 1
#define LV_MODEL_SKIP 2

typedef struct lv_chain lv_chain;

/* Workspace bytes; 0 for invalid arguments (s is ignored unless the model
 * is LV_MODEL_SKIP). */
size_t lv_chain_footprint(int64_t n, int k, int r_max, lv_mode mode, int model, int s);
lv_status lv_chain_create(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode,
                          int model, int s, void* workspace, size_t ws_bytes, void* stream,
                          lv_chain** out);
/* One update Delta A = U V^T (U, V n x r device, ldu, ldv >= r, r <= r_max). */
lv_status lv_chain_update(lv_chain* c, const void* U, const void* V, int64_t r, int64_t ldu,
                          int64_t ldv, void* stream);
/* Copy stored A^power (a power the model stores) to out (n x n, ldo >= n). */
lv_status lv_chain_read(const lv_chain* c, int power, void* out, int64_t ldo, void* stream);
/* Number of stored matrices (-1 for NULL); their powers, ascending, go to
 * powers[0 .. min(count, cap)) when powers is non-null. */
int lv_chain_powers(const lv_chain* c, int* powers, int cap);
/* Release the handle (the caller frees the workspace).  NULL is ignored. */
void lv_chain_destroy(lv_chain* c);

/* ---------------------------------------------------------------- OLS
 *
 * Ordinary least squares kept current under rank-1 changes of the data
 * (Sec. 5.1, with the Sherman-Morrison formula of Sec. 4): X is m x n
 * (predictors, m >= n), Y is m x p (responses), W = (X^T X)^{-1} and the
 * estimate beta = W X^T Y (n x p).  For Delta X = u v^T,
 *     Delta(X^T X) = p1 q1^T + p2 q2^T,  p1 = q2 = v,  q1 = X^T u,
 *                    p2 = X^T u + v (u^T u),
 * W takes the two outer products in turn by Sherman-Morrison (Delta W =
 * R S^T, rank 2) and Delta beta = R S^T X^T Y + W v u^T Y + R S^T v u^T Y,
 * all from the old X and W; X, X^T Y, W and beta are then updated.  Per
 * update: one read of W, one read and write of W, O(m n) for X^T u and
 * X += u v^T (O(n) with lv_ols_update_row), O(n p) for beta.  Both
 * X^T X and its updated value must be nonsingular (the formula's
 * condition; a singular update gives non-finite values).
 * Creation (re-evaluation) forms X^T X and X^T Y in double, inverts by the
 * Newton-Schulz iteration on the double matrix cores (synchronizes the
 * stream once per iteration; LV_EINVAL if X^T X is singular or too
 * ill-conditioned for the mode), and rounds W, X^T Y and beta once to the mode's type.
 * Modes LV_FP64, LV_FP32; 1 <= n <= 32768, n <= m <= 2^22, 1 <= p <= 64.
 * X, Y (device, leading dimensions ldx >= n, ldy >= p) are copied. */
#define LV_OLS_BETA 0      /* n x p */
#define LV_OLS_INVERSE 1   /* W, n x n */
#define LV_OLS_X 2         /* the current data, m x n */

typedef struct lv_ols lv_ols;

size_t lv_ols_footprint(int64_t m, int64_t n, int64_t p, lv_mode mode);
lv_status lv_ols_create(const void* X, int64_t m, int64_t n, int64_t ldx, const void* Y, int64_t p,
                        int64_t ldy, lv_mode mode, void* workspace, size_t ws_bytes, void* stream,
                        lv_ols** out);
/* Delta X = u v^T; u (m elements) and v (n elements) on the device. */
lv_status lv_ols_update(lv_ols* o, const void* u, const void* v, void* stream);
/* Row change Delta X = e_row dx^T (dx: n elements on the device). */
lv_status lv_ols_update_row(lv_ols* o, int64_t row, const void* dx, void* stream);
/* Copy LV_OLS_BETA, LV_OLS_INVERSE or LV_OLS_X to out (device, ld ldo). */
lv_status lv_ols_read(const lv_ols* o, int what, void* out, int64_t ldo, void* stream);
/* Creation diagnostics: Newton-Schulz iterations, the final residual
 * max|Z W - I| and the infinity-norm condition number ||Z|| ||W|| (creation
 * fails when it exceeds 0.1 / unit roundoff of the mode). */
lv_status lv_ols_info(const lv_ols* o, int* iterations, double* residual, double* cond);
void lv_ols_destroy(lv_ols* o);

/* ---------------------------------------------------------------- linear model
 *
 * The general form T_{i+1} = A T_i + B under the linear model (Sec. 3.2,
 * Table 1; App. B, linear model), T_0, B n x p: every T_1 .. T_k is stored
 * and kept current under Delta A = U V^T by one of Table 2's strategies:
 *   LV_GLIN_REEVAL  A += U V^T, then T_i = A T_{i-1} + B, i = 1 .. k;
 *   LV_GLIN_HYBRID  Delta T_1 = U (V^T T_0),
 *                   Delta T_i = A Delta T_{i-1} + U (V^T (T_{i-1} + Delta T_{i-1})),
 *                   dense n x p deltas from the old A and T;
 *   LV_GLIN_INCR    factored Delta T_i = Y_i Z_i^T, Y_1 = U, Z_1 = T_0^T V,
 *                   Y_i = [U, A Y_{i-1} + U (V^T Y_{i-1})],
 *                   Z_i = [T_{i-1}^T V, Z_{i-1}] (old A and T; widths i r);
 * (hybrid and incremental then apply A += U V^T).  Creation evaluates the
 * iteration in double and rounds once.  Modes LV_FP64, LV_FP32;
 * 1 <= k <= 256; 1 <= p <= 4096 (p <= 64 padded to a power of two, wider p
 * to a multiple of 128, whose products with A run on the MFMA GEMM);
 * LV_GLIN_INCR needs k * r_max rounded up to a power of two <= 128.
 * Workspace, streams, ownership and errors as for lv_view. */
#define LV_GLIN_REEVAL 0
#define LV_GLIN_HYBRID 1
#define LV_GLIN_INCR 2

typedef struct lv_glin lv_glin;

size_t lv_glin_footprint(int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy);
lv_status lv_glin_create(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode,
                         const void* T0, int64_t ldt, const void* B, int64_t ldb, int64_t p,
                         int strategy, void* workspace, size_t ws_bytes, void* stream, lv_glin** out);
/* One update Delta A = U V^T (U, V n x r device, ldu, ldv >= r, r <= r_max). */
lv_status lv_glin_update(lv_glin* g, const void* U, const void* V, int64_t r, int64_t ldu,
                         int64_t ldv, void* stream);
/* Copy T_i (0 <= i <= k; T_0 is the fixed start) to out (n x p, ldo >= p). */
lv_status lv_glin_read(const lv_glin* g, int i, void* out, int64_t ldo, void* stream);
void lv_glin_destroy(lv_glin* g);

#ifdef __cplusplus
}
#endif

#endif /* LINVIEW_H */
