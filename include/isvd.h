/*
 * isvd.h -- C ABI of the MI355X incremental-SVD engine (libisvd.so).
 *
 * The engine maintains, for every data stream, a rank-k truncated SVD
 * A_t ~ U_t Sigma_t V_t^T of a dense matrix A_t that grows by appended rows
 * and columns and changes by single-entry updates, following the paper's
 * problem setting (Section 2.1) and its engine loop (Algorithm 1):
 *
 *   isvd_init          (U, Sigma, V) = TruncatedSVD(A_0, k), A = A_0      (Alg. 1 init)
 *   isvd_append_row    A <- [A; x^T],  RowAppendUpdate                     (Sec. 2.2.1, Alg. A1)
 *   isvd_append_col    A <- [A, y],    ColAppendUpdateViaTranspose         (Sec. 2.2.2, Alg. A2)
 *   isvd_update_entry  A_ij += delta,  RankOneUpdate: U' S' V'^T =
 *                      P_U (A_hat + delta e_i e_j^T) P_V                   (Sec. 2.3, eq. rank1-projection)
 *   isvd_refresh       (U, Sigma, V) = TruncatedSVD(A_t, k)                 (Sec. 2.4.1)
 *   isvd_metrics       N_t, EVR, errors, angles, timings                  (Sec. 2.4.2, 2.5)
 *   isvd_causal_center expanding-mean centering of return rows          (Sec. 5.1)
 *   isvd_covariance    low-rank covariance V diag(sigma^2) V^T / (t - 1)   (Sec. 5.3, eq. low-rank-covariances)
 *   isvd_risk          portfolio volatility, risk and covariance errors   (Sec. 5.3, eqs. cov-error, portfolio-vol, risk-error)
 *   isvd_tick          one batched step: many streams' updates in one launch sequence
 *
 * Every update truncates back to the stream's rank and then evaluates the
 * stream's refresh policy (Section 3); a policy that fires refreshes the
 * stream before its next update.
 *
 * Conventions
 *  - All functions return an isvd_status (0 = success, < 0 = error) and never
 *    throw; isvd_last_error() describes the most recent failure on the
 *    calling thread.  On any error no state is changed unless stated.
 *  - Matrices are row-major.  `lda`/`ldu`/`ldv` are leading dimensions in
 *    elements.  dtype is ISVD_DTYPE_F32 or ISVD_DTYPE_F64.
 *  - Payloads (A_0, x, y) are borrowed: `on_device` = 0 means a host pointer
 *    (copied before the call returns), 1 means a device pointer on the
 *    engine's GPU, read by kernels ordered on `hip_stream`; the caller keeps
 *    it alive and unmodified until that stream has passed the call.
 *  - `hip_stream` is a hipStream_t (NULL = the default stream).  All device
 *    work of a call is ordered on it; calls return without waiting for the
 *    GPU unless stated.
 *  - The engine owns all per-stream device state (A, U, V, Sigma, trackers).
 *    One host thread at a time may use an engine.
 *  - Non-finite entries of a host payload are caught before any work is
 *    enqueued (ISVD_E_NONFINITE).  In a device payload they are caught on
 *    the device: the update is rejected and the stream's state is left as it
 *    was; the stream then rejects every further update until the next
 *    isvd_metrics call, which reports ISVD_E_NONFINITE in `status` (with the
 *    count in `n_rejected`), re-synchronises the host's view of the shape
 *    and re-opens the stream.
 */
#ifndef ISVD_H
#define ISVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isvd_engine isvd_engine;   /* opaque */
typedef int64_t isvd_id;                  /* stream handle, >= 0 */
typedef int32_t isvd_status;

enum {
    ISVD_OK = 0,
    ISVD_E_INVAL = -1,      /* bad argument (null pointer, k out of range, bad enum) */
    ISVD_E_SHAPE = -2,      /* payload length differs from the stream's n_t (row) or m_t (column) */
    ISVD_E_RANGE = -3,      /* entry index outside [0, m_t) x [0, n_t) */
    ISVD_E_NONFINITE = -4,  /* payload or delta not finite; update rejected */
    ISVD_E_NOMEM = -5,      /* device allocation failed */
    ISVD_E_BUDGET = -6,     /* the stream would exceed the engine's HBM budget */
    ISVD_E_DEVICE = -7,     /* HIP runtime error */
    ISVD_E_STATE = -8,      /* unknown / released stream id, or engine in wrong mode */
    ISVD_E_CONVERGE = -9,   /* Jacobi core or refresh did not converge */
    ISVD_E_CAPACITY = -10   /* the stream reached its row / column capacity */
};

enum { ISVD_DTYPE_F32 = 0, ISVD_DTYPE_F64 = 1 };

/* Storage / arithmetic of a stream.  The core SVD, the residual norm, the
 * re-orthogonalisation pass and all trackers are FP64 in every mode. */
enum {
    ISVD_FP64 = 0,          /* A, U, V and all products in FP64 */
    ISVD_FP32 = 1,          /* A, U, V, projections and rotations in FP32 */
    ISVD_BF16ROT = 2        /* as ISVD_FP32, but the U / V rotations on the
                               BF16 matrix cores (operands rounded to BF16, FP32 accumulation):
                               faster, with an orthogonality drift of about 2^-8 per update
                               that refreshes repair */
};

enum { ISVD_ROW = 0, ISVD_COL = 1, ISVD_ENTRY = 2 };

enum {
    ISVD_POL_NONE = 0,
    ISVD_POL_PERIODIC = 1,  /* refresh iff t = 0 mod period (eq. periodic-refresh-rule) */
    ISVD_POL_ERROR = 2,     /* at t = 0 mod check_every: refresh iff frob_ratio > gamma
                               and t - t_last >= t_min (eq. error-refresh-rule) */
    ISVD_POL_ANGLE = 3,     /* refresh iff theta_ref > theta_max (Section 3.3) */
    ISVD_POL_ADAPTIVE = 4,  /* EVR / novelty rank rule + periodic refresh (Section 3.4):
                               grow by one on the next append when EVR < tau - band or
                               the append had rho / ||x|| > eta; otherwise shrink by one
                               when EVR without the last triplet >= tau + band; rank in
                               [max(k_min, 1), k_max] */
    ISVD_POL_DRIFT = 5      /* drift surrogate without A (Sections 3.2-3.3): refresh once the
                               step angles of U accumulated since the last refresh exceed
                               theta_max and t - t_last >= t_min.  The largest principal
                               angle satisfies the triangle inequality, so the sum bounds
                               the angle between the span at the last refresh (zero-padded)
                               and the current one, as long as the rank does not change */
};

typedef struct {
    int32_t kind;           /* ISVD_POL_* */
    int32_t angle_scope;    /* columns the angle is measured on; 0 = leading gap-separated */
    int64_t period;         /* PERIODIC / ADAPTIVE refresh period (0 = none) */
    int64_t check_every;    /* ERROR: evaluation cadence */
    int64_t t_min;          /* ERROR / ANGLE / DRIFT: minimum spacing between refreshes */
    double gamma;           /* ERROR threshold on frob_ratio */
    double theta_max;       /* ANGLE / DRIFT threshold, radians */
    double tau, band, eta;  /* ADAPTIVE: EVR target, hysteresis band, novelty threshold */
    int32_t k_min, k_max;   /* ADAPTIVE rank bounds (k_max also sizes the buffers) */
} isvd_policy;

typedef struct {
    int64_t m0, n0;         /* shape of A_0 */
    int64_t m_cap, n_cap;   /* capacity: largest m_t / n_t the stream may reach (>= m0, n0) */
    int32_t k;              /* target rank, 1 <= k <= min(m0, n0, 128) */
    int32_t precision;      /* ISVD_FP64 / ISVD_FP32 / ISVD_BF16ROT */
    double tol_rel;         /* new direction iff rho > tol_rel * ||x|| (0 = 1e-10 FP64, 1e-5 FP32) */
    int32_t refresh_iters;  /* -1 (default): a stream of at most 4096 columns refreshes in Gram form
                               until every leading Ritz pair meets refresh_tol (a stopping rule);
                               wider streams, and any value >= 0, run that many block subspace
                               iterations on A (8 at init, 3 otherwise when -1) */
    int32_t oversample;     /* refresh block size = min(n, k + oversample) (-1 = default) */
    isvd_policy policy;
    double refresh_tol;     /* Gram-form stopping rule: Ritz residual ||G v - theta v|| <= refresh_tol
                               * theta_1 for the leading k pairs, G = A^T A (0 = 1e-16 FP64, i.e.
                               until the residuals stop falling at rounding level; 1e-10 otherwise) */
    int32_t a_on_host;      /* 1: the stored matrix A lives in pinned host memory mapped into the
                               device's address space, not in HBM; updates write it and refreshes
                               and exact metrics read it over the host link (for streams whose
                               refreshes are rare, e.g. under ISVD_POL_DRIFT).  0: in HBM */
} isvd_config;

typedef struct {
    int64_t t, m, n;        /* updates applied, current shape */
    int64_t n_refresh, t_last_refresh, n_rejected;
    int32_t k;              /* current rank */
    int32_t status;         /* ISVD_OK or the error of the last rejected request */
    int32_t sweeps;         /* Jacobi sweeps of the last core */
    int32_t new_direction;  /* last append: rho > tol */
    double fro2_A;          /* N_t = ||A_t||_F^2 (recurrences of Section 2.5.2) */
    double sigma2_sum;      /* ||Sigma_t||_F^2 */
    double evr;             /* eq. evr */
    double rho, novelty;    /* last append: ||z|| and ||z|| / ||x|| */
    double frob_error;      /* E_inc = ||A_t - U S V^T||_F      (NaN unless compute_exact) */
    double frob_opt;        /* E_opt = sqrt(N_t - sum of the leading Ritz values sigma^2 of a
                               refresh, as many as the model's rank): the error of the best
                               approximation of that rank (NaN unless compute_exact) */
    double frob_gap, frob_ratio;   /* eq. frob-ratio; NaN if undefined or not computed */
    double ortho_U, ortho_V;       /* ||Q^T Q - I||_2 (NaN unless compute_exact) */
    double update_time_us;  /* wall-clock of the last immediate-mode update (host-timed) */
    double opt_time_us;     /* wall-clock of the last refresh (host-timed) */
    double angle_ref;       /* theta_ref, radians: largest principal angle between U_ref
                               (stored at the last refresh) and U_t on U_ref's rows, on the
                               angle scope (Section 2.4.2); tracked every update for
                               ISVD_POL_ANGLE streams, formed directly with compute_exact,
                               else NaN */
    /* Drift signals of the last applied update, formed by the update itself
       without reading A (the cheap surrogates of the error- and angle-based
       refresh, Sections 3.2-3.3; NaN before the first update):
       step_angle_U: largest principal angle, radians, between span(U_{t-1})
                     (zero-padded to the new rows) and span(U_t); 0 when the
                     rank grew (the new span contains the old) and for entry
                     updates (both spans are kept);
       step_angle_V: the same for V;
       spectrum_change: ||sigma_t - sigma_{t-1}||_2 / ||sigma_{t-1}||_2, the
                     shorter vector zero-padded (NaN if sigma_{t-1} = 0). */
    double step_angle_U, step_angle_V, spectrum_change;
    /* Last refresh (or initial SVD): Rayleigh-Ritz rounds of the Gram form (0 for the
       A form), and 1 if the stopping rule held (always 1 for the A form, whose
       iteration count is fixed). */
    int32_t refresh_rounds, refresh_converged;
    /* Step angles of U summed since the last refresh (the ISVD_POL_DRIFT
       quantity; NaN for streams whose policy does not track it). */
    double drift_U;
    /* theta_opt, radians: largest principal angle between span(U_t) and the
       span of the leading (model rank) left singular vectors of A_t (the
       angle metric to the optimal subspace, Section 3.3), from the refresh
       the exact metrics compute (NaN unless compute_exact). */
    double angle_opt;
} isvd_metrics_t;

/* One request of a batched tick. */
typedef struct {
    isvd_id id;
    int32_t kind;           /* ISVD_ROW / ISVD_COL / ISVD_ENTRY */
    int32_t dtype;          /* payload dtype; must equal the stream's storage type */
    const void* payload;    /* device pointer, length n_t (ROW) or m_t (COL); unused for ENTRY */
    int64_t len;
    int64_t i, j;
    double delta;
} isvd_request;

/* Engine on HIP device `device`.  hbm_budget_bytes bounds the device memory
 * of all streams together (0 = no bound). */
isvd_status isvd_engine_create(int32_t device, uint64_t hbm_budget_bytes, isvd_engine** out);
isvd_status isvd_engine_destroy(isvd_engine* eng);

/* Bytes of device memory isvd_init would reserve for `cfg` (0 on invalid cfg). */
uint64_t isvd_stream_bytes(const isvd_config* cfg);

/* Algorithm 1 init: allocate the stream, copy A_0 (m0 x n0, leading dim lda,
 * in `dtype`) into its A, set N_0 = ||A_0||_F^2, and compute
 * TruncatedSVD(A_0, k) with the refresh routine, U_ref = U.  The copy and
 * the norm are ordered on hip_stream; the SVD runs on one of the engine's
 * refresh lanes after them, and the stream is busy (isvd_stream_busy) until
 * it is done: every later call on the stream orders itself after it.  A
 * host A_0 is copied before the call returns.  Does not wait for the SVD.
 * Errors: INVAL (cfg), BUDGET, NOMEM, DEVICE; a Rayleigh-Ritz SVD that does
 * not converge is reported (CONVERGE) by the next call on the stream. */
isvd_status isvd_init(isvd_engine* eng, const isvd_config* cfg, const void* A0, int64_t lda,
                      int32_t dtype, int32_t on_device, void* hip_stream, isvd_id* out);

/* Create `count` streams at once, each as isvd_init with A0[q] on the
 * device (leading dimension lda[q], dtype[q]): the initial TruncatedSVDs
 * (Sec. 2.4.1) of the FP32 streams whose SVD runs in the A form go as one
 * segmented batch (isvd_set_segmented_refresh), the others one by one on the
 * refresh lanes, as isvd_init does.  ids[q] receives stream q's id.  On an
 * error while creating stream q the streams before it stay valid and
 * *created = q; if the batched SVD cannot be queued, every stream of the call
 * is released and *created = 0.  Errors: those of isvd_init. */
isvd_status isvd_init_batch(isvd_engine* eng, int32_t count, const isvd_config* cfgs, const void* const* A0,
                            const int64_t* lda, const int32_t* dtype, void* hip_stream, isvd_id* ids,
                            int32_t* created);

/* Like isvd_init, but the stream starts from the given factors instead of
 * TruncatedSVD(A_0, k) (checkpoint restore; running two precisions from one
 * state): U (m0 x k, ldu), S (k, non-increasing), V (n0 x k, ldv) are FP64
 * host arrays, converted to the stream's storage type.  N_0 = ||A_0||_F^2
 * and U_ref = U.  Waits for the device. */
isvd_status isvd_init_from_factors(isvd_engine* eng, const isvd_config* cfg, const void* A0, int64_t lda,
                                   int32_t dtype, int32_t on_device, const double* U, int64_t ldu,
                                   const double* S, const double* V, int64_t ldv, void* hip_stream,
                                   isvd_id* out);

/* Row append (Alg. A1) + truncation + policy.  x has n = n_t entries.
 * Errors: STATE, SHAPE, CAPACITY, INVAL (dtype), DEVICE. */
isvd_status isvd_append_row(isvd_engine* eng, isvd_id id, const void* x, int64_t n,
                            int32_t dtype, int32_t on_device, void* hip_stream);

/* Column append (Alg. A2) + truncation + policy.  y has m = m_t entries. */
isvd_status isvd_append_col(isvd_engine* eng, isvd_id id, const void* y, int64_t m,
                            int32_t dtype, int32_t on_device, void* hip_stream);

/* Rank-1 entry update (Alg. A3): A_ij += delta, then the in-subspace core
 * update.  Errors: STATE, RANGE (i, j), NONFINITE (delta), DEVICE. */
isvd_status isvd_update_entry(isvd_engine* eng, isvd_id id, int64_t i, int64_t j, double delta,
                              void* hip_stream);

/* Refresh (Section 2.4.1): recompute TruncatedSVD(A_t, k_t) by block subspace
 * iteration warm-started from V_t (exact when the block spans all n_t
 * columns); store_reference != 0 also sets U_ref = U.  Waits for the device. */
isvd_status isvd_refresh(isvd_engine* eng, isvd_id id, int32_t store_reference, void* hip_stream);

/* For callers that cannot allocate device memory (serving loops and harnesses
 * that forbid hipMalloc after start-up): isvd_refresh with its whole workspace
 * in a static device array of ISVD_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends (its address is looked
 * up when an engine is created on that GPU).  Same computation, same results
 * bit for bit, same ordering on hip_stream; the call still waits on the host
 * for the Gram form's per-round decisions, as isvd_refresh does.
 * The array is shared by every engine and call on that GPU and keeps the
 * last call's contents: calls that overlap on one GPU (two host threads, or
 * two streams whose refreshes are in flight together) race on it.
 * Errors: as isvd_refresh; NOMEM when the stream's refresh needs more
 * workspace than the array holds (nothing is enqueued; about m x (k + os)
 * elements of the storage type plus, in the Gram form, 8 n^2 bytes and the
 * blocks); INVAL for store_reference = 0 on an angle-policy stream (keeping
 * the old reference needs tracker workspace that only isvd_refresh
 * allocates). */
#define ISVD_NOALLOC_SCRATCH_BYTES (64u << 20)
isvd_status isvd_refresh_noalloc(isvd_engine* eng, isvd_id id, int32_t store_reference, void* hip_stream);

/* Metrics of the stream.  Waits for the device.  compute_exact != 0 adds
 * E_inc (one pass over A), E_opt = sqrt(||A||_F^2 - sum of the k leading
 * squared Ritz values of a refresh-style subspace iteration that does not
 * replace the factors; exact when the refresh block spans all columns, else
 * an upper bound) and the orthogonality of U and V.  The error policy uses
 * the same computation at its check ticks and commits that iteration's
 * result as the refresh when it fires. */
isvd_status isvd_metrics(isvd_engine* eng, isvd_id id, int32_t compute_exact, void* hip_stream,
                         isvd_metrics_t* out);

/* ---- Factor readout of a returns stream (the paper's finance study, Sec. 5) ----
 *
 * Causal de-meaning (Sec. 5.1): for each column j in turn over the rows,
 * mu_t = mu_{t-1} + (r_t - mu_{t-1}) / t and R_t = r_t - mu_t, so the first
 * centred row is zero.  r: `rows` x n device rows (leading dimension n, dtype
 * ISVD_DTYPE_F32 or ISVD_DTYPE_F64); out: device rows of the same shape and
 * dtype receiving R_{t0+1} .. R_{t0+rows} (may be r itself); mu: device FP64
 * n-vector holding mu_{t0} on entry (not read when t0 = 0) and
 * mu_{t0+rows} on exit.  All arithmetic in FP64, one thread per column,
 * rows in order, so the result does not depend on how the rows are split
 * across calls.  Needs no engine; ordered on hip_stream.
 * Errors: INVAL (null pointers, rows < 1, n < 1, t0 < 0, dtype), DEVICE. */
isvd_status isvd_causal_center(const void* r, void* out, int64_t rows, int64_t n, int32_t dtype, double* mu,
                               int64_t t0, void* hip_stream);

/* Low-rank covariance of the stream's factors (eq. low-rank-covariances,
 * the incremental one): cov = V diag(sigma_1^2 .. sigma_k^2) V^T / (m_t - 1),
 * n_t x n_t, FP64, row-major with leading dimension ldc >= n_t, written to the
 * device buffer cov (caller-owned).  Asynchronous: ordered on hip_stream
 * after the stream's pending work (a refresh on a lane, pending U rotations);
 * the kernel takes the rank from the device.  Errors: STATE (unknown id),
 * INVAL (null cov, ldc < n_t, m_t < 2), DEVICE. */
isvd_status isvd_covariance(isvd_engine* eng, isvd_id id, double* cov, int64_t ldc, void* hip_stream);

typedef struct {
    double vol_inc;   /* sqrt(w^T Sigma_inc,k w) from the stream's factors (eq. portfolio-vol) */
    double vol_full;  /* the same from TruncatedSVD(A_t, k); NaN unless exact */
    double err_risk;  /* |vol_inc - vol_full| / vol_full (eq. risk-error); NaN unless exact */
    double err_cov;   /* ||Sigma_inc,k - Sigma_full,k||_F / ||Sigma_full,k||_F (eq. cov-error); NaN unless exact */
} isvd_risk_t;

/* Portfolio volatility of weights w (host FP64, n = n_t entries) under the
 * stream's low-rank covariance.  exact != 0 also computes TruncatedSVD(A_t, k)
 * by the refresh's subspace iteration (exact when the block spans all
 * columns; nothing of the stream changes) and the two errors against it.
 * err_cov comes from k x k products: with D = diag(sigma^2) / (m_t - 1),
 * ||V1 D1 V1^T - V2 D2 V2^T||_F^2 = sum_ij d1_i d1_j (V1^T V1)_ij^2
 * + sum_ij d2_i d2_j (V2^T V2)_ij^2 - 2 sum_ij d1_i d2_j (V1^T V2)_ij^2, in FP64;
 * the three terms cancel down to err_cov^2, which leaves err_cov exact to
 * about sqrt(k eps64) absolute (1e-7 at k = 64; the paper's errors range from
 * 5e-4 up).  Waits for the device.
 * Errors: STATE, SHAPE (n != n_t), INVAL (null w or out, m_t < 2), CONVERGE, DEVICE. */
isvd_status isvd_risk(isvd_engine* eng, isvd_id id, const double* w, int64_t n, int32_t exact, isvd_risk_t* out,
                      void* hip_stream);

/* FP64 host copies of the factors: U (m_t x k, ldu), S (k), V (n_t x k, ldv).
 * Any pointer may be NULL to skip it.  Waits for the device. */
isvd_status isvd_get_factors(isvd_engine* eng, isvd_id id, double* U, int64_t ldu, double* S,
                             double* V, int64_t ldv, void* hip_stream);

/* FP64 host copy of A_t (m_t x n_t, lda).  Waits for the device. */
isvd_status isvd_get_matrix(isvd_engine* eng, isvd_id id, double* A, int64_t lda, void* hip_stream);

/* Current shape and rank (host-side view; no device access). */
isvd_status isvd_shape(isvd_engine* eng, isvd_id id, int64_t* m, int64_t* n, int32_t* k);

/* Free the stream's device memory; the id becomes invalid.  Waits for the
 * device, unless the block cache keeps the memory (isvd_set_block_cache). */
isvd_status isvd_release(isvd_engine* eng, isvd_id id);

/* Block cache for engines that create and release many streams (serving):
 * with bytes > 0, isvd_release keeps a stream's device block (up to `bytes`
 * in all) instead of freeing it, once the stream's own refresh has ended,
 * recording then an event on each of the engine's streams; a later isvd_init
 * whose block needs at most that size and at least four fifths of it reuses
 * the block, its work on the caller's stream ordered after those events.
 * Neither call then waits for the whole device, except that blocks past
 * the cap are freed 32 at a time after one wait.  A release during the
 * stream's own refresh returns at once; the block joins the cache when that
 * refresh has ended (checked by later releases and creations).  The caller
 * must have completed, or ordered before that later isvd_init's stream, any work it
 * queued on its own streams that touches the released stream.  Streams with
 * deferred U or A in host memory are freed as before.  bytes = 0 (the
 * default) frees every release at once; lowering the cap below what is
 * cached frees the cache.  When a new block does not fit the device, the
 * cache is freed and the allocation tried again.  Errors: INVAL. */
isvd_status isvd_set_block_cache(isvd_engine* eng, uint64_t bytes);

/* Batched tick: apply `count` requests to `count` distinct streams as one
 * sequence of batched launches on hip_stream (per-stream order is the order
 * of successive ticks), then evaluate each stream's policy and refresh the
 * streams whose policy fired.  Payloads must be device pointers in the
 * stream's storage dtype.  Validation happens for all requests before any
 * work is enqueued; on error nothing is applied.  Does not wait for the
 * device unless a policy needs device metrics.
 * Lanes: hip_stream uploads the requests and forks the update lanes (the
 * engine's own streams): the projections, cores and V rotations of the
 * 64-column rank bucket (and wider) run on one, the narrower ones' on
 * another -- with deferred U, the 32-column bucket on a second and the
 * 16- and 8-column ones on a third -- and hip_stream joins them all before
 * its next operation.
 * Pipelining: the U rotations run on the engine's rotation streams.  When
 * every request is a row append of a stream without a refresh policy, they
 * may still run after hip_stream has passed the call, overlapping the next
 * tick's projections and cores; every call that reads or replaces stream
 * state (metrics, factors, matrix, refresh, single updates, a tick that
 * reads U) first orders its stream after them, and isvd_sync does so
 * explicitly.  Otherwise the tick joins them into hip_stream before
 * returning.  With deferred U (isvd_set_deferred_u) each group's U rotation
 * follows its V rotation on its update lane instead, and the whole tick
 * ends on hip_stream.  Every read of a payload is ordered before hip_stream's next
 * operation (row payloads are not read by U rotations), so a payload may be
 * freed or overwritten in hip_stream's order as soon as the call returns.
 * Refreshes: the refreshes that a tick's policies fire (periodic, angle,
 * adaptive) run concurrently on the engine's refresh lanes (streams of
 * default priority, one host thread and one workspace per lane) and are not
 * joined into hip_stream: a stream under refresh is busy (isvd_stream_busy)
 * until its refresh is done, and every later call on that stream (a tick
 * that includes it, a single update, metrics, factors, matrix, refresh)
 * orders itself after it, so results do not depend on the overlap.  The
 * error policy's checks run in the tick, on hip_stream.
 * Errors: STATE, SHAPE, RANGE, CAPACITY, INVAL (duplicate stream, dtype),
 * CONVERGE (a lane refresh of a stream in the tick did not converge). */
isvd_status isvd_tick(isvd_engine* eng, int32_t count, const isvd_request* reqs, void* hip_stream);

/* Order hip_stream after every U rotation still pending on the engine's
 * rotation stream and every refresh queued on the refresh lanes (see
 * isvd_tick).  Does not wait on the host. */
isvd_status isvd_sync(isvd_engine* eng, void* hip_stream);

/* *busy = 1 while a refresh fired by a tick still runs for stream id on a
 * refresh lane, else 0 (does not wait).  A scheduler may leave busy streams
 * out of the next tick, so that their refresh overlaps the other streams'
 * updates.  Errors: STATE, INVAL, CONVERGE (the finished refresh did not
 * converge). */
isvd_status isvd_stream_busy(isvd_engine* eng, isvd_id id, int32_t* busy);

/* enable != 0 (the default): row-append ticks may leave their U rotations
 * pending (see isvd_tick) for throughput; 0: every tick joins them before
 * returning, for the shortest tick latency. */
isvd_status isvd_set_pipelining(isvd_engine* eng, int32_t enable);

/* Captured ticks (off by default).  With deferred U on, a tick whose
 * requests are all row appends of streams without a refresh policy is run
 * as one replay of a HIP graph that records its whole launch sequence (the
 * request upload, every bucket's projections, core and rotations on the
 * engine's update lanes, the joins).  The first tick of a request set --
 * the same streams in the same order -- captures the graph (a few ms); later
 * ticks of that set write their request records into the graph's pinned
 * buffer and launch it once, so the host's cost per tick is one launch.
 * Results are bit for bit those of the uncaptured tick.  A few request sets
 * are cached; other ticks run as before.  Disabling frees the cache. */
isvd_status isvd_set_tick_graphs(isvd_engine* eng, int32_t enable);

/* Segmented refresh batches (on by default): the refreshes that the
 * policies of one tick fire (Sec. 3: periodic, angle, adaptive rank; the
 * TruncatedSVD of Sec. 2.4.1), for FP32 streams whose refresh runs in the A
 * form (a block spanning all columns, or refresh_iters >= 0), are computed
 * together: one launch per refresh phase covers all of them, each stream's
 * workspace in its own region of one engine buffer.  Every stream's result
 * is bit for bit that of its own refresh.  enable = 0 refreshes them one by
 * one on the refresh lanes.  Errors: INVAL. */
isvd_status isvd_set_segmented_refresh(isvd_engine* eng, int32_t enable);

/* Deferred U (Brand's factorised update of the left basis, U = U0 W, W a
 * k x k FP64 matrix kept with W^-1): enable != 0 lets row appends of
 * eligible streams (FP32 storage, rank up to 64, no angle / error / adaptive
 * policy) change W alone -- the new row of U0 is b W'^-1 with b the new row of
 * U, W' = W A with A the core's rotation restricted to the old rows -- instead
 * of rotating all m rows of U (Alg. A1's U' = [[U, 0], [0, 1]] U_K, the same
 * matrix in factored form).  V still rotates every append, in place.  An
 * append that would change the rank or whose new row carries more than half
 * of its column's weight rotates U explicitly (W folded into the rotation),
 * and so does every (m / 8k)-th row append of a stream (at most every 256th),
 * staggered across streams, which keeps W within a few percent of
 * orthogonal.  Column appends, entry updates, factor read-back and exact
 * metrics make U explicit first (one pass U0 W); a refresh resets W to I.
 * 0 (the default) makes every deferred U explicit on hip_stream and rotates
 * U on every append again.  Allocates the W buffers of existing eligible
 * streams when enabling.  Errors: INVAL, DEVICE. */
isvd_status isvd_set_deferred_u(isvd_engine* eng, int32_t enable, void* hip_stream);

/* The engine's rotation stream (a hipStream_t).  A pipelined tick (explicit
 * U, row appends of streams without a refresh policy) leaves its U rotations
 * on it; every other tick -- deferred U included -- ends on the caller's
 * stream.  So a tick's updates are all done once both the caller's stream
 * and this stream have passed it: record an event on each (refreshes the
 * tick fired may still run; see isvd_tick). */
isvd_status isvd_rotation_stream(isvd_engine* eng, void** out);

/* GPU time of one kernel launch of the update sequence, collected while
 * profiling is on (HIP events recorded around the launch on its stream). */
typedef struct {
    int32_t phase;          /* 0 projection pass 1, 1 projection pass 2, 2 core,
                               3 rotation of U, 4 rotation of V */
    int32_t kc;             /* rank bucket of the launch (capacity of its U / V rows) */
    int32_t fp64;           /* 1 if the launch works on FP64 storage */
    int32_t nreq;           /* requests served by the launch */
    int64_t blocks;         /* blocks launched */
    double ms;              /* GPU time */
} isvd_launch_time;

/* enable != 0: drop earlier records and start timing every update launch;
 * enable == 0: stop. */
isvd_status isvd_profile(isvd_engine* eng, int32_t enable);

/* Copy up to `cap` records (oldest first) to `out`, the number available to
 * *count.  Waits for the recorded launches to finish. */
isvd_status isvd_profile_read(isvd_engine* eng, isvd_launch_time* out, int32_t cap, int32_t* count);

/* Block shapes of the FP32 matrix-core rotation: variant v runs
 * {rows per block, 16-row tiles per wave step, prefetch of the next step} =
 * 0: {256, 1, yes}, 1: {512, 1, yes} (default), 2: {1024, 1, yes},
 * 3: {1024, 2, no}, 4: {2048, 2, no}. */
#define ISVD_ROT_VARIANTS 5

/* Tile autotuner.  For each rank bucket of the FP32 matrix-core rotation
 * (8, 16, 32, 64), times every variant on a synthetic batch of 64 bases of
 * 32768 x bucket (plus 1024 x bucket) -- about 1.1 GB of HBM for the widest
 * bucket, allocated for the call and freed before it returns -- and keeps
 * the fastest for later launches (a variant replaces an earlier, faster-so-far
 * one only when it is at least 3% faster, so near-equal shapes resolve to
 * the lower index and repeated tunings agree).  variant_out (4 entries, may be NULL)
 * receives the choices, ms_out (4 x ISVD_ROT_VARIANTS entries, bucket major,
 * may be NULL) the mean time of one launch per variant.  Waits for the
 * device.  Errors: NOMEM, DEVICE. */
isvd_status isvd_autotune(isvd_engine* eng, void* hip_stream, int32_t* variant_out, double* ms_out);

/* Use variant (0 .. ISVD_ROT_VARIANTS-1) for the FP32 rotation of bucket kc
 * (8, 16, 32, 64).  Errors: INVAL. */
isvd_status isvd_set_rotation_variant(isvd_engine* eng, int32_t kc, int32_t variant);

/* ------------------------------------------------------------------ serving
 * A server schedules update requests of many streams onto one engine:
 * requests queue per stream in arrival order; each scheduling step retires
 * streams whose lifetime is complete, admits waiting streams in FIFO order
 * while their footprint (isvd_stream_bytes) fits the HBM budget, and
 * launches one tick of the oldest queued request of every admitted stream
 * that is not busy with a refresh, among the requests whose arrival time has
 * passed (continuous batching: requests that
 * arrive while ticks run on the device join the next tick; up to
 * max_inflight ticks overlap on the device, and refreshes fired by a tick
 * overlap the following ticks of the other streams).
 * A request whose length or indices no longer fit its stream completes at
 * once with ISVD_E_SHAPE and is not part of a tick.  Times are seconds on
 * the server's host clock (isvd_server_clock); completion times come from
 * an event after each tick's last work.  One host thread per server. */
typedef struct isvd_server isvd_server;   /* opaque */

typedef struct {
    uint64_t hbm_budget;    /* bytes the admitted streams may hold (0 = no limit) */
    int32_t max_batch;      /* most requests per tick (0 = no limit) */
    int32_t max_inflight;   /* ticks on the device before a step waits for the oldest (>= 1) */
} isvd_server_config;

typedef struct {
    int64_t req;            /* id from isvd_server_submit */
    int64_t ticket;         /* stream ticket */
    int32_t kind;           /* ISVD_ROW / ISVD_COL / ISVD_ENTRY */
    int32_t status;         /* ISVD_OK or the error of the request */
    double arrival_s;       /* as submitted */
    double admit_s;         /* when its stream was admitted */
    double launch_s;        /* when its tick was launched */
    double done_s;          /* when its tick had finished on the device */
} isvd_completion;

typedef struct {
    int64_t waiting, admitted, retired;   /* streams */
    int64_t queued;                        /* requests not yet launched */
    uint64_t hbm_used;                     /* footprint of the admitted streams */
    int32_t inflight_ticks, pad;
    int64_t ticks, tick_requests;          /* ticks launched and the requests they carried */
    double host_admit_s;                   /* host seconds in admissions (isvd_init) */
    double host_tick_s;                    /* host seconds in isvd_tick (policy decisions included) */
    double host_wait_s;                    /* host seconds blocked on in-flight ticks */
    double host_release_s;                 /* host seconds releasing retired streams */
} isvd_server_stats_t;

/* hip_stream: the stream the server's ticks and admissions run on. */
isvd_status isvd_server_create(isvd_engine* eng, const isvd_server_config* cfg, void* hip_stream,
                               isvd_server** out);
isvd_status isvd_server_destroy(isvd_server* srv);
double isvd_server_clock(isvd_server* srv);
const char* isvd_server_error(isvd_server* srv);

/* Register a stream (admitted later by isvd_init with this config and A0, a
 * device pointer the caller keeps valid until then); lifetime = requests
 * after whose completion the stream is released (0 = kept).  *ticket names
 * the stream in the server.  Errors: INVAL, BUDGET (larger than the budget). */
isvd_status isvd_server_add_stream(isvd_server* srv, const isvd_config* cfg, const void* A0, int64_t lda,
                                   int32_t dtype, int64_t lifetime, int64_t* ticket);

/* Queue a request (its id field is ignored; payloads are device pointers
 * kept valid until the request completes).  Errors: INVAL, STATE. */
isvd_status isvd_server_submit(isvd_server* srv, int64_t ticket, const isvd_request* req, double arrival_s,
                               int64_t* req_id);

/* isvd_server_submit for count requests (tickets[q], reqs[q], arrival_s[q]);
 * req_ids may be NULL.  Stops at the first error (earlier ones stay queued). */
isvd_status isvd_server_submit_many(isvd_server* srv, int32_t count, const int64_t* tickets,
                                    const isvd_request* reqs, const double* arrival_s, int64_t* req_ids);

/* One scheduling step (see above); *launched = requests in the tick launched. */
isvd_status isvd_server_step(isvd_server* srv, int32_t* launched);

/* Wait for every launched tick and stamp its requests. */
isvd_status isvd_server_drain(isvd_server* srv);

/* Move up to cap completion records (oldest first) to out; *count = moved. */
isvd_status isvd_server_poll(isvd_server* srv, isvd_completion* out, int32_t cap, int32_t* count);

isvd_status isvd_server_stats(isvd_server* srv, isvd_server_stats_t* out);

/* Engine stream id of a ticket (-1 before admission) and its state
 * (0 waiting, 1 admitted, 2 retired). */
isvd_status isvd_server_stream(isvd_server* srv, int64_t ticket, isvd_id* id, int32_t* state);

/* Message for the last error on this thread ("" if none). */
const char* isvd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ISVD_H */
