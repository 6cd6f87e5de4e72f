/*
 * tsgpu: trapping-set search of the modified Cole importance-sampling method
 * (V. Usatyuk, "A Modified Cole's Importance Sampling Method for Low Error Floor
 * QC-LDPC Codes Construction", arXiv 2208.05795) on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every call returns a ts_status (0 = TS_OK, negative = error); the text
 * of the last error of the calling thread is returned by ts_last_error().
 *
 * Conventions
 *  - Indices are 0-based.  For a QC code the variable in block column j at
 *    circulant position c is j*z + c, the check in block row i at position r is
 *    i*z + r (Section II).
 *  - The caller owns every input and output array; inputs are copied or consumed
 *    before the call returns.  ts_ctx and ts_code are opaque and owned by the
 *    library until ts_destroy / ts_free_code.
 *  - Arrays named in ts_search_opts.mem == TS_MEM_DEVICE must be device memory on
 *    the context's device (e.g. torch tensors); otherwise host memory.
 *  - Every synchronous call on a context runs on the context's stream and
 *    returns after that stream has finished the call's work.  Synchronous calls
 *    on one context are serialised by an internal mutex; separate contexts are
 *    independent.  Submitted jobs (ts_submit) run on the serving workers' own
 *    streams, concurrently with each other and with synchronous calls.
 *  - No CPU fallback exists: without a usable HIP device, ts_create fails with
 *    TS_E_DEVICE.
 */
#ifndef TSGPU_H
#define TSGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ts_ctx ts_ctx;
typedef struct ts_code ts_code;

typedef enum {
    TS_OK = 0,
    TS_E_INVAL = -1,     /* bad argument, shape or code */
    TS_E_NOMEM = -2,     /* device or host allocation failed */
    TS_E_DEVICE = -3,    /* HIP runtime error or no usable device */
    TS_E_STATE = -4,     /* object used in the wrong state (e.g. wrong context) */
    TS_E_BUSY = -5,      /* admission refused (memory budget) */
    TS_E_TRUNC = -6,     /* output buffer too small; sizes were still reported */
    TS_E_CANCELLED = -7  /* job cancelled */
} ts_status;

/* ---- context --------------------------------------------------------------- */

typedef struct {
    int32_t device;        /* HIP device ordinal */
    void *hip_stream;      /* borrowed hipStream_t; NULL = the library creates one */
    /* optional device allocator (both NULL = hipMalloc/hipFree); alloc returns
     * NULL on failure */
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
    size_t hbm_budget_bytes;   /* 0 = no limit; the serving admission check uses it */
    size_t rec_buffer_bytes;   /* device buffer for the candidate error sets of one search
                                * launch; 0 = 256 MiB.  Never smaller than one pattern's
                                * worst case; a launch whose candidates overflow it is
                                * re-run in smaller chunks (same results and statistics) */
} ts_ctx_opts;

/* Creates a context on opts->device.  opts may be NULL (device 0, own stream).
 * Errors: TS_E_DEVICE (no device / HIP failure), TS_E_INVAL. */
int ts_create(const ts_ctx_opts *opts, ts_ctx **out);
/* Frees the context and every code still loaded on it.  Queued served jobs are
 * cancelled and running ones finish first.  No other call on the context may
 * be in progress or follow (including ts_poll waits of other threads). */
int ts_destroy(ts_ctx *ctx);
/* Message of the last failed call on this thread ("" if none).  Valid until the
 * thread's next call. */
const char *ts_last_error(void);

/* ---- codes (Section II, eq. 1-3) ------------------------------------------ */

#define TS_CODE_CSR 1
#define TS_CODE_QC 2

typedef struct {
    int32_t kind;              /* TS_CODE_CSR or TS_CODE_QC */
    /* CSR form: H with rows = checks; row_ptr[m+1] (int64), col_idx[nnz] */
    int32_t n, m;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    /* QC form: mb x nb exponent matrix, row-major; -1 = zero block P^inf,
     * 0..z-1 = the circulant P^s whose row r has its one in column (r+s) mod z */
    int32_t mb, nb, z;
    const int32_t *shifts;
} ts_code_desc;

/* Validates and expands the code, computes its girth (shortest Tanner-graph
 * cycle, 0 = none) and uploads the graph to the device.  Host arrays only.
 * Rejects (TS_E_INVAL): out-of-range entries, duplicate edges, empty columns,
 * checks of degree < 2, n or m above 2^24. */
int ts_load_code(ts_ctx *ctx, const ts_code_desc *desc, ts_code **out);

typedef struct {
    int32_t n, m;
    int64_t e;          /* edges (nonzeros of H) */
    int32_t girth;      /* 0 = cycle-free */
    int32_t z;          /* circulant size, 0 for CSR codes */
    int32_t dv_max, dc_max;
    int32_t n_layers;   /* layers of the layered min-sum schedule: the block rows
                         * of a QC code, else the greedy variable-disjoint
                         * colouring of the checks; 0 = more than 64 layers
                         * (TS_DEC_LNMS_Q4 is then rejected) */
    int32_t streamed_qc;   /* 1: the streamed-frame decoder of this QC code derives
                            * its neighbour and message-slot indices from the
                            * circulant shifts instead of reading index tables */
} ts_code_info_t;
int ts_code_info(const ts_code *code, ts_code_info_t *out);
/* Check-major CSR of the expanded H (host arrays row_ptr[m+1], col[e]). */
int ts_code_csr(const ts_code *code, int64_t *row_ptr, int32_t *col);
int ts_free_code(ts_ctx *ctx, ts_code *code);

/* ---- impulse patterns (Section III, impulse tree of Fig. 3) ----------------- */

#define TS_PAT_SINGLES 1   /* every variable alone (width 1) */
#define TS_PAT_PAIRS 2     /* every pair at Tanner distance 2 or 4 (width 2) */
#define TS_PAT_TRIPLES 3   /* every {v1,v2,v3} on a tree path v1-c-v2-c'-v3, c != c' (width 3) */
/* OR-ed into the kind for a QC code: one pattern per orbit of the circulant
 * shift v = jz + c -> jz + (c + t) mod z (the automorphism of Section II), namely
 * the one equal to its canonical form (the lexicographically smallest sorted
 * image).  The family lists are unions of whole orbits and the decoders commute
 * with the shift, so searching the reduced list finds the same canonical TS with
 * the same k*; only first_pattern indexes the shorter list.  About z-fold
 * fewer patterns.  TS_E_INVAL for a code loaded in CSR form. */
#define TS_PAT_QC_ORBITS 0x100

/* Writes the sorted pattern list of one family (row-major, width = kind & 0xff)
 * to the host array out when cap (in patterns) allows; *n_out = number of
 * patterns.  Returns TS_E_TRUNC when cap is too small (out untouched). */
int ts_make_patterns(ts_ctx *ctx, const ts_code *code, int32_t kind, int32_t *out,
                     int64_t cap, int64_t *n_out);

/* ---- impulse search with bisection (Section III) --------------------------- */

#define TS_DEC_OMS_I8 0     /* offset min-sum, saturating int8 messages */
#define TS_DEC_SPA_F32 1    /* sum-product: float32 phi arithmetic; channel values,
                             * messages and APP sums stored as Q20 fixed point
                             * (int32, step 2^-20) */
/* quantised normalised layered min-sum (Section III, Fig. 2): channel values
 * and check-to-variable messages on 4 bits ([-7, 7]; llr_scale sets the
 * channel scale, q = sat7(round(llr_scale h))), variable-to-check messages and
 * APP values on 6 bits ([-31, 31]), check magnitude floor(3/4 min), layers =
 * block rows of a QC code, else checks in index order each in the first layer
 * holding none of its variables; k_den must be 16.  Register layout only. */
#define TS_DEC_LNMS_Q4 2
#define TS_EXTRACT_PATH 0      /* candidates from every failing decode of the bisection */
#define TS_EXTRACT_CRITICAL 1  /* candidates from the decode at k* only */
#define TS_MEM_HOST 0
#define TS_MEM_DEVICE 1
/* Decoder layouts.  Register: one workgroup per frame with the messages in
 * registers and the APP values in LDS (codes whose checks fit one workgroup).
 * Streamed: one workgroup per frame with the messages in global memory (any
 * code whose APP values fit in LDS, n up to about 39k).  Both compute the same
 * integers, so results do not depend on the layout. */
#define TS_LAYOUT_AUTO 0       /* autotuned among the layouts and shapes that fit */
#define TS_LAYOUT_REGISTER 1
#define TS_LAYOUT_STREAMED 2   /* either streamed variant (autotuned) */
/* The streamed layout's two variants, forced: GATHER rebuilds each APP sum in
 * a variable pass that reads the variable's messages back; ACCUM adds the
 * messages into a second LDS array with integer atomics during the check pass
 * (8 bytes of LDS per variable instead of 4; n up to about 19k).  Statistics
 * report both as TS_LAYOUT_STREAMED, with checks_per_thread = 0 (GATHER) or 1
 * (ACCUM). */
#define TS_LAYOUT_STREAMED_GATHER 3
#define TS_LAYOUT_STREAMED_ACCUM 4

typedef struct {
    int32_t decoder;           /* TS_DEC_* */
    int32_t max_iter;          /* flooding iterations per decode, 1..64 */
    int32_t oms_offset;        /* OMS offset beta on the int8 scale (>= 0) */
    double ebn0_db, rate;      /* sigma^2 = 1/(2 rate 10^(ebn0/10)), h = 2/sigma^2 */
    double llr_scale;          /* OMS: int8 value of an unperturbed bit is round(llr_scale*h) */
    int32_t k_max;             /* amplitude grid eps_k = k/k_den, k = 0..k_max */
    int32_t k_den;             /* OMS requires 16 */
    int32_t a_max;             /* largest TS kept, 1..16 */
    int32_t extract_mode;      /* TS_EXTRACT_* */
    int32_t collect_from_iter; /* first iteration whose error set is sieved; -1 = girth/2 */
    int32_t mem;               /* TS_MEM_HOST / TS_MEM_DEVICE for patterns and outputs */
    int32_t layout;            /* TS_LAYOUT_*; TS_E_INVAL if the forced layout does not fit */
    int32_t full_iterations;   /* 0: a decode that reaches a fixed point (no check message
                                * changes in an iteration, so every later iteration repeats
                                * the last one) stops computing and fills in its remaining
                                * iterations; nonzero: compute every iteration.  Results are
                                * identical; statistics count computed iterations only. */
} ts_search_opts;

typedef struct {            /* caller-owned arrays of n_patterns entries */
    int32_t *k_crit;        /* critical grid index k*, -1 = decoded at every amplitude */
    int32_t *iters_crit;    /* iterations of the decode at k* (0 if k* = -1) */
    int32_t *iters_lo;      /* iterations of the last successful decode on the path */
    int32_t *tmin_crit;     /* first minimum-syndrome iteration at k* (0 if k* = -1) */
    int32_t *n_cand;        /* nonempty candidate sets with a <= a_max (before dedup) */
} ts_search_out;

/* For every pattern (row p of patterns[n_patterns][width], entries -1 = unused,
 * width 1..16) the impulse bits get h(1 - eps), all others h, on the all-zero
 * BPSK codeword.  The decode at k_max runs first; if it fails, bisection on
 * [0, k_max] finds k* (fail at k*, success at k*-1).  From failing decodes the
 * error sets S(x_t) of iterations collect_from_iter..last are sieved into
 * S1 = Tree(S u I) and S2 = Tree(TS(S u I)) when |S u I| <= 2 a_max; every
 * nonempty result with a <= a_max is canonicalised to its QC-orbit
 * representative and merged into the code's TS table (read by ts_collect).
 * Tree(V): variables of the 2-core of the subgraph induced by V.  TS(V): V plus
 * every outside variable with two checks in one connected component of it. */
int ts_impulse_search(ts_ctx *ctx, ts_code *code, const ts_search_opts *opts,
                      const int32_t *patterns, int32_t n_patterns, int32_t width,
                      ts_search_out *out);

/* ---- collected trapping sets (Section II TS(a,b), Section III ordering) ----- */

typedef struct {
    int32_t a, b;            /* |set|, odd-degree checks of the induced subgraph */
    int32_t orbit;           /* size of its QC shift orbit (1 for CSR codes) */
    int32_t first_pattern;   /* smallest pattern index that produced it */
    int32_t k_crit;          /* smallest k* among the patterns that produced it */
    int32_t reserved;
    int64_t bits_off;        /* offset of its variables in the bits array */
} ts_record;

/* Copies the code's TS table, ordered by b/a, then a, then the canonical tuple.
 * recs[cap] and bits[bits_cap] are host arrays; cap = 0 queries sizes only.
 * *n_out / *bits_out always receive the full sizes; TS_E_TRUNC if they exceed
 * the capacities. */
int ts_collect(ts_ctx *ctx, const ts_code *code, ts_record *recs, int64_t cap,
               int64_t *n_out, int32_t *bits, int64_t bits_cap, int64_t *bits_out);
/* Empties the code's TS table. */
int ts_reset_ts(ts_ctx *ctx, ts_code *code);

/* ---- importance sampling of one TS (Section I/II, Cole's TS weighting) ------ */

#define TS_IS_COUNT_ALL 0   /* every failing frame counts */
#define TS_IS_COUNT_TS 1    /* only failing frames whose final hard decision has every
                             * bit of T in error (the frames of T's own error event) */
#define TS_SHIFT_EPS 0      /* shift < 0: s = eps* of the SPA impulse on the whole set */
#define TS_SHIFT_PILOT 1    /* shift < 0: s chosen by pilot runs (ts_is_estimate) */
#define TS_SHIFT_MIX 2      /* shift < 0: a mixture of the shifts eps* k/16, k = 0..16
                             * (ts_is_estimate) */

typedef struct {
    int32_t max_iter;        /* SPA iterations */
    double ebn0_db, rate;
    double shift;            /* mean shift s of the TS bits; < 0: chosen by shift_rule */
    int64_t n_frames;        /* >= 2 */
    uint64_t seed;           /* Philox key */
    uint64_t frame_base;     /* first frame counter (resumable streams) */
    uint32_t stream;         /* Philox stream tag */
    int32_t layout;          /* TS_LAYOUT_* (AUTO: register layout when it fits) */
    int32_t full_iterations; /* as in ts_search_opts (also for the eps* searches) */
    int32_t count_mode;      /* TS_IS_COUNT_ALL or TS_IS_COUNT_TS */
    int32_t shift_rule;      /* TS_SHIFT_EPS, TS_SHIFT_PILOT or TS_SHIFT_MIX (shift < 0) */
    int64_t pilot_frames;    /* TS_SHIFT_PILOT: frames per grid point (0: 2000) */
} ts_is_opts;

typedef struct {
    double p_hat, var, ci_lo, ci_hi, sum_w, sum_w2;
    int64_t n, n_fail;
    double shift_used;
} ts_is_result;

/* Importance sampling of one set T (Section I/II, Cole's TS weighting; the
 * estimator is a reading, the paper leaves it open).  Frame f draws
 * n_v ~ N(0,1) from Philox4x32-10 (counter (v>>2, f_lo, f_hi, stream), key =
 * seed, Box-Muller), receives y_v = 1 - s[v in T] + sigma n_v, is decoded by
 * the sum-product decoder, and contributes 1[counted] w, where counted is
 * "failed" (TS_IS_COUNT_ALL) or "ended in T's own error event: every bit of T
 * and at most 2a bits in all decided 1" (TS_IS_COUNT_TS), and
 * w = exp(-a s^2/(2 sigma^2) + (s/sigma) sum_{v in T} n_v) is the likelihood
 * ratio.  P = mean, Var = sample variance / K, 95% CI = P +- 1.96 sqrt(Var).
 * The shift s: the given one (shift >= 0); eps* of the SPA impulse on the
 * whole set (TS_SHIFT_EPS); the grid point eps* (1/2 + i/16), i = 0..8, whose
 * pilot estimate (its own frames frame_base + 2^40 + i P, P = pilot_frames)
 * has the least relative variance among points with >= 10 counted frames
 * (TS_SHIFT_PILOT); or, TS_SHIFT_MIX, the frames split in frame order over
 * the 17 shifts s_k = eps* k/16 (frame f in component floor(17 f / K)), each
 * counted frame weighted by the balance heuristic
 * w = 1 / sum_k (K_k/K) exp((s_k/sigma) D - a s_k^2/(2 sigma^2)),
 * D = sum_{v in T} (1 - y_v)/sigma (shift_used reports eps*).  fail_out
 * (optional host array [n_frames]) receives each frame's flags: bit 0 the
 * decode failed, bit 1 it ended in T's own error event. */
int ts_is_estimate(ts_ctx *ctx, ts_code *code, const int32_t *ts_bits, int32_t a,
                   const ts_is_opts *opts, ts_is_result *res, uint8_t *fail_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call an allocator): ts_is_estimate with
 * no device allocation.  Every device buffer of the call lives in one fixed
 * device array of 32 MiB, set up by ts_create on the context's device and held
 * by each GPU the library runs on until the process ends.  Same arguments,
 * results and statistics as ts_is_estimate; the caller still owns ts_bits,
 * res and fail_out (host).  Limits: shift >= 0 (no eps* or pilot search),
 * n_frames <= 2^21, and codes whose IS launch shape is the register layout
 * (whose frames stay in LDS and registers, fixed-point exit included).  Calls
 * on one GPU share the array:
 * calls that overlap on a GPU (two contexts on one device, used from two
 * threads) race; calls on one context are serialised.  Errors: TS_E_INVAL
 * beyond the limits (with the limit in the message), as ts_is_estimate
 * otherwise. */
int ts_is_estimate_noalloc(ts_ctx *ctx, ts_code *code, const int32_t *ts_bits, int32_t a,
                           const ts_is_opts *opts, ts_is_result *res, uint8_t *fail_out);

/* ---- cycle / EMD spectrum (Section II, Table II) ------------------------- */

/* Simple cycles of length 4..max_len of a QC code through the position-0
 * variable of every block column, found by walking exponent chains on the base
 * matrix (a walk closes when its alternating shift sum is 0 mod z, Section II),
 * bucketed by length and EMD (the number of (cycle variable, check) incidences
 * whose check meets the cycle in exactly one variable):
 * out[(len / 2) * (emd_max + 1) + emd] (caller-owned, overwritten) counts
 * (cycle, position-0 variable) incidences, so an orbit of cycles of length 2l
 * adds l.  EMD above emd_max is counted at emd_max.  Host computation.
 * Errors: TS_E_INVAL (CSR-form code, max_len not even in 4..16). */
int ts_cycle_emd(ts_ctx *ctx, const ts_code *code, int32_t max_len, int32_t emd_max, int64_t *out);

/* ---- TS spectrum and union bound (Section III; Tables III and IV) -------- */

/* The code's TS table counted by (a, b): counts[a * (b_max + 1) + b] for
 * 0 <= a <= a_max, 0 <= b <= b_max (caller-owned, overwritten), each canonical
 * TS counted once (by_orbit != 0, one per QC orbit) or with its orbit size
 * (by_orbit == 0, every set of the code).  Sets beyond the bounds are not
 * counted.  Errors: TS_E_INVAL (a_max outside 1..16, b_max outside 0..1024). */
int ts_spectrum(ts_ctx *ctx, const ts_code *code, int32_t a_max, int32_t b_max, int32_t by_orbit,
                int64_t *counts);

typedef struct {
    int32_t n_ts;            /* the first n_ts sets of the code's TS table, in its order */
    int32_t n_snr;
    const double *ebn0_db;   /* [n_snr] host array */
    int32_t max_iter;        /* SPA iterations */
    double rate;             /* design rate for sigma */
    double shift;            /* IS mean shift; < 0: chosen per (set, SNR) by shift_rule */
    int64_t n_frames;        /* frames per (set, SNR), >= 2 */
    uint64_t seed;           /* Philox key; stream tag of (set t, SNR i) = (i << 16) | t */
    int32_t layout;          /* TS_LAYOUT_* */
    int32_t count_mode;      /* TS_IS_COUNT_ALL or TS_IS_COUNT_TS (as in ts_is_opts) */
    int32_t shift_rule;      /* TS_SHIFT_EPS, TS_SHIFT_PILOT or TS_SHIFT_MIX (as in ts_is_opts) */
    int64_t pilot_frames;    /* as in ts_is_opts */
} ts_ub_opts;

typedef struct {
    double ebn0_db;
    double fer;              /* sum over the sets of orbit x P_hat */
    double var;              /* sum over the sets of orbit^2 x Var(P_hat) */
    double ci_lo, ci_hi;     /* fer -+ 1.96 sqrt(var) */
} ts_ub_point;

/* Union bound on the frame error rate of the code's decoder (Section III):
 * FER(SNR) ~ sum over the canonical sets T of orbit(T) x P_T(SNR), each P_T an
 * importance-sampling estimate as in ts_is_estimate.  All n_ts x n_snr
 * estimates run as one batch.  out[n_snr] receives the bound per SNR; per_ts,
 * if not NULL, [n_snr][n_ts] the individual estimates.  Errors: TS_E_INVAL
 * (fewer than n_ts sets in the table, n_ts x n_snr > 4096, bad options). */
int ts_union_bound(ts_ctx *ctx, ts_code *code, const ts_ub_opts *opts, ts_ub_point *out,
                   ts_is_result *per_ts);

/* ---- serving: continuous batching of submitted jobs ------------------------ */

#define TS_JOB_SEARCH 1
#define TS_JOB_IS 2
#define TS_JOB_QUEUED 0
#define TS_JOB_RUNNING 1
#define TS_JOB_DONE 2
#define TS_JOB_CANCELLED 3

typedef struct {
    int32_t kind;              /* TS_JOB_SEARCH or TS_JOB_IS */
    ts_code *code;             /* a code loaded on the same context */
    /* TS_JOB_SEARCH: as ts_impulse_search; search.mem must be TS_MEM_HOST and
     * patterns[n_patterns][width] is copied at submission */
    ts_search_opts search;
    const int32_t *patterns;
    int32_t n_patterns, width;
    /* TS_JOB_IS: as ts_is_estimate; ts_bits[a] is copied at submission */
    ts_is_opts is;
    const int32_t *ts_bits;
    int32_t a;
} ts_job_desc;

typedef struct {
    int32_t state;             /* TS_JOB_QUEUED / RUNNING / DONE / CANCELLED */
    int32_t status;            /* ts_status of a finished job (TS_E_CANCELLED if cancelled) */
    double submit_ms, start_ms, end_ms;   /* milliseconds since ts_create */
    int64_t edge_updates;
    int64_t device_bytes;      /* the admission estimate of the job */
    int64_t n_ts, n_bits;      /* search jobs: size of the job's TS list */
    int32_t n_patterns;
    int32_t reserved;
    ts_is_result is;           /* IS jobs: the estimate */
} ts_job_info;

/* Starts `slots` serving workers (1..16), each with its own HIP stream (default
 * priority) and stream-ordered device allocations.  Optional: the first
 * ts_submit starts 4.  The device-memory budget is ts_ctx_opts.hbm_budget_bytes,
 * or half of the free device memory when that is 0.  TS_E_STATE if started. */
int ts_serve_start(ts_ctx *ctx, int32_t slots);
/* Queues a job (inputs copied) and returns its id.  A job starts as soon as a
 * worker is free and its memory estimate fits beside the running jobs (first
 * fit in submission order).  Each search job has its own TS table, so its
 * results are those of the same call run alone.  TS_E_BUSY if the job alone
 * exceeds the budget; TS_E_INVAL on bad arguments (checked at submission).
 * Thread-safe. */
int ts_submit(ts_ctx *ctx, const ts_job_desc *job, uint64_t *job_id);
/* Reports a job's state; wait != 0 blocks until it is done or cancelled.  A
 * failed job's message is available through ts_last_error(). Thread-safe. */
int ts_poll(ts_ctx *ctx, uint64_t job_id, int32_t wait, ts_job_info *info);
/* Copies a finished search job's outputs: per-pattern arrays into out (host,
 * n_patterns each, any may be NULL) and its ordered TS list into recs[cap] /
 * bits[bits_cap] (cap = bits_cap = 0 skips it; TS_E_TRUNC if too small). */
int ts_job_outputs(ts_ctx *ctx, uint64_t job_id, ts_search_out *out, ts_record *recs,
                   int64_t cap, int32_t *bits, int64_t bits_cap);
/* Cancels a queued job at once; a running job finishes its kernels and is then
 * reported as cancelled with no results.  Thread-safe. */
int ts_cancel(ts_ctx *ctx, uint64_t job_id);
/* Runs jobs[n_jobs] (search and IS jobs on any codes of this context, as for
 * ts_submit) as one batch: jobs whose decoder kernel shape is the same share
 * ONE persistent launch whose workgroups take patterns / frames of all of them
 * from a single queue; launches of different shapes overlap on side streams;
 * nothing returns to the host until every decode is done.  Each job's results
 * equal those of the same call run alone.  Synchronous and serialised with the
 * other calls of the context.  On return the jobs are finished jobs of the
 * serving store: read them with ts_poll / ts_job_outputs and free them with
 * ts_release, using the ids written to job_ids[n_jobs].  Errors: TS_E_INVAL if
 * any job fails validation (nothing runs), at most 4096 jobs. */
int ts_run_batch(ts_ctx *ctx, const ts_job_desc *jobs, int32_t n_jobs, uint64_t *job_ids);

/* Frees a finished or cancelled job's results; TS_E_BUSY while in flight. */
int ts_release(ts_ctx *ctx, uint64_t job_id);

/* ---- measurements of the last call ---------------------------------------- */

typedef struct {
    double decode_ms;        /* summed HIP-event time of the decode kernels */
    double extract_ms;       /* same for the sieve/canonicalise/insert kernels */
    double total_ms;         /* the whole call on the stream */
    int64_t decodes;         /* decodes executed */
    int64_t edge_updates;    /* sum over decodes of computed iterations x edges (iterations
                              * filled in after a fixed point are not counted) */
    int64_t candidates;      /* raw candidate error sets written */
    int32_t decode_launches;
    int32_t extract_launches;
    int32_t block_threads;   /* workgroup size of the decode kernel */
    int32_t grid_blocks;     /* workgroups of the decode kernel */
    int32_t layout;          /* TS_LAYOUT_REGISTER / TS_LAYOUT_STREAMED of the last decode */
    int32_t checks_per_thread;   /* register layout: checks per thread */
} ts_stats;
int ts_get_stats(ts_ctx *ctx, ts_stats *out);

/* Measurement aid (not a step of the paper's method): the device's LDS read
 * bandwidth in bytes/s, the best of three timed launches of a kernel whose
 * workgroups (20 per compute unit, 32 KB of LDS each) read their LDS with
 * bank-conflict-free 16-byte loads.  Runs on the context's stream and waits
 * for it; allocates and frees a small device buffer.  TS_E_INVAL on null
 * arguments, TS_E_DEVICE / TS_E_NOMEM on runtime failures. */
int ts_probe_lds(ts_ctx *ctx, double *bytes_per_s);

#ifdef __cplusplus
}
#endif
#endif /* TSGPU_H */
