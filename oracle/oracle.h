/*
 * CPU oracle for the trapping-set (TS) search of the modified Cole importance
 * sampling method (Usatyuk, arXiv 2208.05795).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code with the library under paper_2208_05795_amd/ and includes nothing from
 * there.
 *
 * Every function below follows the paper as cited; where the paper is silent
 * the documented reading is stated beside the function.  Indices are 0-based;
 * a QC code's variable j*Z+c is column c of block column j, its check i*Z+r is
 * row r of block row i.
 *
 * Parity status of each part:
 *   code expansion, girth .......... pinned (Table II/V cycle counts, hand graphs)
 *   Tree / TS / (a,b) / canonical .. pinned (hand graphs, Table III structural cells,
 *                                    brute force, shift invariance)
 *   OMS decoder arithmetic ......... pinned (hand-computed iterations)
 *   SPA decoder arithmetic ......... pinned (exact MAP on cycle-free graphs)
 *   Philox4x32-10 .................. pinned (an independent implementation, rocRAND)
 *   IS estimator ................... pinned (closed-form Gaussian tail)
 *   bisection k*, iteration counts,  parity unpinned by the paper: its decoder is
 *   TS lists, IS numbers ........... unspecified; checked oracle <-> device only
 */
#ifndef TS_ORACLE_H
#define TS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- code (Section II, eq. 1-3) ------------------------------------------ */
typedef struct or_code or_code;

/* QC form: mb x nb exponents, -1 = zero block, else 0..z-1.  Block (i,j) with
 * exponent s puts H[i*z + r][j*z + (r+s) mod z] = 1 (P^s = identity shifted
 * right s times).  Returns NULL on invalid input. */
or_code *or_code_qc(int mb, int nb, int z, const int32_t *shifts);
/* CSR form: rows = checks.  Returns NULL on invalid input (range, duplicates,
 * empty rows or columns). */
or_code *or_code_csr(int n, int m, const int64_t *row_ptr, const int32_t *col);
void or_code_free(or_code *c);
/* n, m, e (edges), girth (0 = no cycle), z (0 = not QC) */
void or_code_info(const or_code *c, int32_t *n, int32_t *m, int64_t *e,
                  int32_t *girth, int32_t *z);
/* Check-major CSR of the expanded H: row_ptr[m+1], col[e] (columns sorted). */
void or_code_csr_out(const or_code *c, int64_t *row_ptr, int32_t *col);

/* ---- channel (Section III, error-impulse rule) ---------------------------- */
/* sigma^2 = 1 / (2 R 10^(EbN0/10)), h = 2 / sigma^2 */
double or_sigma2(double ebn0_db, double rate);
/* int8 channel value of an unperturbed bit: sat127(round_half_away(scale*h)) */
int or_q_base(double ebn0_db, double rate, double scale);
/* int8 channel value of an impulse bit at grid point k (eps = k/16):
 * round_half_away(q_base * (16 - k) / 16), saturated to [-127, 127] */
int or_q_impulse(int q_base, int k);

/* ---- decoders (flooding message passing, Section III) --------------------- */
/* Outputs of one decode. */
typedef struct {
    int32_t fail;     /* final hard decision != all-zero */
    int32_t iters;    /* iterations executed (1..max_iter) */
    int32_t tmin;     /* first iteration of minimum syndrome weight */
    int32_t wmin;     /* that minimum syndrome weight */
} or_dec_result;

/* Offset min-sum on saturated int8 messages.  q_llr[n] are int8 channel values.
 * hist (optional, [max_iter][n] bytes) receives the hard decision of every
 * iteration; synd (optional, [max_iter]) the syndrome weight. */
or_dec_result or_decode_oms(const or_code *c, const int32_t *q_llr, int max_iter,
                            int offset, uint8_t *hist, int32_t *synd);
/* Same, also returning the final APP values (app_out[n], optional). */
or_dec_result or_decode_oms_ex(const or_code *c, const int32_t *q_llr, int max_iter,
                               int offset, uint8_t *hist, int32_t *synd, int32_t *app_out);
/* Sum-product in double precision.  llr[n] are channel LLRs. */
or_dec_result or_decode_spa(const or_code *c, const double *llr, int max_iter,
                            uint8_t *hist, int32_t *synd, double *app_out);
/* Same with early stopping switchable (0 = always run max_iter iterations;
 * used by the exact-MAP pin on cycle-free graphs). */
or_dec_result or_decode_spa_ex(const or_code *c, const double *llr, int max_iter,
                               uint8_t *hist, int32_t *synd, double *app_out,
                               int early_stop);

/* Conditioning probe of the sum-product decoder (not the method itself): the
 * same decode with the channel values and every check-to-variable message
 * rounded to a multiple of 2^-grid (halves to even; grid 0 = or_decode_spa_ex).
 * A decode whose outputs change under this rounding depends on the arithmetic
 * precision of the messages, so no fixed-precision decoder can be held to its
 * double-precision outputs element by element. */
or_dec_result or_decode_spa_grid(const or_code *c, const double *llr, int max_iter,
                                 uint8_t *hist, int32_t *synd, double *app_out,
                                 int early_stop, int grid);

/* Quantised normalised layered min-sum (Section III, Fig. 2; the 4/4/6-bit
 * reading): channel values and check-to-variable messages in [-7, 7],
 * variable-to-check messages and APP values in [-31, 31], check magnitude =
 * floor(3/4 min), layers processed in order with immediate APP updates.
 * q_llr[n] are 4-bit channel values (saturated on entry). */
or_dec_result or_decode_lnms(const or_code *c, const int32_t *q_llr, int max_iter, uint8_t *hist,
                             int32_t *synd, int32_t *app_out);
/* Layers of that schedule: block rows of a QC code; otherwise each check, in
 * index order, in the first layer holding none of its variables.  layer[m];
 * returns the number of layers (-1 if more than 64). */
int or_layers(const or_code *c, int32_t *layer);
/* 4-bit channel values: sat7(round_half_away(scale h)); impulse bits
 * sat7(round_half_away(q_base (16 - k) / 16)). */
int or_q4_base(double ebn0_db, double rate, double scale);
int or_q4_impulse(int q_base, int k);

/* ---- impulse patterns (Section III, impulse tree of Fig. 3) --------------- */
#define OR_PAT_SINGLES 1  /* every variable alone */
#define OR_PAT_PAIRS 2    /* every pair at Tanner distance 2 or 4 */
#define OR_PAT_TRIPLES 3  /* every set {v1,v2,v3} on a tree path v1-c-v2-c'-v3, c != c' */
/* Writes sorted patterns (width = kind, row-major) into out when cap allows;
 * returns the number of patterns (or -1 on bad kind). */
int64_t or_patterns(const or_code *c, int kind, int32_t *out, int64_t cap);

/* ---- set functions on the Tanner graph (Section II and III) ------------- */
/* b = number of odd-degree checks of the subgraph induced by set[k]. */
int or_count_b(const or_code *c, const int32_t *set, int k);
/* Tree(V): variables of the 2-core of the induced subgraph.  Returns size. */
int or_tree(const or_code *c, const int32_t *set, int k, int32_t *out);
/* TS(V): V plus every outside variable with >= 2 checks in one connected
 * component of the induced subgraph (one pass).  out must hold
 * k + k*dv_max*dc_max entries.  Returns size. */
int or_ts_closure(const or_code *c, const int32_t *set, int k, int32_t *out);
/* Minimal representative of the QC shift orbit and the orbit size. */
int or_canon(const or_code *c, const int32_t *set, int k, int32_t *out, int32_t *orbit);

/* ---- impulse search with bisection (Section III) ------------------------- */
#define OR_DEC_OMS 0
#define OR_DEC_SPA 1
#define OR_DEC_LNMS 2     /* quantised normalised layered min-sum (k_den = 16) */
#define OR_EXTRACT_PATH 0
#define OR_EXTRACT_CRITICAL 1
typedef struct {
    int32_t decoder;           /* OR_DEC_OMS / OR_DEC_SPA / OR_DEC_LNMS */
    int32_t max_iter;
    int32_t oms_offset;        /* beta */
    double ebn0_db, rate;
    double llr_scale;          /* int8 LSB = 1/llr_scale */
    int32_t k_max;             /* grid points 0..k_max */
    int32_t k_den;             /* eps = k / k_den (16 for OMS) */
    int32_t a_max;             /* largest TS kept */
    int32_t extract_mode;      /* OR_EXTRACT_* */
    int32_t collect_from_iter; /* -1 = floor(girth/2) */
    int32_t threads;           /* 0 = OpenMP default */
    int32_t spa_grid;          /* 0; g > 0: the conditioning probe of or_decode_spa_grid */
} or_search_opts;

typedef struct or_ts_list or_ts_list;
/* Runs the search; per-pattern outputs are arrays of n_patterns.  The TS list
 * is deduplicated by canonical representative and ordered by (b/a, a, lex). */
int or_search(const or_code *c, const or_search_opts *o, const int32_t *patterns,
              int32_t n_patterns, int32_t width, int32_t *k_crit, int32_t *iters_crit,
              int32_t *iters_lo, int32_t *tmin_crit, int32_t *n_cand,
              int64_t *decodes, int64_t *edge_updates, or_ts_list **out);
int64_t or_ts_count(const or_ts_list *l);
/* Record i: a, b, orbit, first pattern, smallest k*; bits into set (a entries). */
void or_ts_get(const or_ts_list *l, int64_t i, int32_t *a, int32_t *b, int32_t *orbit,
               int32_t *first_pattern, int32_t *k_crit, int32_t *set);
void or_ts_free(or_ts_list *l);

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Standard normals of variables v = 0..n-1 for one frame (Box-Muller on the
 * Philox words of counter (v>>2, frame_lo, frame_hi, stream)). */
void or_normals(uint64_t seed, uint64_t frame, uint32_t stream, int n, double *out);

/* ---- importance sampling (Section I / II, Cole's TS weighting) ----------- */
#define OR_IS_SPA 0
#define OR_IS_LINEAR 1   /* test decoder: fails iff sum_{v in T} y_v < 0 */
#define OR_IS_COUNT_ALL 0  /* every failure counts */
#define OR_IS_COUNT_TS 1   /* only T's error events: at the end every bit of T and at most
                            * 2a bits in all in error */
typedef struct {
    int32_t decoder;        /* OR_IS_SPA, or OR_IS_LINEAR for the closed-form pin */
    int32_t max_iter;
    double ebn0_db, rate;
    double shift;           /* mean shift s of the TS bits (y = 1 - s + sigma n) */
    int64_t n_frames;
    uint64_t seed;
    uint64_t frame_base;
    uint32_t stream;        /* Philox stream tag */
    int32_t threads;
    int32_t count_mode;     /* OR_IS_COUNT_ALL / OR_IS_COUNT_TS */
    int32_t n_mix;          /* 0: every frame at `shift`; m > 0: a mixture of m shifts */
    double mix_s0, mix_ds;  /* component k: shift mix_s0 + k mix_ds (see or_is.c) */
} or_is_opts;
typedef struct {
    double p_hat, var, ci_lo, ci_hi, sum_w, sum_w2;
    int64_t n, n_fail;
    double shift_used;
} or_is_result;
/* fail_out (optional, [n_frames]) receives each frame's flags: bit 0 = the
 * decode failed, bit 1 = it ended in T's error event (OR_IS_COUNT_TS). */
int or_is_estimate(const or_code *c, const int32_t *ts, int a, const or_is_opts *o,
                   or_is_result *res, uint8_t *fail_out, int64_t *edge_updates);
/* Pilot-chosen mean shift over the grid eps* (1/2 + i/16), i = 0..8, pilot_frames
 * frames per point (see or_is.c); rv_out[9] optional. */
double or_is_pilot_shift(const or_code *c, const int32_t *ts, int a, const or_is_opts *o,
                         double eps_star, int64_t pilot_frames, double *rv_out);
/* Critical impulse amplitude of the SPA decoder on the whole set (grid 2^-10). */
double or_spa_eps_star(const or_code *c, const int32_t *ts, int a, double ebn0_db,
                       double rate, int max_iter, double eps_max);

/* ---- brute-force tools (pins) --------------------------------------------- */
/* All connected variable sets with |S| <= a_max whose induced subgraph is its
 * own 2-core.  counts[a*(bmax+1)+b] += 1 per set; orbits likewise counts
 * distinct canonical representatives.  Returns the number of sets. */
int64_t or_brute_ts(const or_code *c, int a_max, int b_max, int64_t *counts,
                    int64_t *orbits);
/* Lists the canonical representatives of those sets (a, b, then a entries
 * padded to a_max), sorted; returns the count (writes when cap allows). */
int64_t or_brute_ts_list(const or_code *c, int a_max, int32_t *out, int64_t cap);
/* Exact minimum distance by Gray-code enumeration of all codewords
 * (requires code dimension <= 40).  Returns -1 if too large. */
int or_dmin(const or_code *c, int32_t *word_out);
/* Simple cycles of length 4..max_len through each variable of block column
 * position 0 (QC codes), bucketed by EMD: out[(len/2)*(emd_max+1)+emd] counts
 * (cycle, variable-of-position-0) incidences.  per_row / per_col (optional,
 * [mb] and [nb] per length) count incidences of cycles with block rows/cols. */
int or_cycle_emd(const or_code *c, int max_len, int emd_max, int64_t *out,
                 int64_t *per_row, int64_t *per_col);

#ifdef __cplusplus
}
#endif
#endif
