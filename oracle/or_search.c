/* Impulse search of the modified Cole method, oracle version (test
 * infrastructure only).
 *
 * Section III: for every root variable an impulse tree VN1-CN1-VN2-CN2-VN3-CN3
 * is built and impulse sets are drawn from its variable layers.  Impulse bits
 * get the channel value h(1 - eps), all other bits h (h = 2/sigma^2, BPSK over
 * AWGN, all-zero codeword).  The decoder runs iteration by iteration; when an
 * impulse is not decoded, the error sets S(x_t) of the iterations from
 * floor(girth/2) on are sieved into
 *     S1(x_t) = Tree(S(x_t) U I),   S2(x_t) = Tree(TS(S(x_t) U I)),
 * I = the impulse set, and every nonempty result is a trapping-set candidate.
 *
 * Readings taken where the paper is silent:
 *   - amplitude grid eps_k = k / k_den, k = 0..k_max; decode at k_max first, no
 *     failure => k* = -1; else bisection on [0, k_max] (fail(mid) ? hi : lo)
 *     down to hi - lo = 1, k* = hi (D(0) is the noiseless decode and succeeds);
 *   - candidates are taken from every failing decode on the bisection path
 *     (or only from the decode at k*), at iterations collect_from .. last,
 *     only when |S(x_t) U I| <= 2 a_max, and kept when 1 <= a <= a_max;
 *   - candidates are deduplicated by their canonical QC-orbit representative;
 *     each keeps the smallest producing pattern index and the smallest k* of
 *     its producing patterns;
 *   - output order (a total order refining the b/a rule of Section III):
 *     ascending b/a, then a, then the canonical tuple.
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "or_internal.h"

/* ---- impulse patterns ---------------------------------------------------- */

static int cmp_triple(const void *a, const void *b) {
    const int32_t *x = a, *y = b;
    for (int i = 0; i < 3; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

int64_t or_patterns(const or_code *c, int kind, int32_t *out, int64_t cap) {
    int64_t cnt = 0;
    if (kind == OR_PAT_SINGLES) {
        for (int v = 0; v < c->n; v++) {
            if (cnt < cap) out[cnt] = v;
            cnt++;
        }
        return cnt;
    }
    if (kind == OR_PAT_PAIRS) {
        /* v at distance 2 (shares a check with u) or 4 (shares a check with a
         * variable at distance 2) */
        uint8_t *d2 = malloc((size_t)c->n), *d4 = malloc((size_t)c->n);
        for (int u = 0; u < c->n; u++) {
            memset(d2, 0, (size_t)c->n);
            memset(d4, 0, (size_t)c->n);
            for (int64_t p = c->vptr[u]; p < c->vptr[u + 1]; p++) {
                int ch = c->vchk[p];
                for (int64_t q = c->row_ptr[ch]; q < c->row_ptr[ch + 1]; q++) d2[c->col[q]] = 1;
            }
            d2[u] = 0;
            for (int w = 0; w < c->n; w++) {
                if (!d2[w]) continue;
                for (int64_t p = c->vptr[w]; p < c->vptr[w + 1]; p++) {
                    int ch = c->vchk[p];
                    for (int64_t q = c->row_ptr[ch]; q < c->row_ptr[ch + 1]; q++) d4[c->col[q]] = 1;
                }
            }
            for (int v = u + 1; v < c->n; v++)
                if (d2[v] || d4[v]) {
                    if (cnt < cap) { out[2 * cnt] = u; out[2 * cnt + 1] = v; }
                    cnt++;
                }
        }
        free(d2);
        free(d4);
        return cnt;
    }
    if (kind == OR_PAT_TRIPLES) {
        /* every path v1 - c - v2 - c' - v3 with c != c', as a sorted set */
        int64_t room = 1024, k = 0;
        int32_t *all = malloc(sizeof(int32_t) * 3 * (size_t)room);
        for (int v1 = 0; v1 < c->n; v1++)
            for (int64_t p = c->vptr[v1]; p < c->vptr[v1 + 1]; p++) {
                int ch = c->vchk[p];
                for (int64_t q = c->row_ptr[ch]; q < c->row_ptr[ch + 1]; q++) {
                    int v2 = c->col[q];
                    if (v2 == v1) continue;
                    for (int64_t p2 = c->vptr[v2]; p2 < c->vptr[v2 + 1]; p2++) {
                        int ch2 = c->vchk[p2];
                        if (ch2 == ch) continue;
                        for (int64_t q2 = c->row_ptr[ch2]; q2 < c->row_ptr[ch2 + 1]; q2++) {
                            int v3 = c->col[q2];
                            if (v3 == v1 || v3 == v2) continue;
                            if (k == room) {
                                room *= 2;
                                all = realloc(all, sizeof(int32_t) * 3 * (size_t)room);
                            }
                            int32_t *t = all + 3 * k;
                            t[0] = v1;
                            t[1] = v2;
                            t[2] = v3;
                            or_sort_i32(t, 3);
                            k++;
                        }
                    }
                }
            }
        qsort(all, (size_t)k, 3 * sizeof(int32_t), cmp_triple);
        for (int64_t i = 0; i < k; i++) {
            if (i > 0 && cmp_triple(all + 3 * i, all + 3 * (i - 1)) == 0) continue;
            if (cnt < cap) memcpy(out + 3 * cnt, all + 3 * i, 3 * sizeof(int32_t));
            cnt++;
        }
        free(all);
        return cnt;
    }
    return -1;
}

static void sort_records(int32_t *d, int64_t n, int stride, int by_output);

/* ---- growable record store ------------------------------------------------ */

typedef struct {
    int32_t *d;
    int64_t n, cap;  /* in records */
    int stride;
} recs;

static void recs_push(recs *r, const int32_t *rec) {
    if (r->n == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 16;
        r->d = realloc(r->d, sizeof(int32_t) * (size_t)r->stride * (size_t)r->cap);
    }
    memcpy(r->d + (size_t)r->n * r->stride, rec, sizeof(int32_t) * (size_t)r->stride);
    r->n++;
}

/* record layout: a, b, orbit, pattern, k*, canon[a_max] */
#define R_HDR 5

struct or_ts_list {
    int32_t *d;
    int64_t n;
    int stride;
};

/* ---- one pattern ------------------------------------------------------------ */

typedef struct {
    const or_code *c;
    const or_search_opts *o;
    int q_base;
    double h;
    int t0, cap;
    int32_t *q;      /* [n] int8 channel values */
    double *llr;     /* [n] */
    uint8_t *hist;   /* [max_iter * n] */
    uint8_t *hist_keep;
    int32_t *u, *s1, *tsu, *s2, *canon;
} worker;

static or_dec_result decode_at(worker *w, const int32_t *pat, int width, int k,
                               uint8_t *hist) {
    const or_code *c = w->c;
    if (w->o->decoder == OR_DEC_OMS) {
        for (int v = 0; v < c->n; v++) w->q[v] = w->q_base;
        for (int i = 0; i < width; i++)
            if (pat[i] >= 0) w->q[pat[i]] = or_q_impulse(w->q_base, k);
        return or_decode_oms(c, w->q, w->o->max_iter, w->o->oms_offset, hist, NULL);
    }
    if (w->o->decoder == OR_DEC_LNMS) {
        for (int v = 0; v < c->n; v++) w->q[v] = w->q_base;
        for (int i = 0; i < width; i++)
            if (pat[i] >= 0) w->q[pat[i]] = or_q4_impulse(w->q_base, k);
        return or_decode_lnms(c, w->q, w->o->max_iter, hist, NULL, NULL);
    }
    double eps = (double)k / (double)w->o->k_den;
    for (int v = 0; v < c->n; v++) w->llr[v] = w->h;
    for (int i = 0; i < width; i++)
        if (pat[i] >= 0) w->llr[pat[i]] = w->h * (1.0 - eps);
    return or_decode_spa_grid(c, w->llr, w->o->max_iter, hist, NULL, NULL, 1, w->o->spa_grid);
}

static int emit(worker *w, recs *out, const int32_t *set, int a, int pattern) {
    if (a < 1 || a > w->o->a_max) return 0;
    int32_t rec[R_HDR + 64];
    int32_t orbit;
    or_canon(w->c, set, a, w->canon, &orbit);
    memset(rec, 0xff, sizeof(rec));
    rec[0] = a;
    rec[1] = or_count_b(w->c, set, a);
    rec[2] = orbit;
    rec[3] = pattern;
    rec[4] = 0; /* k* filled in after the bisection */
    memcpy(rec + R_HDR, w->canon, sizeof(int32_t) * (size_t)a);
    recs_push(out, rec);
    return 1;
}

static int extract(worker *w, const uint8_t *hist, int iters, const int32_t *pat,
                   int width, int pattern, recs *out) {
    const or_code *c = w->c;
    int emitted = 0;
    for (int t = w->t0; t <= iters; t++) {
        const uint8_t *x = hist + (size_t)(t - 1) * c->n;
        int k = 0, over = 0;
        for (int v = 0; v < c->n; v++) {
            int in = x[v];
            for (int i = 0; i < width && !in; i++) in = (pat[i] == v);
            if (in) {
                if (k == w->cap) { over = 1; break; }
                w->u[k++] = v;
            }
        }
        if (over) continue;   /* |S(x_t) U I| > 2 a_max */
        int a1 = or_tree(c, w->u, k, w->s1);
        emitted += emit(w, out, w->s1, a1, pattern);
        int kt = or_ts_closure(c, w->u, k, w->tsu);
        int a2 = or_tree(c, w->tsu, kt, w->s2);
        emitted += emit(w, out, w->s2, a2, pattern);
    }
    return emitted;
}

int or_search(const or_code *c, const or_search_opts *o, const int32_t *patterns,
              int32_t n_patterns, int32_t width, int32_t *k_crit, int32_t *iters_crit,
              int32_t *iters_lo, int32_t *tmin_crit, int32_t *n_cand, int64_t *decodes,
              int64_t *edge_updates, or_ts_list **out) {
    if (o->max_iter < 1 || o->a_max < 1 || o->a_max > 64 || o->k_max < 1 || width < 1)
        return -1;
    int stride = R_HDR + o->a_max;
    recs *per = calloc((size_t)n_patterns + 1, sizeof(recs));
    int64_t dec_total = 0, eu_total = 0;
    int t0 = o->collect_from_iter >= 0 ? o->collect_from_iter : c->girth / 2;
    if (t0 < 1) t0 = 1;
    int threads = o->threads;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#else
    threads = 1;
#endif

#pragma omp parallel num_threads(threads) reduction(+ : dec_total, eu_total)
    {
        worker w;
        memset(&w, 0, sizeof(w));
        w.c = c;
        w.o = o;
        w.q_base = o->decoder == OR_DEC_LNMS ? or_q4_base(o->ebn0_db, o->rate, o->llr_scale)
                                             : or_q_base(o->ebn0_db, o->rate, o->llr_scale);
        w.h = 2.0 / or_sigma2(o->ebn0_db, o->rate);
        w.t0 = t0;
        w.cap = 2 * o->a_max;
        w.q = malloc(sizeof(int32_t) * (size_t)c->n);
        w.llr = malloc(sizeof(double) * (size_t)c->n);
        w.hist = malloc((size_t)o->max_iter * (size_t)c->n);
        w.hist_keep = malloc((size_t)o->max_iter * (size_t)c->n);
        size_t big = (size_t)w.cap * (1 + (size_t)c->dv_max * (size_t)c->dc_max) + 8;
        w.u = malloc(sizeof(int32_t) * big);
        w.s1 = malloc(sizeof(int32_t) * big);
        w.tsu = malloc(sizeof(int32_t) * big);
        w.s2 = malloc(sizeof(int32_t) * big);
        w.canon = malloc(sizeof(int32_t) * big);

#pragma omp for schedule(dynamic, 16)
        for (int32_t p = 0; p < n_patterns; p++) {
            const int32_t *pat = patterns + (size_t)p * width;
            recs *ro = &per[p];
            ro->stride = stride;
            int ncand = 0;
            or_dec_result r = decode_at(&w, pat, width, o->k_max, w.hist);
            dec_total++;
            eu_total += (int64_t)r.iters * c->e;
            if (!r.fail) {
                k_crit[p] = -1;
                iters_crit[p] = 0;
                tmin_crit[p] = 0;
                iters_lo[p] = r.iters;
                n_cand[p] = 0;
                continue;
            }
            int keep_iters = r.iters;
            if (o->extract_mode == OR_EXTRACT_PATH)
                ncand += extract(&w, w.hist, r.iters, pat, width, p, ro);
            else
                memcpy(w.hist_keep, w.hist, (size_t)o->max_iter * (size_t)c->n);
            int lo = 0, hi = o->k_max;
            int it_hi = r.iters, tm_hi = r.tmin, it_lo = 1;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                r = decode_at(&w, pat, width, mid, w.hist);
                dec_total++;
                eu_total += (int64_t)r.iters * c->e;
                if (r.fail) {
                    hi = mid;
                    it_hi = r.iters;
                    tm_hi = r.tmin;
                    if (o->extract_mode == OR_EXTRACT_PATH)
                        ncand += extract(&w, w.hist, r.iters, pat, width, p, ro);
                    else {
                        memcpy(w.hist_keep, w.hist, (size_t)o->max_iter * (size_t)c->n);
                        keep_iters = r.iters;
                    }
                } else {
                    lo = mid;
                    it_lo = r.iters;
                }
            }
            if (o->extract_mode != OR_EXTRACT_PATH)
                ncand += extract(&w, w.hist_keep, keep_iters, pat, width, p, ro);
            k_crit[p] = hi;
            iters_crit[p] = it_hi;
            tmin_crit[p] = tm_hi;
            iters_lo[p] = it_lo;
            n_cand[p] = ncand;
            for (int64_t i = 0; i < ro->n; i++) ro->d[(size_t)i * stride + 4] = hi;
        }
        free(w.q);
        free(w.llr);
        free(w.hist);
        free(w.hist_keep);
        free(w.u);
        free(w.s1);
        free(w.tsu);
        free(w.s2);
        free(w.canon);
    }
    if (decodes) *decodes = dec_total;
    if (edge_updates) *edge_updates = eu_total;

    /* merge: identical canonical sets become one record */
    int64_t total = 0;
    for (int32_t p = 0; p < n_patterns; p++) total += per[p].n;
    int32_t *all = malloc(sizeof(int32_t) * (size_t)stride * (size_t)(total ? total : 1));
    int64_t k = 0;
    for (int32_t p = 0; p < n_patterns; p++) {
        if (per[p].n)
            memcpy(all + (size_t)k * stride, per[p].d,
                   sizeof(int32_t) * (size_t)stride * (size_t)per[p].n);
        k += per[p].n;
        free(per[p].d);
    }
    free(per);
    /* sort by (a, canonical tuple) so that equal sets are adjacent */
    sort_records(all, total, stride, 0);
    or_ts_list *l = calloc(1, sizeof(or_ts_list));
    l->stride = stride;
    l->d = malloc(sizeof(int32_t) * (size_t)stride * (size_t)(total ? total : 1));
    int64_t nu = 0;
    for (int64_t i = 0; i < total; i++) {
        int32_t *r = all + (size_t)i * stride;
        int32_t *last = nu ? l->d + (size_t)(nu - 1) * stride : NULL;
        int same = last && last[0] == r[0] &&
                   memcmp(last + R_HDR, r + R_HDR, sizeof(int32_t) * (size_t)r[0]) == 0;
        if (same) {
            if (r[3] < last[3]) last[3] = r[3];
            if (r[4] < last[4]) last[4] = r[4];
        } else {
            memcpy(l->d + (size_t)nu * stride, r, sizeof(int32_t) * (size_t)stride);
            nu++;
        }
    }
    free(all);
    l->n = nu;
    sort_records(l->d, nu, stride, 1);
    *out = l;
    return 0;
}

/* ---- record ordering -------------------------------------------------------- */

static int g_by_output;

static int rec_cmp(const void *pa, const void *pb) {
    const int32_t *x = pa, *y = pb;
    if (g_by_output) {
        /* b/a ascending, compared exactly as b_x * a_y vs b_y * a_x */
        int64_t l = (int64_t)x[1] * y[0], r = (int64_t)y[1] * x[0];
        if (l != r) return l < r ? -1 : 1;
    }
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    for (int i = 0; i < x[0]; i++)
        if (x[R_HDR + i] != y[R_HDR + i]) return x[R_HDR + i] < y[R_HDR + i] ? -1 : 1;
    return 0;
}

/* qsort has no context argument; the oracle sorts from one thread only */
static void sort_records(int32_t *d, int64_t n, int stride, int by_output) {
    g_by_output = by_output;
    qsort(d, (size_t)n, sizeof(int32_t) * (size_t)stride, rec_cmp);
}

int64_t or_ts_count(const or_ts_list *l) { return l->n; }

void or_ts_get(const or_ts_list *l, int64_t i, int32_t *a, int32_t *b, int32_t *orbit,
               int32_t *first_pattern, int32_t *k_crit, int32_t *set) {
    const int32_t *r = l->d + (size_t)i * l->stride;
    *a = r[0];
    *b = r[1];
    *orbit = r[2];
    *first_pattern = r[3];
    *k_crit = r[4];
    if (set) memcpy(set, r + R_HDR, sizeof(int32_t) * (size_t)r[0]);
}

void or_ts_free(or_ts_list *l) {
    if (!l) return;
    free(l->d);
    free(l);
}
