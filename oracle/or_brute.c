/* Brute-force tools that pin the oracle (test infrastructure only).
 *
 *  - or_brute_ts: every connected variable set S with |S| <= a_max whose
 *    induced subgraph is its own 2-core, with its b (Section II's TS(a,b)).
 *    Sets are enumerated exactly once each by Wernicke's ESU procedure over the
 *    variable graph (variables adjacent iff they share a check).
 *  - or_dmin: exact minimum distance (Section II: TS(d_min, 0) are the
 *    minimum-weight codewords) by Gray-code enumeration of the null space of H.
 *  - or_cycle_emd: simple cycles and their EMD (Section II: number of checks
 *    joined to exactly one variable of the cycle), by depth-first search from
 *    the position-0 variable of every block column of a QC code.
 */
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

/* ---- ESU enumeration of connected sets ------------------------------------ */

typedef struct {
    const or_code *c;
    int a_max, b_max;
    int32_t **nbr;  /* variable graph */
    int *deg;
    int32_t set[64];
    int ns;
    uint8_t *in_set;
    int *adj_cnt;   /* number of set members adjacent to each variable */
    int64_t nsets;
    int64_t *counts;
    int32_t *list;  /* canonical records: a, b, canon[a_max] */
    int64_t nlist, caplist;
    int32_t *tmp;
} esu;

static int is_own_2core(const or_code *c, const int32_t *s, int k) {
    for (int i = 0; i < k; i++) {
        int strong = 0;
        for (int64_t p = c->vptr[s[i]]; p < c->vptr[s[i] + 1]; p++) {
            int ch = c->vchk[p], shared = 0;
            for (int j = 0; j < k && !shared; j++) {
                if (j == i) continue;
                for (int64_t q = c->vptr[s[j]]; q < c->vptr[s[j] + 1]; q++)
                    if (c->vchk[q] == ch) { shared = 1; break; }
            }
            strong += shared;
        }
        if (strong < 2) return 0;
    }
    return 1;
}

static void esu_visit(esu *e) {
    if (!is_own_2core(e->c, e->set, e->ns)) return;
    int b = or_count_b(e->c, e->set, e->ns);
    e->nsets++;
    if (b <= e->b_max && e->counts) e->counts[e->ns * (e->b_max + 1) + b]++;
    int stride = 2 + e->a_max;
    if (e->nlist == e->caplist) {
        e->caplist = e->caplist ? 2 * e->caplist : 1024;
        e->list = realloc(e->list, sizeof(int32_t) * (size_t)stride * (size_t)e->caplist);
    }
    int32_t *r = e->list + (size_t)e->nlist * stride;
    int32_t orbit;
    for (int i = 0; i < stride; i++) r[i] = -1;
    r[0] = e->ns;
    r[1] = b;
    or_canon(e->c, e->set, e->ns, r + 2, &orbit);
    e->nlist++;
}

static void esu_extend(esu *e, const int32_t *ext, int next, int root) {
    esu_visit(e);
    if (e->ns == e->a_max) return;
    int32_t *mine = malloc(sizeof(int32_t) * ((size_t)next + 1));
    memcpy(mine, ext, sizeof(int32_t) * (size_t)next);
    int left = next;
    while (left > 0) {
        int w = mine[--left];
        /* ext' = remaining ext plus exclusive neighbours of w greater than root */
        int32_t *ext2 = malloc(sizeof(int32_t) * ((size_t)left + (size_t)e->deg[w] + 1));
        int n2 = left;
        memcpy(ext2, mine, sizeof(int32_t) * (size_t)left);
        for (int i = 0; i < e->deg[w]; i++) {
            int u = e->nbr[w][i];
            if (u > root && !e->in_set[u] && e->adj_cnt[u] == 0) ext2[n2++] = u;
        }
        e->set[e->ns++] = w;
        e->in_set[w] = 1;
        for (int i = 0; i < e->deg[w]; i++) e->adj_cnt[e->nbr[w][i]]++;
        esu_extend(e, ext2, n2, root);
        for (int i = 0; i < e->deg[w]; i++) e->adj_cnt[e->nbr[w][i]]--;
        e->in_set[w] = 0;
        e->ns--;
        free(ext2);
    }
    free(mine);
}

static int cmp_rec_global_stride;
static int cmp_rec(const void *pa, const void *pb) {
    const int32_t *x = pa, *y = pb;
    for (int i = 0; i < cmp_rec_global_stride; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

static int64_t brute_run(const or_code *c, int a_max, int b_max, int64_t *counts,
                         int64_t *orbits, int list_mode, int32_t *out, int64_t cap) {
    if (a_max < 1 || a_max > 16) return -1;
    esu e;
    memset(&e, 0, sizeof(e));
    e.c = c;
    e.a_max = a_max;
    e.b_max = b_max;
    e.counts = counts;
    e.nbr = malloc(sizeof(int32_t *) * (size_t)c->n);
    e.deg = calloc((size_t)c->n, sizeof(int));
    uint8_t *mark = calloc((size_t)c->n, 1);
    int32_t *buf = malloc(sizeof(int32_t) * (size_t)c->n);
    for (int v = 0; v < c->n; v++) {
        int k = 0;
        for (int64_t p = c->vptr[v]; p < c->vptr[v + 1]; p++) {
            int ch = c->vchk[p];
            for (int64_t q = c->row_ptr[ch]; q < c->row_ptr[ch + 1]; q++) {
                int u = c->col[q];
                if (u != v && !mark[u]) { mark[u] = 1; buf[k++] = u; }
            }
        }
        for (int i = 0; i < k; i++) mark[buf[i]] = 0;
        e.nbr[v] = malloc(sizeof(int32_t) * ((size_t)k + 1));
        memcpy(e.nbr[v], buf, sizeof(int32_t) * (size_t)k);
        e.deg[v] = k;
    }
    e.in_set = calloc((size_t)c->n, 1);
    e.adj_cnt = calloc((size_t)c->n, sizeof(int));
    for (int v = 0; v < c->n; v++) {
        int32_t *ext = malloc(sizeof(int32_t) * ((size_t)e.deg[v] + 1));
        int next = 0;
        for (int i = 0; i < e.deg[v]; i++)
            if (e.nbr[v][i] > v) ext[next++] = e.nbr[v][i];
        e.set[0] = v;
        e.ns = 1;
        e.in_set[v] = 1;
        for (int i = 0; i < e.deg[v]; i++) e.adj_cnt[e.nbr[v][i]]++;
        esu_extend(&e, ext, next, v);
        for (int i = 0; i < e.deg[v]; i++) e.adj_cnt[e.nbr[v][i]]--;
        e.in_set[v] = 0;
        free(ext);
    }
    /* distinct canonical representatives */
    int stride = 2 + a_max;
    cmp_rec_global_stride = stride;
    qsort(e.list, (size_t)e.nlist, sizeof(int32_t) * (size_t)stride, cmp_rec);
    int64_t nd = 0;
    for (int64_t i = 0; i < e.nlist; i++) {
        int32_t *r = e.list + (size_t)i * stride;
        if (i > 0 && cmp_rec(r, r - stride) == 0) continue;
        if (orbits && r[1] <= b_max) orbits[r[0] * (b_max + 1) + r[1]]++;
        if (out && nd < cap) memcpy(out + (size_t)nd * stride, r, sizeof(int32_t) * (size_t)stride);
        nd++;
    }
    for (int v = 0; v < c->n; v++) free(e.nbr[v]);
    free(e.nbr);
    free(e.deg);
    free(mark);
    free(buf);
    free(e.in_set);
    free(e.adj_cnt);
    free(e.list);
    return list_mode ? nd : e.nsets;
}

int64_t or_brute_ts(const or_code *c, int a_max, int b_max, int64_t *counts, int64_t *orbits) {
    return brute_run(c, a_max, b_max, counts, orbits, 0, NULL, 0);
}

int64_t or_brute_ts_list(const or_code *c, int a_max, int32_t *out, int64_t cap) {
    return brute_run(c, a_max, 1 << 20, NULL, NULL, 1, out, cap);
}

/* ---- exact minimum distance ---------------------------------------------- */

int or_dmin(const or_code *c, int32_t *word_out) {
    int n = c->n, m = c->m;
    if (n <= 0 || n > 128) return -1;
    /* rows of H as 128-bit masks */
    uint64_t (*h)[2] = calloc((size_t)m, sizeof(*h));
    for (int r = 0; r < m; r++)
        for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++)
            h[r][c->col[k] >> 6] |= 1ull << (c->col[k] & 63);
    int *pivot_col = malloc(sizeof(int) * (size_t)m);
    int rank = 0;
    for (int col = 0; col < n && rank < m; col++) {
        int sel = -1;
        for (int r = rank; r < m; r++)
            if ((h[r][col >> 6] >> (col & 63)) & 1) { sel = r; break; }
        if (sel < 0) continue;
        uint64_t t0 = h[sel][0], t1 = h[sel][1];
        h[sel][0] = h[rank][0];
        h[sel][1] = h[rank][1];
        h[rank][0] = t0;
        h[rank][1] = t1;
        for (int r = 0; r < m; r++)
            if (r != rank && ((h[r][col >> 6] >> (col & 63)) & 1)) {
                h[r][0] ^= h[rank][0];
                h[r][1] ^= h[rank][1];
            }
        pivot_col[rank++] = col;
    }
    int kdim = n - rank;
    if (kdim > 40) { free(h); free(pivot_col); return -1; }
    uint8_t *is_pivot = calloc((size_t)n, 1);
    for (int i = 0; i < rank; i++) is_pivot[pivot_col[i]] = 1;
    /* null-space basis: one vector per free column */
    uint64_t (*basis)[2] = calloc((size_t)kdim + 1, sizeof(*basis));
    int b = 0;
    for (int f = 0; f < n; f++) {
        if (is_pivot[f]) continue;
        basis[b][f >> 6] |= 1ull << (f & 63);
        for (int i = 0; i < rank; i++)
            if ((h[i][f >> 6] >> (f & 63)) & 1)
                basis[b][pivot_col[i] >> 6] |= 1ull << (pivot_col[i] & 63);
        b++;
    }
    uint64_t w0 = 0, w1 = 0, best0 = 0, best1 = 0;
    int best = n + 1;
    for (uint64_t g = 1; g < (1ull << kdim); g++) {
        int bit = __builtin_ctzll(g);   /* Gray code: flip one basis vector */
        w0 ^= basis[bit][0];
        w1 ^= basis[bit][1];
        int wt = __builtin_popcountll(w0) + __builtin_popcountll(w1);
        if (wt < best) { best = wt; best0 = w0; best1 = w1; }
    }
    if (word_out) {
        int k = 0;
        for (int v = 0; v < n; v++)
            if (((v < 64 ? best0 : best1) >> (v & 63)) & 1) word_out[k++] = v;
    }
    free(h);
    free(pivot_col);
    free(is_pivot);
    free(basis);
    return best;
}

/* ---- cycles and EMD ------------------------------------------------------- */

typedef struct {
    const or_code *c;
    int max_len, emd_max;
    int64_t *out, *per_row, *per_col;
    int path[32];     /* node ids: variables < n, checks n + r */
    uint8_t *used;
} cyc;

static void cyc_record(cyc *s, int len) {
    const or_code *c = s->c;
    int l = len / 2;
    /* EMD: checks joined to exactly one variable of the cycle */
    int emd = 0;
    for (int i = 0; i < len; i += 2) {
        int v = s->path[i];
        for (int64_t p = c->vptr[v]; p < c->vptr[v + 1]; p++) {
            int ch = c->vchk[p], hits = 0;
            for (int j = 0; j < len; j += 2) {
                int u = s->path[j];
                for (int64_t q = c->vptr[u]; q < c->vptr[u + 1]; q++)
                    if (c->vchk[q] == ch) hits++;
            }
            if (hits == 1) emd++;
        }
    }
    if (emd > s->emd_max) emd = s->emd_max;
    s->out[l * (s->emd_max + 1) + emd]++;
    if (s->per_row)
        for (int i = 1; i < len; i += 2)
            s->per_row[l * c->mb + (s->path[i] - c->n) / c->z]++;
    if (s->per_col)
        for (int i = 0; i < len; i += 2) s->per_col[l * c->nb + s->path[i] / c->z]++;
}

static void cyc_dfs(cyc *s, int depth) {
    const or_code *c = s->c;
    int x = s->path[depth - 1];
    if (x < c->n) {  /* at a variable: step to a check */
        for (int64_t p = c->vptr[x]; p < c->vptr[x + 1]; p++) {
            int y = c->n + c->vchk[p];
            if (s->used[y]) continue;
            if (depth >= s->max_len) continue;
            s->used[y] = 1;
            s->path[depth] = y;
            cyc_dfs(s, depth + 1);
            s->used[y] = 0;
        }
    } else {         /* at a check: close the cycle or step to a variable */
        int r = x - c->n;
        for (int64_t q = c->row_ptr[r]; q < c->row_ptr[r + 1]; q++) {
            int y = c->col[q];
            if (y == s->path[0] && depth >= 4) {
                /* count each cycle once: first check smaller than last check */
                if (s->path[1] < x) cyc_record(s, depth);
                continue;
            }
            if (s->used[y] || depth + 1 >= s->max_len) continue;
            s->used[y] = 1;
            s->path[depth] = y;
            cyc_dfs(s, depth + 1);
            s->used[y] = 0;
        }
    }
}

int or_cycle_emd(const or_code *c, int max_len, int emd_max, int64_t *out,
                 int64_t *per_row, int64_t *per_col) {
    if (c->z == 0 || max_len > 30) return -1;
    cyc s;
    memset(&s, 0, sizeof(s));
    s.c = c;
    s.max_len = max_len;
    s.emd_max = emd_max;
    s.out = out;
    s.per_row = per_row;
    s.per_col = per_col;
    s.used = calloc((size_t)c->n + (size_t)c->m, 1);
    for (int j = 0; j < c->nb; j++) {
        int root = j * c->z;
        s.path[0] = root;
        s.used[root] = 1;
        cyc_dfs(&s, 1);
        s.used[root] = 0;
    }
    free(s.used);
    return 0;
}
