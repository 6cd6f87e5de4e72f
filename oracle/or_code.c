/* Code construction for the oracle (test infrastructure only).
 *
 * QC expansion follows Section II, eq. (1)-(3): P is the L x L circulant with
 * P_ij = 1 iff i+1 = j (mod L), so P^k has the 1 of row r in column (r+k) mod L,
 * and exponent -1 stands for the zero block P^inf.  Girth is the length of the
 * shortest cycle of the expanded Tanner graph, found by breadth-first search. */
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void or_sort_i32(int32_t *a, int k) { qsort(a, (size_t)k, sizeof(int32_t), cmp_i32); }

/* shortest cycle length over BFS trees rooted at every variable node */
static int compute_girth(const or_code *c) {
    int nn = c->n + c->m;
    int *dist = malloc(sizeof(int) * nn);
    int *par = malloc(sizeof(int) * nn);
    int *queue = malloc(sizeof(int) * nn);
    int best = 0;
    for (int root = 0; root < c->n; root++) {
        for (int i = 0; i < nn; i++) dist[i] = -1;
        int qh = 0, qt = 0;
        dist[root] = 0;
        par[root] = -1;
        queue[qt++] = root;
        while (qh < qt) {
            int x = queue[qh++];
            if (best && 2 * dist[x] + 1 >= best) break;
            /* neighbours: node ids < n are variables, >= n are checks */
            int64_t lo, hi;
            if (x < c->n) { lo = c->vptr[x]; hi = c->vptr[x + 1]; }
            else { lo = c->row_ptr[x - c->n]; hi = c->row_ptr[x - c->n + 1]; }
            for (int64_t k = lo; k < hi; k++) {
                int y = (x < c->n) ? c->n + c->vchk[k] : c->col[k];
                if (y == par[x]) continue;
                if (dist[y] < 0) {
                    dist[y] = dist[x] + 1;
                    par[y] = x;
                    queue[qt++] = y;
                } else {
                    int len = dist[x] + dist[y] + 1;
                    if (!best || len < best) best = len;
                }
            }
        }
    }
    free(dist);
    free(par);
    free(queue);
    return best;
}

static or_code *finish(or_code *c) {
    /* variable-side adjacency */
    c->vptr = calloc((size_t)c->n + 1, sizeof(int64_t));
    c->vchk = malloc(sizeof(int32_t) * (size_t)(c->e ? c->e : 1));
    c->vedge = malloc(sizeof(int64_t) * (size_t)(c->e ? c->e : 1));
    for (int64_t k = 0; k < c->e; k++) c->vptr[c->col[k] + 1]++;
    for (int v = 0; v < c->n; v++) c->vptr[v + 1] += c->vptr[v];
    int64_t *fill = malloc(sizeof(int64_t) * ((size_t)c->n + 1));
    memcpy(fill, c->vptr, sizeof(int64_t) * ((size_t)c->n + 1));
    for (int r = 0; r < c->m; r++)       /* rows in order, so checks come sorted */
        for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++) {
            int v = c->col[k];
            c->vchk[fill[v]] = r;
            c->vedge[fill[v]] = k;
            fill[v]++;
        }
    free(fill);
    c->dv_max = 0;
    c->dc_max = 0;
    for (int v = 0; v < c->n; v++) {
        int d = (int)(c->vptr[v + 1] - c->vptr[v]);
        if (d == 0) { or_code_free(c); return NULL; }
        if (d > c->dv_max) c->dv_max = d;
    }
    for (int r = 0; r < c->m; r++) {
        int d = (int)(c->row_ptr[r + 1] - c->row_ptr[r]);
        if (d == 0) { or_code_free(c); return NULL; }
        if (d > c->dc_max) c->dc_max = d;
    }
    c->girth = compute_girth(c);
    return c;
}

or_code *or_code_qc(int mb, int nb, int z, const int32_t *shifts) {
    if (mb <= 0 || nb <= 0 || z <= 0) return NULL;
    for (int i = 0; i < mb * nb; i++)
        if (shifts[i] < -1 || shifts[i] >= z) return NULL;
    or_code *c = calloc(1, sizeof(or_code));
    c->n = nb * z;
    c->m = mb * z;
    c->z = z;
    c->mb = mb;
    c->nb = nb;
    int64_t e = 0;
    for (int i = 0; i < mb * nb; i++) e += (shifts[i] >= 0) ? z : 0;
    c->e = e;
    c->row_ptr = calloc((size_t)c->m + 1, sizeof(int64_t));
    c->col = malloc(sizeof(int32_t) * (size_t)(e ? e : 1));
    int64_t k = 0;
    for (int i = 0; i < mb; i++)
        for (int r = 0; r < z; r++) {
            int row = i * z + r;
            int64_t start = k;
            for (int j = 0; j < nb; j++) {
                int s = shifts[i * nb + j];
                if (s < 0) continue;
                c->col[k++] = j * z + (r + s) % z;   /* row r of P^s */
            }
            or_sort_i32(c->col + start, (int)(k - start));
            c->row_ptr[row + 1] = k;
        }
    return finish(c);
}

or_code *or_code_csr(int n, int m, const int64_t *row_ptr, const int32_t *col) {
    if (n <= 0 || m <= 0 || row_ptr[0] != 0) return NULL;
    for (int r = 0; r < m; r++)
        if (row_ptr[r + 1] < row_ptr[r]) return NULL;
    int64_t e = row_ptr[m];
    for (int64_t k = 0; k < e; k++)
        if (col[k] < 0 || col[k] >= n) return NULL;
    or_code *c = calloc(1, sizeof(or_code));
    c->n = n;
    c->m = m;
    c->e = e;
    c->row_ptr = malloc(sizeof(int64_t) * ((size_t)m + 1));
    memcpy(c->row_ptr, row_ptr, sizeof(int64_t) * ((size_t)m + 1));
    c->col = malloc(sizeof(int32_t) * (size_t)(e ? e : 1));
    memcpy(c->col, col, sizeof(int32_t) * (size_t)e);
    for (int r = 0; r < m; r++) {
        int64_t lo = row_ptr[r], hi = row_ptr[r + 1];
        or_sort_i32(c->col + lo, (int)(hi - lo));
        for (int64_t k = lo + 1; k < hi; k++)
            if (c->col[k] == c->col[k - 1]) { or_code_free(c); return NULL; }
    }
    return finish(c);
}

void or_code_free(or_code *c) {
    if (!c) return;
    free(c->row_ptr);
    free(c->col);
    free(c->vptr);
    free(c->vchk);
    free(c->vedge);
    free(c);
}

void or_code_info(const or_code *c, int32_t *n, int32_t *m, int64_t *e, int32_t *girth,
                  int32_t *z) {
    if (n) *n = c->n;
    if (m) *m = c->m;
    if (e) *e = c->e;
    if (girth) *girth = c->girth;
    if (z) *z = c->z;
}

void or_code_csr_out(const or_code *c, int64_t *row_ptr, int32_t *col) {
    memcpy(row_ptr, c->row_ptr, sizeof(int64_t) * ((size_t)c->m + 1));
    memcpy(col, c->col, sizeof(int32_t) * (size_t)c->e);
}
