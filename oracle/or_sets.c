/* Set functions on the Tanner graph for the oracle (test infrastructure only).
 *
 * TS(a,b) (Section II): a variable nodes, b = odd-degree checks of the subgraph
 * they induce (the induced subgraph holds the variables and every check joined
 * to one of them).
 *
 * Section III defines two set maps; the readings used here:
 *   Tree(V): the largest subset of V whose induced subgraph has no tree-like
 *            part, read as the variable set of the 2-core of G[V] (repeatedly
 *            drop variables with fewer than two checks that are joined to at
 *            least two surviving variables);
 *   TS(V):   V together with every variable outside V that adds a new cycle to
 *            G[V], read as "has at least two checks lying in one connected
 *            component of G[V]", evaluated once against G[V].
 *
 * The QC shift automorphism (abstract; Section II): shifting every circulant
 * position by the same t maps the Tanner graph onto itself, variable j*z+c to
 * j*z+(c+t) mod z.  The canonical representative of a set is the
 * lexicographically smallest sorted image over all t, and its orbit size is
 * z divided by the number of t that fix the set.
 */
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

/* per-call scratch: check counters (zeroed on return) */
typedef struct {
    int32_t *cnt;    /* [m] */
    int32_t *touched;
    int ntouched;
} chk_count;

static void cc_init(const or_code *c, chk_count *cc, int k) {
    cc->cnt = calloc((size_t)c->m, sizeof(int32_t));
    cc->touched = malloc(sizeof(int32_t) * ((size_t)k * c->dv_max + 1));
    cc->ntouched = 0;
}

static void cc_add_set(const or_code *c, chk_count *cc, const int32_t *set, int k,
                       const uint8_t *alive) {
    for (int i = 0; i < k; i++) {
        if (alive && !alive[i]) continue;
        int v = set[i];
        for (int64_t p = c->vptr[v]; p < c->vptr[v + 1]; p++) {
            int ch = c->vchk[p];
            if (cc->cnt[ch] == 0) cc->touched[cc->ntouched++] = ch;
            cc->cnt[ch]++;
        }
    }
}

static void cc_clear(chk_count *cc) {
    for (int i = 0; i < cc->ntouched; i++) cc->cnt[cc->touched[i]] = 0;
    cc->ntouched = 0;
}

static void cc_free(chk_count *cc) {
    free(cc->cnt);
    free(cc->touched);
}

int or_count_b(const or_code *c, const int32_t *set, int k) {
    chk_count cc;
    cc_init(c, &cc, k);
    cc_add_set(c, &cc, set, k, NULL);
    int b = 0;
    for (int i = 0; i < cc.ntouched; i++) b += cc.cnt[cc.touched[i]] & 1;
    cc_free(&cc);
    return b;
}

int or_tree(const or_code *c, const int32_t *set, int k, int32_t *out) {
    uint8_t *alive = malloc((size_t)k + 1);
    memset(alive, 1, (size_t)k + 1);
    chk_count cc;
    cc_init(c, &cc, k);
    int changed = 1;
    while (changed) {
        changed = 0;
        cc_add_set(c, &cc, set, k, alive);
        uint8_t *drop = calloc((size_t)k + 1, 1);
        for (int i = 0; i < k; i++) {
            if (!alive[i]) continue;
            int strong = 0;   /* checks of v shared with another surviving variable */
            for (int64_t p = c->vptr[set[i]]; p < c->vptr[set[i] + 1]; p++)
                if (cc.cnt[c->vchk[p]] >= 2) strong++;
            if (strong < 2) drop[i] = 1;
        }
        for (int i = 0; i < k; i++)
            if (drop[i]) { alive[i] = 0; changed = 1; }
        free(drop);
        cc_clear(&cc);
    }
    int a = 0;
    for (int i = 0; i < k; i++)
        if (alive[i]) out[a++] = set[i];
    or_sort_i32(out, a);
    free(alive);
    cc_free(&cc);
    return a;
}

static int uf_find(int *p, int x) {
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

int or_ts_closure(const or_code *c, const int32_t *set, int k, int32_t *out) {
    /* components of G[V]: variables joined through a shared check */
    int *parent = malloc(sizeof(int) * ((size_t)k + 1));
    for (int i = 0; i < k; i++) parent[i] = i;
    int32_t *chk_first = malloc(sizeof(int32_t) * (size_t)c->m);  /* a set index on each check */
    for (int r = 0; r < c->m; r++) chk_first[r] = -1;
    for (int i = 0; i < k; i++)
        for (int64_t p = c->vptr[set[i]]; p < c->vptr[set[i] + 1]; p++) {
            int ch = c->vchk[p];
            if (chk_first[ch] < 0) chk_first[ch] = i;
            else {
                int a = uf_find(parent, chk_first[ch]), b = uf_find(parent, i);
                if (a != b) parent[a] = b;
            }
        }
    uint8_t *in_set = calloc((size_t)c->n, 1);
    for (int i = 0; i < k; i++) in_set[set[i]] = 1;
    uint8_t *added = calloc((size_t)c->n, 1);
    int a = 0;
    for (int i = 0; i < k; i++) out[a++] = set[i];
    for (int i = 0; i < k; i++)
        for (int64_t p = c->vptr[set[i]]; p < c->vptr[set[i] + 1]; p++) {
            int ch = c->vchk[p];
            for (int64_t q = c->row_ptr[ch]; q < c->row_ptr[ch + 1]; q++) {
                int u = c->col[q];
                if (in_set[u] || added[u]) continue;
                /* does u have two checks in one component of G[V]? */
                int hit = 0;
                for (int64_t p1 = c->vptr[u]; p1 < c->vptr[u + 1] && !hit; p1++) {
                    int c1 = c->vchk[p1];
                    if (chk_first[c1] < 0) continue;
                    for (int64_t p2 = p1 + 1; p2 < c->vptr[u + 1]; p2++) {
                        int c2 = c->vchk[p2];
                        if (chk_first[c2] < 0) continue;
                        if (uf_find(parent, chk_first[c1]) == uf_find(parent, chk_first[c2])) {
                            hit = 1;
                            break;
                        }
                    }
                }
                if (hit) {
                    added[u] = 1;
                    out[a++] = u;
                }
            }
        }
    or_sort_i32(out, a);
    free(parent);
    free(chk_first);
    free(in_set);
    free(added);
    return a;
}

static int lex_cmp(const int32_t *x, const int32_t *y, int k) {
    for (int i = 0; i < k; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

int or_canon(const or_code *c, const int32_t *set, int k, int32_t *out, int32_t *orbit) {
    int32_t *base = malloc(sizeof(int32_t) * ((size_t)k + 1));
    memcpy(base, set, sizeof(int32_t) * (size_t)k);
    or_sort_i32(base, k);
    if (c->z == 0) {
        memcpy(out, base, sizeof(int32_t) * (size_t)k);
        *orbit = 1;
        free(base);
        return k;
    }
    int z = c->z;
    int32_t *img = malloc(sizeof(int32_t) * ((size_t)k + 1));
    int fixed = 0;
    memcpy(out, base, sizeof(int32_t) * (size_t)k);
    for (int t = 0; t < z; t++) {
        for (int i = 0; i < k; i++) img[i] = (base[i] / z) * z + (base[i] % z + t) % z;
        or_sort_i32(img, k);
        if (lex_cmp(img, out, k) < 0) memcpy(out, img, sizeof(int32_t) * (size_t)k);
        if (lex_cmp(img, base, k) == 0) fixed++;
    }
    *orbit = z / fixed;
    free(base);
    free(img);
    return k;
}
