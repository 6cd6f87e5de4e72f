/* Flooding message-passing decoders of the oracle (test infrastructure only).
 *
 * The paper runs "unrolled" message-passing iterations on the all-zero
 * codeword and reads the hard decision after each iteration (Section III); it
 * does not fix the decoder.  The two decoders here are the readings used by the
 * whole project:
 *
 *   offset min-sum (OMS), int8 messages:
 *     v2c = sat127(APP_v - c2v)                     (sat127: clamp to [-127,127])
 *     c2v = prod_{v' != v} sgn(v2c') * max(min_{v' != v} |v2c'| - beta, 0)
 *           with sgn(0) = +1
 *     APP_v = lambda_v + sum_c c2v                  (exact integers)
 *
 *   sum-product (SPA), double precision:
 *     v2c = APP_v - c2v
 *     c2v = prod_{v' != v} sgn(v2c') * phi( sum_{v' != v} phi(min(|v2c'|, 30)) )
 *     phi(x) = -ln tanh(x/2) = ln(1 + 2/(e^x - 1)), evaluated at max(x, 2^-20)
 *     APP_v = lambda_v + sum_c c2v
 *
 * Both start from c2v = 0 (so APP = lambda before iteration 1).  After every
 * iteration t the hard decision is x_v = [APP_v < 0] and the syndrome weight
 * w_t = number of unsatisfied checks (Section III, w_H(H x_iter)).  Decoding
 * stops at the first t with w_t = 0 or at max_iter.  It fails iff the final x
 * is not all-zero (this includes stopping on a nonzero codeword).  tmin is the
 * first t reaching min_t w_t (the S(min_iter w_H) set of Section III).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

static int sat127(int x) { return x > 127 ? 127 : (x < -127 ? -127 : x); }

/* syndrome weight of the hard decision x */
static int syndrome_weight(const or_code *c, const uint8_t *x) {
    int w = 0;
    for (int r = 0; r < c->m; r++) {
        int par = 0;
        for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++) par ^= x[c->col[k]];
        w += par;
    }
    return w;
}

or_dec_result or_decode_oms_ex(const or_code *c, const int32_t *q_llr, int max_iter,
                               int offset, uint8_t *hist, int32_t *synd, int32_t *app_out) {
    or_dec_result res = {0, 0, 0, 0};
    int32_t *c2v = calloc((size_t)c->e, sizeof(int32_t));
    int32_t *v2c = malloc(sizeof(int32_t) * (size_t)c->e);
    int32_t *app = malloc(sizeof(int32_t) * (size_t)c->n);
    uint8_t *x = malloc((size_t)c->n);
    for (int v = 0; v < c->n; v++) app[v] = q_llr[v];
    int wbest = -1;
    int t;
    for (t = 1; t <= max_iter; t++) {
        /* variable-to-check messages from the previous APP */
        for (int r = 0; r < c->m; r++)
            for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++)
                v2c[k] = sat127(app[c->col[k]] - c2v[k]);
        /* check-node update, excluding the target edge explicitly */
        for (int r = 0; r < c->m; r++)
            for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++) {
                int sign = 1, mn = 1 << 30;
                for (int64_t k2 = c->row_ptr[r]; k2 < c->row_ptr[r + 1]; k2++) {
                    if (k2 == k) continue;
                    if (v2c[k2] < 0) sign = -sign;
                    int a = abs(v2c[k2]);
                    if (a < mn) mn = a;
                }
                int mag = mn - offset;
                if (mag < 0) mag = 0;
                c2v[k] = sign * mag;
            }
        /* variable-node update */
        for (int v = 0; v < c->n; v++) {
            int s = q_llr[v];
            for (int64_t k = c->vptr[v]; k < c->vptr[v + 1]; k++) s += c2v[c->vedge[k]];
            app[v] = s;
            x[v] = (uint8_t)(s < 0);
        }
        int w = syndrome_weight(c, x);
        if (hist) memcpy(hist + (size_t)(t - 1) * c->n, x, (size_t)c->n);
        if (synd) synd[t - 1] = w;
        if (wbest < 0 || w < wbest) { wbest = w; res.tmin = t; }
        if (w == 0) break;
    }
    res.iters = t > max_iter ? max_iter : t;
    res.wmin = wbest;
    res.fail = 0;
    for (int v = 0; v < c->n; v++) res.fail |= x[v];
    if (app_out) memcpy(app_out, app, sizeof(int32_t) * (size_t)c->n);
    free(c2v);
    free(v2c);
    free(app);
    free(x);
    return res;
}

or_dec_result or_decode_oms(const or_code *c, const int32_t *q_llr, int max_iter,
                            int offset, uint8_t *hist, int32_t *synd) {
    return or_decode_oms_ex(c, q_llr, max_iter, offset, hist, synd, NULL);
}

static double phi(double x) {
    if (x < 0x1p-20) x = 0x1p-20;
    return log1p(2.0 / expm1(x));
}

/* Rounds x to a multiple of 2^-grid, halves to even (grid 0: x unchanged). */
static double on_grid(double x, int grid) {
    if (grid <= 0) return x;
    return nearbyint(ldexp(x, grid)) * ldexp(1.0, -grid);
}

or_dec_result or_decode_spa_grid(const or_code *c, const double *llr_in, int max_iter,
                                 uint8_t *hist, int32_t *synd, double *app_out,
                                 int early_stop, int grid) {
    or_dec_result res = {0, 0, 0, 0};
    double *c2v = calloc((size_t)c->e, sizeof(double));
    double *v2c = malloc(sizeof(double) * (size_t)c->e);
    double *app = malloc(sizeof(double) * (size_t)c->n);
    double *llr = malloc(sizeof(double) * (size_t)c->n);
    uint8_t *x = malloc((size_t)c->n);
    for (int v = 0; v < c->n; v++) llr[v] = on_grid(llr_in[v], grid);
    for (int v = 0; v < c->n; v++) app[v] = llr[v];
    int wbest = -1;
    int t;
    for (t = 1; t <= max_iter; t++) {
        for (int r = 0; r < c->m; r++)
            for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++)
                v2c[k] = app[c->col[k]] - c2v[k];
        for (int r = 0; r < c->m; r++)
            for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++) {
                int sign = 1;
                double sum = 0.0;
                for (int64_t k2 = c->row_ptr[r]; k2 < c->row_ptr[r + 1]; k2++) {
                    if (k2 == k) continue;
                    if (v2c[k2] < 0) sign = -sign;
                    double a = fabs(v2c[k2]);
                    if (a > 30.0) a = 30.0;
                    sum += phi(a);
                }
                c2v[k] = on_grid(sign * phi(sum), grid);
            }
        for (int v = 0; v < c->n; v++) {
            double s = llr[v];
            for (int64_t k = c->vptr[v]; k < c->vptr[v + 1]; k++) s += c2v[c->vedge[k]];
            app[v] = s;
            x[v] = (uint8_t)(s < 0);
        }
        int w = syndrome_weight(c, x);
        if (hist) memcpy(hist + (size_t)(t - 1) * c->n, x, (size_t)c->n);
        if (synd) synd[t - 1] = w;
        if (wbest < 0 || w < wbest) { wbest = w; res.tmin = t; }
        if (w == 0 && early_stop) break;
    }
    res.iters = t > max_iter ? max_iter : t;
    res.wmin = wbest;
    res.fail = 0;
    for (int v = 0; v < c->n; v++) res.fail |= x[v];
    if (app_out) memcpy(app_out, app, sizeof(double) * (size_t)c->n);
    free(c2v);
    free(v2c);
    free(app);
    free(llr);
    free(x);
    return res;
}

or_dec_result or_decode_spa_ex(const or_code *c, const double *llr, int max_iter,
                               uint8_t *hist, int32_t *synd, double *app_out,
                               int early_stop) {
    return or_decode_spa_grid(c, llr, max_iter, hist, synd, app_out, early_stop, 0);
}

/* ---- quantised normalised layered min-sum (Section III, Fig. 2) ---------- */
/* Reading of the paper's "quantized normalized layered min-sum, 4/4/6 bits":
 * channel values and check-to-variable messages on 4 bits ([-7, 7]),
 * variable-to-check messages and APP values on 6 bits ([-31, 31]); the check
 * rule scales the min-sum magnitude by 3/4 (rounded down); the layers are the
 * block rows of a QC code, otherwise the checks in index order each put in the
 * first layer that holds none of its variables. */

static int sat7(int x) { return x > 7 ? 7 : (x < -7 ? -7 : x); }
static int sat31(int x) { return x > 31 ? 31 : (x < -31 ? -31 : x); }

int or_layers(const or_code *c, int32_t *layer) {
    if (c->z > 0) {
        for (int r = 0; r < c->m; r++) layer[r] = r / c->z;
        return c->mb;
    }
    /* owner[v * cap + L] = 1 if layer L holds a check of variable v */
    int n_layers = 0, cap = 64;
    uint8_t *owner = calloc((size_t)c->n * cap, 1);
    for (int r = 0; r < c->m; r++) {
        int L = 0;
        for (;; L++) {
            if (L >= cap) { free(owner); return -1; }
            int clash = 0;
            for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1] && !clash; k++)
                clash = owner[(size_t)c->col[k] * cap + L];
            if (!clash) break;
        }
        layer[r] = L;
        for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++)
            owner[(size_t)c->col[k] * cap + L] = 1;
        if (L + 1 > n_layers) n_layers = L + 1;
    }
    free(owner);
    return n_layers;
}

or_dec_result or_decode_lnms(const or_code *c, const int32_t *q_llr, int max_iter, uint8_t *hist,
                             int32_t *synd, int32_t *app_out) {
    or_dec_result res = {0, 0, 0, 0};
    int32_t *layer = malloc(sizeof(int32_t) * (size_t)(c->m > 0 ? c->m : 1));
    int n_layers = or_layers(c, layer);
    int32_t *c2v = calloc((size_t)c->e, sizeof(int32_t));
    int32_t *v2c = malloc(sizeof(int32_t) * (size_t)c->e);
    int32_t *app = malloc(sizeof(int32_t) * (size_t)c->n);
    uint8_t *x = malloc((size_t)c->n);
    for (int v = 0; v < c->n; v++) app[v] = sat7(q_llr[v]);
    int wbest = -1, t;
    for (t = 1; t <= max_iter; t++) {
        for (int L = 0; L < n_layers; L++)
            for (int r = 0; r < c->m; r++) {
                if (layer[r] != L) continue;
                for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++)
                    v2c[k] = sat31(app[c->col[k]] - c2v[k]);
                /* each edge from the other edges of the check */
                for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++) {
                    int sign = 1, mn = 1 << 30;
                    for (int64_t k2 = c->row_ptr[r]; k2 < c->row_ptr[r + 1]; k2++) {
                        if (k2 == k) continue;
                        if (v2c[k2] < 0) sign = -sign;
                        int a = abs(v2c[k2]);
                        if (a < mn) mn = a;
                    }
                    c2v[k] = sign * sat7((3 * mn) / 4);
                }
                for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; k++)
                    app[c->col[k]] = sat31(v2c[k] + c2v[k]);
            }
        for (int v = 0; v < c->n; v++) x[v] = (uint8_t)(app[v] < 0);
        int w = syndrome_weight(c, x);
        if (hist) memcpy(hist + (size_t)(t - 1) * c->n, x, (size_t)c->n);
        if (synd) synd[t - 1] = w;
        if (wbest < 0 || w < wbest) { wbest = w; res.tmin = t; }
        if (w == 0) break;
    }
    res.iters = t > max_iter ? max_iter : t;
    res.wmin = wbest;
    res.fail = 0;
    for (int v = 0; v < c->n; v++) res.fail |= x[v];
    if (app_out) memcpy(app_out, app, sizeof(int32_t) * (size_t)c->n);
    free(layer);
    free(c2v);
    free(v2c);
    free(app);
    free(x);
    return res;
}

int or_q4_base(double ebn0_db, double rate, double scale) {
    double h = 2.0 / or_sigma2(ebn0_db, rate);
    return sat7((int)lround(scale * h));
}

int or_q4_impulse(int q_base, int k) {
    long n = (long)q_base * (16 - k);
    long mag = (labs(n) + 8) / 16;
    long q = n < 0 ? -mag : mag;
    return sat7((int)(q > 1000 ? 1000 : (q < -1000 ? -1000 : q)));
}

/* ---- channel values ------------------------------------------------------ */

double or_sigma2(double ebn0_db, double rate) {
    return 1.0 / (2.0 * rate * pow(10.0, ebn0_db / 10.0));
}

int or_q_base(double ebn0_db, double rate, double scale) {
    double h = 2.0 / or_sigma2(ebn0_db, rate);
    return sat127((int)lround(scale * h));   /* lround rounds half away from zero */
}

int or_q_impulse(int q_base, int k) {
    /* lambda = h (1 - eps), eps = k/16, computed on the int8 scale from q_base */
    long n = (long)q_base * (16 - k);
    long mag = (labs(n) + 8) / 16;
    long q = n < 0 ? -mag : mag;
    return sat127((int)(q > 1000 ? 1000 : (q < -1000 ? -1000 : q)));
}

or_dec_result or_decode_spa(const or_code *c, const double *llr, int max_iter,
                            uint8_t *hist, int32_t *synd, double *app_out) {
    return or_decode_spa_ex(c, llr, max_iter, hist, synd, app_out, 1);
}
