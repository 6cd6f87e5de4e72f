/* Importance-sampling weighting of a trapping set, oracle version (test
 * infrastructure only).
 *
 * Section I and II: the error-floor contribution of a TS is weighted by
 * importance sampling (Cole's method) before the union bound.  The paper does
 * not spell out the estimator; the reading used here is the mean-shift
 * estimator:
 *   y_v = 1 - s [v in T] + sigma n_v,  n_v ~ N(0,1),   lambda_v = 2 y_v / sigma^2
 *   w   = exp(-a s^2 / (2 sigma^2) + (s / sigma) sum_{v in T} n_v)
 *   P   = (1/K) sum_f 1[fail_f] w_f,
 *   Var = (1/(K(K-1))) sum_f (1[fail_f] w_f - P)^2,   95% CI = P +- 1.96 sqrt(Var)
 * with the SPA decoder of or_decode.c.  w is the likelihood ratio of the
 * unshifted over the shifted Gaussian density of the a shifted bits.  Which
 * failures count (count_mode): every failure, or only T's own error events,
 * whose final hard decision has every bit of T in error and at most 2a bits in
 * error in all (the failures of the union bound's term for T; wide decoding
 * failures and other sets' events are not T's).
 *
 * A mixture of m shifts s_k = mix_s0 + k mix_ds (multiple importance sampling
 * with the balance heuristic): frame f is drawn at the shift of component
 * j = floor(f m / K), so the components hold K_k frames each, in frame order,
 * and a counted frame weighs
 *   w = p(y) / sum_k (K_k / K) p_k(y),   p the unshifted and p_k the
 * shifted Gaussian densities of the a TS bits; with D = sum_{v in T} (1 - y_v) / sigma,
 * p_k(y) / p(y) = exp((s_k / sigma) D - a s_k^2 / (2 sigma^2)).
 *
 * Noise comes from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): counter (v>>2, frame_lo, frame_hi,
 * stream), key = the 64-bit seed; the four words give the normals of variables
 * 4(v>>2)..4(v>>2)+3 by the Box-Muller transform on u = (x + 1/2) 2^-32.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "or_internal.h"

/* Philox S-box constants and Weyl key increments, as published by Salmon et al. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

void or_normals(uint64_t seed, uint64_t frame, uint32_t stream, int n, double *out) {
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int g = 0; 4 * g < n; g++) {
        uint32_t ctr[4] = {(uint32_t)g, (uint32_t)frame, (uint32_t)(frame >> 32), stream};
        uint32_t x[4];
        or_philox4x32_10(ctr, key, x);
        double u[4];
        for (int i = 0; i < 4; i++) u[i] = ((double)x[i] + 0.5) * 0x1p-32;
        double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
        double nv[4] = {r0 * cos(two_pi * u[1]), r0 * sin(two_pi * u[1]),
                        r1 * cos(two_pi * u[3]), r1 * sin(two_pi * u[3])};
        for (int i = 0; i < 4 && 4 * g + i < n; i++) out[4 * g + i] = nv[i];
    }
}

static int spa_impulse_fails(const or_code *c, const int32_t *ts, int a, double h,
                             int k, int max_iter, double *llr) {
    for (int v = 0; v < c->n; v++) llr[v] = h;
    for (int i = 0; i < a; i++) llr[ts[i]] = h * (1.0 - (double)k / 1024.0);
    return or_decode_spa(c, llr, max_iter, NULL, NULL, NULL).fail;
}

double or_spa_eps_star(const or_code *c, const int32_t *ts, int a, double ebn0_db,
                       double rate, int max_iter, double eps_max) {
    double h = 2.0 / or_sigma2(ebn0_db, rate);
    double *llr = malloc(sizeof(double) * (size_t)c->n);
    int k_max = (int)lround(eps_max * 1024.0);
    double out = -1.0;
    if (spa_impulse_fails(c, ts, a, h, k_max, max_iter, llr)) {
        int lo = 0, hi = k_max;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (spa_impulse_fails(c, ts, a, h, mid, max_iter, llr)) hi = mid;
            else lo = mid;
        }
        out = hi / 1024.0;
    }
    free(llr);
    return out;
}

int or_is_estimate(const or_code *c, const int32_t *ts, int a, const or_is_opts *o,
                   or_is_result *res, uint8_t *fail_out, int64_t *edge_updates) {
    if (o->n_frames < 2 || a < 1 || o->max_iter < 1) return -1;
    if (o->count_mode != OR_IS_COUNT_ALL && o->count_mode != OR_IS_COUNT_TS) return -1;
    double sigma2 = or_sigma2(o->ebn0_db, o->rate), sigma = sqrt(sigma2);
    uint8_t *in_t = calloc((size_t)c->n, 1);
    for (int i = 0; i < a; i++) in_t[ts[i]] = 1;
    double *wf = malloc(sizeof(double) * (size_t)o->n_frames);   /* 1[fail] w per frame */
    uint8_t *failv = malloc((size_t)o->n_frames);
    int64_t eu = 0;
    int threads = o->threads;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#else
    threads = 1;
#endif
#pragma omp parallel num_threads(threads) reduction(+ : eu)
    {
        double *nz = malloc(sizeof(double) * ((size_t)c->n + 4));
        double *llr = malloc(sizeof(double) * (size_t)c->n);
        double *app = malloc(sizeof(double) * (size_t)c->n);
#pragma omp for schedule(dynamic, 64)
        for (int64_t f = 0; f < o->n_frames; f++) {
            or_normals(o->seed, o->frame_base + (uint64_t)f, o->stream, c->n, nz);
            double s = o->shift;
            if (o->n_mix > 0) s = o->mix_s0 + (double)((f * o->n_mix) / o->n_frames) * o->mix_ds;
            double sum_t = 0.0, sum_y = 0.0;
            for (int v = 0; v < c->n; v++) {
                double y = 1.0 - (in_t[v] ? s : 0.0) + sigma * nz[v];
                llr[v] = 2.0 * y / sigma2;
                if (in_t[v]) {
                    sum_t += nz[v];
                    sum_y += y;
                }
            }
            or_dec_result r;
            if (o->decoder == OR_IS_LINEAR) {
                r.fail = sum_y < 0.0;
                r.iters = 0;
                memcpy(app, llr, sizeof(double) * (size_t)c->n);
            } else {
                r = or_decode_spa(c, llr, o->max_iter, NULL, NULL, app);
            }
            eu += (int64_t)r.iters * c->e;
            /* T's own error event: every bit of T decided 1 at the end of the
             * decode, and at most 2a bits in error in all */
            int t_err = r.fail, n_err = 0;
            for (int i = 0; i < a && t_err; i++) t_err = app[ts[i]] < 0.0;
            for (int v = 0; v < c->n; v++) n_err += app[v] < 0.0;
            t_err = t_err && n_err <= 2 * a;
            const int counted = o->count_mode == OR_IS_COUNT_TS ? t_err : r.fail;
            double w;
            if (o->n_mix > 0) {
                /* D = sum over T of (1 - y_v) / sigma = a s / sigma - sum_t */
                const double D = a * s / sigma - sum_t;
                double den = 0.0;
                for (int k = 0; k < o->n_mix; k++) {
                    const double sk = o->mix_s0 + k * o->mix_ds;
                    const int64_t f0 = (k * o->n_frames + o->n_mix - 1) / o->n_mix;
                    const int64_t f1 = ((k + 1) * o->n_frames + o->n_mix - 1) / o->n_mix;
                    den += (double)(f1 - f0) / (double)o->n_frames *
                           exp((sk / sigma) * D - a * sk * sk / (2.0 * sigma2));
                }
                w = 1.0 / den;
            } else {
                w = exp(-a * s * s / (2.0 * sigma2) + (s / sigma) * sum_t);
            }
            wf[f] = counted ? w : 0.0;
            failv[f] = (uint8_t)(r.fail | (t_err << 1));
        }
        free(nz);
        free(llr);
        free(app);
    }
    /* sums in frame order */
    double sw = 0.0, sw2 = 0.0;
    int64_t nf = 0;
    for (int64_t f = 0; f < o->n_frames; f++) {
        sw += wf[f];
        sw2 += wf[f] * wf[f];
        nf += o->count_mode == OR_IS_COUNT_TS ? (failv[f] >> 1) & 1 : failv[f] & 1;
    }
    double K = (double)o->n_frames;
    double p = sw / K;
    double ss = 0.0;
    for (int64_t f = 0; f < o->n_frames; f++) ss += (wf[f] - p) * (wf[f] - p);
    double var = ss / (K * (K - 1.0));
    res->p_hat = p;
    res->var = var;
    res->ci_lo = p - 1.96 * sqrt(var);
    res->ci_hi = p + 1.96 * sqrt(var);
    res->sum_w = sw;
    res->sum_w2 = sw2;
    res->n = o->n_frames;
    res->n_fail = nf;
    res->shift_used = o->n_mix > 0 ? o->mix_s0 + (o->n_mix - 1) * o->mix_ds : o->shift;
    if (edge_updates) *edge_updates = eu;
    if (fail_out) memcpy(fail_out, failv, (size_t)o->n_frames);
    free(in_t);
    free(wf);
    free(failv);
    return 0;
}

/* Mean shift chosen by pilot runs (a reading of Cole's weighting, which leaves
 * the shift open).  The grid is s_i = eps* (1/2 + i/16), i = 0..8; pilot i
 * runs P frames with the estimate's options at s_i, on frame counters
 * frame_base + 2^40 + i P (its own frames, none shared with the estimate).
 * The chosen shift has the smallest relative variance Var / P_hat^2 among the
 * grid points with at least 10 counted failures (the first such point on
 * ties); without one it is eps*.  rv_out[9] (optional) receives each point's
 * relative variance (-1 where it does not qualify). */
double or_is_pilot_shift(const or_code *c, const int32_t *ts, int a, const or_is_opts *o,
                         double eps_star, int64_t pilot_frames, double *rv_out) {
    double best = -1.0, shift = eps_star;
    for (int i = 0; i <= 8; i++) {
        or_is_opts po = *o;
        po.shift = eps_star * (0.5 + i / 16.0);
        po.n_frames = pilot_frames;
        po.frame_base = o->frame_base + (1ull << 40) + (uint64_t)i * (uint64_t)pilot_frames;
        or_is_result r;
        double rv = -1.0;
        if (or_is_estimate(c, ts, a, &po, &r, NULL, NULL) == 0 && r.n_fail >= 10 && r.p_hat > 0.0)
            rv = r.var / (r.p_hat * r.p_hat);
        if (rv_out) rv_out[i] = rv;
        if (rv >= 0.0 && (best < 0.0 || rv < best)) {
            best = rv;
            shift = po.shift;
        }
    }
    return shift;
}
