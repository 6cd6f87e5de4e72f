// The code's trapping-set spectrum and the union bound on the frame error rate
// (Section III): FER(SNR) ~ sum over the canonical TS T of orbit(T) x P_T(SNR),
// P_T from importance sampling of T (Section I/II).  Every (TS, SNR) estimate is
// one IS job; all of them run as one batch.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

using namespace tsg;

extern "C" {

int ts_spectrum(ts_ctx *ctx, const ts_code *code, int32_t a_max, int32_t b_max, int32_t by_orbit,
                int64_t *counts) {
    clear_error();
    if (!ctx || !code || !counts) { set_error("null argument"); return TS_E_INVAL; }
    if (a_max < 1 || a_max > kMaxAmax || b_max < 0 || b_max > 1024) { set_error("a_max must be 1..%d, b_max 0..1024", kMaxAmax); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    const std::vector<int32_t> *rp = nullptr, *bp = nullptr;
    const int rc = table_readout(ctx, code, &rp, &bp);
    if (rc) return rc;
    const std::vector<int32_t> &rh = *rp;
    std::memset(counts, 0, sizeof(int64_t) * (size_t)(a_max + 1) * (b_max + 1));
    for (size_t i = 0; i + 4 < rh.size(); i += 5) {
        const int a = rh[i], b = rh[i + 1], orbit = rh[i + 2];
        if (a > a_max || b > b_max) continue;
        counts[(size_t)a * (b_max + 1) + b] += by_orbit ? 1 : orbit;
    }
    return TS_OK;
}

int ts_union_bound(ts_ctx *ctx, ts_code *code, const ts_ub_opts *o, ts_ub_point *out,
                   ts_is_result *per_ts) {
    clear_error();
    if (!ctx || !code || !o || !out || (o->n_snr > 0 && !o->ebn0_db)) { set_error("null argument"); return TS_E_INVAL; }
    if (o->n_ts < 1 || o->n_snr < 1 || (int64_t)o->n_ts * o->n_snr > 4096) {
        set_error("need 1 <= n_ts, 1 <= n_snr, n_ts x n_snr <= 4096");
        return TS_E_INVAL;
    }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    const std::vector<int32_t> *rp = nullptr, *bp = nullptr;
    int rc = table_readout(ctx, code, &rp, &bp);
    if (rc) return rc;
    const std::vector<int32_t> rh = *rp, bh = *bp;   // copies: the jobs point into them
    const int n_avail = (int)(rh.size() / 5);
    if (n_avail < o->n_ts) {
        set_error("the code's TS table holds %d sets, %d requested", n_avail, o->n_ts);
        return TS_E_INVAL;
    }
    // bits offsets of the first n_ts records (the table read-out concatenates them)
    std::vector<int64_t> off(o->n_ts + 1, 0);
    for (int t = 0; t < o->n_ts; ++t) off[t + 1] = off[t] + rh[5 * t];
    std::vector<BatchJob> jobs;
    std::vector<ts_is_result> res((size_t)o->n_ts * o->n_snr);
    for (int si = 0; si < o->n_snr; ++si)
        for (int t = 0; t < o->n_ts; ++t) {
            BatchJob b;
            b.kind = TS_JOB_IS;
            b.code = code;
            b.io.max_iter = o->max_iter;
            b.io.ebn0_db = o->ebn0_db[si];
            b.io.rate = o->rate;
            b.io.shift = o->shift;
            b.io.n_frames = o->n_frames;
            b.io.seed = o->seed;
            b.io.frame_base = 0;
            b.io.stream = ((uint32_t)si << 16) | (uint32_t)t;
            b.io.layout = o->layout;
            b.io.count_mode = o->count_mode;
            b.io.shift_rule = o->shift_rule;
            b.io.pilot_frames = o->pilot_frames;
            b.ts_bits = bh.data() + off[t];
            b.a = rh[5 * t];
            b.is = &res[(size_t)si * o->n_ts + t];
            rc = check_is_opts(code, b.ts_bits, b.a, &b.io);
            if (rc) return rc;
            jobs.push_back(b);
        }
    ctx->main.stats = ts_stats{};
    rc = run_batch(ctx->main, jobs);
    if (rc) return rc;
    for (const BatchJob &b : jobs)
        if (b.status != TS_OK) {
            set_error("%s", b.err.c_str());
            return b.status;
        }
    for (int si = 0; si < o->n_snr; ++si) {
        double fer = 0.0, var = 0.0;
        for (int t = 0; t < o->n_ts; ++t) {
            const ts_is_result &r = res[(size_t)si * o->n_ts + t];
            const double orbit = (double)rh[5 * t + 2];
            fer += orbit * r.p_hat;
            var += orbit * orbit * r.var;
        }
        out[si].ebn0_db = o->ebn0_db[si];
        out[si].fer = fer;
        out[si].var = var;
        out[si].ci_lo = fer - 1.96 * std::sqrt(var);
        out[si].ci_hi = fer + 1.96 * std::sqrt(var);
    }
    if (per_ts) std::memcpy(per_ts, res.data(), res.size() * sizeof(ts_is_result));
    return TS_OK;
}

}  // extern "C"
