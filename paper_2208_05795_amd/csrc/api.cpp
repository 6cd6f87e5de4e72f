// C ABI of the tsgpu library: context and code lifecycle, the impulse search
// driver (chunking, candidate buffer, table growth), importance sampling and
// the TS read-out.  The work of a call runs on an executor (stream, events,
// staging, statistics): the context's own one for the synchronous calls, a
// serving worker's one for submitted jobs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace tsg {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

std::string last_error_copy() { return g_err; }

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace tsg

using namespace tsg;

void *ts_exec::dalloc(size_t bytes) {
    if (bytes == 0) bytes = 4;
    void *p = nullptr;
    if (stream_alloc) {
        const hipError_t e = ctx->pool ? hipMallocFromPoolAsync(&p, bytes, ctx->pool, stream)
                                       : hipMallocAsync(&p, bytes, stream);
        return e == hipSuccess ? p : nullptr;
    }
    if (ctx->alloc) return ctx->alloc(bytes, ctx->user);
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void ts_exec::dfree(void *p) {
    if (!p) return;
    if (stream_alloc) (void)hipFreeAsync(p, stream);
    else if (ctx->free_fn) ctx->free_fn(p, ctx->user);
    else (void)hipFree(p);
}

int ts_exec::bulk_buf(size_t bytes, unsigned char **p) {
    if (bytes > bulk_cap) {
        TSG_HIP(hipStreamSynchronize(stream));   // a copy may still use the old one
        if (bulk) (void)hipHostFree(bulk);
        bulk = nullptr;
        bulk_cap = 0;
        size_t cap = (size_t)1 << 20;
        while (cap < bytes) cap <<= 1;
        TSG_HIP(hipHostMalloc((void **)&bulk, cap, hipHostMallocDefault));
        bulk_cap = cap;
    }
    *p = bulk;
    return TS_OK;
}

int ts_exec::stage(const void *src, size_t bytes, void **dev, int *slot) {
    if (bytes > kJobSlotBytes) {
        tsg::set_error("job descriptors exceed %zu bytes", kJobSlotBytes);
        return TS_E_INVAL;
    }
    const int i = job_next;
    job_next = (job_next + 1) % kJobSlots;
    if (job_used[i]) TSG_HIP(hipEventSynchronize(job_ev[i]));   // its last launch has run
    std::memcpy(job_host + (size_t)i * kJobSlotBytes, src, bytes);
    TSG_HIP(hipMemcpyAsync(job_dev + (size_t)i * kJobSlotBytes, job_host + (size_t)i * kJobSlotBytes,
                           bytes, hipMemcpyHostToDevice, stream));
    *dev = job_dev + (size_t)i * kJobSlotBytes;
    *slot = i;
    return TS_OK;
}

void ts_exec::staged(int slot) {
    if (slot < 0) return;
    (void)hipEventRecord(job_ev[slot], stream);
    job_used[slot] = true;
}



namespace tsg {

double sigma2_of(double ebn0_db, double rate) { return 1.0 / (2.0 * rate * std::pow(10.0, ebn0_db / 10.0)); }

int sat127(long v) { return (int)(v > 127 ? 127 : (v < -127 ? -127 : v)); }

int64_t rec_capacity(const ts_search_opts *o, int t0, int64_t P, bool sieve, size_t max_bytes,
                     int64_t *worst) {
    const int d_fail_max = 2 + (int)std::ceil(std::log2((double)o->k_max));
    const int64_t wp = sieve ? (int64_t)d_fail_max * std::max(1, o->max_iter - t0 + 1) : 0;
    int64_t cap = std::min<int64_t>((int64_t)(max_bytes / (kRecStride * 4)), wp * P);
    cap = std::max<int64_t>(std::max<int64_t>(cap, wp), 1);
    if (worst) *worst = wp;
    return cap;
}

int first_iter(const ts_code *code, const ts_search_opts *o) {
    int t0 = o->collect_from_iter >= 0 ? o->collect_from_iter : code->girth / 2;
    return t0 < 1 ? 1 : t0;
}

// Search launch parameters of opts that do not depend on buffers.
void fill_search_launch(const ts_code *code, const ts_search_opts *o, int t0, int32_t width,
                        SearchLaunch *a) {
    const double h = 2.0 / sigma2_of(o->ebn0_db, o->rate);
    a->code = &code->dev;
    a->decoder = o->decoder;
    a->max_iter = o->max_iter;
    a->offset = o->oms_offset;
    const long q = std::lround(std::min(o->llr_scale * h, 1e6));   // saturated below anyway
    a->q_base = o->decoder == TS_DEC_LNMS_Q4 ? (int)(q > 7 ? 7 : (q < -7 ? -7 : q)) : sat127(q);
    a->k_max = o->k_max;
    a->k_den = o->k_den;
    a->h = (float)h;
    a->t0 = t0;
    a->cap = 2 * o->a_max;
    a->a_max = o->a_max;
    a->extract_mode = o->extract_mode;
    a->width = width;
    a->fp_exit = o->full_iterations ? 0 : 1;
}

size_t search_bytes_estimate(const ts_code *code, const ts_search_opts *o, int64_t P, int32_t width) {
    const int64_t cap = rec_capacity(o, first_iter(code, o), P, true, code->ctx->rec_bytes, nullptr);
    size_t scr = 0;   // decoder scratch of the largest streamed shape the autotuner may try
    std::vector<SearchPlan> shapes;
    if (plan_candidates(code->ctx, code, o->decoder, o->max_iter, &shapes) == TS_OK)
        for (const SearchPlan &p : shapes)
            scr = std::max(scr, (size_t)std::min<int64_t>(p.grid, std::max<int64_t>(P, 1)) * p.slot_bytes);
    return (size_t)P * (width + 5) * 4 + (size_t)cap * kRecStride * 4 + table_bytes(1 << 16) + scr + 4096;
}

int check_search_opts(const ts_code *code, const ts_search_opts *o, int32_t width) {
    if (o->decoder != TS_DEC_OMS_I8 && o->decoder != TS_DEC_SPA_F32 && o->decoder != TS_DEC_LNMS_Q4) {
        set_error("unknown decoder %d", o->decoder);
        return TS_E_INVAL;
    }
    if (o->decoder == TS_DEC_LNMS_Q4 && code->dev.n_layers == 0) {
        set_error("the code needs more than 64 layers for the layered decoder");
        return TS_E_INVAL;
    }
    if (o->max_iter < 1 || o->max_iter > kMaxIter) { set_error("max_iter must be 1..%d", kMaxIter); return TS_E_INVAL; }
    if (o->a_max < 1 || o->a_max > kMaxAmax) { set_error("a_max must be 1..%d", kMaxAmax); return TS_E_INVAL; }
    if (o->k_max < 1 || o->k_max > (1 << 24)) { set_error("k_max must be 1..2^24"); return TS_E_INVAL; }
    if (o->decoder != TS_DEC_SPA_F32 && o->k_den != 16) { set_error("the integer decoders use k_den = 16"); return TS_E_INVAL; }
    if (o->k_den < 1) { set_error("k_den must be positive"); return TS_E_INVAL; }
    if (o->oms_offset < 0 || o->oms_offset > 127) { set_error("oms_offset must be 0..127"); return TS_E_INVAL; }
    if (!(o->rate > 0.0 && o->rate <= 1.0) || !(o->llr_scale > 0.0)) { set_error("rate / llr_scale out of range"); return TS_E_INVAL; }
    if (!std::isfinite(o->ebn0_db) || !std::isfinite(o->llr_scale)) { set_error("Eb/N0 and llr_scale must be finite"); return TS_E_INVAL; }
    if (o->extract_mode != TS_EXTRACT_PATH && o->extract_mode != TS_EXTRACT_CRITICAL) { set_error("bad extract_mode"); return TS_E_INVAL; }
    if (o->mem != TS_MEM_HOST && o->mem != TS_MEM_DEVICE) { set_error("bad mem kind"); return TS_E_INVAL; }
    if (o->layout < TS_LAYOUT_AUTO || o->layout > TS_LAYOUT_STREAMED_ACCUM) { set_error("bad layout"); return TS_E_INVAL; }
    if (width < 1 || width > kMaxWidth) { set_error("width must be 1..%d", kMaxWidth); return TS_E_INVAL; }
    if (code->dv_max > kDvMax) { set_error("variable degree %d above the sieve's limit %d", code->dv_max, kDvMax); return TS_E_INVAL; }
    return TS_OK;
}

// Autotuner: times every candidate launch shape twice on a probe of the job's
// own patterns (candidate writing off) and keeps the best score per (code,
// decoder, iteration count, layout request).  Shapes only change the schedule,
// never the results.  Score of a probe time: a streamed shape must beat a
// register one by 10%, since in batches its message traffic meets other
// launches in L2 and the MALL (probes run alone) while register frames stay
// on chip.
static float tune_score(const SearchPlan &p, float ms) { return p.kind == kPlanStreamed ? 1.1f * ms : ms; }

static int tune_shape(ts_exec &ex, const std::vector<SearchPlan> &cands,
                      const SearchLaunch &base, int64_t P, SearchPlan *best) {
    // each shape's probe: sixteen patterns per workgroup of that shape (fewer
    // let the tail of a few long bisections decide), taken at an even stride
    // over the whole list (pattern lists are ordered by kind, and decode
    // lengths differ between kinds); shapes are compared by time per pattern
    int64_t probe_max = 0;
    for (const SearchPlan &p : cands) probe_max = std::max<int64_t>(probe_max, 16 * (int64_t)p.grid);
    probe_max = std::min(probe_max, P);
    DBuf sample(ex, probe_max < P ? (size_t)probe_max * base.width * 4 : 0);
    if (probe_max < P && !sample.p) {
        set_error("device allocation of the tuning probe failed");
        return TS_E_NOMEM;
    }
    const size_t row = (size_t)base.width * 4;
    int64_t sampled = 0;   // probe size the sample buffer holds
    float best_ms = 0.0f;  // best score per pattern
    for (const SearchPlan &p : cands) {
        const int64_t probe = std::min<int64_t>(16 * (int64_t)p.grid, P);
        const int *pat = base.patterns;
        if (probe < P) {
            if (sampled != probe) {
                TSG_HIP(hipMemcpy2DAsync(sample.p, row, base.patterns, (size_t)(P / probe) * row, row,
                                         (size_t)probe, hipMemcpyDeviceToDevice, ex.stream));
                sampled = probe;
            }
            pat = sample.as<int>();
        }
        float ms_min = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {   // the faster of two timings
            // a shape already 1.5x slower than the best needs no second timing
            if (rep == 1 && best_ms > 0.0f && tune_score(p, ms_min) / (float)probe > 1.5f * best_ms) break;
            SearchLaunch a = base;
            a.t0 = a.max_iter + 1;   // no candidate is written while timing
            a.patterns = pat;
            a.n_patterns = (int)probe;
            a.pat_base = 0;
            int rc = launch_fill(ex.stream, a.queue, 0, 2);
            if (rc) return rc;
            TSG_HIP(hipEventRecord(ex.ev[0], ex.stream));
            rc = launch_search(ex, p, a);
            if (rc) return rc;
            TSG_HIP(hipEventRecord(ex.ev[1], ex.stream));
            TSG_HIP(hipStreamSynchronize(ex.stream));
            float ms = 0.0f;
            TSG_HIP(hipEventElapsedTime(&ms, ex.ev[0], ex.ev[1]));
            if (rep == 0 || ms < ms_min) ms_min = ms;
        }
        const float score = tune_score(p, ms_min) / (float)probe;
        if (best_ms == 0.0f || score < best_ms) {
            best_ms = score;
            *best = p;
        }
    }
    return TS_OK;
}

static bool same_shape(const SearchPlan &p, const SearchShape &s) {
    return p.kind == s.kind && p.cpt == s.cpt && p.block == s.block && p.save_lds == s.save_lds;
}

static size_t scratch_bytes(const SearchPlan &p, int64_t P) {
    return (size_t)std::min<int64_t>(p.grid, std::max<int64_t>(P, 1)) * p.slot_bytes;
}

// Candidate shapes of a search (restricted to the requested layout) and the
// one to use: the autotuner's earlier choice for (decoder, iterations, layout),
// else the first; need_tune when there is no choice yet and a probe is worth it.
static int select_shape(ts_ctx *ctx, ts_code *code, const ts_search_opts *o, int64_t P,
                        std::vector<SearchPlan> *shapes, SearchPlan *plan, bool *need_tune) {
    int rc = plan_candidates(ctx, code, o->decoder, o->max_iter, shapes);
    if (rc) return rc;
    if (o->layout != TS_LAYOUT_AUTO) {
        shapes->erase(std::remove_if(shapes->begin(), shapes->end(),
                                     [&](const SearchPlan &p) { return !layout_accepts(o->layout, p); }),
                      shapes->end());
        if (shapes->empty()) {
            set_error("the requested decoder layout does not fit this code");
            return TS_E_INVAL;
        }
    }
    *plan = shapes->front();
    *need_tune = false;
    const int tune_key = (o->layout * 2 + o->decoder) * 1000 + o->max_iter;
    std::lock_guard<std::mutex> g(code->tune_mu);
    auto it = code->tuned.find(tune_key);
    if (it != code->tuned.end()) {
        for (const SearchPlan &p : *shapes)
            if (same_shape(p, it->second)) *plan = p;
    } else {
        *need_tune = shapes->size() > 1 && P >= 256;
    }
    return TS_OK;
}

static int is_tune_key(int max_iter, int layout) { return 500000 + layout * 1000 + max_iter; }

// IS counterpart of select_shape.
static int select_is_shape(ts_ctx *ctx, ts_code *code, int max_iter, int layout, int64_t K,
                           std::vector<SearchPlan> *shapes, SearchPlan *plan, bool *need_tune) {
    int rc = plan_is_candidates(ctx, code, max_iter, layout, shapes);
    if (rc) return rc;
    *plan = shapes->front();
    *need_tune = false;
    std::lock_guard<std::mutex> g(code->tune_mu);
    auto it = code->tuned.find(is_tune_key(max_iter, layout));
    if (it != code->tuned.end()) {
        for (const SearchPlan &p : *shapes)
            if (same_shape(p, it->second)) *plan = p;
    } else {
        *need_tune = shapes->size() > 1 && K >= 1024;
    }
    return TS_OK;
}

// Batches plan every job with its code's cached shape.  A job whose code has
// none yet for the job's (decoder, iterations, layout), and which is as large
// as a plain call that would tune (256 patterns / 1024 frames), first runs the
// plain call on a probe of its own patterns or frames (at most 8192; results
// discarded, statistics restored), which tunes and caches the shape.  Never
// fails: a probe that cannot run leaves the code untuned.
int tune_for_batch(ts_exec &ex, std::vector<BatchJob> &jobs) {
    const ts_stats keep = ex.stats;
    hipStream_t s = ex.stream;
    for (BatchJob &b : jobs) {
        ts_code *code = b.code;
        int rc = TS_OK;
        if (b.kind == TS_JOB_SEARCH) {
            if (b.n_patterns < 256) continue;
            {
                std::lock_guard<std::mutex> g(code->tune_mu);
                if (code->tuned.count((b.so.layout * 2 + b.so.decoder) * 1000 + b.so.max_iter)) continue;
            }
            const int64_t P = std::min<int64_t>(b.n_patterns, 8192);
            DBuf d_pat(ex, (size_t)P * b.width * 4), d_out(ex, (size_t)5 * P * 4);
            if (!d_pat.p || !d_out.p) continue;
            if (hipMemcpyAsync(d_pat.p, b.patterns, (size_t)P * b.width * 4, hipMemcpyHostToDevice, s) != hipSuccess)
                continue;
            int32_t *outs[5];
            for (int i = 0; i < 5; ++i) outs[i] = d_out.as<int32_t>() + (size_t)i * P;
            DevTable none{};
            rc = run_search(ex, code, none, &b.so, d_pat.as<int32_t>(), P, b.width, outs, false);
        } else {
            if (b.io.n_frames < 1024) continue;
            {
                std::lock_guard<std::mutex> g(code->tune_mu);
                if (code->tuned.count(is_tune_key(b.io.max_iter, b.io.layout))) continue;
            }
            ts_is_opts io = b.io;
            io.n_frames = std::min<int64_t>(io.n_frames, 8192);
            if (io.shift < 0.0) io.shift = 1.0;   // no eps* search for a timing probe
            ts_is_result res{};
            rc = run_is(ex, code, b.ts_bits, b.a, &io, &res, nullptr);
        }
        // tuning is an optimisation: a probe that fails (the batch reports the
        // job's own error) leaves the code untuned
        if (rc) clear_error();
    }
    (void)hipStreamSynchronize(s);
    ex.stats = keep;
    return TS_OK;
}

int plan_is_shape(ts_exec &ex, ts_code *code, int max_iter, int layout, SearchPlan *plan) {
    std::vector<SearchPlan> shapes;
    bool need_tune = false;
    return select_is_shape(ex.ctx, code, max_iter, layout, 0, &shapes, plan, &need_tune);
}

int plan_search_shape(ts_exec &ex, ts_code *code, const ts_search_opts *o, int64_t P, SearchPlan *plan) {
    std::vector<SearchPlan> shapes;
    bool need_tune = false;
    return select_shape(ex.ctx, code, o, P, &shapes, plan, &need_tune);
}

// Runs the search on device-resident patterns / outputs into `table`.  With
// sieve = false no candidate is written (only k* and the iteration counts).
int run_search(ts_exec &ex, ts_code *code, DevTable &table, const ts_search_opts *o,
               const int32_t *d_pat, int64_t P, int32_t width, int32_t *const d_out[5], bool sieve) {
    ts_ctx *ctx = ex.ctx;
    hipStream_t s = ex.stream;
    std::vector<SearchPlan> shapes;
    SearchPlan plan;
    bool need_tune = false;
    const int tune_key = (o->layout * 2 + o->decoder) * 1000 + o->max_iter;
    int rc = select_shape(ctx, code, o, P, &shapes, &plan, &need_tune);
    if (rc) return rc;
    size_t scr_bytes = scratch_bytes(plan, P);
    if (need_tune)
        for (const SearchPlan &p : shapes) scr_bytes = std::max(scr_bytes, scratch_bytes(p, P));
    DBuf scratch(ex, scr_bytes);
    if (scr_bytes && !scratch.p) { set_error("device allocation of the decoder scratch failed"); return TS_E_NOMEM; }
    int t0 = first_iter(code, o);
    if (!sieve) t0 = o->max_iter + 1;   // no iteration qualifies: nothing is written

    DBuf misc(ex, 64 * 4);
    if (!misc.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    int *d_misc = misc.as<int>();
    // misc layout: [0] queue, [1] rec_count, [2] err, [4..7] counters (2 x u64)
    rc = launch_fill(s, d_misc, 0, 64);
    if (rc) return rc;
    const int64_t rec_cap = rec_capacity(o, t0, P, sieve, ctx->rec_bytes, nullptr);
    DBuf recs(ex, (size_t)rec_cap * kRecStride * 4);
    if (!recs.p) { set_error("device allocation of the candidate buffer failed"); return TS_E_NOMEM; }

    SearchLaunch a{};
    fill_search_launch(code, o, t0, width, &a);
    a.k_crit = d_out[0];
    a.iters_crit = d_out[1];
    a.iters_lo = d_out[2];
    a.tmin_crit = d_out[3];
    a.n_cand = d_out[4];
    a.queue = d_misc;
    a.rec_count = d_misc + 1;
    a.err = d_misc + 2;
    a.counters = (unsigned long long *)(d_misc + 4);
    a.recs = recs.as<int>();
    a.rec_cap = (int)rec_cap;
    a.gscr = scr_bytes ? scratch.as<unsigned char>() : nullptr;

    if (need_tune) {
        a.patterns = d_pat;
        rc = tune_shape(ex, shapes, a, P, &plan);
        if (rc) return rc;
        std::lock_guard<std::mutex> g(code->tune_mu);
        SearchShape sh;
        sh.kind = plan.kind;
        sh.cpt = plan.cpt;
        sh.block = plan.block;
        sh.save_lds = plan.save_lds;
        code->tuned[tune_key] = sh;
        rc = launch_fill(s, d_misc, 0, 64);   // the probe's counters are not the job's
        if (rc) return rc;
    }
    if (sieve) {
        rc = table_init(ex, table, 1 << 16);
        if (rc) return rc;
    }
    TSG_HIP(hipEventRecord(ex.ev[4], s));
    int64_t chunk = P, pos = 0, cands = 0;
    double dec_ms = 0.0, sieve_ms = 0.0;
    // decodes and computed iterations of the accepted chunks (a chunk whose
    // candidates overflow the buffer is re-run, and its first run not counted)
    unsigned long long cnt[2] = {0, 0};
    while (pos < P) {
        const int64_t len = std::min<int64_t>(chunk, P - pos);
        rc = launch_fill(s, d_misc, 0, 2);   // queue, rec_count
        if (rc) return rc;
        rc = launch_fill(s, d_misc + 4, 0, 4);   // the chunk's counters
        if (rc) return rc;
        a.patterns = d_pat + pos * width;
        a.n_patterns = (int)len;
        a.pat_base = (int)pos;
        TSG_HIP(hipEventRecord(ex.ev[0], s));
        rc = launch_search(ex, plan, a);
        if (rc) return rc;
        TSG_HIP(hipEventRecord(ex.ev[1], s));
        TSG_HIP(hipMemcpyAsync(ex.pinned, d_misc, 32, hipMemcpyDeviceToHost, s));
        TSG_HIP(hipStreamSynchronize(s));
        float ms = 0.0f;
        TSG_HIP(hipEventElapsedTime(&ms, ex.ev[0], ex.ev[1]));
        dec_ms += ms;
        ex.stats.decode_launches++;
        const int64_t nrec = ex.pinned[1];
        if (ex.pinned[2] & 1) { set_error("pattern entry out of range"); return TS_E_INVAL; }
        if (nrec > rec_cap) {
            if (len == 1) { set_error("candidate buffer too small for one pattern"); return TS_E_NOMEM; }
            chunk = std::max<int64_t>(1, len / 2);   // re-run this chunk in smaller pieces
            continue;
        }
        {
            unsigned long long c[2];
            std::memcpy(c, ex.pinned + 4, 16);
            cnt[0] += c[0];
            cnt[1] += c[1];
        }
        if (sieve && nrec > 0) {
            cands += nrec;
            rc = table_grow_if_needed(ex, table, 2 * nrec);
            if (rc) return rc;
            TSG_HIP(hipEventRecord(ex.ev[2], s));
            rc = launch_sieve(ex, code->dev, table, a, (int)nrec);
            if (rc) return rc;
            TSG_HIP(hipEventRecord(ex.ev[3], s));
            TSG_HIP(hipStreamSynchronize(s));
            TSG_HIP(hipEventElapsedTime(&ms, ex.ev[2], ex.ev[3]));
            sieve_ms += ms;
            ex.stats.extract_launches++;
        }
        pos += len;
    }
    TSG_HIP(hipMemcpyAsync(ex.pinned, d_misc, 32, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipEventRecord(ex.ev[5], s));
    TSG_HIP(hipStreamSynchronize(s));
    float tot = 0.0f;
    TSG_HIP(hipEventElapsedTime(&tot, ex.ev[4], ex.ev[5]));
    const int err = ex.pinned[2];
    ex.stats.decode_ms += dec_ms;
    ex.stats.extract_ms += sieve_ms;
    ex.stats.total_ms += tot;
    ex.stats.decodes += (int64_t)cnt[0];
    ex.stats.edge_updates += (int64_t)cnt[1] * code->e;
    ex.stats.candidates += cands;
    ex.stats.block_threads = plan.block;
    ex.stats.grid_blocks = (int)std::min<int64_t>(plan.grid, P);
    ex.stats.layout = plan.kind == kPlanRegister ? TS_LAYOUT_REGISTER : TS_LAYOUT_STREAMED;
    ex.stats.checks_per_thread = plan.cpt;
    if (err & 1) { set_error("pattern entry out of range"); return TS_E_INVAL; }
    if (err & 4) { set_error("TS table insert timed out"); return TS_E_DEVICE; }
    if (err & 8) { set_error("TS table full"); return TS_E_NOMEM; }
    if (err & 16) { set_error("corrupt candidate record"); return TS_E_DEVICE; }
    return TS_OK;
}

// eps* of the noiseless SPA impulse on the whole set (device bits d_t), grid
// 2^-10 up to 32: the default mean shift of the IS frames.
static ts_search_opts eps_search_opts(const ts_is_opts *o) {
    ts_search_opts so{};
    so.decoder = TS_DEC_SPA_F32;
    so.max_iter = o->max_iter;
    so.ebn0_db = o->ebn0_db;
    so.rate = o->rate;
    so.llr_scale = 4.0;
    so.k_max = 32 * 1024;
    so.k_den = 1024;
    so.a_max = 1;
    so.extract_mode = TS_EXTRACT_CRITICAL;
    so.collect_from_iter = -1;
    so.mem = TS_MEM_DEVICE;
    so.layout = o->layout;
    so.full_iterations = o->full_iterations;
    return so;
}

// eps* of several sets of one code under the same IS options: one search
// launch with one pattern per set (a pattern's decodes do not depend on the
// other patterns of the launch), so every value is the one is_eps_shift gives.
int is_eps_shifts(ts_exec &ex, ts_code *code, const ts_is_opts *o,
                  const std::vector<std::vector<int32_t>> &sets, double *shift) {
    hipStream_t s = ex.stream;
    const int J = (int)sets.size();
    if (J == 0) return TS_OK;
    int W = 1;
    for (const auto &t : sets) W = std::max(W, (int)t.size());
    std::vector<int32_t> pat((size_t)J * W, -1), kc(J);
    for (int j = 0; j < J; ++j) {
        std::vector<int32_t> t = sets[j];
        std::sort(t.begin(), t.end());
        std::copy(t.begin(), t.end(), pat.begin() + (size_t)j * W);
    }
    const ts_search_opts so = eps_search_opts(o);
    DBuf d_pat(ex, pat.size() * 4), outs(ex, (size_t)5 * J * 4);
    if (!d_pat.p || !outs.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    TSG_HIP(hipMemcpyAsync(d_pat.p, pat.data(), pat.size() * 4, hipMemcpyHostToDevice, s));
    int32_t *d_out[5];
    for (int i = 0; i < 5; ++i) d_out[i] = outs.as<int32_t>() + (size_t)i * J;
    DevTable none{};
    int rc = run_search(ex, code, none, &so, d_pat.as<int32_t>(), J, W, d_out, false);
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(kc.data(), d_out[0], (size_t)J * 4, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < J; ++j) {
        if (kc[j] < 0) {
            set_error("the impulse on the whole set never fails; give a shift");
            return TS_E_INVAL;
        }
        shift[j] = kc[j] / 1024.0;
    }
    return TS_OK;
}

int is_eps_shift(ts_exec &ex, ts_code *code, const int32_t *d_t, int32_t a, const ts_is_opts *o,
                 double *shift) {
    hipStream_t s = ex.stream;
    const ts_search_opts so = eps_search_opts(o);
    DBuf outs(ex, 5 * 4);
    if (!outs.p) return TS_E_NOMEM;
    int32_t *d_out[5];
    for (int i = 0; i < 5; ++i) d_out[i] = outs.as<int32_t>() + i;
    DevTable none{};
    int rc = run_search(ex, code, none, &so, d_t, 1, a, d_out, false);
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(ex.pinned, d_out[0], 4, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipStreamSynchronize(s));
    const int32_t kc = ex.pinned[0];
    if (kc < 0) {
        set_error("the impulse on the whole set never fails; give a shift");
        return TS_E_INVAL;
    }
    *shift = kc / 1024.0;
    return TS_OK;
}

// Mean shift chosen by pilot runs (TS_SHIFT_PILOT; a reading of Cole's
// weighting, which leaves the shift open).  Grid point i of a request (eps*
// its set's impulse threshold) is s_i = eps* (kPilotF0 + i kPilotDf); its
// pilot estimate uses the request's options with P frames of its own, frame
// counters frame_base + kPilotFrameOffset + i P (the request's stream), so the
// pilot shares no frame with the estimate itself.  The chosen point has the
// smallest relative variance Var / P_hat^2 among the points with at least
// kPilotMinFail counted failures (ties: the smaller shift); without such a
// point the shift is eps*.  All pilots of all requests run as one batch.
constexpr int kPilotPoints = 9;
constexpr double kPilotF0 = 0.5, kPilotDf = 0.0625;
constexpr int64_t kPilotDefaultFrames = 2000;
constexpr int kPilotMinFail = 10;
constexpr uint64_t kPilotFrameOffset = 1ull << 40;

int pilot_shifts(ts_exec &ex, std::vector<PilotReq> &reqs) {
    if (reqs.empty()) return TS_OK;
    std::vector<BatchJob> jobs;
    std::vector<ts_is_result> res(reqs.size() * kPilotPoints);
    for (size_t r = 0; r < reqs.size(); ++r) {
        const PilotReq &q = reqs[r];
        const int64_t P = q.io.pilot_frames > 0 ? q.io.pilot_frames : kPilotDefaultFrames;
        for (int i = 0; i < kPilotPoints; ++i) {
            BatchJob b;
            b.kind = TS_JOB_IS;
            b.code = q.code;
            b.io = q.io;
            b.io.shift = q.eps * (kPilotF0 + i * kPilotDf);
            b.io.n_frames = P;
            b.io.frame_base = q.io.frame_base + kPilotFrameOffset + (uint64_t)i * (uint64_t)P;
            b.ts_bits = q.bits;
            b.a = q.a;
            b.is = &res[r * kPilotPoints + i];
            jobs.push_back(b);
        }
    }
    const int rc = run_batch(ex, jobs);
    if (rc) return rc;
    for (const BatchJob &b : jobs)
        if (b.status != TS_OK) {
            set_error("%s", b.err.c_str());
            return b.status;
        }
    for (size_t r = 0; r < reqs.size(); ++r) {
        double best = -1.0, shift = reqs[r].eps;
        for (int i = 0; i < kPilotPoints; ++i) {
            const ts_is_result &x = res[r * kPilotPoints + i];
            if (x.n_fail < kPilotMinFail || !(x.p_hat > 0.0)) continue;
            const double rv = x.var / (x.p_hat * x.p_hat);
            if (best < 0.0 || rv < best) {
                best = rv;
                shift = x.shift_used;
            }
        }
        *reqs[r].shift = shift;
    }
    return TS_OK;
}

// The mixture of TS_SHIFT_MIX up to eps* (a reading of Cole's weighting): the
// frames are split evenly, in frame order, over the shifts
// eps* (kMixF0 + k kMixDf), k < kMixPoints, and every counted frame is weighted
// by the balance heuristic over all of them (the likelihood ratio of the
// unshifted density over the mixture density).  The unshifted component
// bounds every weight by the number of components, and the others cover the
// set's displacements up to eps*, so no frame's weight can run away the way a
// single shift's does for failures far from it.
void set_mixture(IsLaunch *L, double eps) {
    L->n_mix = kMixPoints;
    L->mix_s0 = eps * kMixF0;
    L->mix_ds = eps * kMixDf;
}

// IS estimate from the fixed-order sums red = {sum w, sum w^2, failures,
// sum (w - p)^2} of K frames.
void is_fill_result(const double red[4], int64_t K, double shift, ts_is_result *res) {
    const double p = red[0] / (double)K;
    const double var = red[3] / ((double)K * (double)(K - 1));
    res->p_hat = p;
    res->var = var;
    res->ci_lo = p - 1.96 * std::sqrt(var);
    res->ci_hi = p + 1.96 * std::sqrt(var);
    res->sum_w = red[0];
    res->sum_w2 = red[1];
    res->n = K;
    res->n_fail = (int64_t)std::llround(red[2]);
    res->shift_used = shift;
}

int check_is_opts(const ts_code *code, const int32_t *ts_bits, int32_t a, const ts_is_opts *o) {
    if (a < 1 || a > kMaxWidth || !ts_bits) { set_error("TS size must be 1..%d", kMaxWidth); return TS_E_INVAL; }
    if (o->n_frames < 2 || o->n_frames > (1ll << 31) - 1) { set_error("n_frames must be 2..2^31-1"); return TS_E_INVAL; }
    if (o->max_iter < 1 || o->max_iter > kMaxIter) { set_error("max_iter must be 1..%d", kMaxIter); return TS_E_INVAL; }
    if (!(o->rate > 0.0 && o->rate <= 1.0)) { set_error("rate out of range"); return TS_E_INVAL; }
    if (!std::isfinite(o->ebn0_db) || !std::isfinite(o->shift)) { set_error("Eb/N0 and shift must be finite"); return TS_E_INVAL; }
    if (o->layout < TS_LAYOUT_AUTO || o->layout > TS_LAYOUT_STREAMED_ACCUM) { set_error("bad layout"); return TS_E_INVAL; }
    if (o->count_mode != TS_IS_COUNT_ALL && o->count_mode != TS_IS_COUNT_TS) { set_error("bad count_mode"); return TS_E_INVAL; }
    if (o->shift_rule != TS_SHIFT_EPS && o->shift_rule != TS_SHIFT_PILOT && o->shift_rule != TS_SHIFT_MIX) {
        set_error("bad shift_rule");
        return TS_E_INVAL;
    }
    if (o->pilot_frames < 0 || o->pilot_frames > (1ll << 24)) { set_error("pilot_frames must be 0..2^24"); return TS_E_INVAL; }
    std::vector<int32_t> t(ts_bits, ts_bits + a);
    std::sort(t.begin(), t.end());
    for (int i = 0; i < a; ++i)
        if (t[i] < 0 || t[i] >= code->n || (i && t[i] == t[i - 1])) {
            set_error("TS bits must be distinct variables of the code");
            return TS_E_INVAL;
        }
    return TS_OK;
}

int run_is(ts_exec &ex, ts_code *code, const int32_t *ts_bits, int32_t a, const ts_is_opts *o,
           ts_is_result *res, uint8_t *fail_out) {
    hipStream_t s = ex.stream;
    int rc0 = check_is_opts(code, ts_bits, a, o);
    if (rc0) return rc0;
    std::vector<int32_t> t(ts_bits, ts_bits + a);
    std::sort(t.begin(), t.end());
    double shift = o->shift;
    DBuf d_t(ex, kMaxWidth * 4);
    if (!d_t.p) return TS_E_NOMEM;
    TSG_HIP(hipMemcpyAsync(d_t.p, t.data(), a * 4, hipMemcpyHostToDevice, s));
    if (shift < 0.0) {
        int rc = is_eps_shift(ex, code, d_t.as<int32_t>(), a, o, &shift);
        if (rc) return rc;
        if (o->shift_rule == TS_SHIFT_PILOT) {
            std::vector<PilotReq> req(1);
            req[0] = PilotReq{code, t.data(), a, *o, shift, &shift};
            rc = pilot_shifts(ex, req);
            if (rc) return rc;
        }
    }
    const int64_t K = o->n_frames;
    DBuf d_fail(ex, (size_t)K), d_wf(ex, (size_t)K * 8), d_misc(ex, 64 * 4), d_red(ex, 8 * 8),
        d_part(ex, (size_t)is_reduce_parts(K) * 3 * 8);
    if (!d_fail.p || !d_wf.p || !d_misc.p || !d_red.p || !d_part.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    int rc = launch_fill(s, d_misc.as<int>(), 0, 64);
    if (rc) return rc;
    IsLaunch L{};
    L.code = &code->dev;
    L.max_iter = o->max_iter;
    L.sigma2 = sigma2_of(o->ebn0_db, o->rate);
    L.shift = shift;
    L.n_frames = K;
    L.seed = o->seed;
    L.frame_base = o->frame_base;
    L.stream = o->stream;
    L.fp_exit = o->full_iterations ? 0 : 1;
    L.count_mode = o->count_mode;
    if (o->shift < 0.0 && o->shift_rule == TS_SHIFT_MIX) set_mixture(&L, shift);
    L.ts = d_t.as<int32_t>();
    L.a = a;
    L.fail = d_fail.as<unsigned char>();
    L.wf = d_wf.as<double>();
    L.counters = (unsigned long long *)(d_misc.as<int>() + 4);
    std::vector<SearchPlan> shapes;
    SearchPlan plan;
    bool need_tune = false;
    rc = select_is_shape(ex.ctx, code, o->max_iter, o->layout, K, &shapes, &plan, &need_tune);
    if (rc) return rc;
    size_t scr = 0;
    for (const SearchPlan &p : need_tune ? shapes : std::vector<SearchPlan>{plan})
        scr = std::max(scr, (size_t)std::min<int64_t>(p.grid, K) * p.slot_bytes);
    DBuf scratch(ex, scr);
    if (scr && !scratch.p) { set_error("device allocation of the decoder scratch failed"); return TS_E_NOMEM; }
    L.gscr = scr ? scratch.as<unsigned char>() : nullptr;
    // one IS launch of `frames` frames with shape p; ms_out: its duration
    auto launch = [&](const SearchPlan &p, int64_t frames, float *ms_out) -> int {
        IsJob job{};
        job.a = make_is_dev(L, p);
        job.cd = code->dev;
        job.item0 = 0;
        void *dj = nullptr;
        int slot = -1;
        int r = ex.stage(&job, sizeof(job), &dj, &slot);
        if (r) return r;
        TSG_HIP(hipEventRecord(ex.ev[0], s));
        r = launch_is_jobs(s, p, (const IsJob *)dj, 1, d_misc.as<int>(), frames);
        ex.staged(slot);
        if (r) return r;
        TSG_HIP(hipEventRecord(ex.ev[1], s));
        if (ms_out) {
            TSG_HIP(hipStreamSynchronize(s));
            TSG_HIP(hipEventElapsedTime(ms_out, ex.ev[0], ex.ev[1]));
        }
        return TS_OK;
    };
    if (need_tune) {
        // Autotuner: every shape twice on the job's first frames; the best is
        // kept for (code, iterations, layout request).  Frames only depend on
        // their Philox counters, so the real run below recomputes them exactly.
        int64_t probe = 0;
        for (const SearchPlan &p : shapes) probe = std::max<int64_t>(probe, 2 * (int64_t)p.grid);
        probe = std::min(probe, K);
        float best = 0.0f;
        for (const SearchPlan &p : shapes) {
            float ms_min = 0.0f;
            for (int rep = 0; rep < 2; ++rep) {   // the faster of two timings
                rc = launch_fill(s, d_misc.as<int>(), 0, 64);
                if (rc) return rc;
                float ms = 0.0f;
                rc = launch(p, probe, &ms);
                if (rc) return rc;
                if (rep == 0 || ms < ms_min) ms_min = ms;
            }
            const float score = tune_score(p, ms_min);
            if (best == 0.0f || score < best) {
                best = score;
                plan = p;
            }
        }
        std::lock_guard<std::mutex> g(code->tune_mu);
        SearchShape sh;
        sh.kind = plan.kind;
        sh.cpt = plan.cpt;
        sh.block = plan.block;
        sh.save_lds = plan.save_lds;
        code->tuned[is_tune_key(o->max_iter, o->layout)] = sh;
        rc = launch_fill(s, d_misc.as<int>(), 0, 64);
        if (rc) return rc;
    }
    const int grid = (int)std::min<int64_t>(plan.grid, K), block = plan.block;
    rc = launch(plan, K, nullptr);
    if (rc) return rc;
    const RedJob rj = make_red_job(make_is_dev(L, plan), L.wf, L.fail, K, d_red.as<double>(),
                                   d_part.as<double>());
    rc = launch_is_reduce(s, rj, 0);
    if (rc) return rc;
    rc = launch_is_reduce(s, rj, 1);
    if (rc) return rc;
    double red[4];
    TSG_HIP(hipMemcpyAsync(ex.pinned, d_red.p, 32, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipMemcpyAsync(ex.pinned + 8, d_misc.as<int>() + 4, 16, hipMemcpyDeviceToHost, s));
    if (fail_out) TSG_HIP(hipMemcpyAsync(fail_out, d_fail.p, (size_t)K, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipEventRecord(ex.ev[2], s));
    TSG_HIP(hipStreamSynchronize(s));
    std::memcpy(red, ex.pinned, 32);
    unsigned long long cnt[2];
    std::memcpy(cnt, ex.pinned + 8, 16);
    float ms = 0.0f, tot = 0.0f;
    TSG_HIP(hipEventElapsedTime(&ms, ex.ev[0], ex.ev[1]));
    TSG_HIP(hipEventElapsedTime(&tot, ex.ev[0], ex.ev[2]));
    is_fill_result(red, K, shift, res);
    ex.stats.decode_ms += ms;
    ex.stats.total_ms += tot;
    ex.stats.decodes += K;
    ex.stats.edge_updates += (int64_t)cnt[1] * code->e;
    ex.stats.decode_launches += 1;
    ex.stats.block_threads = block;
    ex.stats.grid_blocks = grid;
    ex.stats.layout = plan.kind == kPlanRegister ? TS_LAYOUT_REGISTER : TS_LAYOUT_STREAMED;
    ex.stats.checks_per_thread = plan.cpt;
    return TS_OK;
}

}  // namespace tsg

namespace {

int exec_init(ts_exec &ex, ts_ctx *ctx, hipStream_t stream, bool stream_alloc) {
    ex.ctx = ctx;
    if (stream) {
        ex.stream = stream;
    } else {
        // default priority: stream priorities are left alone
        TSG_HIP(hipStreamCreateWithFlags(&ex.stream, hipStreamNonBlocking));
        ex.own_stream = true;
    }
    ex.stream_alloc = stream_alloc;
    if (stream_alloc && !ctx->pool) {
        // A pool of the context's own (the device's default pool is left as it
        // is), which keeps freed memory instead of returning it at every
        // synchronisation: serving batches allocate an arena per batch.  Where
        // it cannot be made, the workers allocate from the default pool.
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = ctx->device;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) == hipSuccess && pool) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            ctx->pool = pool;
        } else {
            (void)hipGetLastError();
        }
    }
    for (auto &e : ex.ev) TSG_HIP(hipEventCreate(&e));
    TSG_HIP(hipHostMalloc((void **)&ex.pinned, 64 * sizeof(int), hipHostMallocDefault));
    for (auto &e : ex.job_ev) TSG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    TSG_HIP(hipHostMalloc((void **)&ex.job_host, ts_exec::kJobSlots * ts_exec::kJobSlotBytes,
                          hipHostMallocDefault));
    TSG_HIP(hipMalloc((void **)&ex.job_dev, ts_exec::kJobSlots * ts_exec::kJobSlotBytes));
    return TS_OK;
}

void exec_fini(ts_exec &ex) {
    if (ex.stream) (void)hipStreamSynchronize(ex.stream);
    for (auto &e : ex.ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ex.job_ev)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < ts_exec::kSide; ++i) {
        if (ex.side[i]) {
            (void)hipStreamSynchronize(ex.side[i]);
            (void)hipStreamDestroy(ex.side[i]);
        }
        if (ex.side_ev[i]) (void)hipEventDestroy(ex.side_ev[i]);
    }
    if (ex.join_ev) (void)hipEventDestroy(ex.join_ev);
    if (ex.pinned) (void)hipHostFree(ex.pinned);
    if (ex.bulk) (void)hipHostFree(ex.bulk);
    if (ex.job_host) (void)hipHostFree(ex.job_host);
    if (ex.job_dev) (void)hipFree(ex.job_dev);
    if (ex.own_stream && ex.stream) (void)hipStreamDestroy(ex.stream);
    ex = ts_exec{};
}

}  // namespace

namespace tsg {
int exec_create(ts_exec &ex, ts_ctx *ctx) { return exec_init(ex, ctx, nullptr, true); }
void exec_destroy(ts_exec &ex) { exec_fini(ex); }
int table_readout(ts_ctx *ctx, const ts_code *code, const std::vector<int32_t> **recs,
                  const std::vector<int32_t> **bits) {
    if (code->readout_version != code->table_version) {
        code->readout_version = ~0ull;
        const int rc = collect_table(ctx->main, code->table, code->readout_recs, code->readout_bits);
        if (rc) return rc;
        code->readout_version = code->table_version;
    }
    *recs = &code->readout_recs;
    *bits = &code->readout_bits;
    return TS_OK;
}

}  // namespace tsg

extern "C" {

const char *ts_last_error(void) { return g_err.c_str(); }

int ts_create(const ts_ctx_opts *opts, ts_ctx **out) {
    clear_error();
    if (!out) { set_error("null output"); return TS_E_INVAL; }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        set_error("no HIP device available");
        return TS_E_DEVICE;
    }
    const int dev = opts ? opts->device : 0;
    if (dev < 0 || dev >= ndev) { set_error("device %d out of range", dev); return TS_E_INVAL; }
    if ((opts && opts->alloc) != (opts && opts->free)) {
        set_error("alloc and free must be given together");
        return TS_E_INVAL;
    }
    TSG_HIP(hipSetDevice(dev));
    ts_ctx *c = new (std::nothrow) ts_ctx();
    if (!c) { set_error("out of host memory"); return TS_E_NOMEM; }
    c->device = dev;
    c->t0 = now_ms();
    if (opts) {
        c->alloc = opts->alloc;
        c->free_fn = opts->free;
        c->user = opts->user;
        c->budget = opts->hbm_budget_bytes;
        if (opts->rec_buffer_bytes) c->rec_bytes = opts->rec_buffer_bytes;
    }
    int ncu = 0, lds = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        delete c;
        set_error("device query failed");
        return TS_E_DEVICE;
    }
    c->num_cu = ncu;
    c->lds_per_block = (size_t)lds;
    int rc = noalloc_init(dev);   // the no-allocation entry point's scratch on this device
    if (rc) {
        delete c;
        return rc;
    }
    rc = exec_init(c->main, c, opts ? (hipStream_t)opts->hip_stream : nullptr, false);
    if (rc) {
        exec_fini(c->main);
        delete c;
        return rc;
    }
    *out = c;
    return TS_OK;
}

int ts_free_code(ts_ctx *ctx, ts_code *code) {
    clear_error();
    if (!ctx || !code) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    if (code->jobs_in_flight.load() > 0) { set_error("code has submitted jobs in flight"); return TS_E_BUSY; }
    (void)hipStreamSynchronize(ctx->main.stream);
    table_free(ctx->main, code->table);
    for (void *p : code->dev_allocs) ctx->main.dfree(p);
    ctx->codes.erase(std::remove(ctx->codes.begin(), ctx->codes.end(), code), ctx->codes.end());
    delete code;
    return TS_OK;
}

int ts_destroy(ts_ctx *ctx) {
    clear_error();
    if (!ctx) return TS_OK;
    server_stop(ctx);
    {
        std::lock_guard<std::recursive_mutex> g(ctx->mu);
        while (!ctx->codes.empty()) ts_free_code(ctx, ctx->codes.back());
        exec_fini(ctx->main);
        // the workers (stopped above) have freed their memory into the pool
        if (ctx->pool) (void)hipMemPoolDestroy(ctx->pool);
    }
    delete ctx;
    return TS_OK;
}

int ts_load_code(ts_ctx *ctx, const ts_code_desc *desc, ts_code **out) {
    clear_error();
    if (!ctx || !desc || !out) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    *out = nullptr;
    ts_code *c = new (std::nothrow) ts_code();
    if (!c) { set_error("out of host memory"); return TS_E_NOMEM; }
    c->ctx = ctx;
    int rc = build_code(desc, c);
    if (rc == TS_OK) rc = upload_code(ctx->main, c);
    if (rc != TS_OK) {
        for (void *p : c->dev_allocs) ctx->main.dfree(p);
        delete c;
        return rc;
    }
    ctx->codes.push_back(c);
    *out = c;
    return TS_OK;
}

int ts_code_info(const ts_code *code, ts_code_info_t *out) {
    clear_error();
    if (!code || !out) { set_error("null argument"); return TS_E_INVAL; }
    out->n = code->n;
    out->m = code->m;
    out->e = code->e;
    out->girth = code->girth;
    out->z = code->z;
    out->dv_max = code->dv_max;
    out->dc_max = code->dc_max;
    out->n_layers = code->dev.n_layers;
    out->streamed_qc = code->dev.q_ok;
    return TS_OK;
}

int ts_code_csr(const ts_code *code, int64_t *row_ptr, int32_t *col) {
    clear_error();
    if (!code || !row_ptr || !col) { set_error("null argument"); return TS_E_INVAL; }
    std::memcpy(row_ptr, code->row_ptr.data(), code->row_ptr.size() * 8);
    std::memcpy(col, code->col.data(), code->col.size() * 4);
    return TS_OK;
}

int ts_make_patterns(ts_ctx *ctx, const ts_code *code, int32_t kind, int32_t *out, int64_t cap,
                     int64_t *n_out) {
    clear_error();
    if (!ctx || !code || !n_out || (cap > 0 && !out)) { set_error("null argument"); return TS_E_INVAL; }
    const int64_t n = make_patterns(code, kind, nullptr, 0);
    if (n < 0) {
        set_error((kind & TS_PAT_QC_ORBITS) && code->z <= 0 ? "orbit reduction needs a code in QC form"
                                                            : "unknown pattern kind %d", kind);
        return TS_E_INVAL;
    }
    *n_out = n;
    if (cap < n) {
        if (cap > 0) set_error("pattern buffer holds %lld, need %lld", (long long)cap, (long long)n);
        return cap > 0 ? TS_E_TRUNC : TS_OK;
    }
    make_patterns(code, kind, out, cap);
    return TS_OK;
}

int ts_get_stats(ts_ctx *ctx, ts_stats *out) {
    clear_error();
    if (!ctx || !out) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    *out = ctx->main.stats;
    return TS_OK;
}

int ts_reset_ts(ts_ctx *ctx, ts_code *code) {
    clear_error();
    if (!ctx || !code) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    (void)hipStreamSynchronize(ctx->main.stream);
    table_free(ctx->main, code->table);
    ++code->table_version;
    return TS_OK;
}

int ts_impulse_search(ts_ctx *ctx, ts_code *code, const ts_search_opts *o, const int32_t *patterns,
                      int32_t n_patterns, int32_t width, ts_search_out *out) {
    clear_error();
    if (!ctx || !code || !o || !out) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    ts_exec &ex = ctx->main;
    ex.stats = ts_stats{};
    int rc = check_search_opts(code, o, width);
    if (rc) return rc;
    ++code->table_version;   // the search may add sets to the table
    if (n_patterns < 0) { set_error("negative pattern count"); return TS_E_INVAL; }
    if (n_patterns == 0) return TS_OK;
    if (!patterns || !out->k_crit || !out->iters_crit || !out->iters_lo || !out->tmin_crit || !out->n_cand) {
        set_error("null pattern or output array");
        return TS_E_INVAL;
    }
    const size_t P = (size_t)n_patterns;
    int32_t *d_out[5] = {out->k_crit, out->iters_crit, out->iters_lo, out->tmin_crit, out->n_cand};
    if (o->mem == TS_MEM_DEVICE)
        return run_search(ex, code, code->table, o, patterns, (int64_t)P, width, d_out, true);
    for (size_t i = 0; i < P * (size_t)width; ++i)
        if (patterns[i] < -1 || patterns[i] >= code->n) {
            set_error("pattern entry %d out of range", patterns[i]);
            return TS_E_INVAL;
        }
    DBuf pat_buf(ex, P * width * 4), out_buf(ex, P * 5 * 4);
    if (!pat_buf.p || !out_buf.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    TSG_HIP(hipMemcpyAsync(pat_buf.p, patterns, P * width * 4, hipMemcpyHostToDevice, ex.stream));
    int32_t *dev_out[5];
    for (int i = 0; i < 5; ++i) dev_out[i] = out_buf.as<int32_t>() + i * P;
    rc = run_search(ex, code, code->table, o, pat_buf.as<int32_t>(), (int64_t)P, width, dev_out, true);
    if (rc) return rc;
    // the five output arrays are one device block: one copy, then host copies
    unsigned char *h = nullptr;
    rc = ex.bulk_buf(P * 5 * 4, &h);
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(h, out_buf.p, P * 5 * 4, hipMemcpyDeviceToHost, ex.stream));
    TSG_HIP(hipStreamSynchronize(ex.stream));
    for (int i = 0; i < 5; ++i) std::memcpy(d_out[i], h + (size_t)i * P * 4, P * 4);
    return TS_OK;
}

int ts_is_estimate(ts_ctx *ctx, ts_code *code, const int32_t *ts_bits, int32_t a,
                   const ts_is_opts *o, ts_is_result *res, uint8_t *fail_out) {
    clear_error();
    if (!ctx || !code || !ts_bits || !o || !res) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    ctx->main.stats = ts_stats{};
    return run_is(ctx->main, code, ts_bits, a, o, res, fail_out);
}

int ts_collect(ts_ctx *ctx, const ts_code *code, ts_record *recs, int64_t cap, int64_t *n_out,
               int32_t *bits, int64_t bits_cap, int64_t *bits_out) {
    clear_error();
    if (!ctx || !code || !n_out || !bits_out) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    const std::vector<int32_t> *rp = nullptr, *bp = nullptr;
    int rc = table_readout(ctx, code, &rp, &bp);
    if (rc) return rc;
    const std::vector<int32_t> &rh = *rp, &bh = *bp;
    const int64_t n = (int64_t)rh.size() / 5;
    *n_out = n;
    *bits_out = (int64_t)bh.size();
    if (cap == 0 && bits_cap == 0) return TS_OK;
    if (cap < n || bits_cap < (int64_t)bh.size()) {
        set_error("collect buffers too small (%lld records, %lld bits needed)", (long long)n,
                  (long long)bh.size());
        return TS_E_TRUNC;
    }
    if (!recs || (!bits && !bh.empty())) { set_error("null output array"); return TS_E_INVAL; }
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *r = rh.data() + i * 5;
        recs[i].a = r[0];
        recs[i].b = r[1];
        recs[i].orbit = r[2];
        recs[i].first_pattern = r[3];
        recs[i].k_crit = r[4];
        recs[i].reserved = 0;
        recs[i].bits_off = off;
        off += r[0];
    }
    if (!bh.empty()) std::memcpy(bits, bh.data(), bh.size() * 4);
    return TS_OK;
}

}  // extern "C"
