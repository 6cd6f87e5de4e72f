// C ABI of the tsgpu library: context and code lifecycle, the impulse search
// driver (chunking, candidate buffer, table growth) and the TS read-out.
#include <algorithm>
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

}  // namespace tsg

using namespace tsg;

void *ts_ctx::dalloc(size_t bytes) {
    if (bytes == 0) bytes = 4;
    if (alloc) return alloc(bytes, user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void ts_ctx::dfree(void *p) {
    if (!p) return;
    if (free_fn) free_fn(p, user);
    else (void)hipFree(p);
}

namespace {

// RAII device buffer from the context allocator
struct DBuf {
    ts_ctx *ctx;
    void *p = nullptr;
    DBuf(ts_ctx *c, size_t bytes) : ctx(c) { p = c->dalloc(bytes); }
    ~DBuf() { ctx->dfree(p); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    template <class T> T *as() { return (T *)p; }
};

double sigma2_of(double ebn0_db, double rate) { return 1.0 / (2.0 * rate * std::pow(10.0, ebn0_db / 10.0)); }

int sat127(long v) { return (int)(v > 127 ? 127 : (v < -127 ? -127 : v)); }

}  // namespace

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
    if (opts) {
        c->alloc = opts->alloc;
        c->free_fn = opts->free;
        c->user = opts->user;
        c->budget = opts->hbm_budget_bytes;
    }
    if (opts && opts->hip_stream) {
        c->stream = (hipStream_t)opts->hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            set_error("stream creation failed");
            return TS_E_DEVICE;
        }
        c->own_stream = true;
    }
    int ncu = 0, lds = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        set_error("device query failed");
        return TS_E_DEVICE;
    }
    c->num_cu = ncu;
    c->lds_per_block = (size_t)lds;
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            set_error("event creation failed");
            return TS_E_DEVICE;
        }
    if (hipHostMalloc((void **)&c->pinned, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        set_error("pinned allocation failed");
        return TS_E_NOMEM;
    }
    *out = c;
    return TS_OK;
}

int ts_free_code(ts_ctx *ctx, ts_code *code) {
    clear_error();
    if (!ctx || !code) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    (void)hipStreamSynchronize(ctx->stream);
    table_free(ctx, code);
    for (void *p : code->dev_allocs) ctx->dfree(p);
    ctx->codes.erase(std::remove(ctx->codes.begin(), ctx->codes.end(), code), ctx->codes.end());
    delete code;
    return TS_OK;
}

int ts_destroy(ts_ctx *ctx) {
    clear_error();
    if (!ctx) return TS_OK;
    {
        std::lock_guard<std::recursive_mutex> g(ctx->mu);
        while (!ctx->codes.empty()) ts_free_code(ctx, ctx->codes.back());
        (void)hipStreamSynchronize(ctx->stream);
        for (auto &e : ctx->ev)
            if (e) (void)hipEventDestroy(e);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
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
    if (rc == TS_OK) rc = upload_code(ctx, c);
    if (rc != TS_OK) {
        for (void *p : c->dev_allocs) ctx->dfree(p);
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
    if (n < 0) { set_error("unknown pattern kind %d", kind); return TS_E_INVAL; }
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
    *out = ctx->stats;
    return TS_OK;
}

int ts_reset_ts(ts_ctx *ctx, ts_code *code) {
    clear_error();
    if (!ctx || !code) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    (void)hipStreamSynchronize(ctx->stream);
    return table_free(ctx, code);
}

}  // extern "C"

namespace {

// Runs the search on device-resident patterns / outputs.  With sieve = false no
// candidate is written (only k* and the iteration counts are produced).
int run_search(ts_ctx *ctx, ts_code *code, const ts_search_opts *o, const int32_t *d_pat,
               int64_t P, int32_t width, int32_t *const d_out[5], bool sieve) {
    SearchPlan plan;
    int rc = plan_search(ctx, code, o->decoder, o->max_iter, &plan);
    if (rc) return rc;
    const double s2 = sigma2_of(o->ebn0_db, o->rate);
    const double h = 2.0 / s2;
    const int q_base = sat127(std::lround(o->llr_scale * h));
    int t0 = o->collect_from_iter >= 0 ? o->collect_from_iter : code->girth / 2;
    if (t0 < 1) t0 = 1;
    if (!sieve) t0 = o->max_iter + 1;   // no iteration qualifies: nothing is written

    DBuf misc(ctx, 64 * 4);
    if (!misc.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    int *d_misc = misc.as<int>();
    // misc layout: [0] queue, [1] rec_count, [2] err, [4..7] counters (2 x u64)
    rc = launch_fill(ctx, d_misc, 0, 64);
    if (rc) return rc;

    // candidate record buffer: at most 256 MB, at least one pattern's worst case
    const int d_fail_max = 2 + (int)std::ceil(std::log2((double)o->k_max));
    const int64_t worst_per_pat = sieve ? (int64_t)d_fail_max * std::max(1, o->max_iter - t0 + 1) : 0;
    int64_t rec_cap = std::min<int64_t>((256ll << 20) / (kRecStride * 4), worst_per_pat * P);
    rec_cap = std::max<int64_t>(std::max<int64_t>(rec_cap, worst_per_pat), 1);
    DBuf recs(ctx, (size_t)rec_cap * kRecStride * 4);
    if (!recs.p) { set_error("device allocation of the candidate buffer failed"); return TS_E_NOMEM; }

    SearchLaunch a{};
    a.code = &code->dev;
    a.decoder = o->decoder;
    a.max_iter = o->max_iter;
    a.offset = o->oms_offset;
    a.q_base = q_base;
    a.k_max = o->k_max;
    a.k_den = o->k_den;
    a.h = (float)h;
    a.t0 = t0;
    a.cap = 2 * o->a_max;
    a.a_max = o->a_max;
    a.extract_mode = o->extract_mode;
    a.width = width;
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

    if (sieve) {
        rc = table_init(ctx, code, 1 << 16);
        if (rc) return rc;
    }
    TSG_HIP(hipEventRecord(ctx->ev[4], ctx->stream));
    int64_t chunk = P, pos = 0, cands = 0;
    double dec_ms = 0.0, sieve_ms = 0.0;
    while (pos < P) {
        const int64_t len = std::min<int64_t>(chunk, P - pos);
        rc = launch_fill(ctx, d_misc, 0, 2);   // queue, rec_count
        if (rc) return rc;
        a.patterns = d_pat + pos * width;
        a.n_patterns = (int)len;
        a.pat_base = (int)pos;
        TSG_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
        rc = launch_search(ctx, plan, a);
        if (rc) return rc;
        TSG_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
        TSG_HIP(hipMemcpyAsync(ctx->pinned, d_misc, 16, hipMemcpyDeviceToHost, ctx->stream));
        TSG_HIP(hipStreamSynchronize(ctx->stream));
        float ms = 0.0f;
        TSG_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        dec_ms += ms;
        ctx->stats.decode_launches++;
        const int64_t nrec = ctx->pinned[1];
        if (ctx->pinned[2] & 1) { set_error("pattern entry out of range"); return TS_E_INVAL; }
        if (nrec > rec_cap) {
            if (len == 1) { set_error("candidate buffer too small for one pattern"); return TS_E_NOMEM; }
            chunk = std::max<int64_t>(1, len / 2);   // re-run this chunk in smaller pieces
            continue;
        }
        if (sieve && nrec > 0) {
            cands += nrec;
            rc = table_grow_if_needed(ctx, code, 2 * nrec);
            if (rc) return rc;
            TSG_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
            rc = launch_sieve(ctx, code, a, (int)nrec);
            if (rc) return rc;
            TSG_HIP(hipEventRecord(ctx->ev[3], ctx->stream));
            TSG_HIP(hipStreamSynchronize(ctx->stream));
            TSG_HIP(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
            sieve_ms += ms;
            ctx->stats.extract_launches++;
        }
        pos += len;
    }
    TSG_HIP(hipMemcpyAsync(ctx->pinned, d_misc, 32, hipMemcpyDeviceToHost, ctx->stream));
    TSG_HIP(hipEventRecord(ctx->ev[5], ctx->stream));
    TSG_HIP(hipStreamSynchronize(ctx->stream));
    float tot = 0.0f;
    TSG_HIP(hipEventElapsedTime(&tot, ctx->ev[4], ctx->ev[5]));
    const int err = ctx->pinned[2];
    unsigned long long cnt[2];
    std::memcpy(cnt, ctx->pinned + 4, 16);
    ctx->stats.decode_ms += dec_ms;
    ctx->stats.extract_ms += sieve_ms;
    ctx->stats.total_ms += tot;
    ctx->stats.decodes += (int64_t)cnt[0];
    ctx->stats.edge_updates += (int64_t)cnt[1] * code->e;
    ctx->stats.candidates += cands;
    ctx->stats.block_threads = plan.block;
    ctx->stats.grid_blocks = (int)std::min<int64_t>(plan.grid, P);
    if (err & 1) { set_error("pattern entry out of range"); return TS_E_INVAL; }
    if (err & 4) { set_error("TS table insert timed out"); return TS_E_DEVICE; }
    if (err & 8) { set_error("TS table full"); return TS_E_NOMEM; }
    if (err & 16) { set_error("corrupt candidate record"); return TS_E_DEVICE; }
    return TS_OK;
}

int check_search_opts(const ts_code *code, const ts_search_opts *o, int32_t width) {
    if (o->decoder != TS_DEC_OMS_I8 && o->decoder != TS_DEC_SPA_F32) {
        set_error("unknown decoder %d", o->decoder);
        return TS_E_INVAL;
    }
    if (o->max_iter < 1 || o->max_iter > kMaxIter) { set_error("max_iter must be 1..%d", kMaxIter); return TS_E_INVAL; }
    if (o->a_max < 1 || o->a_max > kMaxAmax) { set_error("a_max must be 1..%d", kMaxAmax); return TS_E_INVAL; }
    if (o->k_max < 1 || o->k_max > (1 << 24)) { set_error("k_max must be 1..2^24"); return TS_E_INVAL; }
    if (o->decoder == TS_DEC_OMS_I8 && o->k_den != 16) { set_error("the int8 decoder uses k_den = 16"); return TS_E_INVAL; }
    if (o->k_den < 1) { set_error("k_den must be positive"); return TS_E_INVAL; }
    if (o->oms_offset < 0 || o->oms_offset > 127) { set_error("oms_offset must be 0..127"); return TS_E_INVAL; }
    if (!(o->rate > 0.0 && o->rate <= 1.0) || !(o->llr_scale > 0.0)) { set_error("rate / llr_scale out of range"); return TS_E_INVAL; }
    if (o->extract_mode != TS_EXTRACT_PATH && o->extract_mode != TS_EXTRACT_CRITICAL) { set_error("bad extract_mode"); return TS_E_INVAL; }
    if (o->mem != TS_MEM_HOST && o->mem != TS_MEM_DEVICE) { set_error("bad mem kind"); return TS_E_INVAL; }
    if (width < 1 || width > kMaxWidth) { set_error("width must be 1..%d", kMaxWidth); return TS_E_INVAL; }
    if (code->dv_max > kDvMax) { set_error("variable degree %d above the sieve's limit %d", code->dv_max, kDvMax); return TS_E_INVAL; }
    return TS_OK;
}

}  // namespace

extern "C" {

int ts_impulse_search(ts_ctx *ctx, ts_code *code, const ts_search_opts *o, const int32_t *patterns,
                      int32_t n_patterns, int32_t width, ts_search_out *out) {
    clear_error();
    if (!ctx || !code || !o || !out) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    ctx->stats = ts_stats{};
    int rc = check_search_opts(code, o, width);
    if (rc) return rc;
    if (n_patterns < 0) { set_error("negative pattern count"); return TS_E_INVAL; }
    if (n_patterns == 0) return TS_OK;
    if (!patterns || !out->k_crit || !out->iters_crit || !out->iters_lo || !out->tmin_crit || !out->n_cand) {
        set_error("null pattern or output array");
        return TS_E_INVAL;
    }
    const size_t P = (size_t)n_patterns;
    int32_t *d_out[5] = {out->k_crit, out->iters_crit, out->iters_lo, out->tmin_crit, out->n_cand};
    if (o->mem == TS_MEM_DEVICE) return run_search(ctx, code, o, patterns, (int64_t)P, width, d_out, true);
    for (size_t i = 0; i < P * (size_t)width; ++i)
        if (patterns[i] < -1 || patterns[i] >= code->n) {
            set_error("pattern entry %d out of range", patterns[i]);
            return TS_E_INVAL;
        }
    DBuf pat_buf(ctx, P * width * 4), out_buf(ctx, P * 5 * 4);
    if (!pat_buf.p || !out_buf.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    TSG_HIP(hipMemcpyAsync(pat_buf.p, patterns, P * width * 4, hipMemcpyHostToDevice, ctx->stream));
    int32_t *dev_out[5];
    for (int i = 0; i < 5; ++i) dev_out[i] = out_buf.as<int32_t>() + i * P;
    rc = run_search(ctx, code, o, pat_buf.as<int32_t>(), (int64_t)P, width, dev_out, true);
    if (rc) return rc;
    for (int i = 0; i < 5; ++i)
        TSG_HIP(hipMemcpyAsync(d_out[i], dev_out[i], P * 4, hipMemcpyDeviceToHost, ctx->stream));
    TSG_HIP(hipStreamSynchronize(ctx->stream));
    return TS_OK;
}

int ts_is_estimate(ts_ctx *ctx, ts_code *code, const int32_t *ts_bits, int32_t a,
                   const ts_is_opts *o, ts_is_result *res, uint8_t *fail_out) {
    clear_error();
    if (!ctx || !code || !ts_bits || !o || !res) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    ctx->stats = ts_stats{};
    if (a < 1 || a > kMaxWidth) { set_error("TS size must be 1..%d", kMaxWidth); return TS_E_INVAL; }
    if (o->n_frames < 2 || o->n_frames > (1ll << 31) - 1) { set_error("n_frames must be 2..2^31-1"); return TS_E_INVAL; }
    if (o->max_iter < 1 || o->max_iter > kMaxIter) { set_error("max_iter must be 1..%d", kMaxIter); return TS_E_INVAL; }
    if (!(o->rate > 0.0 && o->rate <= 1.0)) { set_error("rate out of range"); return TS_E_INVAL; }
    std::vector<int32_t> t(ts_bits, ts_bits + a);
    std::sort(t.begin(), t.end());
    for (int i = 0; i < a; ++i)
        if (t[i] < 0 || t[i] >= code->n || (i && t[i] == t[i - 1])) {
            set_error("TS bits must be distinct variables of the code");
            return TS_E_INVAL;
        }
    double shift = o->shift;
    DBuf d_t(ctx, kMaxWidth * 4);
    if (!d_t.p) return TS_E_NOMEM;
    TSG_HIP(hipMemcpyAsync(d_t.p, t.data(), a * 4, hipMemcpyHostToDevice, ctx->stream));
    if (shift < 0.0) {
        // eps* of the noiseless SPA impulse on the whole set, grid 2^-10 up to 32
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
        DBuf outs(ctx, 5 * 4);
        if (!outs.p) return TS_E_NOMEM;
        int32_t *d_out[5];
        for (int i = 0; i < 5; ++i) d_out[i] = outs.as<int32_t>() + i;
        int rc = run_search(ctx, code, &so, d_t.as<int32_t>(), 1, a, d_out, false);
        if (rc) return rc;
        int32_t kc = 0;
        TSG_HIP(hipMemcpy(&kc, d_out[0], 4, hipMemcpyDeviceToHost));
        if (kc < 0) {
            set_error("the impulse on the whole set never fails; give a shift");
            return TS_E_INVAL;
        }
        shift = kc / 1024.0;
    }
    const int64_t K = o->n_frames;
    DBuf d_fail(ctx, (size_t)K), d_wf(ctx, (size_t)K * 8), d_misc(ctx, 64 * 4), d_red(ctx, 8 * 8);
    if (!d_fail.p || !d_wf.p || !d_misc.p || !d_red.p) { set_error("device allocation failed"); return TS_E_NOMEM; }
    int rc = launch_fill(ctx, d_misc.as<int>(), 0, 64);
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
    L.ts = d_t.as<int32_t>();
    L.a = a;
    L.fail = d_fail.as<unsigned char>();
    L.wf = d_wf.as<double>();
    L.queue = d_misc.as<int>();
    L.counters = (unsigned long long *)(d_misc.as<int>() + 4);
    int grid = 0, block = 0;
    TSG_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
    rc = launch_is(ctx, code, L, &grid, &block);
    if (rc) return rc;
    TSG_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
    rc = launch_is_reduce(ctx, L.wf, L.fail, K, 0, 0.0, d_red.as<double>());
    if (rc) return rc;
    double red[4];
    TSG_HIP(hipMemcpyAsync(red, d_red.p, 32, hipMemcpyDeviceToHost, ctx->stream));
    TSG_HIP(hipStreamSynchronize(ctx->stream));
    const double p = red[0] / (double)K;
    rc = launch_is_reduce(ctx, L.wf, L.fail, K, 1, p, d_red.as<double>());
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(red, d_red.p, 32, hipMemcpyDeviceToHost, ctx->stream));
    unsigned long long cnt[2];
    TSG_HIP(hipMemcpyAsync(cnt, d_misc.as<int>() + 4, 16, hipMemcpyDeviceToHost, ctx->stream));
    if (fail_out) TSG_HIP(hipMemcpyAsync(fail_out, d_fail.p, (size_t)K, hipMemcpyDeviceToHost, ctx->stream));
    TSG_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
    TSG_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.0f, tot = 0.0f;
    TSG_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    TSG_HIP(hipEventElapsedTime(&tot, ctx->ev[0], ctx->ev[2]));
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
    ctx->stats.decode_ms += ms;
    ctx->stats.total_ms += tot;
    ctx->stats.decodes += K;
    ctx->stats.edge_updates += (int64_t)cnt[1] * code->e;
    ctx->stats.decode_launches += 1;
    ctx->stats.block_threads = block;
    ctx->stats.grid_blocks = grid;
    return TS_OK;
}

int ts_collect(ts_ctx *ctx, const ts_code *code, ts_record *recs, int64_t cap, int64_t *n_out,
               int32_t *bits, int64_t bits_cap, int64_t *bits_out) {
    clear_error();
    if (!ctx || !code || !n_out || !bits_out) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    std::vector<int32_t> rh, bh;
    int rc = collect_table(ctx, code, rh, bh);
    if (rc) return rc;
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
