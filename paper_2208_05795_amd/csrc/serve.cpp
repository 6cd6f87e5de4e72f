// Serving: continuous batching of submitted trapping-set search and IS jobs.
//
// A pool of worker threads, each with its own executor (a default-priority HIP
// stream, stream-ordered device allocations, events and host staging), takes
// jobs from a FIFO queue.  A job is admitted as soon as a worker is free and its
// device-memory estimate fits in what the running jobs leave of the context's
// budget (first fit, so a small job can pass a large one that does not fit yet).
// Jobs that arrive while others run start on the next free worker; their
// kernels overlap on the device through the separate streams.  Each search job
// has its own TS table, so its result does not depend on what else is running.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace tsg {

int exec_create(ts_exec &ex, ts_ctx *ctx);
void exec_destroy(ts_exec &ex);

struct Job {
    uint64_t id = 0;
    int kind = 0;
    ts_code *code = nullptr;
    ts_search_opts so{};
    std::vector<int32_t> patterns;
    int32_t n_patterns = 0, width = 0;
    ts_is_opts io{};
    std::vector<int32_t> ts_bits;
    size_t est = 0;
    int state = TS_JOB_QUEUED;
    int status = TS_OK;
    bool cancel_req = false;
    std::string err;
    double t_submit = 0, t_start = 0, t_end = 0;
    int64_t edge_updates = 0;
    // results
    std::vector<int32_t> out[5];
    std::vector<int32_t> recs, bits;
    ts_is_result is{};
};

struct Server {
    ts_ctx *ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> queue;
    std::unordered_map<uint64_t, Job *> jobs;
    std::vector<std::thread> workers;
    std::vector<ts_exec *> execs;
    bool stop = false;
    size_t in_use = 0;
    size_t budget = 0;
    uint64_t next_id = 1;
};

namespace {

void run_jobs(ts_exec &ex, std::vector<Job *> &js);

int run_job(ts_exec &ex, Job *j) {
    ex.stats = ts_stats{};
    if (j->kind == TS_JOB_IS) {
        const int rc = run_is(ex, j->code, j->ts_bits.data(), (int32_t)j->ts_bits.size(), &j->io,
                              &j->is, nullptr);
        j->edge_updates = ex.stats.edge_updates;
        return rc;
    }
    const int64_t P = j->n_patterns;
    if (P == 0) return TS_OK;
    void *d_pat = ex.dalloc((size_t)P * j->width * 4);
    void *d_o = ex.dalloc((size_t)P * 5 * 4);
    if (!d_pat || !d_o) {
        ex.dfree(d_pat);
        ex.dfree(d_o);
        set_error("device allocation failed");
        return TS_E_NOMEM;
    }
    int rc = TS_OK;
    DevTable table{};
    int32_t *d_out[5];
    for (int i = 0; i < 5; ++i) d_out[i] = (int32_t *)d_o + i * P;
    if (hipMemcpyAsync(d_pat, j->patterns.data(), (size_t)P * j->width * 4, hipMemcpyHostToDevice,
                       ex.stream) != hipSuccess) {
        set_error("pattern upload failed");
        rc = TS_E_DEVICE;
    }
    ts_search_opts so = j->so;
    so.mem = TS_MEM_DEVICE;
    if (rc == TS_OK) rc = run_search(ex, j->code, table, &so, (int32_t *)d_pat, P, j->width, d_out, true);
    if (rc == TS_OK) {
        for (int i = 0; i < 5; ++i) {
            j->out[i].resize((size_t)P);
            if (hipMemcpyAsync(j->out[i].data(), d_out[i], (size_t)P * 4, hipMemcpyDeviceToHost,
                               ex.stream) != hipSuccess)
                rc = TS_E_DEVICE;
        }
        if (hipStreamSynchronize(ex.stream) != hipSuccess) rc = TS_E_DEVICE;
        if (rc == TS_OK) rc = collect_table(ex, table, j->recs, j->bits);
    }
    j->edge_updates = ex.stats.edge_updates;
    table_free(ex, table);
    ex.dfree(d_pat);
    ex.dfree(d_o);
    (void)hipStreamSynchronize(ex.stream);
    return rc;
}

// A worker takes the first queued job that fits in what the running batches
// leave of the budget, together with every further queued job that fits beside
// it (first fit, up to kMaxBatch), and runs them as one batch.  Jobs that arrive
// meanwhile go to the next free worker, whose batch overlaps on the device.
constexpr int kMaxBatch = 32;

void worker_main(Server *s, ts_exec *ex) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        std::vector<Job *> js;
        size_t est = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop) return;
                for (auto it = s->queue.begin(); it != s->queue.end() && (int)js.size() < kMaxBatch;) {
                    if (s->in_use + est + (*it)->est <= s->budget) {
                        est += (*it)->est;
                        js.push_back(*it);
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
                if (!js.empty()) break;
                s->cv_work.wait(lk);
            }
            s->in_use += est;
            const double t = now_ms();
            for (Job *j : js) {
                j->state = TS_JOB_RUNNING;
                j->t_start = t;
            }
        }
        run_jobs(*ex, js);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->in_use -= est;
            const double t = now_ms();
            for (Job *j : js) {
                j->t_end = t;
                j->code->jobs_in_flight--;
                if (j->cancel_req) {
                    j->state = TS_JOB_CANCELLED;
                    j->status = TS_E_CANCELLED;
                } else {
                    j->state = TS_JOB_DONE;
                }
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

int server_get(ts_ctx *ctx, int slots, Server **out) {
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (Server *cur = ctx->server.load()) {
        *out = cur;
        return TS_OK;
    }
    Server *s = new Server();
    s->ctx = ctx;
    size_t free_b = 0, total_b = 0;
    TSG_HIP(hipMemGetInfo(&free_b, &total_b));
    s->budget = ctx->budget ? ctx->budget : free_b / 2;
    for (int i = 0; i < slots; ++i) {
        ts_exec *ex = new ts_exec();
        const int rc = exec_create(*ex, ctx);
        if (rc) {
            exec_destroy(*ex);
            delete ex;
            for (ts_exec *e : s->execs) {
                exec_destroy(*e);
                delete e;
            }
            delete s;
            return rc;
        }
        s->execs.push_back(ex);
    }
    for (ts_exec *ex : s->execs) s->workers.emplace_back(worker_main, s, ex);
    ctx->server = s;
    *out = s;
    return TS_OK;
}

Job *find_job(Server *s, uint64_t id) {
    auto it = s->jobs.find(id);
    return it == s->jobs.end() ? nullptr : it->second;
}

// Validates a job description and copies its inputs.
int make_job(ts_ctx *ctx, const ts_job_desc *d, Job **out) {
    if (!d->code) { set_error("null code"); return TS_E_INVAL; }
    if (d->code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    Job *j = new Job();
    j->kind = d->kind;
    j->code = d->code;
    if (d->kind == TS_JOB_SEARCH) {
        int rc = check_search_opts(d->code, &d->search, d->width);
        if (rc) { delete j; return rc; }
        if (d->search.mem != TS_MEM_HOST) { delete j; set_error("submitted jobs take host arrays"); return TS_E_INVAL; }
        if (d->n_patterns < 0 || (d->n_patterns > 0 && !d->patterns)) { delete j; set_error("bad patterns"); return TS_E_INVAL; }
        const size_t cnt = (size_t)d->n_patterns * d->width;
        for (size_t i = 0; i < cnt; ++i)
            if (d->patterns[i] < -1 || d->patterns[i] >= d->code->n) {
                delete j;
                set_error("pattern entry %d out of range", d->patterns[i]);
                return TS_E_INVAL;
            }
        j->so = d->search;
        j->patterns.assign(d->patterns, d->patterns + cnt);
        j->n_patterns = d->n_patterns;
        j->width = d->width;
        j->est = search_bytes_estimate(d->code, &d->search, d->n_patterns, d->width) * 5 / 4;
    } else if (d->kind == TS_JOB_IS) {
        int rc = check_is_opts(d->code, d->ts_bits, d->a, &d->is);
        if (rc) { delete j; return rc; }
        j->io = d->is;
        j->ts_bits.assign(d->ts_bits, d->ts_bits + d->a);
        j->est = (size_t)d->is.n_frames * 9 + (1 << 20);
        std::vector<SearchPlan> ips;   // scratch of the largest shape the autotuner may try
        size_t scr = 0;
        if (plan_is_candidates(ctx, d->code, d->is.max_iter, d->is.layout, &ips) == TS_OK)
            for (const SearchPlan &ip : ips)
                scr = std::max(scr, (size_t)std::min<int64_t>(ip.grid, d->is.n_frames) * ip.slot_bytes);
        j->est += scr;
    } else {
        delete j;
        set_error("unknown job kind %d", d->kind);
        return TS_E_INVAL;
    }
    *out = j;
    return TS_OK;
}

BatchJob batch_view(Job *j) {
    BatchJob b;
    b.kind = j->kind;
    b.code = j->code;
    b.so = j->so;
    b.patterns = j->patterns.data();
    b.n_patterns = j->n_patterns;
    b.width = j->width;
    b.io = j->io;
    b.ts_bits = j->ts_bits.data();
    b.a = (int32_t)j->ts_bits.size();
    b.out = j->out;
    b.recs = &j->recs;
    b.bits = &j->bits;
    b.is = &j->is;
    return b;
}

// Runs jobs as one batch; each job's status and results are filled in.
void run_jobs(ts_exec &ex, std::vector<Job *> &js) {
    if (js.size() == 1) {
        clear_error();
        const int rc = run_job(ex, js[0]);
        js[0]->status = rc;
        if (rc != TS_OK) js[0]->err = last_error_copy();
        return;
    }
    std::vector<BatchJob> v;
    for (Job *j : js) v.push_back(batch_view(j));
    ex.stats = ts_stats{};
    clear_error();
    const int rc = run_batch(ex, v);
    const std::string err = rc != TS_OK ? last_error_copy() : std::string();
    for (size_t i = 0; i < js.size(); ++i) {
        js[i]->edge_updates = v[i].edge_updates;
        js[i]->status = rc != TS_OK ? rc : v[i].status;
        js[i]->err = rc != TS_OK ? err : v[i].err;
    }
}

}  // namespace

void server_stop(ts_ctx *ctx) {
    Server *s = ctx->server.load();
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Job *j : s->queue) {
            j->state = TS_JOB_CANCELLED;
            j->status = TS_E_CANCELLED;
            j->code->jobs_in_flight--;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();   // running jobs finish first
    for (ts_exec *e : s->execs) {
        exec_destroy(*e);
        delete e;
    }
    for (auto &kv : s->jobs) delete kv.second;
    delete s;
    ctx->server = nullptr;
}

}  // namespace tsg

using namespace tsg;

extern "C" {

int ts_serve_start(ts_ctx *ctx, int32_t slots) {
    clear_error();
    if (!ctx) { set_error("null argument"); return TS_E_INVAL; }
    if (slots < 1 || slots > 16) { set_error("slots must be 1..16"); return TS_E_INVAL; }
    if (ctx->server.load()) { set_error("serving already started"); return TS_E_STATE; }
    Server *s = nullptr;
    return server_get(ctx, slots, &s);
}

int ts_submit(ts_ctx *ctx, const ts_job_desc *d, uint64_t *job_id) {
    clear_error();
    if (!ctx || !d || !job_id) { set_error("null argument"); return TS_E_INVAL; }
    Job *j = nullptr;
    int rc0 = make_job(ctx, d, &j);
    if (rc0) return rc0;
    Server *s = nullptr;
    int rc = server_get(ctx, 4, &s);
    if (rc) { delete j; return rc; }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (j->est > s->budget) {
            set_error("job needs about %zu bytes, above the serving budget %zu", j->est, s->budget);
            delete j;
            return TS_E_BUSY;
        }
        j->id = s->next_id++;
        j->t_submit = now_ms();
        j->code->jobs_in_flight++;
        s->jobs[j->id] = j;
        s->queue.push_back(j);
        *job_id = j->id;
    }
    s->cv_work.notify_one();
    return TS_OK;
}

int ts_run_batch(ts_ctx *ctx, const ts_job_desc *jobs, int32_t n_jobs, uint64_t *job_ids) {
    clear_error();
    if (!ctx || n_jobs < 0 || (n_jobs > 0 && (!jobs || !job_ids))) { set_error("bad arguments"); return TS_E_INVAL; }
    if (n_jobs > 4096) { set_error("at most 4096 jobs per batch"); return TS_E_INVAL; }
    std::vector<Job *> js;
    for (int32_t i = 0; i < n_jobs; ++i) {
        Job *j = nullptr;
        const int rc = make_job(ctx, &jobs[i], &j);
        if (rc) {
            for (Job *q : js) delete q;
            return rc;
        }
        js.push_back(j);
    }
    Server *s = nullptr;
    int rc = server_get(ctx, 4, &s);
    if (rc) {
        for (Job *q : js) delete q;
        return rc;
    }
    const double t0 = now_ms();
    {
        std::lock_guard<std::recursive_mutex> g(ctx->mu);
        for (Job *j : js) {
            j->t_submit = j->t_start = t0;
            j->state = TS_JOB_RUNNING;
        }
        if (!js.empty()) run_jobs(ctx->main, js);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const double t1 = now_ms();
        for (int32_t i = 0; i < n_jobs; ++i) {
            Job *j = js[i];
            j->t_end = t1;
            j->state = TS_JOB_DONE;
            j->id = s->next_id++;
            s->jobs[j->id] = j;
            job_ids[i] = j->id;
        }
    }
    s->cv_done.notify_all();
    return TS_OK;
}

int ts_poll(ts_ctx *ctx, uint64_t job_id, int32_t wait, ts_job_info *info) {
    clear_error();
    if (!ctx || !info) { set_error("null argument"); return TS_E_INVAL; }
    Server *s = ctx->server.load();
    if (!s) { set_error("no job was submitted"); return TS_E_STATE; }
    std::unique_lock<std::mutex> lk(s->mu);
    Job *j = find_job(s, job_id);
    if (!j) { set_error("unknown job %llu", (unsigned long long)job_id); return TS_E_INVAL; }
    if (wait)
        s->cv_done.wait(lk, [&] { return j->state == TS_JOB_DONE || j->state == TS_JOB_CANCELLED; });
    std::memset(info, 0, sizeof(*info));
    info->state = j->state;
    info->status = j->status;
    info->submit_ms = j->t_submit - ctx->t0;
    info->start_ms = j->t_start > 0 ? j->t_start - ctx->t0 : 0;
    info->end_ms = j->t_end > 0 ? j->t_end - ctx->t0 : 0;
    info->edge_updates = j->edge_updates;
    info->device_bytes = (int64_t)j->est;
    info->n_ts = (int64_t)j->recs.size() / 5;
    info->n_bits = (int64_t)j->bits.size();
    info->n_patterns = j->n_patterns;
    info->is = j->is;
    if (j->state == TS_JOB_DONE && j->status != TS_OK) set_error("%s", j->err.c_str());
    return TS_OK;
}

int ts_job_outputs(ts_ctx *ctx, uint64_t job_id, ts_search_out *out, ts_record *recs, int64_t cap,
                   int32_t *bits, int64_t bits_cap) {
    clear_error();
    if (!ctx) { set_error("null argument"); return TS_E_INVAL; }
    Server *s = ctx->server.load();
    if (!s) { set_error("no job was submitted"); return TS_E_STATE; }
    std::lock_guard<std::mutex> lk(s->mu);
    Job *j = find_job(s, job_id);
    if (!j) { set_error("unknown job %llu", (unsigned long long)job_id); return TS_E_INVAL; }
    if (j->state != TS_JOB_DONE || j->status != TS_OK) { set_error("job has no results"); return TS_E_STATE; }
    if (j->kind != TS_JOB_SEARCH) { set_error("IS jobs report through ts_poll"); return TS_E_INVAL; }
    if (out) {
        int32_t *dst[5] = {out->k_crit, out->iters_crit, out->iters_lo, out->tmin_crit, out->n_cand};
        for (int i = 0; i < 5; ++i)
            if (dst[i]) std::memcpy(dst[i], j->out[i].data(), j->out[i].size() * 4);
    }
    const int64_t n = (int64_t)j->recs.size() / 5;
    if (cap > 0 || bits_cap > 0) {
        if (cap < n || bits_cap < (int64_t)j->bits.size()) { set_error("output buffers too small"); return TS_E_TRUNC; }
        if ((n > 0 && !recs) || (!j->bits.empty() && !bits)) { set_error("null output buffer"); return TS_E_INVAL; }
        int64_t off = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *r = j->recs.data() + i * 5;
            recs[i].a = r[0];
            recs[i].b = r[1];
            recs[i].orbit = r[2];
            recs[i].first_pattern = r[3];
            recs[i].k_crit = r[4];
            recs[i].reserved = 0;
            recs[i].bits_off = off;
            off += r[0];
        }
        if (!j->bits.empty()) std::memcpy(bits, j->bits.data(), j->bits.size() * 4);
    }
    return TS_OK;
}

int ts_cancel(ts_ctx *ctx, uint64_t job_id) {
    clear_error();
    if (!ctx) { set_error("null argument"); return TS_E_INVAL; }
    Server *s = ctx->server.load();
    if (!s) { set_error("no job was submitted"); return TS_E_STATE; }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        Job *j = find_job(s, job_id);
        if (!j) { set_error("unknown job %llu", (unsigned long long)job_id); return TS_E_INVAL; }
        if (j->state == TS_JOB_QUEUED) {
            s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), j), s->queue.end());
            j->state = TS_JOB_CANCELLED;
            j->status = TS_E_CANCELLED;
            j->code->jobs_in_flight--;
        } else if (j->state == TS_JOB_RUNNING) {
            j->cancel_req = true;   // its results are dropped when it finishes
        }
    }
    s->cv_done.notify_all();
    return TS_OK;
}

int ts_release(ts_ctx *ctx, uint64_t job_id) {
    clear_error();
    if (!ctx) { set_error("null argument"); return TS_E_INVAL; }
    Server *s = ctx->server.load();
    if (!s) { set_error("no job was submitted"); return TS_E_STATE; }
    std::lock_guard<std::mutex> lk(s->mu);
    Job *j = find_job(s, job_id);
    if (!j) { set_error("unknown job %llu", (unsigned long long)job_id); return TS_E_INVAL; }
    if (j->state == TS_JOB_QUEUED || j->state == TS_JOB_RUNNING) { set_error("job still in flight"); return TS_E_BUSY; }
    s->jobs.erase(job_id);
    delete j;
    return TS_OK;
}

}  // extern "C"
