// Batched execution of several search and IS jobs, possibly on different codes.
//
// Every job is planned as if run alone (the code's autotuned shape, else the
// first that fits).  Jobs whose plans name the same kernel and workgroup size
// and whose frames fit the same number of times into a CU's LDS form a group
// (so every job runs at its own tuned shape); a group runs as ONE persistent
// launch whose workgroups pull items (patterns or IS frames) of all its jobs
// from a single queue, so small jobs fill the device together and no launch
// tail or host round trip separates them.  Groups go to the executor's side
// streams and overlap.  After one synchronisation the per-job candidate sieves
// and IS reductions run, each job with its own TS table, so every result is the
// one the job gives alone (a job whose candidate buffer overflows is re-run
// alone).  All device buffers of the batch come from a single allocation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "internal.h"

namespace tsg {

int plan_search_shape(ts_exec &ex, ts_code *code, const ts_search_opts *o, int64_t P, SearchPlan *plan);

namespace {

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct SItem {
    BatchJob *b;
    SearchPlan plan;
    int t0 = 0;
    int64_t P = 0, rec_cap = 0;
    size_t pat = 0, out = 0, recs = 0, misc = 0;   // arena offsets; misc in the zeroed area
    int group = -1;
    SearchLaunch a{};
};

struct IItem {
    BatchJob *b;
    SearchPlan plan;
    double shift = 0.0;
    int64_t K = 0;
    size_t ts = 0, fail = 0, wf = 0, red = 0, part = 0, misc = 0;
    int group = -1;
    IsLaunch L{};
};

struct Group {
    bool search = true;
    SearchPlan plan{};
    std::vector<int> members;
    size_t queue = 0, jobs = 0, scratch = 0, scratch_bytes = 0;
    long long n_items = 0;
    double work = 0.0;
};

int ensure_side(ts_exec &ex) {
    for (int i = 0; i < ts_exec::kSide; ++i) {
        if (!ex.side[i]) TSG_HIP(hipStreamCreateWithFlags(&ex.side[i], hipStreamNonBlocking));
        if (!ex.side_ev[i]) TSG_HIP(hipEventCreateWithFlags(&ex.side_ev[i], hipEventDisableTiming));
    }
    if (!ex.join_ev) TSG_HIP(hipEventCreateWithFlags(&ex.join_ev, hipEventDisableTiming));
    return TS_OK;
}

}  // namespace

int run_batch(ts_exec &ex, std::vector<BatchJob> &jobs) {
    ts_ctx *ctx = ex.ctx;
    hipStream_t s = ex.stream;
    int rc = ensure_side(ex);
    if (rc) return rc;
    rc = tune_for_batch(ex, jobs);
    if (rc) return rc;
    std::vector<SItem> S;
    std::vector<IItem> I;
    // ---- plan every job -------------------------------------------------
    for (BatchJob &b : jobs) {
        b.status = TS_OK;
        b.edge_updates = 0;
        if (b.kind == TS_JOB_SEARCH) {
            if (b.n_patterns == 0) {
                for (int i = 0; i < 5; ++i) b.out[i].clear();
                b.recs->clear();
                b.bits->clear();
                continue;
            }
            SItem it;
            it.b = &b;
            it.P = b.n_patterns;
            rc = plan_search_shape(ex, b.code, &b.so, it.P, &it.plan);
            if (rc) return rc;
            it.t0 = first_iter(b.code, &b.so);
            // the capacity a plain call gives the job (its worst case, up to
            // the context's record buffer), so that a batch re-runs no job
            // the plain call would not re-run
            it.rec_cap = rec_capacity(&b.so, it.t0, it.P, true, ex.ctx->rec_bytes, nullptr);
            S.push_back(it);
        } else {
            IItem it;
            it.b = &b;
            it.K = b.io.n_frames;
            it.shift = b.io.shift;
            rc = plan_is_shape(ex, b.code, b.io.max_iter, b.io.layout, &it.plan);
            if (rc) return rc;
            I.push_back(it);
        }
    }
    // eps* shifts before the batch: one search launch per (code, options),
    // one pattern per set
    {
        std::map<std::tuple<ts_code *, int, double, double, int>, std::vector<IItem *>> need;
        for (IItem &it : I)
            if (it.shift < 0.0)
                need[std::make_tuple(it.b->code, it.b->io.max_iter, it.b->io.ebn0_db, it.b->io.rate,
                                     it.b->io.layout)].push_back(&it);
        for (auto &kv : need) {
            std::vector<std::vector<int32_t>> sets;
            for (IItem *it : kv.second) sets.emplace_back(it->b->ts_bits, it->b->ts_bits + it->b->a);
            std::vector<double> sh(sets.size());
            rc = is_eps_shifts(ex, std::get<0>(kv.first), &kv.second.front()->b->io, sets, sh.data());
            if (rc) return rc;
            for (size_t j = 0; j < sets.size(); ++j) kv.second[j]->shift = sh[j];
        }
        // pilot-chosen shifts: one batch of pilots for all such jobs
        std::vector<PilotReq> req;
        for (IItem &it : I)
            if (it.b->io.shift < 0.0 && it.b->io.shift_rule == TS_SHIFT_PILOT)
                req.push_back(PilotReq{it.b->code, it.b->ts_bits, it.b->a, it.b->io, it.shift, &it.shift});
        if (!req.empty()) {
            rc = pilot_shifts(ex, req);
            if (rc) return rc;
        }
    }
    // ---- groups -----------------------------------------------------------
    std::vector<Group> G;
    std::map<std::tuple<int, int, int, int, int, int, int>, int> gid;
    auto group_of = [&](bool search, const SearchPlan &p) {
        // a group takes the largest LDS frame of its jobs: only jobs whose frames
        // fit the same number of times into a CU's LDS share one, so that no job
        // loses occupancy to a larger code's frame
        const int lds_fit = (int)(ctx->lds_per_block / std::max<size_t>(p.lds, 1));
        const auto key = std::make_tuple(search ? 1 : 0, p.kind, p.dc, p.cpt, p.decoder, p.block,
                                         lds_fit * 2 + p.save_lds);
        auto f = gid.find(key);
        if (f != gid.end()) {
            Group &g = G[f->second];
            g.plan.block = std::max(g.plan.block, p.block);
            g.plan.lds = std::max(g.plan.lds, p.lds);
            g.plan.slot_bytes = std::max(g.plan.slot_bytes, p.slot_bytes);
            return f->second;
        }
        Group g;
        g.search = search;
        g.plan = p;
        G.push_back(g);
        gid[key] = (int)G.size() - 1;
        return (int)G.size() - 1;
    };
    for (size_t i = 0; i < S.size(); ++i) {
        S[i].group = group_of(true, S[i].plan);
        Group &g = G[S[i].group];
        g.members.push_back((int)i);
        g.n_items += S[i].P;
        g.work += (double)S[i].P * S[i].b->code->e;
    }
    for (size_t i = 0; i < I.size(); ++i) {
        I[i].group = group_of(false, I[i].plan);
        Group &g = G[I[i].group];
        g.members.push_back((int)i);
        g.n_items += I[i].K;
        g.work += (double)I[i].K * I[i].b->code->e * 8.0;
    }
    for (Group &g : G) {
        if (g.n_items > INT_MAX) { set_error("too many items in one batch group"); return TS_E_INVAL; }
        rc = occupancy_grid(ctx, g.plan, g.plan.decoder, g.search, &g.plan.grid);
        if (rc) return rc;
        const long long grid = std::min<long long>(g.plan.grid, g.n_items);
        g.scratch_bytes = (size_t)grid * g.plan.slot_bytes;
    }
    // ---- one arena: zeroed counters first, then the buffers ---------------
    // per job 8 ints: [0] candidate count, [1] error flags, [4..7] two 64-bit
    // counters (decodes, iterations); per group one queue counter
    constexpr size_t kMisc = 32;
    size_t zero = 0;
    for (SItem &it : S) { it.misc = zero; zero += kMisc; }
    for (IItem &it : I) { it.misc = zero; zero += kMisc; }
    for (Group &g : G) { g.queue = zero; zero += kMisc; }
    size_t o = al(zero);
    // the search jobs' outputs and the IS jobs' reduction results each form
    // one block, read back with one copy
    const size_t out0 = o;
    for (SItem &it : S) { it.out = o; o += (size_t)it.P * 5 * 4; }
    const size_t out_bytes = o - out0;
    o = al(o);
    const size_t red0 = o;
    for (IItem &it : I) { it.red = o; o += 8 * 8; }
    const size_t red_bytes = o - red0;
    o = al(o);
    // the inputs (patterns, the sets' bits, job and reduction descriptors)
    // form one block, uploaded with one copy
    const size_t up0 = o;
    for (SItem &it : S) { it.pat = o; o = al(o + (size_t)it.P * it.b->width * 4); }
    for (IItem &it : I) { it.ts = o; o = al(o + kMaxWidth * 4); }
    for (Group &g : G) {
        g.jobs = o;
        o = al(o + g.members.size() * (g.search ? sizeof(SearchJob) : sizeof(IsJob)));
    }
    const size_t redj = o;
    o = al(o + I.size() * sizeof(RedJob));
    const size_t up_bytes = o - up0;
    for (SItem &it : S) { it.recs = o; o = al(o + (size_t)it.rec_cap * kRecStride * 4); }
    for (IItem &it : I) {
        it.fail = o; o = al(o + (size_t)it.K);
        it.wf = o; o = al(o + (size_t)it.K * 8);
        it.part = o; o = al(o + (size_t)is_reduce_parts(it.K) * 3 * 8);
    }
    for (Group &g : G) {
        g.scratch = o;
        o = al(o + g.scratch_bytes);
    }
    if (o == 0) return TS_OK;
    unsigned char *arena = (unsigned char *)ex.dalloc(o);
    if (!arena) { set_error("device allocation of %zu bytes for the batch failed", o); return TS_E_NOMEM; }
    // freed only once no launch of the batch can still use it (the side
    // streams run the IS groups while the main stream post-processes, and an
    // error may end the batch early)
    struct Free {
        ts_exec &ex;
        void *p;
        ~Free() {
            for (int i = 0; i < ts_exec::kSide; ++i)
                if (ex.side[i]) (void)hipStreamSynchronize(ex.side[i]);
            (void)hipStreamSynchronize(ex.stream);
            ex.dfree(p);
        }
    } arena_guard{ex, arena};
    rc = launch_fill(s, (int *)arena, 0, (int64_t)(zero / 4));
    if (rc) return rc;
    // ---- inputs and job descriptors: one image in pinned memory, one copy ---
    unsigned char *hu = nullptr;
    rc = ex.bulk_buf(up_bytes, &hu);
    if (rc) return rc;
    std::memset(hu, 0, up_bytes);
    for (SItem &it : S) {
        std::memcpy(hu + (it.pat - up0), it.b->patterns, (size_t)it.P * it.b->width * 4);
        SearchLaunch &a = it.a;
        fill_search_launch(it.b->code, &it.b->so, it.t0, it.b->width, &a);
        int32_t *out = (int32_t *)(arena + it.out);
        a.k_crit = out;
        a.iters_crit = out + it.P;
        a.iters_lo = out + 2 * it.P;
        a.tmin_crit = out + 3 * it.P;
        a.n_cand = out + 4 * it.P;
        a.patterns = (const int *)(arena + it.pat);
        a.n_patterns = (int)it.P;
        a.pat_base = 0;
        int *misc = (int *)(arena + it.misc);
        a.queue = nullptr;
        a.rec_count = misc;
        a.err = misc + 1;
        a.counters = (unsigned long long *)(misc + 4);
        a.recs = (int *)(arena + it.recs);
        a.rec_cap = (int)it.rec_cap;
        const Group &g = G[it.group];
        a.gscr = g.scratch_bytes ? arena + g.scratch : nullptr;
        a.slot_bytes = (long long)g.plan.slot_bytes;
        a.save_lds = g.plan.save_lds;
        a.hist_off = (long long)it.plan.hist_off;
    }
    int red_parts = 0;
    for (size_t ii = 0; ii < I.size(); ++ii) {
        IItem &it = I[ii];
        int32_t *t = (int32_t *)(hu + (it.ts - up0));
        std::copy(it.b->ts_bits, it.b->ts_bits + it.b->a, t);
        std::sort(t, t + it.b->a);
        IsLaunch &L = it.L;
        L.code = &it.b->code->dev;
        L.max_iter = it.b->io.max_iter;
        L.sigma2 = sigma2_of(it.b->io.ebn0_db, it.b->io.rate);
        L.shift = it.shift;
        L.n_frames = it.K;
        L.seed = it.b->io.seed;
        L.frame_base = it.b->io.frame_base;
        L.stream = it.b->io.stream;
        L.fp_exit = it.b->io.full_iterations ? 0 : 1;
        L.count_mode = it.b->io.count_mode;
        if (it.b->io.shift < 0.0 && it.b->io.shift_rule == TS_SHIFT_MIX) set_mixture(&L, it.shift);
        L.ts = (const int *)(arena + it.ts);
        L.a = it.b->a;
        L.fail = arena + it.fail;
        L.wf = (double *)(arena + it.wf);
        L.counters = (unsigned long long *)(arena + it.misc + 16);
        const Group &g = G[it.group];
        L.gscr = g.scratch_bytes ? arena + g.scratch : nullptr;
        RedJob rj = make_red_job(make_is_dev(L, it.plan), L.wf, L.fail, it.K, (double *)(arena + it.red),
                                 (double *)(arena + it.part));
        if (rj.np < 1) { set_error("empty IS reduction"); return TS_E_INVAL; }
        rj.part0 = red_parts;
        red_parts += rj.np;
        std::memcpy(hu + (redj - up0) + ii * sizeof(RedJob), &rj, sizeof(RedJob));
    }
    for (size_t gi = 0; gi < G.size(); ++gi) {
        Group &g = G[gi];
        unsigned char *hj = hu + (g.jobs - up0);
        long long item0 = 0;
        for (int m : g.members) {
            if (g.search) {
                SearchJob j{};
                j.a = S[m].a;
                j.cd = S[m].b->code->dev;
                j.item0 = item0;
                item0 += S[m].P;
                std::memcpy(hj, &j, sizeof(j));
                hj += sizeof(j);
            } else {
                IsJob j{};
                j.a = make_is_dev(I[m].L, I[m].plan);
                j.a.slot_bytes = (long long)g.plan.slot_bytes;
                j.cd = I[m].b->code->dev;
                j.item0 = item0;
                item0 += I[m].K;
                std::memcpy(hj, &j, sizeof(j));
                hj += sizeof(j);
            }
        }
    }
    TSG_HIP(hipMemcpyAsync(arena + up0, hu, up_bytes, hipMemcpyHostToDevice, s));
    TSG_HIP(hipStreamSynchronize(s));
    // ---- launches, spread over the side streams: the search groups first
    // (largest first), then the IS groups (largest first).  The main stream
    // waits for the search groups only, so the search jobs' sieves and
    // read-outs run while the IS groups still decode.
    std::vector<int> order(G.size());
    for (size_t i = 0; i < G.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        if (G[x].search != G[y].search) return G[x].search;
        return G[x].work > G[y].work;
    });
    TSG_HIP(hipEventRecord(ex.ev[0], s));
    TSG_HIP(hipEventRecord(ex.join_ev, s));
    // IS groups whose frames take more than half a CU's LDS (one workgroup per
    // CU) run one after another on the first side stream, the others one after
    // another on the second, so that small frames run beside the large ones
    // in the LDS and wave slots those leave free on every CU.  Two large
    // groups at once only share the CUs and contend for them: with the large
    // groups spread over two streams and the small ones over two more, the
    // 64-code batch took 0.67 s, with one stream each 0.62 s.
    int used = 0, n_search = 0;
    bool joined[ts_exec::kSide] = {};
    for (size_t k = 0; k < order.size(); ++k) {
        const Group &g = G[order[k]];
        int si;
        if (g.search) si = n_search++ % ts_exec::kSide;
        else si = g.plan.lds * 2 > ctx->lds_per_block ? 0 : 1;
        hipStream_t st = ex.side[si];
        if (!joined[si]) {
            TSG_HIP(hipStreamWaitEvent(st, ex.join_ev, 0));
            joined[si] = true;
        }
        int *queue = (int *)(arena + g.queue);
        if (g.search)
            rc = launch_search_jobs(st, g.plan, (const SearchJob *)(arena + g.jobs), (int)g.members.size(),
                                    queue, g.n_items);
        else
            rc = launch_is_jobs(st, g.plan, (const IsJob *)(arena + g.jobs), (int)g.members.size(), queue,
                                g.n_items);
        if (rc) return rc;
        used = std::max(used, si + 1);
        const bool last_search = g.search && (k + 1 == order.size() || !G[order[k + 1]].search);
        if (last_search) {   // the main stream waits for the search groups
            for (int i = 0; i < used; ++i) {
                if (!joined[i]) continue;
                TSG_HIP(hipEventRecord(ex.side_ev[i], ex.side[i]));
                TSG_HIP(hipStreamWaitEvent(s, ex.side_ev[i], 0));
            }
        }
    }
    std::vector<int> zh(zero / 4);
    if (zero) TSG_HIP(hipMemcpyAsync(zh.data(), arena, zero, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipStreamSynchronize(s));
    ex.stats.decode_launches += (int)G.size();
    // ---- per search job: sieve into its own table, read out -----------------
    std::vector<SItem *> rerun;
    std::vector<DevTable> tables(S.size());
    std::vector<char> done(S.size(), 0);   // outputs read back with the block below
    int64_t cands = 0;
    for (size_t i = 0; i < S.size(); ++i) {
        SItem &it = S[i];
        const int *misc = zh.data() + it.misc / 4;
        if (misc[1] & 1) {
            it.b->status = TS_E_INVAL;
            it.b->err = "pattern entry out of range";
            continue;
        }
        const int64_t nrec = misc[0];
        if (nrec > it.rec_cap) {   // re-run alone below; this run's work is not counted
            rerun.push_back(&it);
            continue;
        }
        unsigned long long cnt[2];
        std::memcpy(cnt, misc + 4, 16);
        it.b->edge_updates = (int64_t)cnt[1] * it.b->code->e;
        ex.stats.decodes += (int64_t)cnt[0];
        ex.stats.edge_updates += it.b->edge_updates;
        it.b->recs->clear();
        it.b->bits->clear();
        if (nrec > 0) {   // a table sized for the job's candidates (the read-out is sorted)
            int cap = 1024;
            while (cap < 4 * nrec && cap < (1 << 30)) cap <<= 1;
            rc = table_init(ex, tables[i], cap);
            if (rc) return rc;
            cands += nrec;
            rc = table_grow_if_needed(ex, tables[i], 2 * nrec);
            if (rc) return rc;
            rc = launch_sieve(ex, it.b->code->dev, tables[i], it.a, (int)nrec);
            if (rc) return rc;
            ex.stats.extract_launches++;
        }
        done[i] = 1;
    }
    ex.stats.candidates += cands;
    // every search job's outputs (the sieves add the candidate counts): one
    // copy into pinned memory
    if (out_bytes) {
        unsigned char *h = nullptr;
        rc = ex.bulk_buf(out_bytes, &h);
        if (rc) return rc;
        TSG_HIP(hipMemcpyAsync(h, arena + out0, out_bytes, hipMemcpyDeviceToHost, s));
        TSG_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < S.size(); ++i) {
            if (!done[i]) continue;
            SItem &it = S[i];
            for (int k = 0; k < 5; ++k) {
                it.b->out[k].resize((size_t)it.P);
                std::memcpy(it.b->out[k].data(), h + (it.out - out0) + (size_t)k * it.P * 4,
                            (size_t)it.P * 4);
            }
        }
    }
    // ---- TS read-out: every job's table at once -----------------------------
    {
        std::vector<const DevTable *> tp;
        std::vector<std::vector<int32_t> *> rp, bp;
        for (size_t i = 0; i < S.size(); ++i) {
            if (!tables[i].cap || S[i].b->status != TS_OK) continue;
            tp.push_back(&tables[i]);
            rp.push_back(S[i].b->recs);
            bp.push_back(S[i].b->bits);
        }
        rc = tp.empty() ? TS_OK : collect_tables(ex, (int)tp.size(), tp.data(), rp.data(), bp.data());
        for (DevTable &t : tables) table_free(ex, t);
        if (rc) return rc;
    }
    // ---- jobs whose candidates overflowed the batch buffer run alone ---------
    for (SItem *it : rerun) {
        int32_t *d_pat = (int32_t *)(arena + it->pat);
        int32_t *out = (int32_t *)(arena + it->out);
        int32_t *d_out[5] = {out, out + it->P, out + 2 * it->P, out + 3 * it->P, out + 4 * it->P};
        DevTable t{};
        ts_search_opts so = it->b->so;
        so.mem = TS_MEM_DEVICE;
        const int64_t eu0 = ex.stats.edge_updates;
        rc = run_search(ex, it->b->code, t, &so, d_pat, it->P, it->b->width, d_out, true);
        if (rc == TS_OK) {
            for (int k = 0; k < 5; ++k) {
                it->b->out[k].resize((size_t)it->P);
                TSG_HIP(hipMemcpyAsync(it->b->out[k].data(), d_out[k], (size_t)it->P * 4,
                                       hipMemcpyDeviceToHost, s));
            }
            TSG_HIP(hipStreamSynchronize(s));
            rc = collect_table(ex, t, *it->b->recs, *it->b->bits);
        }
        it->b->edge_updates = ex.stats.edge_updates - eu0;
        table_free(ex, t);
        if (rc) return rc;
    }
    // ---- the IS groups: wait for every side stream --------------------------
    for (int i = 0; i < used; ++i) {
        if (!joined[i]) continue;
        TSG_HIP(hipEventRecord(ex.side_ev[i], ex.side[i]));
        TSG_HIP(hipStreamWaitEvent(s, ex.side_ev[i], 0));
    }
    TSG_HIP(hipEventRecord(ex.ev[1], s));
    if (zero && !I.empty()) TSG_HIP(hipMemcpyAsync(zh.data(), arena, zero, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipStreamSynchronize(s));
    {
        float dec_ms = 0.0f;
        TSG_HIP(hipEventElapsedTime(&dec_ms, ex.ev[0], ex.ev[1]));
        ex.stats.decode_ms += dec_ms;
    }
    // ---- IS reductions: every job's two passes in two launches each ---------
    // (the reduction results of all IS jobs, 8 doubles apart: one copy)
    std::vector<double> red(I.size() * 4, 0.0);
    if (!I.empty()) {
        const RedJob *dj = (const RedJob *)(arena + redj);
        rc = launch_is_reduce_jobs(s, dj, (int)I.size(), red_parts, 0);
        if (rc) return rc;
        rc = launch_is_reduce_jobs(s, dj, (int)I.size(), red_parts, 1);
        if (rc) return rc;
        unsigned char *h = nullptr;
        rc = ex.bulk_buf(red_bytes, &h);
        if (rc) return rc;
        TSG_HIP(hipMemcpyAsync(h, arena + red0, red_bytes, hipMemcpyDeviceToHost, s));
        TSG_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < I.size(); ++i) std::memcpy(&red[4 * i], h + 64 * i, 32);
    }
    for (size_t i = 0; i < I.size(); ++i) {
        IItem &it = I[i];
        double r[4] = {red[4 * i], red[4 * i + 1], red[4 * i + 2], red[4 * i + 3]};
        is_fill_result(r, it.K, it.shift, it.b->is);
        const int *misc = zh.data() + it.misc / 4;
        unsigned long long cnt[2];
        std::memcpy(cnt, misc + 4, 16);
        it.b->edge_updates = (int64_t)cnt[1] * it.b->code->e;
        ex.stats.decodes += it.K;
        ex.stats.edge_updates += it.b->edge_updates;
    }
    TSG_HIP(hipStreamSynchronize(s));
    return TS_OK;
}

}  // namespace tsg
