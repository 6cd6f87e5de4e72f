// ts_is_estimate_noalloc: the importance-sampling estimate of one set without
// any device allocation, for callers that cannot allocate (code under HIP
// graph capture, serving loops that must not touch the allocator).  Every
// device buffer of the call lives in one file-scope device array, `scratch`,
// of kNoAllocScratchBytes, which each GPU holds until the process ends.
//
// Layout of the array (byte offsets; the caller's frame count K decides the
// sizes):
//   [0, 256)            queue and counters (cleared by a fill kernel per call)
//   [256, 320)          the set's sorted bits
//   [320, 384)          the two reduction results
//   [384, p)            reduction partials, 3 doubles per 16384 frames
//   [p, p + K)          per-frame flags
//   [.., .. + 8K)       per-frame sums of the set's normals
// (the register-layout decoder keeps all other state of a frame in LDS and
// registers, its fixed-point exit included)
// Calls on one GPU share the array: calls that overlap on a GPU race, so a
// caller serialises them (ts_ctx calls already are, by the context mutex; two
// contexts on one GPU are not).
#include <algorithm>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace tsg {
namespace {

constexpr size_t kNoAllocScratchBytes = 32ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on each device, from hipGetSymbolAddress (the
// array's name is a host-side stand-in, not a device address).
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Called by ts_create with the context's device current.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d beyond the %d devices the no-allocation scratch tracks", device, kMaxDevices);
        return TS_E_INVAL;
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return TS_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error("hipGetSymbolAddress of the no-allocation scratch failed: %s", hipGetErrorString(e));
        return TS_E_DEVICE;
    }
    g_ptr[device] = (unsigned char *)p;
    return TS_OK;
}

int64_t noalloc_max_frames() {
    // flags and sums (9 bytes a frame) and the partials
    return (int64_t)1 << 21;
}

}  // namespace tsg

using namespace tsg;

extern "C" int ts_is_estimate_noalloc(ts_ctx *ctx, ts_code *code, const int32_t *ts_bits, int32_t a,
                                      const ts_is_opts *o, ts_is_result *res, uint8_t *fail_out) {
    clear_error();
    if (!ctx || !code || !ts_bits || !o || !res) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    int rc = check_is_opts(code, ts_bits, a, o);
    if (rc) return rc;
    if (o->shift < 0.0) {
        set_error("the no-allocation estimate needs a given shift (shift >= 0)");
        return TS_E_INVAL;
    }
    const int64_t K = o->n_frames;
    if (K > noalloc_max_frames()) {
        set_error("n_frames %lld exceeds the no-allocation maximum of %lld", (long long)K,
                  (long long)noalloc_max_frames());
        return TS_E_INVAL;
    }
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_mu);
        base = ctx->device < kMaxDevices ? g_ptr[ctx->device] : nullptr;
    }
    if (!base) { set_error("no-allocation scratch not set up on device %d", ctx->device); return TS_E_STATE; }
    ts_exec &ex = ctx->main;
    hipStream_t s = ex.stream;
    SearchPlan plan;
    rc = plan_is_shape(ex, code, o->max_iter, o->layout, &plan);
    if (rc) return rc;
    if (plan.kind != kPlanRegister) {
        set_error("the no-allocation estimate runs the register layout only; this code's IS shape is "
                  "streamed (needs per-workgroup message slots)");
        return TS_E_INVAL;
    }
    // carve the array
    size_t off = 0;
    int *misc = (int *)(base + off);
    off += 256;
    int32_t *d_t = (int32_t *)(base + off);
    off += 64;
    double *d_red = (double *)(base + off);
    off += 64;
    double *d_part = (double *)(base + off);
    off = al256(off + (size_t)is_reduce_parts(K) * 3 * sizeof(double));
    unsigned char *d_fail = base + off;
    off = al256(off + (size_t)K);
    double *d_wf = (double *)(base + off);
    off = al256(off + (size_t)K * sizeof(double));
    const int grid = (int)std::min<int64_t>(plan.grid, K);
    if (off > kNoAllocScratchBytes) {   // unreachable with noalloc_max_frames()
        set_error("no-allocation scratch too small");
        return TS_E_INVAL;
    }
    int32_t t[kMaxWidth];
    std::copy(ts_bits, ts_bits + a, t);
    std::sort(t, t + a);
    std::memcpy(ex.pinned, t, (size_t)a * 4);
    TSG_HIP(hipMemcpyAsync(d_t, ex.pinned, (size_t)a * 4, hipMemcpyHostToDevice, s));
    rc = launch_fill(s, misc, 0, 64);   // queue and counters start at zero
    if (rc) return rc;
    IsLaunch L{};
    L.code = &code->dev;
    L.max_iter = o->max_iter;
    L.sigma2 = sigma2_of(o->ebn0_db, o->rate);
    L.shift = o->shift;
    L.n_frames = K;
    L.seed = o->seed;
    L.frame_base = o->frame_base;
    L.stream = o->stream;
    L.fp_exit = o->full_iterations ? 0 : 1;
    L.count_mode = o->count_mode;
    L.ts = d_t;
    L.a = a;
    L.fail = d_fail;
    L.wf = d_wf;
    L.counters = (unsigned long long *)(misc + 4);
    L.gscr = nullptr;
    IsJob job{};
    job.a = make_is_dev(L, plan);
    job.cd = code->dev;
    job.item0 = 0;
    void *dj = nullptr;
    int slot = -1;
    rc = ex.stage(&job, sizeof(job), &dj, &slot);
    if (rc) return rc;
    TSG_HIP(hipEventRecord(ex.ev[0], s));
    rc = launch_is_jobs(s, plan, (const IsJob *)dj, 1, misc, K);
    ex.staged(slot);
    if (rc) return rc;
    TSG_HIP(hipEventRecord(ex.ev[1], s));
    const RedJob rj = make_red_job(make_is_dev(L, plan), d_wf, d_fail, K, d_red, d_part);
    rc = launch_is_reduce(s, rj, 0);
    if (rc) return rc;
    rc = launch_is_reduce(s, rj, 1);
    if (rc) return rc;
    double red[4];
    TSG_HIP(hipMemcpyAsync(ex.pinned, d_red, 32, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipMemcpyAsync(ex.pinned + 8, misc + 4, 16, hipMemcpyDeviceToHost, s));
    if (fail_out) TSG_HIP(hipMemcpyAsync(fail_out, d_fail, (size_t)K, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipEventRecord(ex.ev[2], s));
    TSG_HIP(hipStreamSynchronize(s));
    std::memcpy(red, ex.pinned, 32);
    unsigned long long cnt[2];
    std::memcpy(cnt, ex.pinned + 8, 16);
    float ms = 0.0f, tot = 0.0f;
    TSG_HIP(hipEventElapsedTime(&ms, ex.ev[0], ex.ev[1]));
    TSG_HIP(hipEventElapsedTime(&tot, ex.ev[0], ex.ev[2]));
    is_fill_result(red, K, o->shift, res);
    ex.stats = ts_stats{};
    ex.stats.decode_ms = ms;
    ex.stats.total_ms = tot;
    ex.stats.decodes = K;
    ex.stats.edge_updates = (int64_t)cnt[1] * code->e;
    ex.stats.decode_launches = 1;
    ex.stats.block_threads = plan.block;
    ex.stats.grid_blocks = grid;
    ex.stats.layout = TS_LAYOUT_REGISTER;
    ex.stats.checks_per_thread = plan.cpt;
    return TS_OK;
}
