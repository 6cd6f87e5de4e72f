// Measurement aid, not part of the method: the LDS read bandwidth of the
// device, as the reference point for the decoders' LDS traffic.
#include "internal.h"

using namespace tsg;

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWords = 2048;        // 16-byte words of LDS per workgroup (32 KB)
constexpr int kProbeBlocksPerCu = 20;

// Each workgroup fills its LDS array, then every thread reads four 16-byte
// words per round; a wavefront's 64 lanes read 64 consecutive words (no bank
// conflicts) and the rounds walk the array.  A compiler memory barrier ends
// each round, so that no load is hoisted out of the loop or merged with the
// same address of another round (the addresses repeat every two rounds), and
// the sums are written out so that no load is dropped.
__global__ __launch_bounds__(kProbeThreads) void k_lds_probe(unsigned int *out, int rounds) {
    __shared__ uint4 buf[kProbeWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeWords; i += kProbeThreads)
        buf[i] = make_uint4(i, 3u * i + 1u, 5u * i + 2u, 7u * i + 3u);
    __syncthreads();
    unsigned int a = 0, b = 0, c = 0, d = 0;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint4 v = buf[(tid + (4 * r + u) * kProbeThreads) & (kProbeWords - 1)];
            a += v.x;
            b += v.y;
            c += v.z;
            d += v.w;
        }
        __asm__ __volatile__("" ::: "memory");
    }
    out[(size_t)blockIdx.x * kProbeThreads + tid] = a ^ b ^ c ^ d;
}

}  // namespace

extern "C" int ts_probe_lds(ts_ctx *ctx, double *bytes_per_s) {
    clear_error();
    if (!ctx || !bytes_per_s) { set_error("null argument"); return TS_E_INVAL; }
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    ts_exec &ex = ctx->main;
    int cus = 0;
    TSG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int grid = cus * kProbeBlocksPerCu, rounds = 1024;
    unsigned int *out = (unsigned int *)ex.dalloc((size_t)grid * kProbeThreads * sizeof(unsigned int));
    if (!out) { set_error("device allocation failed"); return TS_E_NOMEM; }
    double best = 0.0;
    for (int rep = 0; rep < 3; ++rep) {
        hipLaunchKernelGGL(k_lds_probe, dim3(grid), dim3(kProbeThreads), 0, ex.stream, out, rounds);
        TSG_HIP(hipEventRecord(ex.ev[0], ex.stream));
        hipLaunchKernelGGL(k_lds_probe, dim3(grid), dim3(kProbeThreads), 0, ex.stream, out, rounds);
        TSG_HIP(hipEventRecord(ex.ev[1], ex.stream));
        TSG_HIP(hipEventSynchronize(ex.ev[1]));
        float ms = 0.0f;
        TSG_HIP(hipEventElapsedTime(&ms, ex.ev[0], ex.ev[1]));
        const double bytes = (double)grid * kProbeThreads * rounds * 4 * 16.0;
        if (ms > 0.0f) best = std::max(best, bytes / (ms * 1e-3));
    }
    TSG_HIP(hipGetLastError());
    ex.dfree(out);
    *bytes_per_s = best;
    return TS_OK;
}
