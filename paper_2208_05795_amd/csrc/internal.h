// Internal declarations of the tsgpu library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "tsgpu.h"

namespace tsg {

void set_error(const char *fmt, ...);
void clear_error();

#define TSG_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::tsg::set_error("%s failed: %s", #expr, hipGetErrorString(e_));   \
            return TS_E_DEVICE;                                                \
        }                                                                      \
    } while (0)

// Limits of the device kernels (checked by the host before every launch).
constexpr int kMaxIter = 64;      // iterations per decode
constexpr int kMaxWidth = 16;     // impulse pattern width
constexpr int kMaxAmax = 16;      // largest TS kept
constexpr int kCapMax = 2 * kMaxAmax;  // |S u I| bound for sieving
constexpr int kDvMax = 8;         // variable degree bound of the sieve kernel
constexpr int kRecHdr = 8;        // candidate record header (ints)
constexpr int kRecStride = kRecHdr + kCapMax;

// Device-side description of a code, shared by all kernels.
struct DevCode {
    int n, m, e;
    int dv_max, dc_max;
    int z;                 // 0 = not QC
    const int *row_ptr;    // [m+1] check -> first edge (check-major edges)
    const int *col;        // [e]   variable of each edge
    const int *vptr;       // [n+1] variable -> first entry
    const int *vchk;       // [e]   checks of each variable, ascending
    const int *vedge;      // [e]   edge index of each (variable, check)
    const int *cn_tab;     // [dc_pad][m_tab] padded check neighbour table (-1 = pad)
    const int *vn_tab;     // [dv_pad][n_tab] padded variable -> edge table (-1 = pad)
    int dc_pad, m_tab, dv_pad, n_tab;
};

// Open-addressing TS table on the device, keyed by the canonical QC-orbit
// representative; the full key is compared on every hash match.
struct DevTable {
    unsigned long long *key;   // [cap] 0 = empty
    int *ready;                // [cap] 1 once the slot's key is written
    int *set;                  // [cap][kMaxAmax]
    int *ab;                   // [cap] a | b << 8
    int *orbit;                // [cap]
    int *first;                // [cap] smallest pattern index
    int *kcrit;                // [cap] smallest k*
    int *count;                // [1]   claimed slots
    int cap;                   // power of two
};

struct ts_code_impl;

}  // namespace tsg

struct ts_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *user = nullptr;
    size_t budget = 0;
    std::recursive_mutex mu;
    ts_stats stats{};
    hipEvent_t ev[6] = {};
    std::vector<ts_code *> codes;
    // reusable device scratch
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    int num_cu = 0;
    size_t lds_per_block = 0;
    // pinned host staging for small device -> host reads
    int *pinned = nullptr;

    void *dalloc(size_t bytes);
    void dfree(void *p);
};

struct ts_code {
    ts_ctx *ctx = nullptr;
    int n = 0, m = 0;
    int64_t e = 0;
    int girth = 0, z = 0, mb = 0, nb = 0, dv_max = 0, dc_max = 0;
    std::vector<int64_t> row_ptr;   // host copy, check-major
    std::vector<int32_t> col;
    std::vector<int64_t> vptr;
    std::vector<int32_t> vchk;
    std::vector<int32_t> vedge;
    // device copies
    tsg::DevCode dev{};
    std::vector<void *> dev_allocs;
    tsg::DevTable table{};
    bool table_alloc = false;
};

namespace tsg {

// loader.cpp
int build_code(const ts_code_desc *d, ts_code *c);
int upload_code(ts_ctx *ctx, ts_code *c);
int64_t make_patterns(const ts_code *c, int kind, int32_t *out, int64_t cap);

// table.cpp / ts_kernels.hip
int table_init(ts_ctx *ctx, ts_code *c, int cap);
int table_free(ts_ctx *ctx, ts_code *c);
int table_grow_if_needed(ts_ctx *ctx, ts_code *c, int64_t incoming);

// search (search_kernels.hip)
struct SearchPlan {
    int block;      // threads per workgroup
    int cpt;        // checks per thread
    int dc;         // padded check degree of the kernel
    int vpt;        // variables per thread (SPA)
    int dv;         // padded variable degree of the kernel (SPA)
    size_t lds;     // dynamic LDS bytes
    int grid;       // persistent workgroups
};

struct SearchLaunch {
    const DevCode *code;
    int decoder;
    int max_iter, offset, q_base, k_max, k_den;
    float h;
    int t0, cap, a_max, extract_mode;
    const int *patterns;   // device, chunk-relative rows
    int n_patterns, width, pat_base;
    int *k_crit, *iters_crit, *iters_lo, *tmin_crit, *n_cand;   // device, global index
    int *queue;
    int *recs;
    int rec_cap;
    int *rec_count;
    unsigned long long *counters;   // [0] decodes, [1] iterations
    int *err;
};

int plan_search(ts_ctx *ctx, const ts_code *c, int decoder, int max_iter, SearchPlan *plan);
int launch_search(ts_ctx *ctx, const SearchPlan &plan, const SearchLaunch &a);
int launch_sieve(ts_ctx *ctx, ts_code *c, const SearchLaunch &a, int n_waves_hint);
int launch_fill(ts_ctx *ctx, int *p, int value, int64_t count);

// collect
int collect_table(ts_ctx *ctx, const ts_code *c, std::vector<int32_t> &rec_host,
                  std::vector<int32_t> &bits_host);

// importance sampling (is_kernels.hip)
struct IsLaunch {
    const DevCode *code;
    int max_iter;
    double sigma2, shift;
    int64_t n_frames;
    unsigned long long seed, frame_base;
    unsigned stream;
    const int *ts; int a;
    unsigned char *fail;    // [n_frames]
    double *wf;             // [n_frames]
    int *queue;
    unsigned long long *counters;
};
int launch_is(ts_ctx *ctx, const ts_code *c, const IsLaunch &a, int *grid_out, int *block_out);
// mode 0: out[0..2] = sum w, sum w^2, failures; mode 1: out[3] = sum (w - mean)^2
int launch_is_reduce(ts_ctx *ctx, const double *wf, const unsigned char *fail, int64_t n, int mode,
                     double mean, double *out);

}  // namespace tsg
