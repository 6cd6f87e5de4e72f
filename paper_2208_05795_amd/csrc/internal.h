// Internal declarations of the tsgpu library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tsgpu.h"

namespace tsg {

void set_error(const char *fmt, ...);
void clear_error();
std::string last_error_copy();

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
constexpr int kMixMax = 32;       // components of an IS shift mixture
// The shift mixture of TS_SHIFT_MIX: eps* k/16, k = 0..16
constexpr int kMixPoints = 17;
constexpr double kMixF0 = 0.0, kMixDf = 0.0625;
constexpr int kMaxAmax = 16;      // largest TS kept
constexpr int kCapMax = 2 * kMaxAmax;  // |S u I| bound for sieving
constexpr int kDvMax = 8;         // variable degree bound of the sieve kernel
constexpr int kRecHdr = 8;        // candidate record header (ints)
constexpr int kRecStride = kRecHdr + kCapMax;
// Check-degree classes of the streamed-frame decoder: a check of degree d is
// padded to the smallest class >= d; checks are sorted by degree so each class
// is a contiguous range.  Codes of check degree above 24 use the classes
// without 24 (degrees 17..32 pad to 32).
constexpr int kGClasses[] = {3, 4, 6, 8, 12, 16, 24, 32};
constexpr int kQTabMaxBytes = 16 * 1024;   // LDS budget of the QC index tables
constexpr int kGMaxCls = 8;

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
    // streamed-frame layout: checks sorted by degree into classes; class q holds
    // positions [g_c0[q], g_c0[q+1]) with message slot g_off[q] + j*g_stride[q] + (p - g_c0[q])
    int g_ncls;
    int g_dc[kGMaxCls];
    int g_c0[kGMaxCls + 1];
    int g_stride[kGMaxCls];
    int g_off[kGMaxCls + 1];   // g_off[g_ncls] = total message slots
    const int *g_cn;       // [slots] variable of each message slot (n = padding)
    const int *g_vslot;    // [dv_pad][n_tab] message slot of each (variable, k) edge, -1 = pad
    // streamed layout of a QC code: the same indices computed from per-circulant
    // tables (qc_neighbour / qc_slot) instead of read from g_cn / g_vslot.  q_ok
    // is set only after the loader has checked every computed index against
    // those tables.  q_tab holds int pairs: [mb][q_dc] (j z or -1, shift) per
    // (block row, neighbour slot), then [nb][q_dv] (slot base or -1, shift) per
    // (block column, k-th check); q_rowpos[p] = (block row << 16) | row of the
    // check at sorted position p.
    int q_ok, q_dc, q_dv, q_bytes, q_var_off;   // q_var_off: ints before the column part
    float q_inv_z;
    const int *q_tab;
    const int *q_rowpos;
    // layered schedule: the checks ordered by layer (stable), so that a layer is a
    // contiguous range of positions; lay_of[p] = layer at position p
    // (non-decreasing), cn_lay[j][p] = cn_tab[j][check at p]; n_layers = 0 when
    // no schedule of at most 64 layers exists
    const int *lay_of;
    const int *cn_lay;     // [dc_pad][m_tab]
    int n_layers;
};

// LDS layout of a streamed frame (host and device).
struct LdsG {
    int np, W;
    size_t app, acc, imask, wsyn, pcnt, moved, cls, qtab, extra, total;
};

// qbytes: size of the QC index tables copied to LDS (0 = read g_cn / g_vslot);
// acc: the accumulating variant's second array of np sums
__host__ __device__ inline LdsG lds_layout_g(int n, int T, int qbytes, bool acc = false) {
    LdsG L;
    L.np = (n + 1 + 63) & ~63;
    L.W = L.np >> 6;
    size_t o = 0;
    L.app = o;
    o += (size_t)L.np * 4;
    L.acc = o;
    if (acc) o += (size_t)L.np * 4;
    o = (o + 15) & ~(size_t)15;
    L.imask = o;
    o += (size_t)L.W * 8;
    L.wsyn = o;
    o += (size_t)(T + 2) * 4;
    L.pcnt = o;
    o += (size_t)(T + 2) * 4;
    L.moved = o;   // per iteration: some check message changed
    o += (size_t)(T + 2) * 4;
    L.cls = o;   // class table: dc, c0, stride, off
    o += (size_t)(4 * kGMaxCls + 2) * 4;
    o = (o + 15) & ~(size_t)15;
    L.qtab = o;
    o += (size_t)qbytes;
    o = (o + 15) & ~(size_t)15;
    L.extra = o;
    o += (size_t)kMaxWidth * 8 + (size_t)kMaxWidth * 4;
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// Variable of neighbour slot j of check (i, r) of a QC code, from its table
// pair e = (j z, shift) of block row i (j z < 0: padding, returns n).
__host__ __device__ inline int qc_neighbour(const int *e, int r, int z, int n) {
    if (e[0] < 0) return n;
    int c = r + e[1];
    if (c >= z) c -= z;
    return e[0] + c;
}

// Message slot of the k-th edge of variable (j, c) of a QC code, from the pair
// e = (slot base, shift) of (block column j, k) (slot base < 0: padding, -1).
__host__ __device__ inline int qc_slot(const int *e, int c, int z) {
    if (e[0] < 0) return -1;
    int r = c - e[1];
    if (r < 0) r += z;
    return e[0] + r;
}

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
    int cap;                   // power of two, 0 = not allocated
};

// A decoder launch shape picked by the autotuner.
struct SearchShape {
    int kind = 0, cpt = 0, block = 0, save_lds = 0;
};

}  // namespace tsg

struct ts_code;

// One executor: a stream and the host/device state a call needs on it.  The
// context owns one for the synchronous calls; every serving worker owns one.
struct ts_exec {
    ts_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool stream_alloc = false;   // allocate with hipMallocAsync on this stream
    hipEvent_t ev[6] = {};
    int *pinned = nullptr;       // host staging for small device -> host reads
    ts_stats stats{};
    // job descriptors: a ring of pinned host slots copied to device slots; a
    // slot is reused once the event recorded after its launch has completed
    static constexpr int kJobSlots = 8;
    static constexpr size_t kJobSlotBytes = 64 * 1024;
    unsigned char *job_host = nullptr;
    unsigned char *job_dev = nullptr;
    hipEvent_t job_ev[kJobSlots] = {};
    bool job_used[kJobSlots] = {};
    int job_next = 0;
    // side streams (default priority) for the concurrent launches of a batch
    static constexpr int kSide = 4;
    hipStream_t side[kSide] = {};
    hipEvent_t side_ev[kSide] = {};
    hipEvent_t join_ev = nullptr;

    // pinned host buffer for bulk transfers (one copy instead of one per
    // array; pageable copies cost a host round trip each)
    unsigned char *bulk = nullptr;
    size_t bulk_cap = 0;

    void *dalloc(size_t bytes);
    void dfree(void *p);
    // a pinned host buffer of at least `bytes` (valid until the next call;
    // growing it first waits for this executor's stream)
    int bulk_buf(size_t bytes, unsigned char **p);
    // copies bytes (<= kJobSlotBytes) of job descriptors into a free slot; the
    // caller launches with *dev and then calls staged(slot)
    int stage(const void *src, size_t bytes, void **dev, int *slot);
    void staged(int slot);
};

// RAII device buffer from an executor
struct DBuf {
    ts_exec &ex;
    void *p = nullptr;
    DBuf(ts_exec &e, size_t bytes) : ex(e) { p = e.dalloc(bytes); }
    ~DBuf() { ex.dfree(p); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    template <class T> T *as() { return (T *)p; }
};

namespace tsg {
struct Server;
}

struct ts_ctx {
    int device = 0;
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *user = nullptr;
    size_t budget = 0;
    size_t rec_bytes = 256ull << 20;   // candidate record buffer of one search launch
    std::recursive_mutex mu;
    ts_exec main;
    std::vector<ts_code *> codes;
    int num_cu = 0;
    size_t lds_per_block = 0;
    std::atomic<tsg::Server *> server{nullptr};   // set once under mu, read without it
    hipMemPool_t pool = nullptr;   // the serving workers' stream-ordered device memory
    double t0 = 0.0;   // creation time (ms, steady clock)
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
    tsg::DevTable table{};          // the code's TS table (synchronous calls)
    // ordered read-out of the table, kept until a call may change the table
    uint64_t table_version = 0;
    mutable uint64_t readout_version = ~0ull;
    mutable std::vector<int32_t> readout_recs, readout_bits;
    std::atomic<int> jobs_in_flight{0};
    // launch shapes chosen by the autotuner, keyed by (decoder, max_iter)
    std::mutex tune_mu;
    std::unordered_map<int, tsg::SearchShape> tuned;
};

namespace tsg {

double now_ms();

// loader.cpp
int build_code(const ts_code_desc *d, ts_code *c);
int upload_code(ts_exec &ex, ts_code *c);
int64_t make_patterns(const ts_code *c, int kind, int32_t *out, int64_t cap);

// ts_kernels.hip
int table_init(ts_exec &ex, DevTable &t, int cap);
void table_free(ts_exec &ex, DevTable &t);
int table_grow_if_needed(ts_exec &ex, DevTable &t, int64_t incoming);
int collect_table(ts_exec &ex, const DevTable &t, std::vector<int32_t> &rec_host,
                  std::vector<int32_t> &bits_host);
// The same for nt tables at once (two synchronisations in all).
int collect_tables(ts_exec &ex, int nt, const DevTable *const *t, std::vector<int32_t> *const *rec_host,
                   std::vector<int32_t> *const *bits_host);
// The code's table in order (collect_table), read again only after a call that
// may have changed it.  Caller holds ctx->mu.
int table_readout(ts_ctx *ctx, const ts_code *code, const std::vector<int32_t> **recs,
                  const std::vector<int32_t> **bits);
size_t table_bytes(int cap);

// search (search_kernels.hip)
enum PlanKind { kPlanRegister = 0, kPlanStreamed = 1 };
struct SearchPlan {
    int kind;       // kPlanRegister: messages in registers; kPlanStreamed: in global memory
    int decoder;    // TS_DEC_* of the kernel (search plans)
    int block;      // threads per workgroup
    int cpt;        // checks per thread (register kind); streamed: 0 gathering, 1 accumulating
    int dc;         // padded check degree of the kernel (streamed: largest class)
    size_t lds;     // dynamic LDS bytes
    int grid;       // persistent workgroups
    size_t slot_bytes;   // global scratch per workgroup (register kind: the layered decoder's message save area)
    size_t hist_off;     // streamed: offset of the iteration history in a slot
    int save_lds = 0;    // register kind: the layered decoder's message save area in LDS (after the frame)
};

// Whether a plan is allowed under a TS_LAYOUT_* request (streamed plans carry
// their variant in cpt: 0 gathering, 1 accumulating).
inline bool layout_accepts(int layout, const SearchPlan &p) {
    switch (layout) {
        case TS_LAYOUT_REGISTER: return p.kind == kPlanRegister;
        case TS_LAYOUT_STREAMED: return p.kind == kPlanStreamed;
        case TS_LAYOUT_STREAMED_GATHER: return p.kind == kPlanStreamed && p.cpt == 0;
        case TS_LAYOUT_STREAMED_ACCUM: return p.kind == kPlanStreamed && p.cpt == 1;
        default: return true;
    }
}


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
    unsigned char *gscr;            // grid x slot_bytes scratch (nullptr: none)
    long long slot_bytes, hist_off;
    int fp_exit;                    // end decodes at a fixed point
    int save_lds;                   // register kind: the layered decoder's message save area in LDS
};

int plan_search(ts_ctx *ctx, const ts_code *c, int decoder, int max_iter, SearchPlan *plan);
int plan_candidates(ts_ctx *ctx, const ts_code *c, int decoder, int max_iter,
                    std::vector<SearchPlan> *out);
int launch_search(ts_exec &ex, const SearchPlan &plan, const SearchLaunch &a);
size_t streamed_slot_bytes(const ts_code *c, int decoder, int max_iter, bool search, size_t *hist_off);
int launch_sieve(ts_exec &ex, const DevCode &cd, const DevTable &t, const SearchLaunch &a,
                 int n_records);
int launch_fill(hipStream_t s, int *p, int value, int64_t count);

// Several jobs in one persistent launch: items (patterns or IS frames) of job j
// are the indices [item0, item0 + count) of the launch's queue.  Kernels copy the
// descriptor of the job they work on into LDS (kJobLds bytes at offset 0,
// followed by kShLds bytes of scratch words and then the frame).
struct SearchJob {
    SearchLaunch a;
    DevCode cd;
    long long item0;
};

struct IsDev {
    int max_iter;
    double sigma2, sigma, shift, wconst;   // wconst = -a s^2 / (2 sigma^2)
    long long n_frames;
    unsigned long long seed, frame_base;
    unsigned stream;
    const int *ts;
    int a;
    unsigned char *fail;
    double *wf;
    unsigned long long *counters;
    unsigned char *gscr;   // per-workgroup scratch (nullptr: none)
    long long slot_bytes, lam_off;
    int fp_exit;           // end decodes at a fixed point
    int count_mode;        // TS_IS_COUNT_ALL / TS_IS_COUNT_TS
    // mixture of shifts (n_mix > 0): frame f takes component j = f n_mix / n_frames,
    // shift mix_s0 + j mix_ds, and the balance-heuristic weight of all components
    int n_mix;
    double mix_s0, mix_ds;
};

struct IsJob {
    IsDev a;
    DevCode cd;
    long long item0;
};

constexpr size_t kJobLds = ((sizeof(SearchJob) > sizeof(IsJob) ? sizeof(SearchJob) : sizeof(IsJob)) + 15) & ~(size_t)15;
// Scratch words of the job header: 32 words, then (search kernels) a staging
// list and the per-pattern cache of candidate sets already recorded
// (kDedupSets entries: record index, size, amplitude index, spare, variables).
constexpr int kDedupSets = 2;
constexpr int kDedupStride = 4 + kCapMax;
constexpr size_t kShLds = (32 + kCapMax + kDedupSets * kDedupStride) * 4;
constexpr size_t kHdrLds = kJobLds + kShLds;

// importance sampling
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
    unsigned long long *counters;
    unsigned char *gscr;    // grid x slot_bytes scratch
    int fp_exit;            // end decodes at a fixed point
    int count_mode;         // TS_IS_COUNT_ALL / TS_IS_COUNT_TS
    int n_mix;              // 0: one shift; else the mixture of IsDev
    double mix_s0, mix_ds;
};
// IS launch shape (plan.slot_bytes of scratch per workgroup)
int plan_is(ts_ctx *ctx, const ts_code *c, int max_iter, int layout, SearchPlan *plan);
int plan_is_candidates(ts_ctx *ctx, const ts_code *c, int max_iter, int layout,
                       std::vector<SearchPlan> *out);
// the IS shape to use: the autotuner's earlier choice, else the first candidate
int plan_is_shape(ts_exec &ex, ts_code *code, int max_iter, int layout, SearchPlan *plan);
IsDev make_is_dev(const IsLaunch &a, const SearchPlan &plan);
// One persistent launch over the items of n_jobs device-resident jobs that share
// the plan's kernel and workgroup size (plan.lds and plan.grid cover them all).
int launch_search_jobs(hipStream_t s, const SearchPlan &plan, const SearchJob *d_jobs, int n_jobs,
                       int *queue, long long n_items);
int launch_is_jobs(hipStream_t s, const SearchPlan &plan, const IsJob *d_jobs, int n_jobs,
                   int *queue, long long n_items);
int occupancy_grid(ts_ctx *ctx, const SearchPlan &plan, int decoder, bool search, int *grid);
// Importance weights of a mixture of m shifts s0 + k ds (m = 0: one shift).
struct MixW {
    int m, a;
    long long n;
    double s0, ds, sigma;
};
// Reduction of the weights of the n IS frames of one job (wf: sums of the
// TS-bit normals, fail: per-frame flags).  mode 0: out[0..2] = sum w, sum w^2,
// counted failures; mode 1: out[3] = sum (w - mean)^2, mean = out[0] / n read
// on the device (after mode 0 on the same stream).  part: device scratch of
// 3 * is_reduce_parts(n) doubles.  In a launch over many jobs, job i takes
// the blocks from part0 on.
struct RedJob {
    const double *wf;
    const unsigned char *fail;
    long long n;
    double wconst, coef;
    MixW mix;
    int cmask, part0, np;
    double *part, *out;
};
int is_reduce_parts(int64_t n);
RedJob make_red_job(const IsDev &d, const double *wf, const unsigned char *fail, int64_t n, double *out,
                    double *part);
int launch_is_reduce(hipStream_t s, const RedJob &j, int mode);
// d_jobs: device array of nj jobs with part0 ascending from 0, total_parts
// blocks in all.
int launch_is_reduce_jobs(hipStream_t s, const RedJob *d_jobs, int nj, int total_parts, int mode);

// api.cpp: the work of one search / IS call on an executor
double sigma2_of(double ebn0_db, double rate);
int first_iter(const ts_code *code, const ts_search_opts *o);
int64_t rec_capacity(const ts_search_opts *o, int t0, int64_t P, bool sieve, size_t max_bytes,
                     int64_t *worst);
void fill_search_launch(const ts_code *code, const ts_search_opts *o, int t0, int32_t width,
                        SearchLaunch *a);
int is_eps_shifts(ts_exec &ex, ts_code *code, const ts_is_opts *o,
                  const std::vector<std::vector<int32_t>> &sets, double *shift);
int is_eps_shift(ts_exec &ex, ts_code *code, const int32_t *d_t, int32_t a, const ts_is_opts *o,
                 double *shift);
void is_fill_result(const double red[4], int64_t K, double shift, ts_is_result *res);
int check_search_opts(const ts_code *code, const ts_search_opts *o, int32_t width);
int run_search(ts_exec &ex, ts_code *code, DevTable &table, const ts_search_opts *o,
               const int32_t *d_pat, int64_t P, int32_t width, int32_t *const d_out[5], bool sieve);
int check_is_opts(const ts_code *code, const int32_t *ts_bits, int32_t a, const ts_is_opts *o);
int run_is(ts_exec &ex, ts_code *code, const int32_t *ts_bits, int32_t a, const ts_is_opts *o,
           ts_is_result *res, uint8_t *fail_out);
size_t search_bytes_estimate(const ts_code *code, const ts_search_opts *o, int64_t P, int32_t width);

// batch.cpp: several search / IS jobs run as one batch on an executor.  Jobs
// that share a kernel shape share one persistent launch; launches of different
// shapes run on the executor's side streams.  Results are those of each job
// run alone.
struct BatchJob {
    int kind = 0;                          // TS_JOB_SEARCH / TS_JOB_IS
    ts_code *code = nullptr;
    ts_search_opts so{};
    const int32_t *patterns = nullptr;     // host [n_patterns][width]
    int32_t n_patterns = 0, width = 0;
    ts_is_opts io{};
    const int32_t *ts_bits = nullptr;      // host [a]
    int32_t a = 0;
    // results
    std::vector<int32_t> *out = nullptr;   // [5] per-pattern outputs (search)
    std::vector<int32_t> *recs = nullptr, *bits = nullptr;
    ts_is_result *is = nullptr;
    int64_t edge_updates = 0;
    int status = TS_OK;
    std::string err;
};
int run_batch(ts_exec &ex, std::vector<BatchJob> &jobs);
// Pilot-chosen IS shifts (TS_SHIFT_PILOT) of several requests, one batch.
struct PilotReq {
    ts_code *code;
    const int32_t *bits;   // host [a]
    int32_t a;
    ts_is_opts io;         // the estimate's options
    double eps;            // eps* of the set (the grid's unit)
    double *shift;         // out
};
int pilot_shifts(ts_exec &ex, std::vector<PilotReq> &reqs);
// TS_SHIFT_MIX: the mixture around eps* on an IS launch
void set_mixture(IsLaunch *L, double eps);
int tune_for_batch(ts_exec &ex, std::vector<BatchJob> &jobs);   // api.cpp

// noalloc.hip: device address of the no-allocation scratch (once per device,
// with the device current)
int noalloc_init(int device);

// serve.cpp
struct Server;
void server_stop(ts_ctx *ctx);

}  // namespace tsg
