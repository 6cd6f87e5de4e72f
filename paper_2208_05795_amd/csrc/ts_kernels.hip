// Trapping-set sieve, canonicalisation and deduplication (Section III), and the
// ordered read-out of the TS table.
//
// One wavefront handles one candidate record U = S(x_t) u I (|U| <= 2 a_max):
//   S1 = Tree(U), S2 = Tree(TS(U)), and every nonempty result with a <= a_max
//   gets its b (odd-degree checks of the induced subgraph), its canonical QC
//   representative and orbit size, and is inserted into the device table.
// Tree(V) is the variable set of the 2-core of G[V] (peeling variables with
// fewer than two checks shared with another surviving variable); TS(V) adds
// every outside variable having two checks in one connected component of G[V].
//
// Every variable TS(U) adds closes a cycle with U inside G[TS(U)], and the
// variables of a cycle survive the 2-core peeling; hence |S2| >= |TS(U) \ U|,
// and when more than a_max variables are added S2 cannot be kept and is not
// built.  That bounds every set handled here by 2 a_max + a_max variables.
//
// Canonical form: the lexicographically smallest sorted image of the set under
// the QC shifts v = j z + c -> j z + (c + t) mod z.  The smallest image maps an
// element of the lowest block column to position 0, so only those shifts are
// tried; the number of shifts reaching it is the stabiliser size, and the orbit
// size is z over it.
//
// Table: open addressing on a 64-bit hash of (a, tuple) with the full tuple
// compared on every hash match; the slot owner publishes the tuple with a
// release store, readers acquire before comparing.
#include <climits>
#include <cstring>

#include "internal.h"
#include "wave.h"

namespace tsg {
namespace {

constexpr int kSetMax = kCapMax + kMaxAmax;
constexpr int kWaves = 4;          // wavefronts per workgroup of the sieve kernel
constexpr int kWtab = 128;         // LDS hash slots for the TS(U) additions
constexpr int kHtab = 512;         // LDS check map (more slots than a set has incidences)
static_assert(kHtab > kSetMax * kDvMax, "the check map must hold every incidence");

struct WaveLds {
    int U[kCapMax];
    int X[kSetMax];
    int alive[kSetMax];
    int inc[kSetMax * kDvMax];
    int isl[kSetMax * kDvMax];   // check-map slot of each incidence's check
    int comp[kCapMax];
    int hkey[kHtab];             // check map: check id (-1 = empty) ...
    int hval[kHtab];             // ... and its count (Tree) or component (TS)
    int wtab[kWtab];
    int wlist[kWtab];
    int S[kSetMax];
    int cand[kMaxAmax];
    int best[kMaxAmax];
    int misc[4];
};

struct SieveArgs {
    DevCode cd;
    DevTable tab;
    const int *recs;
    const int *rec_count;
    int rec_cap;
    const int *k_crit;
    int *n_cand;
    int a_max, extract_mode;
    int *err;
};

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__device__ unsigned long long set_hash(const int *key, int a) {
    unsigned long long h = 0x6a09e667f3bcc909ull ^ (unsigned long long)a;
    for (int i = 0; i < a; ++i) h = mix64(h + (unsigned)key[i] + 0x9e3779b97f4a7c15ull);
    return h ? h : 1ull;
}

// Per-wave check map in LDS (open addressing; it never holds more checks than
// it has slots, so probes end).
__device__ __forceinline__ unsigned check_hash(int c) { return ((unsigned)c * 2654435761u) >> 23; }

__device__ void check_map_clear(WaveLds &w) {
    for (int i = lane_id(); i < kHtab; i += 64) w.hkey[i] = -1;
}

// slot of check c, inserted if absent (lanes may insert concurrently)
__device__ int check_map_slot(WaveLds &w, int c) {
    unsigned s = check_hash(c);
    for (;;) {
        const int old = atomicCAS(&w.hkey[s], -1, c);
        if (old == -1 || old == c) return (int)s;
        s = (s + 1) & (kHtab - 1);
    }
}

// slot of check c, or -1 (no concurrent inserts)
__device__ int check_map_find(const WaveLds &w, int c) {
    unsigned s = check_hash(c);
    for (int p = 0; p < kHtab; ++p) {
        const int k = w.hkey[s];
        if (k == c) return (int)s;
        if (k == -1) return -1;
        s = (s + 1) & (kHtab - 1);
    }
    return -1;
}

// Builds the incidence list of X[0..k) (check of each variable/degree slot).
__device__ void build_incidences(const DevCode &cd, WaveLds &w, int k) {
    const int dv = cd.dv_max;
    for (int idx = lane_id(); idx < k * dv; idx += 64) {
        const int i = idx / dv, d = idx - i * dv;
        const int v = w.X[i];
        const int lo = cd.vptr[v], deg = cd.vptr[v + 1] - lo;
        w.inc[idx] = d < deg ? cd.vchk[lo + d] : -1;
    }
    wave_sync();
}

// Tree(X[0..k)): survivors written sorted to out, returns their number; *b gets
// the number of odd-degree checks of the survivors' induced subgraph.  Each
// peeling round counts, per check, its surviving variables in the check map,
// then drops every variable with fewer than two checks counted twice or more.
__device__ int wave_tree(const DevCode &cd, WaveLds &w, int k, int *out, int *b) {
    const int lane = lane_id(), dv = cd.dv_max, L = k * dv;
    build_incidences(cd, w, k);
    check_map_clear(w);
    if (lane < k) w.alive[lane] = 1;
    wave_sync();
    for (int idx = lane; idx < L; idx += 64) w.isl[idx] = w.inc[idx] >= 0 ? check_map_slot(w, w.inc[idx]) : -1;
    wave_sync();
    for (;;) {
        for (int i = lane; i < kHtab; i += 64) w.hval[i] = 0;
        wave_sync();
        for (int idx = lane; idx < L; idx += 64)
            if (w.isl[idx] >= 0 && w.alive[idx / dv]) atomicAdd(&w.hval[w.isl[idx]], 1);
        wave_sync();
        int drop = 0;
        if (lane < k && w.alive[lane]) {
            int strong = 0;
            for (int d = 0; d < dv; ++d) {
                const int sl = w.isl[lane * dv + d];
                strong += sl >= 0 && w.hval[sl] >= 2;
            }
            drop = strong < 2;
        }
        if (!__any(drop)) break;
        if (drop) w.alive[lane] = 0;
        wave_sync();
    }
    const int keep = lane < k ? w.alive[lane] : 0;
    const unsigned long long mask = __ballot(keep);
    if (keep) out[__popcll(mask & ((1ull << lane) - 1ull))] = w.X[lane];
    // the final counts are those of the survivors: odd ones are the odd checks
    int odd = 0;
    for (int i = lane; i < kHtab; i += 64) odd += w.hkey[i] >= 0 && (w.hval[i] & 1);
    *b = wave_sum(odd);
    wave_sync();
    return __popcll(mask);
}

// TS(U) \ U into w.wlist; returns its size, or a_max + 1 as soon as it exceeds a_max.
__device__ int wave_ts_additions(const DevCode &cd, WaveLds &w, int u, int a_max) {
    const int lane = lane_id(), dv = cd.dv_max, L = u * dv;
    for (int i = 0; i < u; i += 64)
        if (i + lane < u) w.X[i + lane] = w.U[i + lane];
    wave_sync();
    build_incidences(cd, w, u);
    // components of G[U] by label propagation over shared checks
    unsigned adj = 0;
    if (lane < u)
        for (int j = 0; j < u; ++j) {
            if (j == lane) continue;
            bool share = false;
            for (int d = 0; d < dv && !share; ++d) {
                const int c = w.inc[lane * dv + d];
                if (c < 0) continue;
                for (int d2 = 0; d2 < dv; ++d2)
                    if (w.inc[j * dv + d2] == c) { share = true; break; }
            }
            if (share) adj |= 1u << j;
        }
    int comp = lane;
    for (;;) {
        int nc = comp;
        for (int j = 0; j < u; ++j) {
            const int cj = __shfl(comp, j, 64);
            if ((adj >> j) & 1u) nc = min(nc, cj);
        }
        const int changed = nc != comp;
        comp = nc;
        if (!__any(changed)) break;
    }
    if (lane < u) w.comp[lane] = comp;
    for (int i = lane; i < kWtab; i += 64) w.wtab[i] = -1;
    check_map_clear(w);
    if (lane == 0) w.misc[0] = 0;
    wave_sync();
    // check map: every check of U -> its component (U variables that share a
    // check are in one component, so concurrent writers agree)
    for (int idx = lane; idx < L; idx += 64) {
        const int c = w.inc[idx];
        if (c >= 0) w.hval[check_map_slot(w, c)] = w.comp[idx / dv];
    }
    wave_sync();
    // every (incidence, neighbour) pair: dcp lanes per incidence, 64 / dcp
    // incidences per round
    const int dcp = cd.dc_max <= 8 ? 8 : (cd.dc_max <= 16 ? 16 : (cd.dc_max <= 32 ? 32 : 64));
    for (int base = 0; base < L; base += 64 / dcp) {
        const int idx = base + lane / dcp, q = lane & (dcp - 1);
        const int c = idx < L ? w.inc[idx] : -1;
        int v = -1;
        if (c >= 0) {
            const int r0 = cd.row_ptr[c], deg = cd.row_ptr[c + 1] - r0;
            if (q < deg) v = cd.col[r0 + q];
        }
        if (v >= 0) {
            int lo = 0, hi = u;   // binary search in the sorted U
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (w.U[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            if (lo < u && w.U[lo] == v) v = -1;
        }
        bool hit = false;
        if (v >= 0) {
            int comps[kDvMax];
            const int vlo = cd.vptr[v], vdeg = cd.vptr[v + 1] - vlo;
            for (int d = 0; d < vdeg && !hit; ++d) {
                const int sl = check_map_find(w, cd.vchk[vlo + d]);
                const int cp = sl >= 0 ? w.hval[sl] : -1;
                comps[d] = cp;
                if (cp >= 0)
                    for (int d2 = 0; d2 < d; ++d2)
                        if (comps[d2] == cp) { hit = true; break; }
            }
        }
        if (hit) {
            unsigned slot = ((unsigned)v * 2654435761u) & (kWtab - 1);
            for (int p = 0; p < kWtab; ++p) {
                const int old = atomicCAS(&w.wtab[slot], -1, v);
                if (old == -1) {
                    const int pos = atomicAdd(&w.misc[0], 1);
                    if (pos < kWtab) w.wlist[pos] = v;
                    break;
                }
                if (old == v) break;
                slot = (slot + 1) & (kWtab - 1);
            }
        }
        wave_sync();
        if (w.misc[0] > a_max) return a_max + 1;
    }
    return w.misc[0];
}

// Canonical QC representative of S[0..a) (sorted) into w.best; returns the orbit size.
__device__ int wave_canon(const DevCode &cd, WaveLds &w, int a) {
    const int lane = lane_id(), z = cd.z;
    if (z == 0) {
        if (lane < a) w.best[lane] = w.S[lane];
        wave_sync();
        return 1;
    }
    const int s = lane < a ? w.S[lane] : 0;
    const int blk = s / z, pos = s - blk * z;
    const int jmin = w.S[0] / z;
    unsigned long long cands = __ballot(lane < a && blk == jmin);
    int nbest = 0;
    while (cands) {
        const int ci = __ffsll((unsigned long long)cands) - 1;
        cands &= cands - 1;
        const int t = (z - __shfl(pos, ci, 64)) % z;
        const int img = lane < a ? blk * z + (pos + t) % z : INT_MAX;
        int rank = 0;
        for (int j = 0; j < a; ++j) rank += __shfl(img, j, 64) < img;
        if (lane < a) w.cand[rank] = img;
        wave_sync();
        if (nbest == 0) {
            if (lane < a) w.best[lane] = w.cand[lane];
            nbest = 1;
        } else {
            const unsigned long long diff = __ballot(lane < a && w.cand[lane] != w.best[lane]);
            if (!diff) {
                ++nbest;
            } else {
                const int p = __ffsll((unsigned long long)diff) - 1;
                if (w.cand[p] < w.best[p]) {
                    if (lane < a) w.best[lane] = w.cand[lane];
                    nbest = 1;
                }
            }
        }
        wave_sync();
    }
    return z / nbest;
}

__device__ void table_insert(const DevTable &T, const int *key, int a, int b, int orbit,
                             int pattern, int kstar, int *err) {
    const unsigned long long h = set_hash(key, a);
    const unsigned mask = (unsigned)T.cap - 1u;
    unsigned slot = (unsigned)h & mask;
    for (int probe = 0; probe < T.cap; ++probe) {
        const unsigned long long old = atomicCAS(&T.key[slot], 0ull, h);
        if (old == 0ull) {
            for (int i = 0; i < a; ++i) T.set[(size_t)slot * kMaxAmax + i] = key[i];
            T.ab[slot] = a | (b << 8);
            T.orbit[slot] = orbit;
            T.first[slot] = pattern;
            T.kcrit[slot] = kstar;
            __threadfence();
            __hip_atomic_store(&T.ready[slot], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            atomicAdd(T.count, 1);
            return;
        }
        if (old == h) {
            int spins = 0;
            while (__hip_atomic_load(&T.ready[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (++spins > (1 << 22)) {
                    atomicOr(err, 4);
                    return;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            bool same = (T.ab[slot] & 0xff) == a;
            for (int i = 0; i < a && same; ++i) same = T.set[(size_t)slot * kMaxAmax + i] == key[i];
            if (same) {
                atomicMin(&T.first[slot], pattern);
                atomicMin(&T.kcrit[slot], kstar);
                return;
            }
        }
        slot = (slot + 1u) & mask;
    }
    atomicOr(err, 8);
}

// canonicalise w.S[0..a) and insert it (lane 0 inserts)
__device__ void emit_set(const SieveArgs &s, WaveLds &w, int a, int b, int pattern, int kstar) {
    const int orbit = wave_canon(s.cd, w, a);
    if (lane_id() == 0) table_insert(s.tab, w.best, a, b, orbit, pattern, kstar, s.err);
    wave_sync();
}

__global__ __launch_bounds__(kWaves * 64) void k_sieve(SieveArgs s) {
    __shared__ WaveLds lds[kWaves];
    WaveLds &w = lds[threadIdx.x >> 6];
    const int lane = lane_id();
    int nrec = *s.rec_count;
    if (nrec > s.rec_cap) nrec = s.rec_cap;
    const int gw = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int stride = gridDim.x * kWaves;
    for (int r = gw; r < nrec; r += stride) {
        const int *rec = s.recs + (size_t)r * kRecStride;
        const int pattern = rec[0], k = rec[1], mult = rec[3], u = rec[4];
        const int kstar = s.k_crit[pattern];
        if (s.extract_mode == TS_EXTRACT_CRITICAL && k != kstar) continue;
        if (u < 1 || u > kCapMax) {
            if (lane == 0) atomicOr(s.err, 16);
            continue;
        }
        if (lane < u) {
            w.U[lane] = rec[kRecHdr + lane];
            w.X[lane] = rec[kRecHdr + lane];
        }
        wave_sync();
        int emitted = 0, b = 0;
        // S1 = Tree(U)
        int a1 = wave_tree(s.cd, w, u, w.S, &b);
        if (a1 >= 1 && a1 <= s.a_max) {
            emit_set(s, w, a1, b, pattern, kstar);
            ++emitted;
        }
        // S2 = Tree(TS(U))
        const int add = wave_ts_additions(s.cd, w, u, s.a_max);
        if (add <= s.a_max) {
            const int k2 = u + add;
            const int x = lane < u ? w.U[lane] : (lane < k2 ? w.wlist[lane - u] : INT_MAX);
            int rank = 0;
            for (int j = 0; j < k2; ++j) rank += __shfl(x, j, 64) < x;
            wave_sync();
            if (lane < k2) w.X[rank] = x;
            wave_sync();
            int a2 = wave_tree(s.cd, w, k2, w.S, &b);
            if (a2 >= 1 && a2 <= s.a_max) {
                emit_set(s, w, a2, b, pattern, kstar);
                ++emitted;
            }
        }
        if (lane == 0 && emitted) atomicAdd(&s.n_cand[pattern], emitted * mult);
        wave_sync();
    }
}

// ---- table maintenance -------------------------------------------------------

__global__ void k_rehash(DevTable from, DevTable to, int *err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= from.cap) return;
    const unsigned long long h = from.key[i];
    if (!h) return;
    const unsigned mask = (unsigned)to.cap - 1u;
    unsigned slot = (unsigned)h & mask;
    for (int p = 0; p < to.cap; ++p) {
        if (atomicCAS(&to.key[slot], 0ull, h) == 0ull) {
            for (int q = 0; q < kMaxAmax; ++q)
                to.set[(size_t)slot * kMaxAmax + q] = from.set[(size_t)i * kMaxAmax + q];
            to.ab[slot] = from.ab[i];
            to.orbit[slot] = from.orbit[i];
            to.first[slot] = from.first[i];
            to.kcrit[slot] = from.kcrit[i];
            to.ready[slot] = 1;
            atomicAdd(to.count, 1);
            return;
        }
        slot = (slot + 1u) & mask;
    }
    atomicOr(err, 8);
}

// ---- ordered read-out --------------------------------------------------------

__global__ void k_compact(DevTable t, int *idx, int *n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < t.cap && t.key[i]) idx[atomicAdd(n, 1)] = i;
}

// true iff slot x comes after slot y in the output order (b/a, a, tuple);
// -1 marks padding and comes last
__device__ bool after(const DevTable &t, int x, int y) {
    if (x < 0) return y >= 0;
    if (y < 0) return false;
    const int ax = t.ab[x] & 0xff, bx = t.ab[x] >> 8, ay = t.ab[y] & 0xff, by = t.ab[y] >> 8;
    const long long l = (long long)bx * ay, r = (long long)by * ax;
    if (l != r) return l > r;
    if (ax != ay) return ax > ay;
    for (int i = 0; i < ax; ++i) {
        const int p = t.set[(size_t)x * kMaxAmax + i], q = t.set[(size_t)y * kMaxAmax + i];
        if (p != q) return p > q;
    }
    return false;
}

__global__ void k_bitonic(DevTable t, int *idx, int P, int k, int j) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int l = i ^ j;
    if (l <= i) return;
    const int x = idx[i], y = idx[l];
    const bool up = (i & k) == 0;
    if (after(t, x, y) == up) {
        idx[i] = y;
        idx[l] = x;
    }
}

// The whole bitonic network of a table of at most kSortLds entries in one
// workgroup: the slot indices in LDS, a barrier between stages (one launch
// where the global form takes one per stage).  The order is a total order on
// distinct sets, so the result equals the global form's.
constexpr int kSortLds = 8192;
constexpr int kSortThreads = 1024;
__global__ __launch_bounds__(kSortThreads) void k_bitonic_lds(DevTable t, int *idx, int n, int P) {
    __shared__ int sx[kSortLds];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += kSortThreads) sx[i] = i < n ? idx[i] : -1;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += kSortThreads) {
                const int l = i ^ j;
                if (l <= i) continue;
                const int x = sx[i], y = sx[l];
                if (after(t, x, y) == ((i & k) == 0)) {
                    sx[i] = y;
                    sx[l] = x;
                }
            }
            __syncthreads();
        }
    for (int i = tid; i < n; i += kSortThreads) idx[i] = sx[i];
}

__global__ void k_gather(DevTable t, const int *idx, int n, int *out, int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = idx[i];
    int *o = out + (size_t)i * stride;
    o[0] = t.ab[s] & 0xff;
    o[1] = t.ab[s] >> 8;
    o[2] = t.orbit[s];
    o[3] = t.first[s];
    o[4] = t.kcrit[s];
    for (int q = 0; q < kMaxAmax; ++q) o[5 + q] = t.set[(size_t)s * kMaxAmax + q];
}

}  // namespace

int launch_sieve(ts_exec &ex, const DevCode &cd, const DevTable &t, const SearchLaunch &a,
                 int n_records) {
    if (n_records <= 0) return TS_OK;
    SieveArgs s;
    s.cd = cd;
    s.tab = t;
    s.recs = a.recs;
    s.rec_count = a.rec_count;
    s.rec_cap = a.rec_cap;
    s.k_crit = a.k_crit;
    s.n_cand = a.n_cand;
    s.a_max = a.a_max;
    s.extract_mode = a.extract_mode;
    s.err = a.err;
    int grid = (n_records + kWaves - 1) / kWaves;
    const int cap = ex.ctx->num_cu * 8;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(k_sieve, dim3(grid), dim3(kWaves * 64), 0, ex.stream, s);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

size_t table_bytes(int cap) { return (size_t)cap * (8 + 4 * (5 + kMaxAmax)) + 64; }

static int alloc_table(ts_exec &ex, DevTable *t, int cap) {
    const size_t bytes = table_bytes(cap);
    char *p = (char *)ex.dalloc(bytes);
    if (!p) {
        set_error("device allocation of the TS table (%zu bytes) failed", bytes);
        return TS_E_NOMEM;
    }
    t->cap = cap;
    t->key = (unsigned long long *)p;
    t->ready = (int *)(p + (size_t)cap * 8);
    t->ab = t->ready + cap;
    t->orbit = t->ab + cap;
    t->first = t->orbit + cap;
    t->kcrit = t->first + cap;
    t->set = t->kcrit + cap;
    t->count = t->set + (size_t)cap * kMaxAmax;
    // keys, ready flags and the counter start at 0 (fill kernels, not memset)
    int rc = launch_fill(ex.stream, (int *)t->key, 0, (int64_t)cap * 2);
    if (rc) return rc;
    rc = launch_fill(ex.stream, t->ready, 0, cap);
    if (rc) return rc;
    return launch_fill(ex.stream, t->count, 0, 1);
}

int table_init(ts_exec &ex, DevTable &t, int cap) {
    if (t.cap) return TS_OK;
    return alloc_table(ex, &t, cap);
}

void table_free(ts_exec &ex, DevTable &t) {
    if (t.cap) ex.dfree(t.key);
    t = DevTable{};
}

// Makes room for `incoming` more distinct sets at a load factor <= 1/2.
int table_grow_if_needed(ts_exec &ex, DevTable &t, int64_t incoming) {
    int rc = table_init(ex, t, 1 << 16);
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(ex.pinned, t.count, 4, hipMemcpyDeviceToHost, ex.stream));
    TSG_HIP(hipStreamSynchronize(ex.stream));
    const int64_t need = 2 * ((int64_t)ex.pinned[0] + incoming);
    if (need <= t.cap) return TS_OK;
    int64_t cap = t.cap;
    while (cap < need) cap *= 2;
    if (cap > (1 << 30)) {
        set_error("TS table would exceed 2^30 slots");
        return TS_E_NOMEM;
    }
    DevTable nt{};
    rc = alloc_table(ex, &nt, (int)cap);
    if (rc) return rc;
    int *err = (int *)ex.dalloc(16);
    if (!err) return TS_E_NOMEM;
    rc = launch_fill(ex.stream, err, 0, 1);
    if (rc) return rc;
    const int blk = 256;
    hipLaunchKernelGGL(k_rehash, dim3((t.cap + blk - 1) / blk), dim3(blk), 0, ex.stream, t, nt, err);
    TSG_HIP(hipGetLastError());
    TSG_HIP(hipMemcpyAsync(ex.pinned, err, 4, hipMemcpyDeviceToHost, ex.stream));
    TSG_HIP(hipStreamSynchronize(ex.stream));
    ex.dfree(err);
    ex.dfree(t.key);
    t = nt;
    if (ex.pinned[0]) {
        set_error("rehash overflow");
        return TS_E_STATE;
    }
    return TS_OK;
}

int collect_tables(ts_exec &ex, int nt, const DevTable *const *t, std::vector<int32_t> *const *rec_host,
                   std::vector<int32_t> *const *bits_host) {
    size_t idx_total = 0;
    std::vector<size_t> idx_off(nt);
    for (int i = 0; i < nt; ++i) {
        rec_host[i]->clear();
        bits_host[i]->clear();
        idx_off[i] = idx_total;
        idx_total += (size_t)t[i]->cap;   // a power of two: room for the padded sort
    }
    if (!idx_total) return TS_OK;
    hipStream_t s = ex.stream;
    DBuf d_n(ex, (size_t)nt * 4), idx(ex, idx_total * 4);
    if (!d_n.p || !idx.p) return TS_E_NOMEM;
    int rc = launch_fill(s, d_n.as<int>(), 0, nt);
    if (rc) return rc;
    const int blk = 256;
    for (int i = 0; i < nt; ++i) {
        if (!t[i]->cap) continue;
        hipLaunchKernelGGL(k_compact, dim3((t[i]->cap + blk - 1) / blk), dim3(blk), 0, s, *t[i],
                           idx.as<int>() + idx_off[i], d_n.as<int>() + i);
    }
    TSG_HIP(hipGetLastError());
    // the tables' sizes, one copy
    unsigned char *h = nullptr;
    rc = ex.bulk_buf((size_t)nt * 4, &h);
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(h, d_n.p, (size_t)nt * 4, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipStreamSynchronize(s));
    std::vector<int> n(nt);
    std::memcpy(n.data(), h, (size_t)nt * 4);
    const int stride = 5 + kMaxAmax;
    std::vector<size_t> out_off(nt);
    size_t out_total = 0;
    for (int i = 0; i < nt; ++i) {
        out_off[i] = out_total;
        out_total += (size_t)n[i] * stride;
    }
    if (!out_total) return TS_OK;
    DBuf out(ex, out_total * 4);
    if (!out.p) return TS_E_NOMEM;
    for (int i = 0; i < nt; ++i) {
        if (n[i] <= 0) continue;
        int *ix = idx.as<int>() + idx_off[i];
        int P = 1;
        while (P < n[i]) P <<= 1;
        if (P <= kSortLds) {   // one launch, padded in LDS
            hipLaunchKernelGGL(k_bitonic_lds, dim3(1), dim3(kSortThreads), 0, s, *t[i], ix, n[i], P);
        } else {
            // pad to a power of two with -1 (sorts last), one launch per stage
            if (P > n[i]) {
                rc = launch_fill(s, ix + n[i], -1, P - n[i]);
                if (rc) return rc;
            }
            for (int k = 2; k <= P; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1)
                    hipLaunchKernelGGL(k_bitonic, dim3((P + blk - 1) / blk), dim3(blk), 0, s, *t[i], ix, P,
                                       k, j);
        }
        hipLaunchKernelGGL(k_gather, dim3((n[i] + blk - 1) / blk), dim3(blk), 0, s, *t[i], ix, n[i],
                           out.as<int>() + out_off[i], stride);
        TSG_HIP(hipGetLastError());
    }
    // every table's sorted records, one copy
    rc = ex.bulk_buf(out_total * 4, &h);
    if (rc) return rc;
    TSG_HIP(hipMemcpyAsync(h, out.p, out_total * 4, hipMemcpyDeviceToHost, s));
    TSG_HIP(hipStreamSynchronize(s));
    const int32_t *raw = (const int32_t *)h;
    for (int i = 0; i < nt; ++i) {
        std::vector<int32_t> &recs = *rec_host[i];
        std::vector<int32_t> &bits = *bits_host[i];
        recs.resize((size_t)n[i] * 5);
        for (int q0 = 0; q0 < n[i]; ++q0) {
            const int32_t *r = raw + out_off[i] + (size_t)q0 * stride;
            for (int q = 0; q < 5; ++q) recs[(size_t)q0 * 5 + q] = r[q];
            for (int q = 0; q < r[0]; ++q) bits.push_back(r[5 + q]);
        }
    }
    return TS_OK;
}

int collect_table(ts_exec &ex, const DevTable &t, std::vector<int32_t> &rec_host,
                  std::vector<int32_t> &bits_host) {
    const DevTable *tp = &t;
    std::vector<int32_t> *rp = &rec_host, *bp = &bits_host;
    return collect_tables(ex, 1, &tp, &rp, &bp);
}

}  // namespace tsg
