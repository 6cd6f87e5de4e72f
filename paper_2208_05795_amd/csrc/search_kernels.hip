// Impulse search kernels (Section III): error-impulse channel, flooding decoding
// iteration by iteration, bisection on the impulse amplitude and the write-out
// of the error sets that are sieved into trapping-set candidates.
//
// Layout.  One workgroup owns one impulse pattern at a time (persistent grid,
// patterns taken from an atomic queue) and keeps the whole frame on chip for
// all of its decodes: the APP values live in LDS, the check-to-variable
// messages of the checks a thread owns live in that thread's registers, and the
// check neighbour lists are loaded into registers once per kernel.  A thread
// owns checks tid, tid+B, ... (B = workgroup size); for a QC code consecutive
// threads own consecutive rows of a circulant, so their APP reads
// APP[j*z + (r+s) mod z] are consecutive LDS words.  HBM traffic per decode is
// only the pattern and the per-pattern results.
//
// Offset min-sum (int8 messages, exact integer arithmetic):
//   v2c = sat127(APP - c2v); c2v' = sign-product * max(min - beta, 0) over the
//   other edges (min / second-min / argmin per check); APP' = lambda + sum c2v'
//   accumulated with LDS integer atomics (order-free, hence exact).
// Sum-product (float32):
//   c2v' = sign-product * phi(sum_{others} phi(min(|v2c|, 30))), phi(x) =
//   log1p(2 / expm1(max(x, 2^-20))); the exclusive sums come from prefix and
//   suffix sums; c2v' is staged in LDS in edge order and each variable sums its
//   messages in ascending check order (deterministic).
//
// After iteration t the hard decision x_t = [APP_t < 0] and the syndrome weight
// w_t are produced during the next iteration's check pass (it reads the same
// APP values), so one workgroup barrier per iteration suffices for OMS.
#include <climits>
#include <cmath>

#include "internal.h"
#include "wave.h"

namespace tsg {
namespace {

__device__ __forceinline__ int q_impulse(int qb, int k) {
    // round_half_away(qb * (16 - k) / 16), saturated to [-127, 127]
    const long long nv = (long long)qb * (16 - k);
    const long long mag = ((nv < 0 ? -nv : nv) + 8) >> 4;
    long long q = nv < 0 ? -mag : mag;
    q = q > 127 ? 127 : (q < -127 ? -127 : q);
    return (int)q;
}

__device__ __forceinline__ float phi_f(float x) {
    x = fmaxf(x, 0x1p-20f);
    return log1pf(2.0f / expm1f(x));
}

// Shared-memory layout common to both decoders (offsets in bytes from the base).
struct Lds {
    int np, W, T;
    size_t app, c2v, lam, hist, imask, wsyn, pcnt, sh, total;
};

__host__ __device__ inline Lds lds_layout(int decoder, int n, int e, int T) {
    Lds L;
    L.np = (n + 1 + 63) & ~63;   // +1: slot n is a dummy for padded edges
    L.W = L.np >> 6;
    L.T = T;
    size_t o = 0;
    L.app = o;
    o += (size_t)(decoder == TS_DEC_OMS_I8 ? 3 : 1) * L.np * 4;
    L.lam = o;
    if (decoder != TS_DEC_OMS_I8) o += (size_t)L.np * 4;
    L.c2v = o;
    if (decoder != TS_DEC_OMS_I8) o += (size_t)((e + 63) & ~63) * 4;
    o = (o + 15) & ~(size_t)15;
    L.hist = o;
    o += (size_t)T * L.W * 8;
    L.imask = o;
    o += (size_t)L.W * 8;
    L.wsyn = o;
    o += (size_t)(T + 2) * 4;
    L.pcnt = o;
    o += (size_t)(T + 2) * 4;
    L.sh = o;
    o += 32 * 4;
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// Writes the candidate error sets U_t = S(x_t) u I, t = t0..iters, of one
// failing decode to the record buffer (wavefront 0; consecutive equal sets are
// merged into one record with a multiplicity).
__device__ void write_candidates(const SearchLaunch &a, const unsigned long long *hist,
                                 const unsigned long long *imask, int W, int iters,
                                 int pg, int k) {
    if (threadIdx.x < 64) {
        const int lane = lane_id();
        int last = -1, mult = 0;
        for (int t = a.t0; t <= iters; ++t) {
            const unsigned long long *h = hist + (size_t)(t - 1) * W;
            int cnt = 0;
            for (int i = lane; i < W; i += 64) cnt += __popcll(h[i] | imask[i]);
            cnt = wave_sum(cnt);
            if (cnt > a.cap) {
                if (last >= 0 && lane == 0) a.recs[(size_t)last * kRecStride + 3] = mult;
                last = -1;
                continue;
            }
            if (last >= 0) {
                const unsigned long long *hp = h - W;
                int diff = 0;
                for (int i = lane; i < W; i += 64) diff |= ((h[i] | imask[i]) != (hp[i] | imask[i]));
                if (!__any(diff)) {
                    ++mult;
                    continue;
                }
                if (lane == 0) a.recs[(size_t)last * kRecStride + 3] = mult;
            }
            int r = 0;
            if (lane == 0) r = atomicAdd(a.rec_count, 1);
            r = __shfl(r, 0, 64);
            if (r >= a.rec_cap) {   // full: the host re-runs this chunk with fewer patterns
                last = -1;
                continue;
            }
            int *rec = a.recs + (size_t)r * kRecStride;
            if (lane == 0) {
                rec[0] = pg;
                rec[1] = k;
                rec[2] = t;
                rec[3] = 1;
                rec[4] = cnt;
            }
            int off = 0;
            for (int i0 = 0; i0 < W; i0 += 64) {
                const int i = i0 + lane;
                unsigned long long wv = i < W ? (h[i] | imask[i]) : 0ull;
                const int pc = __popcll(wv);
                int pos = off + wave_excl_scan(pc);
                while (wv) {
                    const int b = __ffsll((unsigned long long)wv) - 1;
                    rec[kRecHdr + pos++] = i * 64 + b;
                    wv &= wv - 1;
                }
                off += wave_sum(pc);
            }
            last = r;
            mult = 1;
        }
        if (last >= 0 && lane == 0) a.recs[(size_t)last * kRecStride + 3] = mult;
    }
    __syncthreads();
}

struct DecRes {
    int fail, iters, tmin;
};

// ---------------------------------------------------------------------------
// offset min-sum, int8 messages
// ---------------------------------------------------------------------------
template <int DC, int CPT>
__global__ __launch_bounds__(256) void k_search_oms(SearchLaunch a, DevCode cd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = cd.n, m = cd.m, T = a.max_iter;
    const Lds L = lds_layout(TS_DEC_OMS_I8, n, cd.e, T);
    const int np = L.np, W = L.W;
    int *app = (int *)(smem + L.app);
    unsigned long long *hist = (unsigned long long *)(smem + L.hist);
    unsigned long long *imask = (unsigned long long *)(smem + L.imask);
    int *wsyn = (int *)(smem + L.wsyn);
    int *pcnt = (int *)(smem + L.pcnt);
    int *sh = (int *)(smem + L.sh);
    const int B = blockDim.x, NW = B >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    int nb[CPT][DC];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int chk = tid + c * B;
#pragma unroll
        for (int j = 0; j < DC; ++j) {
            int v = -1;
            if (chk < m && j < cd.dc_pad) v = cd.cn_tab[(size_t)j * cd.m_tab + chk];
            nb[c][j] = v < 0 ? n : v;
        }
    }
    int c2v[CPT][DC];
    unsigned long long my_iters = 0, my_dec = 0;
    int qi = 0;
    const int qb = a.q_base;

    auto lam_of = [&](int v) -> int {
        if (v < n) return ((imask[v >> 6] >> (v & 63)) & 1ull) ? qi : qb;
        return v == n ? 127 : 0;
    };

    auto decode = [&](int k) -> DecRes {
        __syncthreads();   // previous readers of the shared state are done
        qi = q_impulse(qb, k);
        for (int v = tid; v < np; v += B) {
            const int l = lam_of(v);
            app[v] = l;
            app[np + v] = l;
        }
        for (int i = tid; i < T + 2; i += B) {
            wsyn[i] = 0;
            pcnt[i] = 0;
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int j = 0; j < DC; ++j) c2v[c][j] = 0;
        __syncthreads();
        int cur = 0, nxt = 1, spare = 2;
        int iters = T, wmin = INT_MAX, tmin = 0;
        for (int t = 1; t <= T + 1; ++t) {
            const int *A = app + cur * np;
            int *N = app + nxt * np;
            int unsat = 0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                int val[DC];
#pragma unroll
                for (int j = 0; j < DC; ++j) val[j] = A[nb[c][j]];
                int par = 0;
#pragma unroll
                for (int j = 0; j < DC; ++j) par ^= (val[j] < 0);
                unsat += par;
                if (t <= T) {
                    int mn1 = 127, mn2 = 127, idx = 0, sgn = 0;
                    int v2[DC];
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        int x = val[j] - c2v[c][j];
                        x = x > 127 ? 127 : (x < -127 ? -127 : x);
                        if (nb[c][j] == n) x = 127;
                        v2[j] = x;
                        const int ax = x < 0 ? -x : x;
                        sgn ^= (x < 0);
                        if (ax < mn1) {
                            mn2 = mn1;
                            mn1 = ax;
                            idx = j;
                        } else if (ax < mn2) {
                            mn2 = ax;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        int mag = (j == idx ? mn2 : mn1) - a.offset;
                        mag = mag < 0 ? 0 : mag;
                        const int out = (sgn ^ (v2[j] < 0)) ? -mag : mag;
                        c2v[c][j] = out;
                        if (nb[c][j] != n) atomicAdd(&N[nb[c][j]], out);
                    }
                }
            }
            if (t >= 2) {
                const int us = wave_sum(unsat);
                if (lane == 0 && us) atomicAdd(&wsyn[t - 1], us);
                int pc = 0;
                for (int i = wid; i < W; i += NW) {
                    const int v = i * 64 + lane;
                    const unsigned long long mask = __ballot((v < n) && (A[v] < 0));
                    if (lane == 0) hist[(size_t)(t - 2) * W + i] = mask;
                    pc += __popcll(mask);
                }
                if (lane == 0 && pc) atomicAdd(&pcnt[t - 1], pc);
            }
            if (t < T) {
                int *S = app + spare * np;
                for (int v = tid; v < np; v += B) S[v] = lam_of(v);
            }
            __syncthreads();
            if (t >= 2) {
                const int w = wsyn[t - 1];
                if (w < wmin) {
                    wmin = w;
                    tmin = t - 1;
                }
                if (w == 0) {
                    iters = t - 1;
                    break;
                }
            }
            const int tmp = cur;
            cur = nxt;
            nxt = spare;
            spare = tmp;
        }
        DecRes r;
        r.iters = iters;
        r.tmin = tmin;
        r.fail = pcnt[iters] > 0;
        my_iters += iters;
        my_dec += 1;
        return r;
    };

    for (;;) {
        __syncthreads();
        if (tid == 0) sh[0] = atomicAdd(a.queue, 1);
        __syncthreads();
        const int pl = sh[0];
        if (pl >= a.n_patterns) break;
        for (int i = tid; i < W; i += B) imask[i] = 0ull;
        if (tid < kMaxWidth) sh[1 + tid] = tid < a.width ? a.patterns[(size_t)pl * a.width + tid] : -1;
        __syncthreads();
        if (tid < kMaxWidth) {
            const int v = sh[1 + tid];
            if (v >= n || v < -1) atomicOr(a.err, 1);
            else if (v >= 0) atomicOr(&imask[v >> 6], 1ull << (v & 63));
        }
        const int pg = a.pat_base + pl;
        DecRes r = decode(a.k_max);
        int kc = -1, it_hi = 0, tm_hi = 0, it_lo = r.iters;
        if (r.fail) {
            write_candidates(a, hist, imask, W, r.iters, pg, a.k_max);
            int lo = 0, hi = a.k_max;
            it_hi = r.iters;
            tm_hi = r.tmin;
            it_lo = 1;   // D(0) is the noiseless decode: success at the first iteration
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                r = decode(mid);
                if (r.fail) {
                    hi = mid;
                    it_hi = r.iters;
                    tm_hi = r.tmin;
                    write_candidates(a, hist, imask, W, r.iters, pg, mid);
                } else {
                    lo = mid;
                    it_lo = r.iters;
                }
            }
            kc = hi;
        }
        if (tid == 0) {
            a.k_crit[pg] = kc;
            a.iters_crit[pg] = it_hi;
            a.iters_lo[pg] = it_lo;
            a.tmin_crit[pg] = tm_hi;
            a.n_cand[pg] = 0;
        }
    }
    if (tid == 0) {
        atomicAdd(&a.counters[0], my_dec);
        atomicAdd(&a.counters[1], my_iters);
    }
}

// ---------------------------------------------------------------------------
// sum-product, float32
// ---------------------------------------------------------------------------

// Register state of the checks one thread owns.
template <int DC, int CPT>
struct SpaRegs {
    int nb[CPT][DC];
    int ebase[CPT];
    float c2v[CPT][DC];

    __device__ void load(const DevCode &cd) {
        const int B = blockDim.x, tid = threadIdx.x;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int chk = tid + c * B;
            ebase[c] = chk < cd.m ? cd.row_ptr[chk] : 0;
#pragma unroll
            for (int j = 0; j < DC; ++j) {
                int v = -1;
                if (chk < cd.m && j < cd.dc_pad) v = cd.cn_tab[(size_t)j * cd.m_tab + chk];
                nb[c][j] = v < 0 ? cd.n : v;
            }
        }
    }
};

// One SPA decode.  On entry lam[] and app[] hold the channel LLRs, wsyn/pcnt
// are zero and every thread has passed a barrier; c2v is cleared here.  hist
// (optional) receives the hard decision of every iteration.
template <int DC, int CPT>
__device__ DecRes spa_run(const DevCode &cd, SpaRegs<DC, CPT> &R, float *app, const float *lam,
                          float *c2e, unsigned long long *hist, int W, int *wsyn, int *pcnt,
                          int T) {
    const int n = cd.n, B = blockDim.x, NW = B >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int j = 0; j < DC; ++j) R.c2v[c][j] = 0.0f;
    int iters = T, wmin = INT_MAX, tmin = 0;
    for (int t = 1; t <= T + 1; ++t) {
        int unsat = 0;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            float val[DC];
#pragma unroll
            for (int j = 0; j < DC; ++j) val[j] = app[R.nb[c][j]];
            int par = 0;
#pragma unroll
            for (int j = 0; j < DC; ++j) par ^= (R.nb[c][j] != n) & (val[j] < 0.0f);
            unsat += par;
            if (t <= T) {
                float ph[DC];
                int neg[DC];
                int sgn = 0;
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                    const float x = val[j] - R.c2v[c][j];
                    neg[j] = x < 0.0f;
                    sgn ^= neg[j] & (R.nb[c][j] != n);
                    ph[j] = R.nb[c][j] != n ? phi_f(fminf(fabsf(x), 30.0f)) : 0.0f;
                }
                float pre[DC + 1], suf[DC + 1];
                pre[0] = 0.0f;
                suf[DC] = 0.0f;
#pragma unroll
                for (int j = 0; j < DC; ++j) pre[j + 1] = pre[j] + ph[j];
#pragma unroll
                for (int j = DC - 1; j >= 0; --j) suf[j] = suf[j + 1] + ph[j];
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                    const float mag = phi_f(pre[j] + suf[j + 1]);
                    const float out = (sgn ^ neg[j]) ? -mag : mag;
                    R.c2v[c][j] = out;
                    if (R.nb[c][j] != n) c2e[R.ebase[c] + j] = out;
                }
            }
        }
        if (t >= 2) {
            const int us = wave_sum(unsat);
            if (lane == 0 && us) atomicAdd(&wsyn[t - 1], us);
            int pc = 0;
            for (int i = wid; i < W; i += NW) {
                const int v = i * 64 + lane;
                const unsigned long long mask = __ballot((v < n) && (app[v] < 0.0f));
                if (hist && lane == 0) hist[(size_t)(t - 2) * W + i] = mask;
                pc += __popcll(mask);
            }
            if (lane == 0 && pc) atomicAdd(&pcnt[t - 1], pc);
        }
        __syncthreads();
        if (t >= 2) {
            const int w = wsyn[t - 1];
            if (w < wmin) {
                wmin = w;
                tmin = t - 1;
            }
            if (w == 0) {
                iters = t - 1;
                break;
            }
        }
        if (t == T + 1) break;
        // variable pass: APP_t = lambda + messages in ascending check order
        for (int v = tid; v < n; v += B) {
            float s = lam[v];
            for (int d = 0; d < cd.dv_pad; ++d) {
                const int e = cd.vn_tab[(size_t)d * cd.n_tab + v];
                if (e >= 0) s += c2e[e];
            }
            app[v] = s;
        }
        __syncthreads();
    }
    DecRes r;
    r.iters = iters;
    r.tmin = tmin;
    r.fail = pcnt[iters] > 0;
    return r;
}

template <int DC, int CPT>
__global__ __launch_bounds__(256) void k_search_spa(SearchLaunch a, DevCode cd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = cd.n, T = a.max_iter;
    const Lds L = lds_layout(TS_DEC_SPA_F32, n, cd.e, T);
    const int np = L.np, W = L.W;
    float *app = (float *)(smem + L.app);
    float *lam = (float *)(smem + L.lam);
    float *c2e = (float *)(smem + L.c2v);
    unsigned long long *hist = (unsigned long long *)(smem + L.hist);
    unsigned long long *imask = (unsigned long long *)(smem + L.imask);
    int *wsyn = (int *)(smem + L.wsyn);
    int *pcnt = (int *)(smem + L.pcnt);
    int *sh = (int *)(smem + L.sh);
    const int B = blockDim.x, tid = threadIdx.x;

    SpaRegs<DC, CPT> R;
    R.load(cd);
    unsigned long long my_iters = 0, my_dec = 0;
    const float h = a.h;
#define TSG_SPA_DECODE(K, OUT)                                                           \
    do {                                                                                \
        __syncthreads();                                                                \
        const float li_ = h * (1.0f - (float)(K) / (float)a.k_den);                     \
        for (int v = tid; v < np; v += B) {                                             \
            float l_ = 0.0f;                                                            \
            if (v < n) l_ = ((imask[v >> 6] >> (v & 63)) & 1ull) ? li_ : h;             \
            lam[v] = l_;                                                                \
            app[v] = l_;                                                                \
        }                                                                               \
        for (int i = tid; i < T + 2; i += B) {                                          \
            wsyn[i] = 0;                                                                \
            pcnt[i] = 0;                                                                \
        }                                                                               \
        __syncthreads();                                                                \
        OUT = spa_run<DC, CPT>(cd, R, app, lam, c2e, hist, W, wsyn, pcnt, T);           \
        my_iters += OUT.iters;                                                          \
        my_dec += 1;                                                                    \
    } while (0)

    for (;;) {
        __syncthreads();
        if (tid == 0) sh[0] = atomicAdd(a.queue, 1);
        __syncthreads();
        const int pl = sh[0];
        if (pl >= a.n_patterns) break;
        for (int i = tid; i < W; i += B) imask[i] = 0ull;
        if (tid < kMaxWidth) sh[1 + tid] = tid < a.width ? a.patterns[(size_t)pl * a.width + tid] : -1;
        __syncthreads();
        if (tid < kMaxWidth) {
            const int v = sh[1 + tid];
            if (v >= n || v < -1) atomicOr(a.err, 1);
            else if (v >= 0) atomicOr(&imask[v >> 6], 1ull << (v & 63));
        }
        const int pg = a.pat_base + pl;
        DecRes r;
        TSG_SPA_DECODE(a.k_max, r);
        int kc = -1, it_hi = 0, tm_hi = 0, it_lo = r.iters;
        if (r.fail) {
            write_candidates(a, hist, imask, W, r.iters, pg, a.k_max);
            int lo = 0, hi = a.k_max;
            it_hi = r.iters;
            tm_hi = r.tmin;
            it_lo = 1;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                TSG_SPA_DECODE(mid, r);
                if (r.fail) {
                    hi = mid;
                    it_hi = r.iters;
                    tm_hi = r.tmin;
                    write_candidates(a, hist, imask, W, r.iters, pg, mid);
                } else {
                    lo = mid;
                    it_lo = r.iters;
                }
            }
            kc = hi;
        }
        if (tid == 0) {
            a.k_crit[pg] = kc;
            a.iters_crit[pg] = it_hi;
            a.iters_lo[pg] = it_lo;
            a.tmin_crit[pg] = tm_hi;
            a.n_cand[pg] = 0;
        }
    }
    if (tid == 0) {
        atomicAdd(&a.counters[0], my_dec);
        atomicAdd(&a.counters[1], my_iters);
    }
#undef TSG_SPA_DECODE
}

// ---------------------------------------------------------------------------
// importance-sampling frames (float32 SPA on Philox noise)
// ---------------------------------------------------------------------------

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor S-box on a 4 x 32-bit counter, the 2 x 32-bit key bumped by the
// Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c[0];
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c[2];
        const unsigned n0 = (unsigned)(p1 >> 32) ^ c[1] ^ k0;
        const unsigned n2 = (unsigned)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (unsigned)p1;
        c[3] = (unsigned)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

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
    int *queue;
    unsigned long long *counters;
};

__host__ __device__ inline size_t is_lds_bytes(int n, int e, int T, size_t *o_lam, size_t *o_c2v,
                                               size_t *o_misc) {
    const int np = (n + 1 + 63) & ~63;
    size_t o = (size_t)np * 4;   // app
    *o_lam = o;
    o += (size_t)np * 4;
    *o_c2v = o;
    o += (size_t)((e + 63) & ~63) * 4;
    o = (o + 15) & ~(size_t)15;
    *o_misc = o;
    // wsyn[T+2], pcnt[T+2], sh[32] ints, tn[kMaxWidth] doubles, ts[kMaxWidth] ints
    o += (size_t)(2 * (T + 2) + 32) * 4;
    o = (o + 7) & ~(size_t)7;
    o += (size_t)kMaxWidth * 8 + (size_t)kMaxWidth * 4;
    return (o + 15) & ~(size_t)15;
}

template <int DC, int CPT>
__global__ __launch_bounds__(256) void k_is_spa(IsDev a, DevCode cd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = cd.n, T = a.max_iter;
    size_t o_lam, o_c2v, o_misc;
    is_lds_bytes(n, cd.e, T, &o_lam, &o_c2v, &o_misc);
    const int np = (n + 1 + 63) & ~63, W = np >> 6;
    float *app = (float *)smem;
    float *lam = (float *)(smem + o_lam);
    float *c2e = (float *)(smem + o_c2v);
    int *wsyn = (int *)(smem + o_misc);
    int *pcnt = wsyn + (T + 2);
    int *sh = pcnt + (T + 2);
    double *tn = (double *)(((size_t)(sh + 32) + 7) & ~(size_t)7);
    int *tsl = (int *)(tn + kMaxWidth);
    const int B = blockDim.x, tid = threadIdx.x;

    SpaRegs<DC, CPT> R;
    R.load(cd);
    if (tid < kMaxWidth) tsl[tid] = tid < a.a ? a.ts[tid] : -1;
    unsigned long long my_iters = 0;
    const unsigned k0 = (unsigned)a.seed, k1 = (unsigned)(a.seed >> 32);
    const double two_pi = 6.283185307179586476925286766559;
    for (;;) {
        __syncthreads();
        if (tid == 0) sh[0] = atomicAdd(a.queue, 1);
        __syncthreads();
        const int f = sh[0];
        if ((long long)f >= a.n_frames) break;
        const unsigned long long frame = a.frame_base + (unsigned long long)f;
        for (int g = tid; 4 * g < n; g += B) {
            unsigned c[4] = {(unsigned)g, (unsigned)frame, (unsigned)(frame >> 32), a.stream};
            philox4x32_10(c, k0, k1);
            double u[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) u[i] = ((double)c[i] + 0.5) * 0x1p-32;
            const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
            double s0, c0, s1, c1;
            sincos(two_pi * u[1], &s0, &c0);
            sincos(two_pi * u[3], &s1, &c1);
            const double nv[4] = {r0 * c0, r0 * s0, r1 * c1, r1 * s1};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = 4 * g + i;
                if (v >= n) break;
                int slot = -1;
                for (int q = 0; q < a.a; ++q)
                    if (tsl[q] == v) slot = q;
                const double y = 1.0 - (slot >= 0 ? a.shift : 0.0) + a.sigma * nv[i];
                const float l = (float)(2.0 * y / a.sigma2);
                lam[v] = l;
                app[v] = l;
                if (slot >= 0) tn[slot] = nv[i];
            }
        }
        for (int v = n + tid; v < np; v += B) {
            lam[v] = 0.0f;
            app[v] = 0.0f;
        }
        for (int i = tid; i < T + 2; i += B) {
            wsyn[i] = 0;
            pcnt[i] = 0;
        }
        __syncthreads();
        const DecRes r = spa_run<DC, CPT>(cd, R, app, lam, c2e, nullptr, W, wsyn, pcnt, T);
        my_iters += r.iters;
        if (tid == 0) {
            double st = 0.0;
            for (int q = 0; q < a.a; ++q) st += tn[q];
            const double w = exp(a.wconst + (a.shift / a.sigma) * st);
            a.fail[f] = (unsigned char)r.fail;
            a.wf[f] = r.fail ? w : 0.0;
        }
    }
    if (tid == 0) atomicAdd(&a.counters[1], my_iters);
}

// Fixed-order reduction of the per-frame values: thread t sums a contiguous
// range in frame order, then a fixed binary tree combines the threads.
// mode 0: out = {sum w, sum w^2, failures}; mode 1: out[3] = sum (w - mean)^2.
__global__ __launch_bounds__(1024) void k_is_reduce(const double *wf, const unsigned char *fail,
                                                     long long n, int mode, double mean,
                                                     double *out) {
    __shared__ double s0[1024], s1[1024], s2[1024];
    const int t = threadIdx.x, B = blockDim.x;
    const long long per = (n + B - 1) / B;
    const long long lo = (long long)t * per, hi = lo + per < n ? lo + per : n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (long long i = lo; i < hi; ++i) {
        const double w = wf[i];
        if (mode == 0) {
            a0 += w;
            a1 += w * w;
            a2 += (double)fail[i];
        } else {
            a0 += (w - mean) * (w - mean);
        }
    }
    s0[t] = a0;
    s1[t] = a1;
    s2[t] = a2;
    __syncthreads();
    for (int h = B / 2; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
            s2[t] += s2[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (mode == 0) {
            out[0] = s0[0];
            out[1] = s1[0];
            out[2] = s2[0];
        } else {
            out[3] = s0[0];
        }
    }
}

__global__ void k_fill(int *p, int value, long long count) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// ---------------------------------------------------------------------------
// kernel table
// ---------------------------------------------------------------------------
typedef void (*SearchKernel)(SearchLaunch, DevCode);

typedef void (*IsKernel)(IsDev, DevCode);

struct KEntry {
    int dc, cpt;
    SearchKernel oms, spa;
    IsKernel is;
};

#define TSG_K(DC, CPT) {DC, CPT, k_search_oms<DC, CPT>, k_search_spa<DC, CPT>, k_is_spa<DC, CPT>}
const KEntry kTable[] = {
    TSG_K(6, 1),  TSG_K(6, 2),  TSG_K(6, 4),  TSG_K(6, 8),  TSG_K(8, 1),  TSG_K(8, 2),
    TSG_K(8, 4),  TSG_K(8, 8),  TSG_K(12, 1), TSG_K(12, 2), TSG_K(12, 4), TSG_K(16, 1),
    TSG_K(16, 2), TSG_K(16, 4), TSG_K(24, 1), TSG_K(24, 2), TSG_K(32, 1), TSG_K(32, 2),
};
#undef TSG_K

const KEntry *find_kernel(int dc, int cpt) {
    for (const KEntry &k : kTable)
        if (k.dc == dc && k.cpt == cpt) return &k;
    return nullptr;
}

}  // namespace

int plan_search(ts_ctx *ctx, const ts_code *c, int decoder, int max_iter, SearchPlan *plan) {
    static const int dcs[] = {6, 8, 12, 16, 24, 32};
    int dc = 0;
    for (int d : dcs)
        if (d >= c->dc_max) { dc = d; break; }
    if (!dc) {
        set_error("check degree %d above the decoder's limit 32", c->dc_max);
        return TS_E_INVAL;
    }
    const Lds L = lds_layout(decoder, c->n, (int)c->e, max_iter);
    if (L.total > ctx->lds_per_block) {
        set_error("code needs %zu bytes of LDS per workgroup, the device has %zu", L.total,
                  ctx->lds_per_block);
        return TS_E_INVAL;
    }
    // smallest checks-per-thread that keeps the workgroup at <= 256 threads
    // (<= 1024 for large codes), among the instantiated kernels
    int cpt = 0, block = 0;
    for (int lim : {256, 1024}) {
        for (int cp : {1, 2, 4, 8}) {
            if (!find_kernel(dc, cp)) continue;
            const int b = ((c->m + cp - 1) / cp + 63) / 64 * 64;
            if (b <= lim) { cpt = cp; block = b; break; }
        }
        if (cpt) break;
    }
    if (!cpt) {
        set_error("code has too many checks (%d) for one workgroup", c->m);
        return TS_E_INVAL;
    }
    const KEntry *ke = find_kernel(dc, cpt);
    SearchKernel kern = decoder == TS_DEC_OMS_I8 ? ke->oms : ke->spa;
    int per_cu = 0;
    TSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, L.total));
    if (per_cu < 1) {
        set_error("decoder kernel does not fit on a compute unit");
        return TS_E_INVAL;
    }
    plan->block = block;
    plan->cpt = cpt;
    plan->dc = dc;
    plan->vpt = 0;
    plan->dv = 0;
    plan->lds = L.total;
    plan->grid = per_cu * ctx->num_cu;
    return TS_OK;
}

int launch_search(ts_ctx *ctx, const SearchPlan &plan, const SearchLaunch &a) {
    const KEntry *ke = find_kernel(plan.dc, plan.cpt);
    if (!ke) {
        set_error("no kernel for dc %d cpt %d", plan.dc, plan.cpt);
        return TS_E_INVAL;
    }
    SearchKernel kern = a.decoder == TS_DEC_OMS_I8 ? ke->oms : ke->spa;
    const int grid = a.n_patterns < plan.grid ? a.n_patterns : plan.grid;
    if (grid <= 0) return TS_OK;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(plan.block), plan.lds, ctx->stream, a, *a.code);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

int launch_fill(ts_ctx *ctx, int *p, int value, int64_t count) {
    if (count <= 0) return TS_OK;
    const int blk = 256;
    const long long grid = (count + blk - 1) / blk;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)grid), dim3(blk), 0, ctx->stream, p, value,
                       (long long)count);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

int launch_is(ts_ctx *ctx, const ts_code *c, const IsLaunch &a, int *grid_out, int *block_out) {
    static const int dcs[] = {6, 8, 12, 16, 24, 32};
    int dc = 0;
    for (int d : dcs)
        if (d >= c->dc_max) { dc = d; break; }
    if (!dc) { set_error("check degree %d above the decoder's limit 32", c->dc_max); return TS_E_INVAL; }
    size_t o1, o2, o3;
    const size_t lds = is_lds_bytes(c->n, (int)c->e, a.max_iter, &o1, &o2, &o3);
    if (lds > ctx->lds_per_block) {
        set_error("code needs %zu bytes of LDS per workgroup, the device has %zu", lds, ctx->lds_per_block);
        return TS_E_INVAL;
    }
    int cpt = 0, block = 0;
    for (int lim : {256, 1024}) {
        for (int cp : {1, 2, 4, 8}) {
            if (!find_kernel(dc, cp)) continue;
            const int b = ((c->m + cp - 1) / cp + 63) / 64 * 64;
            if (b <= lim) { cpt = cp; block = b; break; }
        }
        if (cpt) break;
    }
    if (!cpt) { set_error("code has too many checks (%d) for one workgroup", c->m); return TS_E_INVAL; }
    IsKernel kern = find_kernel(dc, cpt)->is;
    int per_cu = 0;
    TSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, lds));
    if (per_cu < 1) { set_error("IS kernel does not fit on a compute unit"); return TS_E_INVAL; }
    long long grid = (long long)per_cu * ctx->num_cu;
    if (grid > a.n_frames) grid = a.n_frames;
    IsDev d;
    d.max_iter = a.max_iter;
    d.sigma2 = a.sigma2;
    d.sigma = std::sqrt(a.sigma2);
    d.shift = a.shift;
    d.wconst = -(double)a.a * a.shift * a.shift / (2.0 * a.sigma2);
    d.n_frames = a.n_frames;
    d.seed = a.seed;
    d.frame_base = a.frame_base;
    d.stream = a.stream;
    d.ts = a.ts;
    d.a = a.a;
    d.fail = a.fail;
    d.wf = a.wf;
    d.queue = a.queue;
    d.counters = a.counters;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds, ctx->stream, d, c->dev);
    TSG_HIP(hipGetLastError());
    if (grid_out) *grid_out = (int)grid;
    if (block_out) *block_out = block;
    return TS_OK;
}

int launch_is_reduce(ts_ctx *ctx, const double *wf, const unsigned char *fail, int64_t n, int mode,
                     double mean, double *out) {
    hipLaunchKernelGGL(k_is_reduce, dim3(1), dim3(1024), 0, ctx->stream, wf, fail, (long long)n, mode,
                       mean, out);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

}  // namespace tsg
