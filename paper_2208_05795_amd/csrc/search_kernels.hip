// Decoding kernels of the trapping-set search (Section III) and of the IS
// estimator: error-impulse or noisy channel on the all-zero BPSK codeword,
// flooding message passing iteration by iteration, bisection on the impulse
// amplitude, and the write-out of the error sets that the sieve turns into
// trapping-set candidates.
//
// Layout.  One workgroup owns one frame at a time (persistent grid; patterns or
// IS frames come from an atomic queue) and keeps it on chip for every decode:
//   - the check neighbour lists of the checks a thread owns (tid, tid+B, ...)
//     and their check-to-variable messages live in that thread's registers;
//   - the APP values live in LDS as a ring of three int32 buffers: iteration t
//     reads APP_{t-1}, adds its messages into APP_t (initialised to lambda) with
//     LDS integer atomics, and initialises APP_{t+1}, so one barrier per
//     iteration suffices and the sums are exact whatever the atomic order;
//   - the hard decision x_t = [APP_t < 0] and the syndrome weight w_t are taken
//     during the check pass of iteration t+1, which reads the same APP values.
// For a QC code consecutive threads own consecutive rows of a circulant, so
// their APP accesses j*z + (r+s) mod z hit consecutive LDS words.  HBM traffic
// per decode is the pattern and the per-pattern results only.
//
// Check rules:
//   offset min-sum (int8 scale): v2c = sat127(APP - c2v);
//     c2v' = sign-product * max(min - beta, 0) over the other edges (min,
//     second min and argmin per check);
//   sum-product (float32 arithmetic on Q20 fixed-point APP / messages):
//     c2v' = sign-product * phi(sum_{others} phi(min(|v2c|, 30))),
//     phi(x) = ln((1 + e^-x) / (1 - e^-x)) at max(x, 2^-20), evaluated with the
//     hardware exp2 / log2 / reciprocal, with a series at the end where each of
//     the two evaluations needs one (phi_in, phi_out_q); the exclusive sums
//     come from prefix and suffix sums; messages are rounded to 2^-20.
#include <climits>
#include <type_traits>
#include <cmath>

#include "internal.h"
#include "wave.h"

namespace tsg {
namespace {

constexpr float kQ = 1048576.0f;        // Q20 scale of the sum-product APP values
constexpr float kLamMax = 1024.0f;      // |lambda| bound of the Q20 format

__device__ __forceinline__ int q_impulse(int qb, int k) {
    // round_half_away(qb * (16 - k) / 16), saturated to [-127, 127]
    const long long nv = (long long)qb * (16 - k);
    const long long mag = ((nv < 0 ? -nv : nv) + 8) >> 4;
    long long q = nv < 0 ? -mag : mag;
    q = q > 127 ? 127 : (q < -127 ? -127 : q);
    return (int)q;
}

__device__ __forceinline__ int to_q20(float l) {
    l = fminf(fmaxf(l, -kLamMax), kLamMax);
    return __float2int_rn(l * kQ);
}

// phi(x) = -ln tanh(x/2) = ln((1+u)/(1-u)), u = e^-x, for x >= 0, in two
// forms, each accurate where its result matters.  The check's phi terms and
// their sums are kept in log2 units (phi / ln 2), which the hardware exp2 and
// log2 take and give without conversion.
//
// phi_in: phi / ln 2 of a variable-to-check magnitude |d| (Q20), clamped to
// [2^-20, 30].  Small results must keep their relative accuracy (their sum
// over a check can be tiny, and phi of a tiny sum is large), so below
// u = 1/16 the series 2(u + u^3/3 + u^5/5) / ln 2 replaces the logarithm.
// Large results (x -> 0, where 1 - u cancels) need no care: such a term
// enters the other edges' sums S >= phi_in, where |phi'(S)| <= 2 e^-S ~ x,
// which cancels the 2^-24 / x relative error of 1 - u.
// u = e^-x of the clamped magnitude of d (Q20), then phi_in from u in its two
// regimes: below u = 1/16 the series (exp2 only), above it the logarithm.
__device__ __forceinline__ float phi_in_u(int d) {
    constexpr float kL2eQ = -1.4426950408889634f / 1048576.0f;   // -log2(e) 2^-20
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_fmed3f(fabsf((float)d) * kL2eQ,
                                                          -30.0f * 1.4426950408889634f,
                                                          -0x1p-20f * 1.4426950408889634f));
}
constexpr float kPhiSmallU = 0.0625f;
__device__ __forceinline__ float phi_in_small(float u) {
    const float u2 = u * u;
    return u * (2.8853901f + u2 * (0.96179669f + u2 * 0.57707802f));
}
__device__ __forceinline__ float phi_in_big(float u) {
    return __builtin_amdgcn_logf((1.0f + u) * __builtin_amdgcn_rcpf(1.0f - u));
}

// phi_out: Q20 check-to-variable magnitude phi(S) x 2^20 of an exclusive sum
// given in log2 units, y = S / ln 2 >= 0 (before rounding).  Large results
// need 1 - e^-S without cancellation: its Taylor series in y below
// S = 1/8.  Small results need only the absolute accuracy of the logarithm
// (about 1e-7, below the 2^-20 step).
constexpr float kPhiYMin = 1.3758612e-06f;   // S >= 2^-20
constexpr float kPhiYSeries = 0.18033688f;   // S < 1/8
__device__ __forceinline__ float phi_out_q_den(float y, float den) {
    const float u = __builtin_amdgcn_exp2f(-y);
    return __builtin_amdgcn_logf((1.0f + u) * __builtin_amdgcn_rcpf(den)) * (0.69314718055994531f * 1048576.0f);
}
__device__ __forceinline__ float phi_out_q_plain(float y) {   // y >= kPhiYSeries
    return phi_out_q_den(y, 1.0f - __builtin_amdgcn_exp2f(-y));
}
__device__ __forceinline__ float phi_out_q(float y) {
    const float u = __builtin_amdgcn_exp2f(-y);
    const float ser = y * (0.69314718f - y * (0.24022651f - y * (0.055504109f - y * (0.0096181291f - y * 0.0013333558f))));
    const float den = y < kPhiYSeries ? ser : 1.0f - u;
    return __builtin_amdgcn_logf((1.0f + u) * __builtin_amdgcn_rcpf(den)) * (0.69314718055994531f * 1048576.0f);
}

// A value every lane of the wave holds (read from the LDS job copy), moved to
// scalar registers so that addresses derived from it stay scalar.
template <class T>
__device__ __forceinline__ T uni(T v) {
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    union {
        T t;
        int w[sizeof(T) / 4];
    } u;
    u.t = v;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) u.w[i] = __builtin_amdgcn_readfirstlane(u.w[i]);
    return u.t;
}

// Check rules.  On entry val[j] is APP_{t-1} of the check's j-th neighbour and
// c2v[j] the old message on that edge; on return c2v[j] is the new message.
// Each new message is handed on as soon as it is formed, emit(j, new, new -
// old), so that nothing of the edge stays live to the end of the check.
struct OmsRule {
    static constexpr int kDummy = 127;   // padded edges read as a saturated positive message
    template <int DC, class Emit>
    __device__ static __forceinline__ void update(const int (&val)[DC], int (&c2v)[DC],
                                                  const int (&nb)[DC], int pad_id, int offset,
                                                  Emit &&emit) {
        int mn1 = 127, mn2 = 127, idx = 0, sgn = 0;
        int v2[DC];
#pragma unroll
        for (int j = 0; j < DC; ++j) {
            int x = val[j] - c2v[j];
            x = x > 127 ? 127 : (x < -127 ? -127 : x);
            if (nb[j] == pad_id) x = 127;
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
            int mag = (j == idx ? mn2 : mn1) - offset;
            mag = mag < 0 ? 0 : mag;
            const int m = (sgn ^ (v2[j] < 0)) ? -mag : mag;
            const int d = m - c2v[j];
            c2v[j] = m;
            emit(j, m, d);
        }
    }
};

struct SpaRule {
    // Padded edges read APP = 2^30 (Q20, far above any real message): their
    // v2c stays positive and clamps to 30, so they add phi(30) ~ 1.9e-13 to the
    // check's sums (below the 2^-20 step of the results) and no sign, without
    // a per-edge test.  Real APP values stay below 2^30 + 2^27 in magnitude.
    static constexpr int kDummy = 1 << 30;
    template <int DC, class Emit>
    __device__ static __forceinline__ void update(const int (&val)[DC], int (&c2v)[DC],
                                                  const int (&nb)[DC], int pad, int off, Emit &&emit) {
        update_impl<DC, true>(val, c2v, emit);
    }
    // The per-edge temporaries are the phi terms (which become the exclusive
    // sums in place) and the prefix sums; the v2c signs are bits of one word.
    template <int DC, bool kShortcuts, class Emit>
    __device__ static __forceinline__ void update_impl(const int (&val)[DC], int (&c2v)[DC], Emit &&emit) {
        float ph[DC];
        unsigned neg = 0;   // bit j: the v2c message of edge j is negative
        // Wavefront-uniform shortcuts (impulse frames, kShortcuts): where every
        // lane is in one regime, the other regime's arithmetic (whose result
        // the selection would drop) is skipped.  The values are those of the
        // general form.  The input one (u recomputed on the rare mixed path, so
        // as to hold no extra registers) pays off up to a dozen edges per
        // check; wider checks are rarely in one regime on every lane.
        if constexpr (kShortcuts && DC <= 12) {
            bool small = true;
#pragma unroll
            for (int j = 0; j < DC; ++j) {
                const int d = val[j] - c2v[j];
                neg |= (unsigned)(d < 0) << j;
                const float u = phi_in_u(d);
                ph[j] = phi_in_small(u);
                small &= u < kPhiSmallU;
            }
            if (!__all(small)) {
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                    const float u = phi_in_u(val[j] - c2v[j]);
                    if (!(u < kPhiSmallU)) ph[j] = phi_in_big(u);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < DC; ++j) {
                const int d = val[j] - c2v[j];
                neg |= (unsigned)(d < 0) << j;
                const float u = phi_in_u(d);
                ph[j] = u < kPhiSmallU ? phi_in_small(u) : phi_in_big(u);
            }
        }
        // exclusive sums from prefix and suffix sums (no cancellation): the
        // suffix sums run from the right, in the same order of additions as
        // a suffix array, and ph[j] becomes the exclusive sum of edge j
        float pre[DC];
        pre[1] = ph[0];
#pragma unroll
        for (int j = 1; j + 1 < DC; ++j) pre[j + 1] = pre[j] + ph[j];
        float sf = ph[DC - 1];
        ph[DC - 1] = pre[DC - 1];
#pragma unroll
        for (int j = DC - 2; j >= 1; --j) {
            const float e = pre[j] + sf;
            sf = sf + ph[j];
            ph[j] = e;
        }
        ph[0] = sf;
        bool plain = kShortcuts;
        if constexpr (kShortcuts) {
#pragma unroll
            for (int j = 0; j < DC; ++j) plain &= ph[j] >= kPhiYSeries;
        }
        // sign of the other edges' product applied to the float before the
        // (sign-symmetric) rounding to Q20
        const unsigned par = (unsigned)__builtin_popcount(neg) & 1u;
        auto put = [&](int j, float f) {
            const int sb = (int)((par ^ (neg >> j)) << 31);
            const int m = __float2int_rn(__int_as_float(__float_as_int(f) ^ sb));
            const int d = m - c2v[j];
            c2v[j] = m;
            emit(j, m, d);
        };
        if (kShortcuts && __all(plain)) {
#pragma unroll
            for (int j = 0; j < DC; ++j) put(j, phi_out_q_plain(ph[j]));
        } else {
#pragma unroll
            for (int j = 0; j < DC; ++j) put(j, phi_out_q(fmaxf(ph[j], kPhiYMin)));
        }
    }
};
// The sum-product rule of the noisy IS frames: the same values, without the
// shortcuts (their channel values leave few checks in one regime, and the
// extra paths cost the IS kernels more than they save).
struct SpaIsRule : SpaRule {
    template <int DC, class Emit>
    __device__ static __forceinline__ void update(const int (&val)[DC], int (&c2v)[DC],
                                                  const int (&nb)[DC], int pad, int off, Emit &&emit) {
        update_impl<DC, false>(val, c2v, emit);
    }
};


// Quantised normalised layered min-sum (4-bit channel values and
// check-to-variable messages, 6-bit variable-to-check messages and APP values,
// magnitude floor(3/4 min)); the update is applied layer by layer in
// run_decode_l.  Padded edges read as a saturated positive message.
struct LnmsRule {
    static constexpr int kDummy = 31;
};

__device__ __forceinline__ int sat7(int x) { return x > 7 ? 7 : (x < -7 ? -7 : x); }
__device__ __forceinline__ int sat31(int x) { return x > 31 ? 31 : (x < -31 ? -31 : x); }

__device__ __forceinline__ int q4_impulse(int qb, int k) {
    // round_half_away(qb * (16 - k) / 16), saturated to [-7, 7]
    const long long nv = (long long)qb * (16 - k);
    const long long mag = ((nv < 0 ? -nv : nv) + 8) >> 4;
    long long q = nv < 0 ? -mag : mag;
    q = q > 7 ? 7 : (q < -7 ? -7 : q);
    return (int)q;
}

// Shared-memory layout of a frame (byte offsets): the channel values and a
// ring of three APP buffers (the layered decoder uses two of them).
struct Lds {
    int np, W, T;
    size_t lam, app, hist, imask, wsyn, pcnt, moved, extra, total;
};

__host__ __device__ inline Lds lds_layout(int n, int T, bool with_hist) {
    Lds L;
    L.np = (n + 1 + 63) & ~63;   // +1: slot n is the dummy target of padded edges
    L.W = L.np >> 6;
    L.T = T;
    size_t o = 0;
    L.lam = o;
    o += (size_t)L.np * 4;
    L.app = o;
    o += (size_t)3 * L.np * 4;
    o = (o + 15) & ~(size_t)15;
    L.hist = o;
    if (with_hist) o += (size_t)T * L.W * 8;
    L.imask = o;
    o += (size_t)L.W * 8;
    L.wsyn = o;
    o += (size_t)(T + 2) * 4;
    L.pcnt = o;
    o += (size_t)(T + 2) * 4;
    L.moved = o;
    o += (size_t)(T + 2) * 4;
    o = (o + 15) & ~(size_t)15;
    L.extra = o;   // IS: Philox normals of the TS bits (doubles) and the TS bits
    o += (size_t)kMaxWidth * 8 + (size_t)kMaxWidth * 4;
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

struct Frame {
    int *lam, *app;   // LDS: channel values; APP slots (np apart)
    unsigned long long *hist;   // nullable
    int *wsyn, *pcnt;
    int *moved;   // per iteration: a check message changed
    int *vsave;   // layered decoder: save area of the messages (B x CPT x DC), or nullptr
    int n, np, W, T;
};

struct DecRes {
    int fail, iters, tmin;
    int run;          // iterations computed (below iters when a fixed point ends the decode)
    int nerr;         // 1s in the final hard decision
    const int *app;   // LDS: the APP values of the decode's final hard decision
};

// The neighbours of the thread's checks (padded edges: n), as indices or, with
// kBytes, as byte offsets into an int32 array (the flooding decoder addresses
// both APP slots from them).
template <int DC, int CPT, bool kBytes = false>
__device__ __forceinline__ void load_neighbours(const DevCode &cd, int (&nb)[CPT][DC],
                                                const int *tab = nullptr) {
    const int B = blockDim.x, tid = threadIdx.x;
    if (!tab) tab = cd.cn_tab;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int chk = tid + c * B;
#pragma unroll
        for (int j = 0; j < DC; ++j) {
            int v = -1;
            if (chk < cd.m && j < cd.dc_pad) v = tab[(size_t)j * cd.m_tab + chk];
            nb[c][j] = (v < 0 ? cd.n : v) * (kBytes ? 4 : 1);
        }
    }
}

// One flooding decode.  On entry lam[] holds the channel values (slot n: the
// padding value), APP slots 0 and 1 equal lam[], wsyn/pcnt/moved are zero and
// all threads have passed a barrier.  Iteration t: each thread gathers
// APP_{t-1} (slot cur) for its checks, takes the syndrome bit of x_{t-1},
// applies the rule and adds the new messages into slot nxt (which holds lambda)
// with integer atomics; the hard decision x_{t-1} by ballot; the third slot is
// set to lambda for iteration t + 1; one barrier, then the stop tests.  Integer
// sums are exact and order-free.  The rule also reports each message's change
// (new - old): an iteration in which no message on a real edge changed leaves
// APP_t = APP_{t-1}, and every later iteration repeats it (fixed point).
// nb: byte offsets of the neighbours (padded edges: 4n).
template <class Rule, int DC, int CPT>
__device__ __forceinline__ DecRes run_decode(const Frame &F, const int (&nb)[CPT][DC],
                                             int (&c2v)[CPT][DC], int offset, int fp_exit) {
    const int n = F.n, np = F.np, W = F.W, T = F.T, n4 = F.n * 4;
    const int B = blockDim.x, NW = B >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int j = 0; j < DC; ++j) c2v[c][j] = 0;
    int cur = 0, nxt = 1, spare = 2;
    int iters = T, wmin = INT_MAX, tmin = 0, fixed = 0;
    const int *last = F.app;
    for (int t = 1; t <= T + 1; ++t) {
        const int *A = F.app + cur * np;
        last = A;   // APP_{t-1}: the final values when the decode ends in this iteration
        const char *Ab = (const char *)A;
        char *Nb = (char *)(F.app + nxt * np);
        int unsat = 0;
        unsigned chg = 0;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            int val[DC];
#pragma unroll
            for (int j = 0; j < DC; ++j) val[j] = *(const int *)(Ab + nb[c][j]);
            int par = 0;
#pragma unroll
            for (int j = 0; j < DC; ++j) par ^= (val[j] < 0);
            unsat += par;
            if (t <= T) {
                // Padded edges carry nothing (their dummy slot keeps its
                // value).  The per-edge branch also keeps each atomic next
                // to its message in the schedule: unconditional atomics were
                // issued as one block after the check's arithmetic, which
                // serialised LDS and VALU work (20% slower at 24 edges).
                const int *nbc = nb[c];
                Rule::template update<DC>(val, c2v[c], nb[c], n4, offset, [&](int j, int m, int d) {
                    if (nbc[j] != n4) {
                        atomicAdd((int *)(Nb + nbc[j]), m);
                        chg |= (unsigned)d;
                    }
                });
            }
        }
        if (t >= 2) {
            const int us = wave_sum_bits<count_bits(CPT)>(unsat);   // unsat <= CPT
            if (lane == 0 && us) atomicAdd(&F.wsyn[t - 1], us);
            int pc = 0;
            for (int i = wid; i < W; i += NW) {
                const int v = i * 64 + lane;
                const unsigned long long mask = __ballot((v < n) && (A[v] < 0));
                if (F.hist && lane == 0) F.hist[(size_t)(t - 2) * W + i] = mask;
                pc += __popcll(mask);
            }
            if (lane == 0 && pc) atomicAdd(&F.pcnt[t - 1], pc);
            if (__any(chg != 0u) && lane == 0) F.moved[t] = 1;
        }
        if (t < T) {
            int *S = F.app + spare * np;
            for (int v = tid; v < np; v += B) S[v] = F.lam[v];
        }
        __syncthreads();
        if (t >= 2) {
            const int w = F.wsyn[t - 1];
            if (w < wmin) {
                wmin = w;
                tmin = t - 1;
            }
            if (w == 0) {
                iters = t - 1;
                break;
            }
            if (fp_exit && t <= T && F.moved[t] == 0) {
                fixed = t;
                break;
            }
        }
        const int tmp = cur;
        cur = nxt;
        nxt = spare;
        spare = tmp;
    }
    if (fixed) {
        // No check message changed in iteration t = fixed, so APP_t = APP_{t-1}
        // and every later iteration repeats iteration t - 1 = run: the decode
        // ends at T as if run to the end.  Of the records after run only the
        // number of 1s at T is read here; the candidate writer reads history
        // row run - 1 (the hard decision x_run) for the later ones.
        if (tid == 0) F.pcnt[T] = F.pcnt[fixed - 1];
        __syncthreads();
    }
    DecRes r;
    r.iters = iters;
    r.tmin = tmin;
    r.nerr = F.pcnt[iters];
    r.fail = r.nerr > 0;
    r.run = fixed ? fixed - 1 : iters;
    r.app = last;
    return r;
}

// Writes the candidate error sets U_t = S(x_t) u I, t = t0..iters, of one
// failing decode to the record buffer (wavefront 0).  A record carries a
// multiplicity: consecutive equal sets share one record, and so does a set
// equal to one of the last kDedupSets sets recorded for the same pattern (in
// any of its decodes; in the critical extraction mode only at the same
// amplitude index), whose record then gains the multiplicity.  The sieve
// weighs each record by its multiplicity, so the outcome is that of one record
// per iteration.  dd: staging list and the pattern's cache (header scratch).
// Iterations after `run` repeat iteration `run` (fixed-point exit; their
// history rows are not written, row `run` stands for them): once the previous
// iteration was one of them, the rest only add to the multiplicity.
__device__ void write_candidates(const SearchLaunch &a, const unsigned long long *hist,
                                 const unsigned long long *imask, int W, int iters, int run,
                                 int pg, int k, int *dd) {
    if (threadIdx.x < 64) {
        const int lane = lane_id();
        int *stage = dd;
        int *cache = dd + kCapMax;
        // last >= 0: the current run's own record; -2: merged into record
        // `into`; -1: no record
        int last = -1, into = -1, mult = 0;
        auto finish = [&]() {
            if (lane == 0) {
                if (last >= 0) a.recs[(size_t)last * kRecStride + 3] = mult;
                else if (last == -2) atomicAdd(&a.recs[(size_t)into * kRecStride + 3], mult);
            }
        };
        for (int t = a.t0; t <= iters; ++t) {
            if (t > run && t > a.t0) {   // set(t) = set(t - 1) from here to iters
                if (last != -1) mult += iters - t + 1;
                break;
            }
            const unsigned long long *h = hist + (size_t)((t < run ? t : run) - 1) * W;
            int cnt = 0;
            for (int i = lane; i < W; i += 64) cnt += __popcll(h[i] | imask[i]);
            cnt = wave_sum(cnt);
            if (cnt > a.cap) {
                finish();
                last = -1;
                continue;
            }
            if (last != -1) {
                const unsigned long long *hp = h - W;
                int diff = 0;
                for (int i = lane; i < W; i += 64) diff |= ((h[i] | imask[i]) != (hp[i] | imask[i]));
                if (!__any(diff)) {
                    ++mult;
                    continue;
                }
                finish();
            }
            // the set's variables in ascending order
            int off = 0;
            for (int i0 = 0; i0 < W; i0 += 64) {
                const int i = i0 + lane;
                unsigned long long wv = i < W ? (h[i] | imask[i]) : 0ull;
                const int pc = __popcll(wv);
                int pos = off + wave_excl_scan(pc);
                while (wv) {
                    const int b = __ffsll((unsigned long long)wv) - 1;
                    stage[pos++] = i * 64 + b;
                    wv &= wv - 1;
                }
                off += wave_sum(pc);
            }
            wave_sync();
            int match = -1;
            for (int e = 0; e < kDedupSets && match < 0; ++e) {
                const int *ce = cache + e * kDedupStride;
                if (ce[0] >= 0 && ce[1] == cnt && (a.extract_mode != TS_EXTRACT_CRITICAL || ce[2] == k)) {
                    const bool eq = lane >= cnt || stage[lane] == ce[4 + lane];
                    if (__all(eq)) match = ce[0];
                }
            }
            if (match >= 0) {
                last = -2;
                into = match;
                mult = 1;
                continue;
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
            if (lane < cnt) rec[kRecHdr + lane] = stage[lane];
            // remember the set (entries replaced in turn; the turn is kept in
            // entry 0's spare word)
            const int v = cache[3];
            int *ce = cache + v * kDedupStride;
            wave_sync();
            if (lane < cnt) ce[4 + lane] = stage[lane];
            if (lane == 0) {
                ce[0] = r;
                ce[1] = cnt;
                ce[2] = k;
                cache[3] = (v + 1) % kDedupSets;
            }
            wave_sync();
            last = r;
            mult = 1;
        }
        finish();
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// impulse search: one pattern per workgroup, bisection on the amplitude
// ---------------------------------------------------------------------------
// Workgroup bound of a shape: small register footprints allow 1024 threads.
template <int DC, int CPT>
struct MaxBlock {
    static constexpr int value = DC * CPT <= 16 ? 1024 : (DC * CPT <= 48 ? 512 : 256);
};
template <int DC, int CPT>
struct MaxBlockIs {
    static constexpr int value = MaxBlock<DC, CPT>::value;
};

// Multi-job launches.  Thread 0 pops the next item of the launch and finds its
// job by binary search on the jobs' first items; a workgroup that moves on to
// another job copies that job's descriptor into the LDS header and rebinds its
// decoder (neighbour registers, frame layout).
template <class Job>
__device__ __forceinline__ void pop_item(const Job *jobs, int n_jobs, int *queue, int *sh) {
    if (threadIdx.x == 0) {
        const int it = atomicAdd(queue, 1);
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].item0 <= (long long)it) lo = mid;
            else hi = mid - 1;
        }
        sh[0] = it;
        sh[1] = lo;
    }
}

template <class Job>
__device__ __forceinline__ void load_job(const Job *jobs, int j, unsigned char *smem) {
    const int *src = (const int *)(jobs + j);
    int *dst = (int *)smem;
    for (int i = threadIdx.x; i < (int)(sizeof(Job) / 4); i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Common part of the impulse-search kernels: the pattern queue, the bisection on
// the impulse amplitude, the candidate write-out and the per-pattern results.
// Dec::decode(K) runs one decode of the current pattern (impulse bits in
// Dec::imask) at amplitude index K; Dec::hist() is its history of hard decisions.
template <class Dec>
__device__ __forceinline__ void search_jobs(const SearchJob *jobs, int n_jobs, int *queue,
                                            long long n_items, Dec &dec, unsigned char *smem) {
    const int B = blockDim.x, tid = threadIdx.x;
    const SearchJob &J = *(const SearchJob *)smem;
    const SearchLaunch &a = J.a;
    int *sh = (int *)(smem + kJobLds);
    unsigned char *frame = smem + kHdrLds;
    int cur = -1;
    unsigned long long my_iters = 0, my_dec = 0;
    for (;;) {
        __syncthreads();
        pop_item(jobs, n_jobs, queue, sh);
        __syncthreads();
        const int it = sh[0], j = sh[1];
        if ((long long)it >= n_items) break;
        if (j != cur) {
            if (cur >= 0 && tid == 0) {
                atomicAdd(&a.counters[0], my_dec);
                atomicAdd(&a.counters[1], my_iters);
            }
            my_iters = my_dec = 0;
            __syncthreads();
            load_job(jobs, j, smem);
            dec.bind(J, frame);
            __syncthreads();
            cur = j;
        }
        const int n = J.cd.n, W = dec.W;
        unsigned long long *imask = dec.imask;
        const int pl = it - (int)J.item0;
        for (int i = tid; i < W; i += B) imask[i] = 0ull;
        if (tid < kMaxWidth) sh[2 + tid] = tid < a.width ? a.patterns[(size_t)pl * a.width + tid] : -1;
        __syncthreads();
        if (tid < kMaxWidth) {
            const int v = sh[2 + tid];
            if (v >= n || v < -1) atomicOr(a.err, 1);
            else if (v >= 0) atomicOr(&imask[v >> 6], 1ull << (v & 63));
        }
        const int pg = a.pat_base + pl;
        if (tid == 0) {   // the pattern's cache of recorded sets starts empty
            for (int e = 0; e < kDedupSets; ++e) sh[32 + kCapMax + e * kDedupStride] = -1;
            sh[32 + kCapMax + 3] = 0;
        }
        DecRes r = dec.decode(a.k_max);
        my_iters += r.run;
        my_dec += 1;
        int kc = -1, it_hi = 0, tm_hi = 0, it_lo = r.iters;
        if (r.fail) {
            write_candidates(a, dec.hist(), imask, W, r.iters, r.run, pg, a.k_max, sh + 32);
            int lo = 0, hi = a.k_max;
            it_hi = r.iters;
            tm_hi = r.tmin;
            it_lo = 1;   // D(0) is the noiseless decode: success at the first iteration
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                r = dec.decode(mid);
                my_iters += r.run;
                my_dec += 1;
                if (r.fail) {
                    hi = mid;
                    it_hi = r.iters;
                    tm_hi = r.tmin;
                    write_candidates(a, dec.hist(), imask, W, r.iters, r.run, pg, mid, sh + 32);
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
    if (cur >= 0 && tid == 0) {
        atomicAdd(&a.counters[0], my_dec);
        atomicAdd(&a.counters[1], my_iters);
    }
}

// Channel value of an impulse frame: impulse bits get the amplitude-K value,
// all others the base value (Section III).
template <class Rule>
__device__ __forceinline__ int impulse_lambda(const SearchLaunch &a, int K) {
    if (std::is_same<Rule, OmsRule>::value) return q_impulse(a.q_base, K);
    if (std::is_same<Rule, LnmsRule>::value) return q4_impulse(a.q_base, K);
    return to_q20(a.h * (1.0f - (float)K / (float)a.k_den));
}

template <class Rule>
__device__ __forceinline__ int base_lambda(const SearchLaunch &a) {
    return std::is_same<Rule, SpaRule>::value ? to_q20(a.h) : a.q_base;
}

// Register-resident decoder of one workgroup: the neighbour lists and messages
// of the checks a thread owns stay in its registers.
template <class Rule, int DC, int CPT>
struct RegSearchDec {
    const SearchLaunch *a;
    Frame F;
    unsigned long long *imask;
    int W, offset, fp_exit;
    int nb[CPT][DC];
    int c2v[CPT][DC];

    __device__ __forceinline__ void bind(const SearchJob &J, unsigned char *frame) {
        a = &J.a;
        const int n = uni(J.cd.n), T = uni(J.a.max_iter);
        const Lds L = lds_layout(n, T, true);
        F.lam = (int *)(frame + L.lam);
        F.app = (int *)(frame + L.app);
        F.hist = (unsigned long long *)(frame + L.hist);
        F.wsyn = (int *)(frame + L.wsyn);
        F.pcnt = (int *)(frame + L.pcnt);
        F.moved = (int *)(frame + L.moved);
        F.vsave = nullptr;
        F.n = n;
        F.np = L.np;
        F.W = L.W;
        F.T = T;
        imask = (unsigned long long *)(frame + L.imask);
        W = L.W;
        offset = uni(J.a.offset);
        fp_exit = uni(J.a.fp_exit);
        load_neighbours<DC, CPT, true>(J.cd, nb);
    }

    __device__ __forceinline__ DecRes decode(int K) {
        const int B = blockDim.x, tid = threadIdx.x, n = F.n, np = F.np;
        const int li = impulse_lambda<Rule>(*a, K), lb = base_lambda<Rule>(*a);
        __syncthreads();
        for (int v = tid; v < np; v += B) {
            int l = v == n ? Rule::kDummy : 0;
            if (v < n) l = ((imask[v >> 6] >> (v & 63)) & 1ull) ? li : lb;
            F.lam[v] = l;
            F.app[v] = l;
            F.app[np + v] = l;
        }
        for (int i = tid; i < F.T + 2; i += B) {
            F.wsyn[i] = 0;
            F.pcnt[i] = 0;
            F.moved[i] = 0;
        }
        __syncthreads();
        return run_decode<Rule, DC, CPT>(F, nb, c2v, offset, fp_exit);
    }
    __device__ __forceinline__ const unsigned long long *hist() const { return F.hist; }
};

// Waves per SIMD the register allocator is asked to fit (1 = no request): one
// step above the natural occupancy of the sum-product shapes for which the few
// registers this frees are spilled only outside the decode loop (checked on
// the generated code; the other shapes would spill inside it).
template <class Rule, int DC, int CPT>
struct SearchWaves {
    static constexpr int value =
        !std::is_same<Rule, SpaRule>::value ? 1
        : (DC == 6 && CPT == 1) ? 7 : (DC == 6 && CPT == 2) ? 6 : (DC == 6 && CPT == 4) ? 4
        : (DC == 8 && CPT == 1) ? 6 : (DC == 8 && CPT == 2) ? 5 : (DC == 12 && CPT == 2) ? 4 : 1;
};
template <int DC, int CPT>
struct IsWaves {
    static constexpr int value = (DC == 6 && CPT == 1) ? 8 : (DC == 6 && CPT == 2) ? 6
                                 : (DC == 8 && CPT == 1) ? 7 : (DC == 8 && CPT == 2) ? 5
                                 : (DC == 12 && CPT == 1) ? 5 : 1;
};

template <class Rule, int DC, int CPT>
__global__ __launch_bounds__((MaxBlock<DC, CPT>::value))
__attribute__((amdgpu_waves_per_eu(SearchWaves<Rule, DC, CPT>::value))) void k_search(const SearchJob *jobs, int n_jobs,
                                                                      int *queue, long long n_items) {
    extern __shared__ __align__(16) unsigned char smem[];
    RegSearchDec<Rule, DC, CPT> dec;
    search_jobs(jobs, n_jobs, queue, n_items, dec, smem);
}

// One layered decode (register layout).  On entry APP slot 0 (LDS) holds the
// channel values (slot n: the padding value), wsyn/pcnt are zero and all
// threads have passed a barrier.  Per iteration the layers run in order, one
// barrier each: the checks of a layer touch disjoint variables, so each writes
// its variables' APP values in place.  Then the hard decision x_t, its
// syndrome and history, and the stop test.
template <int DC, int CPT>
__device__ __forceinline__ DecRes run_decode_l(const Frame &F, const int (&nb)[CPT][DC],
                                               const int (&lay)[CPT], int n_layers,
                                               int (&c2v)[CPT][DC]) {
    const int n = F.n, W = F.W, T = F.T;
    const int B = blockDim.x, NW = B >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int *A = F.app;
    int *S = F.app + F.np;   // APP at the start of a verifying sweep (LDS slot 1)
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int j = 0; j < DC; ++j) c2v[c][j] = 0;
    int iters = T, wmin = INT_MAX, tmin = 0, fixed = 0;
    bool verify = false;   // sweep t compares its end state with its start state
    for (int t = 1; t <= T; ++t) {
        if (verify) {
            int *vs = F.vsave + (unsigned)tid * (CPT * DC);
#pragma unroll
            for (int c = 0; c < CPT; ++c)
#pragma unroll
                for (int j = 0; j < DC; ++j) vs[c * DC + j] = c2v[c][j];
            for (int v = tid; v < F.np; v += B) S[v] = A[v];
            __syncthreads();   // the snapshot is complete before layer 0 writes A
        }
        for (int L = 0; L < n_layers; ++L) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (lay[c] != L) continue;
                int v2[DC];
                int mn1 = 31, mn2 = 31, idx = 0, sgn = 0;
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                    int x = sat31(A[nb[c][j]] - c2v[c][j]);
                    if (nb[c][j] == n) x = 31;
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
                    const int mag = sat7((3 * (j == idx ? mn2 : mn1)) >> 2);
                    const int m = (sgn ^ (v2[j] < 0)) ? -mag : mag;
                    c2v[c][j] = m;
                    if (nb[c][j] != n) A[nb[c][j]] = sat31(v2[j] + m);
                }
            }
            __syncthreads();
        }
        int unsat = 0;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (lay[c] < 0) continue;
            int par = 0;
#pragma unroll
            for (int j = 0; j < DC; ++j)
                if (nb[c][j] != n) par ^= (A[nb[c][j]] < 0);
            unsat += par;
        }
        const int us = wave_sum_bits<count_bits(CPT)>(unsat);   // unsat <= CPT
        if (lane == 0 && us) atomicAdd(&F.wsyn[t], us);
        int pc = 0;
        for (int i = wid; i < W; i += NW) {
            const int v = i * 64 + lane;
            const unsigned long long mask = __ballot((v < n) && (A[v] < 0));
            if (F.hist && lane == 0) F.hist[(size_t)(t - 1) * W + i] = mask;
            pc += __popcll(mask);
        }
        if (lane == 0 && pc) atomicAdd(&F.pcnt[t], pc);
        if (verify) {
            const int *vs = F.vsave + (unsigned)tid * (CPT * DC);
            unsigned chg = 0;   // padded edges carry nothing, so they are skipped
#pragma unroll
            for (int c = 0; c < CPT; ++c)
#pragma unroll
                for (int j = 0; j < DC; ++j)
                    if (nb[c][j] != n) chg |= (unsigned)(c2v[c][j] ^ vs[c * DC + j]);
            for (int v = tid; v < n; v += B) chg |= (unsigned)(A[v] ^ S[v]);
            if (__any(chg != 0u) && lane == 0) atomicOr(&F.moved[t], 1);
        }
        __syncthreads();
        const int w = F.wsyn[t];
        if (w < wmin) {
            wmin = w;
            tmin = t;
        }
        if (w == 0) {
            iters = t;
            break;
        }
        if (verify && F.moved[t] == 0) {
            // the sweep left every check message and APP value as it found
            // them: every later sweep repeats it (the decode ends at T)
            fixed = t;
            break;
        }
        // syndrome weight and number of 1s unchanged: check the next sweep
        verify = F.vsave && t >= 2 && t < T && w == F.wsyn[t - 1] && F.pcnt[t] == F.pcnt[t - 1];
    }
    if (fixed) {
        if (tid == 0) F.pcnt[T] = F.pcnt[fixed];
        __syncthreads();
    }
    DecRes r;
    r.iters = iters;
    r.tmin = tmin;
    r.nerr = F.pcnt[iters];
    r.fail = r.nerr > 0;
    r.run = fixed ? fixed : iters;
    r.app = F.app;
    return r;
}

template <int DC, int CPT>
struct LayDec {
    const SearchLaunch *a;
    Frame F;
    unsigned long long *imask;
    int W, n_layers;
    int nb[CPT][DC];
    int lay[CPT];
    int c2v[CPT][DC];

    __device__ __forceinline__ void bind(const SearchJob &J, unsigned char *frame) {
        a = &J.a;
        const int n = uni(J.cd.n), T = uni(J.a.max_iter);
        const Lds L = lds_layout(n, T, true);
        F.lam = nullptr;
        F.app = (int *)(frame + L.app);
        F.hist = (unsigned long long *)(frame + L.hist);
        F.wsyn = (int *)(frame + L.wsyn);
        F.pcnt = (int *)(frame + L.pcnt);
        F.moved = (int *)(frame + L.moved);
        F.vsave = !J.a.fp_exit ? nullptr
                  : J.a.save_lds ? (int *)(frame + L.total)
                  : J.a.gscr ? (int *)uni(J.a.gscr + (size_t)blockIdx.x * J.a.slot_bytes) : nullptr;
        F.n = n;
        F.np = L.np;
        F.W = L.W;
        F.T = T;
        imask = (unsigned long long *)(frame + L.imask);
        W = L.W;
        n_layers = uni(J.cd.n_layers);
        load_neighbours<DC, CPT>(J.cd, nb, J.cd.cn_lay);   // positions in layer order
        const int B = blockDim.x, tid = threadIdx.x, m = uni(J.cd.m);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int chk = tid + c * B;
            lay[c] = chk < m ? J.cd.lay_of[chk] : -1;
        }
    }

    __device__ __forceinline__ DecRes decode(int K) {
        const int B = blockDim.x, tid = threadIdx.x, n = F.n, np = F.np;
        const int li = impulse_lambda<LnmsRule>(*a, K), lb = base_lambda<LnmsRule>(*a);
        __syncthreads();
        for (int v = tid; v < np; v += B) {
            int l = v == n ? LnmsRule::kDummy : 0;
            if (v < n) l = ((imask[v >> 6] >> (v & 63)) & 1ull) ? li : lb;
            F.app[v] = l;
        }
        for (int i = tid; i < F.T + 2; i += B) {
            F.wsyn[i] = 0;
            F.pcnt[i] = 0;
            F.moved[i] = 0;
        }
        __syncthreads();
        return run_decode_l<DC, CPT>(F, nb, lay, n_layers, c2v);
    }
    __device__ __forceinline__ const unsigned long long *hist() const { return F.hist; }
};

// Occupancy the layered kernels keep with the fixed-point test's registers.
template <int DC, int CPT>
struct LayWaves {
    static constexpr int value = (DC == 6 && CPT == 1) ? 6 : (DC == 6 && CPT == 2) ? 5 : 1;
};

template <int DC, int CPT>
__global__ __launch_bounds__((MaxBlock<DC, CPT>::value))
__attribute__((amdgpu_waves_per_eu(LayWaves<DC, CPT>::value))) void k_search_l(const SearchJob *jobs, int n_jobs,
                                                                       int *queue, long long n_items) {
    extern __shared__ __align__(16) unsigned char smem[];
    LayDec<DC, CPT> dec;
    search_jobs(jobs, n_jobs, queue, n_items, dec, smem);
}

// ---------------------------------------------------------------------------
// importance-sampling frames: sum-product on Philox noise
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

// Channel parameters of the IS frames of one job (scalar copies).
struct IsChan {
    unsigned k0, k1, stream;
    int a, n_mix;
    float shift, sigma, two_over_s2;
    unsigned long long frame_base;
    long long n_frames;
    double mix_s0, mix_ds;
};

// The mean shift of frame f: the job's shift, or its mixture component's.
__device__ __forceinline__ float frame_shift(const IsChan &a, int f) {
    if (!a.n_mix) return a.shift;
    const long long j = ((long long)f * a.n_mix) / a.n_frames;
    return (float)(a.mix_s0 + (double)j * a.mix_ds);
}

__device__ __forceinline__ IsChan is_chan(const IsDev &d) {
    IsChan c;
    c.k0 = uni((unsigned)d.seed);
    c.k1 = uni((unsigned)(d.seed >> 32));
    c.stream = uni(d.stream);
    c.a = uni(d.a);
    c.shift = uni((float)d.shift);
    c.sigma = uni((float)d.sigma);
    c.two_over_s2 = uni((float)(2.0 / d.sigma2));
    c.frame_base = uni(d.frame_base);
    c.n_frames = uni(d.n_frames);
    c.n_mix = uni(d.n_mix);
    c.mix_s0 = uni(d.mix_s0);
    c.mix_ds = uni(d.mix_ds);
    return c;
}

// Channel of IS frame `frame` (Section II, mean-shifted noise on the TS bits):
// y_v = 1 - s [v in T] + sigma n_v with n_v from Philox4x32-10 at counter
// (v >> 2, frame, stream) and Box-Muller on u = (x + 0.5) 2^-32, in float32
// (the channel values are then rounded to the Q20 grid, 2^-20, far coarser than
// the float32 error of the normals), lambda_v = 2 y_v / sigma^2.  put(v, lambda)
// stores the values; the normals of the TS bits go to tn.
template <class Put>
__device__ __forceinline__ void is_channel(const IsChan &a, int n, unsigned long long frame,
                                           float shift, const int *tsl, float *tn, Put put) {
    const int B = blockDim.x, tid = threadIdx.x;
    const float two_pi = 6.2831853071795865f;
    for (int g = tid; 4 * g < n; g += B) {
        unsigned c[4] = {(unsigned)g, (unsigned)frame, (unsigned)(frame >> 32), a.stream};
        philox4x32_10(c, a.k0, a.k1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float u0 = ((float)c[2 * h] + 0.5f) * 0x1p-32f;
            const float u1 = ((float)c[2 * h + 1] + 0.5f) * 0x1p-32f;
            const float r = sqrtf(-2.0f * logf(u0));
            float sn, cs;
            sincosf(two_pi * u1, &sn, &cs);
            const float nv[2] = {r * cs, r * sn};
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int v = 4 * g + 2 * h + i;
                if (v >= n) break;
                int slot = -1;
                for (int q = 0; q < a.a; ++q)
                    if (tsl[q] == v) slot = q;
                const float y = 1.0f - (slot >= 0 ? shift : 0.0f) + a.sigma * nv[i];
                put(v, to_q20(y * a.two_over_s2));
                if (slot >= 0) tn[slot] = nv[i];
            }
        }
    }
}

// A finished frame (thread 0): its flags (bit 0 the decode failed, bit 1 it
// ended in the set's own error event: every TS bit decided 1 and at most 2a
// bits in error in all) and the sum of the normals of its TS bits, from which
// the reduction forms the importance weight.
__device__ __forceinline__ void is_finish(const IsDev &a, int f, const DecRes &r, const float *tn,
                                          const int *tsl) {
    double st = 0.0;
    int t_err = r.fail && r.nerr <= 2 * a.a;
    for (int q = 0; q < a.a; ++q) {
        st += (double)tn[q];
        t_err &= r.app[tsl[q]] < 0;
    }
    a.fail[f] = (unsigned char)(r.fail | (t_err << 1));
    a.wf[f] = st;
}

// Common part of the IS kernels: the frame queue over the launch's jobs and
// the per-frame weights.  Dec::decode_frame(f) builds frame f's channel and
// decodes it; Dec::tn holds the normals of the TS bits.
template <class Dec>
__device__ __forceinline__ void is_jobs(const IsJob *jobs, int n_jobs, int *queue, long long n_items,
                                        Dec &dec, unsigned char *smem) {
    const int tid = threadIdx.x;
    const IsJob &J = *(const IsJob *)smem;
    int *sh = (int *)(smem + kJobLds);
    unsigned char *frame = smem + kHdrLds;
    int cur = -1;
    unsigned long long my_iters = 0;
    for (;;) {
        __syncthreads();
        pop_item(jobs, n_jobs, queue, sh);
        __syncthreads();
        const int it = sh[0], j = sh[1];
        if ((long long)it >= n_items) break;
        if (j != cur) {
            if (cur >= 0 && tid == 0) atomicAdd(&J.a.counters[1], my_iters);
            my_iters = 0;
            __syncthreads();
            load_job(jobs, j, smem);
            dec.bind(J, frame);
            __syncthreads();
            cur = j;
        }
        const int f = it - (int)J.item0;
        const DecRes r = dec.decode_frame(f);
        my_iters += r.run;
        if (tid == 0) is_finish(J.a, f, r, dec.tn, dec.tsl);
    }
    if (cur >= 0 && tid == 0) atomicAdd(&J.a.counters[1], my_iters);
}

template <int DC, int CPT>
struct RegIsDec {
    IsChan a;
    Frame F;
    float *tn;
    int *tsl;
    int fp_exit;
    int nb[CPT][DC];
    int c2v[CPT][DC];

    __device__ __forceinline__ void bind(const IsJob &J, unsigned char *frame) {
        a = is_chan(J.a);
        const int n = uni(J.cd.n), T = uni(J.a.max_iter);
        const Lds L = lds_layout(n, T, false);
        F.lam = (int *)(frame + L.lam);
        F.app = (int *)(frame + L.app);
        F.hist = nullptr;
        F.wsyn = (int *)(frame + L.wsyn);
        F.pcnt = (int *)(frame + L.pcnt);
        F.moved = (int *)(frame + L.moved);
        F.vsave = nullptr;
        F.n = n;
        F.np = L.np;
        F.W = L.W;
        F.T = T;
        fp_exit = uni(J.a.fp_exit);
        tn = (float *)(frame + L.extra);
        tsl = (int *)(tn + kMaxWidth);
        const int tid = threadIdx.x;
        if (tid < kMaxWidth) tsl[tid] = tid < J.a.a ? J.a.ts[tid] : -1;
        load_neighbours<DC, CPT, true>(J.cd, nb);
    }

    __device__ __forceinline__ DecRes decode_frame(int f) {
        const int B = blockDim.x, tid = threadIdx.x, n = F.n, np = F.np;
        is_channel(a, n, a.frame_base + (unsigned long long)f, frame_shift(a, f), tsl, tn, [&](int v, int l) {
            F.lam[v] = l;
            F.app[v] = l;
            F.app[np + v] = l;
        });
        for (int v = n + tid; v < np; v += B) {
            F.lam[v] = SpaRule::kDummy;
            F.app[v] = SpaRule::kDummy;
            F.app[np + v] = SpaRule::kDummy;
        }
        for (int i = tid; i < F.T + 2; i += B) {
            F.wsyn[i] = 0;
            F.pcnt[i] = 0;
            F.moved[i] = 0;
        }
        __syncthreads();
        return run_decode<SpaIsRule, DC, CPT>(F, nb, c2v, 0, fp_exit);
    }
};

template <int DC, int CPT>
__global__ __launch_bounds__((MaxBlockIs<DC, CPT>::value))
__attribute__((amdgpu_waves_per_eu(IsWaves<DC, CPT>::value))) void k_is(const IsJob *jobs, int n_jobs,
                                                                    int *queue, long long n_items) {
    extern __shared__ __align__(16) unsigned char smem[];
    RegIsDec<DC, CPT> dec;
    is_jobs(jobs, n_jobs, queue, n_items, dec, smem);
}

// Fixed-order reduction over the frames of the importance weights
// w_f = [frame f failed] exp(-a s^2 / (2 sigma^2) + (s / sigma) sum_{v in T} n_v)
// (wf holds the sums of the TS-bit normals).  Stage 1: workgroup g takes the
// contiguous frame range of chunk g, each thread a contiguous sub-range in frame
// order, combined by a fixed binary tree into part[g].  Stage 2: one workgroup
// combines the parts the same way.  The order depends on n only.
// mode 0: out = {sum w, sum w^2, failures}; mode 1: out[3] = sum (w - mean)^2.
constexpr int kRedThreads = 256;
constexpr long long kRedChunk = 16384;   // frames per stage-1 workgroup

__device__ __forceinline__ void red_tree(double *s0, double *s1, double *s2, int t) {
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
            s2[t] += s2[t + h];
        }
        __syncthreads();
    }
}

// Importance weight of a counted frame f of a mixture of m shifts s_k = s0 + k ds
// (frame f drawn from component j = f m / n): with S = a s_j / sigma - sum_T n,
// the sum of the frame's TS-bit displacements in units of sigma,
// w = 1 / sum_k alpha_k exp((s_k / sigma) S - a s_k^2 / (2 sigma^2)), alpha_k the
// share of frames in component k (the balance heuristic), by log-sum-exp.
__device__ __forceinline__ double mix_term(const MixW &x, int k, double S) {
    const long long f0 = (k * x.n + x.m - 1) / x.m, f1 = ((k + 1) * x.n + x.m - 1) / x.m;
    const double sk = x.s0 + (double)k * x.ds;
    return log((double)(f1 - f0) / (double)x.n) + sk / x.sigma * S - x.a * sk * sk / (2.0 * x.sigma * x.sigma);
}
__device__ double mix_weight(const MixW &x, long long f, double sum_n) {
    const long long j = (f * x.m) / x.n;
    const double S = x.a * (x.s0 + (double)j * x.ds) / x.sigma - sum_n;
    double mx = -1e300;
    for (int k = 0; k < x.m; ++k) mx = fmax(mx, mix_term(x, k, S));
    double t = 0.0;
    for (int k = 0; k < x.m; ++k) t += exp(mix_term(x, k, S) - mx);
    return exp(-(mx + log(t)));
}

// Stage 1 of a job's reduction: block blk of its frames (kRedChunk frames,
// a fixed split over the threads and a fixed tree, so the sums do not depend
// on the launch).  cmask selects the failures that count: 1 every failure,
// 2 those with every TS bit in error.  Mode 1 takes the mean weight from the
// job's mode-0 result on the device.
__device__ void reduce_frames(const RedJob &j, int mode, int blk) {
    __shared__ double s0[kRedThreads], s1[kRedThreads], s2[kRedThreads];
    const int t = threadIdx.x;
    const long long n = j.n;
    const double mean = mode ? j.out[0] / (double)n : 0.0;
    const long long c0 = (long long)blk * kRedChunk;
    const long long c1 = c0 + kRedChunk < n ? c0 + kRedChunk : n;
    const long long per = (kRedChunk + kRedThreads - 1) / kRedThreads;
    const long long lo = c0 + (long long)t * per, hi = lo + per < c1 ? lo + per : c1;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (long long i = lo; i < hi; ++i) {
        const bool counted = (j.fail[i] & j.cmask) != 0;
        const double w = !counted ? 0.0 : j.mix.m ? mix_weight(j.mix, i, j.wf[i]) : exp(j.wconst + j.coef * j.wf[i]);
        if (mode == 0) {
            a0 += w;
            a1 += w * w;
            a2 += counted ? 1.0 : 0.0;
        } else {
            a0 += (w - mean) * (w - mean);
        }
    }
    s0[t] = a0;
    s1[t] = a1;
    s2[t] = a2;
    red_tree(s0, s1, s2, t);
    if (t == 0) {
        j.part[3 * blk] = s0[0];
        j.part[3 * blk + 1] = s1[0];
        j.part[3 * blk + 2] = s2[0];
    }
}

// Stage 2: the job's partial sums in a fixed order; mode 0 writes out[0..2]
// (sum w, sum w^2, counted failures), mode 1 out[3] (sum (w - mean)^2).
__device__ void reduce_parts(const RedJob &j, int mode) {
    __shared__ double s0[kRedThreads], s1[kRedThreads], s2[kRedThreads];
    const int t = threadIdx.x;
    const int per = (j.np + kRedThreads - 1) / kRedThreads;
    const int lo = t * per, hi = lo + per < j.np ? lo + per : j.np;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = lo; i < hi; ++i) {
        a0 += j.part[3 * i];
        a1 += j.part[3 * i + 1];
        a2 += j.part[3 * i + 2];
    }
    s0[t] = a0;
    s1[t] = a1;
    s2[t] = a2;
    red_tree(s0, s1, s2, t);
    if (t == 0) {
        if (mode == 0) {
            j.out[0] = s0[0];
            j.out[1] = s1[0];
            j.out[2] = s2[0];
        } else {
            j.out[3] = s0[0];
        }
    }
}

__global__ __launch_bounds__(kRedThreads) void k_is_reduce(RedJob j, int mode) {
    reduce_frames(j, mode, blockIdx.x);
}
__global__ __launch_bounds__(kRedThreads) void k_is_reduce_final(RedJob j, int mode) { reduce_parts(j, mode); }

// Many jobs in one launch: block b belongs to the last job whose part0 <= b.
__global__ __launch_bounds__(kRedThreads) void k_is_reduce_jobs(const RedJob *jobs, int nj, int mode) {
    const int b = blockIdx.x;
    int lo = 0, hi = nj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].part0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const RedJob j = jobs[lo];
    reduce_frames(j, mode, b - j.part0);
}
__global__ __launch_bounds__(kRedThreads) void k_is_reduce_final_jobs(const RedJob *jobs, int mode) {
    const RedJob j = jobs[blockIdx.x];
    reduce_parts(j, mode);
}

__global__ void k_fill(int *p, int value, long long count) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// ---------------------------------------------------------------------------
// streamed frames: codes whose messages do not fit in registers
// ---------------------------------------------------------------------------
// One workgroup per frame as above, but the check-to-variable messages stream
// through a per-workgroup scratch area in global memory, and the APP values are
// rebuilt from them in a second pass per iteration instead of by atomics:
//   check pass  (thread per check, checks sorted into degree classes): gather
//               APP_{t-1} from LDS, take the syndrome bit of x_{t-1}, read the
//               old messages, apply the check rule, write the new messages;
//   variable pass (thread per variable, wave-contiguous): APP_t = lambda + sum
//               of the variable's new messages, hard decision by ballot.
// Messages are stored edge-major within a class (slot j of consecutive checks
// adjacent), so both passes read and write them coalesced; for a QC code the
// variable pass gathers from consecutive rows of each circulant.  The integer
// arithmetic (int8 / Q20 messages, int32 sums) is that of the register-resident
// decoder, so both give identical results.
struct GFrame {
    int *app;                          // LDS [np]
    const unsigned long long *imask;   // LDS impulse bits (search) or nullptr
    const int *lam_g;                  // global channel values (IS) or nullptr
    int lam_base, lam_imp;
    void *msg;                         // global message slots of this workgroup
    unsigned long long *hist;          // global [T][W] or nullptr
    int *wsyn, *pcnt;                  // LDS
    int *moved;                        // LDS per iteration: a check message changed
    int fp_exit;                       // end the decode at a fixed point
    const int *cdc, *cc0, *cstr, *coff;   // LDS copy of the class table
    const int *g_cn, *g_vslot;         // the code's slot tables
    int ncls, n, np, W, T, m, dv_pad, n_tab;
    int *acc;                          // LDS [np] APP - lambda sums (accumulating variant) or nullptr
    // QC codes: indices computed from the LDS copy of the per-circulant tables
    const int *qtab, *rowpos;
    int qc, qdc, qdv, qvar, z;
    float inv_z;
};

__device__ __forceinline__ int g_lambda(const GFrame &F, int v) {
    if (F.lam_g) return F.lam_g[v];
    return ((F.imask[v >> 6] >> (v & 63)) & 1ull) ? F.lam_imp : F.lam_base;
}

// Check pass of one check (sorted position p, class q); returns the parity of
// the hard decisions of APP_{t-1} on its variables.  chg gathers the bits of
// the changes (new - old) of the messages on real edges (read from t = 2 on).
template <class Rule, int DC, class M, bool kAcc>
__device__ __forceinline__ int check_g(const GFrame &F, int q, int p, int t, int offset,
                                       unsigned &chg) {
    const int stride = F.cstr[q];
    const size_t base = (size_t)F.coff[q] + (size_t)(p - F.cc0[q]);
    int nb[DC], val[DC], c2v[DC];
    if (F.qc) {
        const int rp = F.rowpos[p];
        const int *e = F.qtab + 2 * (rp >> 16) * F.qdc;
#pragma unroll
        for (int j = 0; j < DC; ++j) nb[j] = qc_neighbour(e + 2 * j, rp & 0xffff, F.z, F.n);
    } else {
#pragma unroll
        for (int j = 0; j < DC; ++j) nb[j] = F.g_cn[base + (size_t)j * stride];
    }
#pragma unroll
    for (int j = 0; j < DC; ++j) val[j] = F.app[nb[j]];
    int par = 0;
#pragma unroll
    for (int j = 0; j < DC; ++j) par ^= (val[j] < 0);
    if (t <= F.T) {
        M *msg = (M *)F.msg;
#pragma unroll
        for (int j = 0; j < DC; ++j) c2v[j] = t == 1 ? 0 : (int)msg[base + (size_t)j * stride];
        // the sum-product rule without the wavefront-uniform shortcuts: they
        // save arithmetic that this memory-bound pass does not wait on, and
        // their registers spill here
        // the changes are kept and the messages stored after the rule (stores
        // and atomics inside it cost this pass registers)
        int dv[DC];
        auto keep = [&](int j, int, int d) { dv[j] = d; };
        if constexpr (std::is_same<Rule, SpaRule>::value) SpaRule::update_impl<DC, false>(val, c2v, keep);
        else Rule::template update<DC>(val, c2v, nb, F.n, offset, keep);
#pragma unroll
        for (int j = 0; j < DC; ++j) {
            msg[base + (size_t)j * stride] = (M)c2v[j];
            if (nb[j] != F.n) chg |= (unsigned)dv[j];
        }
        if constexpr (kAcc) {
            // APP_t - lambda accumulated in LDS (exact integer sums, any order)
#pragma unroll
            for (int j = 0; j < DC; ++j)
                if (nb[j] != F.n) atomicAdd(&F.acc[nb[j]], c2v[j]);
        }
    }
    return par;
}

// One decode of a streamed frame.  On entry APP (LDS) holds the channel values
// (slot n: the padding value), wsyn/pcnt are zero, all threads passed a barrier.
template <class Rule, int DCMAX, class M, bool kAcc>
__device__ DecRes run_decode_g(const GFrame &F, int offset) {
    const int n = F.n, W = F.W, T = F.T, mm = F.m;
    const int B = blockDim.x, NW = B >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const M *msg = (const M *)F.msg;
    int iters = T, wmin = INT_MAX, tmin = 0, fixed = 0;
    for (int t = 1; t <= T + 1; ++t) {
        int unsat = 0, q = 0;
        unsigned chg = 0;
        for (int p = tid; p < mm; p += B) {
            while (q + 1 < F.ncls && p >= F.cc0[q + 1]) ++q;
            int par = 0;
            switch (F.cdc[q]) {
#define TSG_GCASE(D)                                                             \
    case D:                                                                      \
        if constexpr (D <= DCMAX && !(DCMAX == 32 && D == 24))                   \
            par = check_g<Rule, D, M, kAcc>(F, q, p, t, offset, chg);            \
        break;
                TSG_GCASE(3) TSG_GCASE(4) TSG_GCASE(6) TSG_GCASE(8)
                TSG_GCASE(12) TSG_GCASE(16) TSG_GCASE(24) TSG_GCASE(32)
#undef TSG_GCASE
                default: break;
            }
            unsat += par;
        }
        if (t >= 2) {
            const int us = wave_sum(unsat);
            if (lane == 0 && us) atomicAdd(&F.wsyn[t - 1], us);
            if (__any(chg != 0u) && lane == 0) F.moved[t] = 1;
        }
        __syncthreads();
        if (t >= 2) {
            const int w = F.wsyn[t - 1];
            if (w < wmin) {
                wmin = w;
                tmin = t - 1;
            }
            if (w == 0) {
                iters = t - 1;
                break;
            }
            // no check message changed in iteration t: APP_t = APP_{t-1}, and
            // every later iteration repeats iteration t - 1 (fixed point)
            if (F.fp_exit && t <= T && F.moved[t] == 0) {
                fixed = t;
                break;
            }
        }
        if (t > T) break;
        int pc = 0;
        for (int i = wid; i < W; i += NW) {
            const int v = i * 64 + lane;
            int x = 0;
            if (v < n && kAcc) {
                const int sum = g_lambda(F, v) + F.acc[v];
                F.acc[v] = 0;
                F.app[v] = sum;
                x = sum < 0;
            } else if (v < n) {
                int sum = g_lambda(F, v);
                if (F.qc) {
                    // block column by a float estimate of v / z, corrected to exact
                    int jc = (int)((float)v * F.inv_z);
                    if (jc * F.z > v) --jc;
                    else if ((jc + 1) * F.z <= v) ++jc;
                    const int cc = v - jc * F.z;
                    const int *e = F.qtab + F.qvar + 2 * jc * F.qdv;
                    for (int k = 0; k < F.qdv; ++k) {
                        const int s = qc_slot(e + 2 * k, cc, F.z);
                        if (s >= 0) sum += (int)msg[s];
                    }
                } else {
                    for (int k = 0; k < F.dv_pad; ++k) {
                        const int e = F.g_vslot[(size_t)k * F.n_tab + v];
                        if (e >= 0) sum += (int)msg[e];
                    }
                }
                F.app[v] = sum;
                x = sum < 0;
            }
            const unsigned long long mask = __ballot(x);
            if (F.hist && lane == 0) F.hist[(size_t)(t - 1) * W + i] = mask;
            pc += __popcll(mask);
        }
        if (lane == 0 && pc) atomicAdd(&F.pcnt[t], pc);
        __syncthreads();
    }
    if (fixed) {
        // as in run_decode: the decode ends at T as if run to the end; the
        // history rows after `run` are not written (the candidate writer
        // reads row `run` for them)
        if (tid == 0) F.pcnt[T] = F.pcnt[fixed - 1];
        __syncthreads();
    }
    DecRes r;
    r.iters = iters;
    r.tmin = tmin;
    r.nerr = F.pcnt[iters];
    r.fail = r.nerr > 0;
    r.run = fixed ? fixed - 1 : iters;
    r.app = F.app;   // APP_{t-1} of the iteration that ended the decode
    return r;
}

// Binds a streamed frame to a job: LDS regions, the workgroup's scratch slot,
// the code's tables and an LDS copy of its class table.
__device__ __forceinline__ void g_bind(const DevCode &cd, int T, unsigned char *frame,
                                       unsigned char *slot, GFrame &F, LdsG &L, bool acc) {
    const int n = uni(cd.n);
    T = uni(T);
    const int qc = uni(cd.q_ok);
    L = lds_layout_g(n, T, qc ? uni(cd.q_bytes) : 0, acc);
    F.acc = acc ? (int *)(frame + L.acc) : nullptr;
    int *cls = (int *)(frame + L.cls);
    const int tid = threadIdx.x;
    if (tid < kGMaxCls) {
        cls[tid] = cd.g_dc[tid];
        cls[2 * kGMaxCls + 1 + tid] = cd.g_stride[tid];
    }
    if (tid < kGMaxCls + 1) {
        cls[kGMaxCls + tid] = cd.g_c0[tid];
        cls[3 * kGMaxCls + 1 + tid] = cd.g_off[tid];
    }
    F.cdc = cls;
    F.cc0 = cls + kGMaxCls;
    F.cstr = cls + 2 * kGMaxCls + 1;
    F.coff = cls + 3 * kGMaxCls + 1;
    F.ncls = uni(cd.g_ncls);
    F.g_cn = uni(cd.g_cn);
    F.g_vslot = uni(cd.g_vslot);
    F.m = uni(cd.m);
    F.dv_pad = uni(cd.dv_pad);
    F.n_tab = uni(cd.n_tab);
    F.app = (int *)(frame + L.app);
    F.wsyn = (int *)(frame + L.wsyn);
    F.pcnt = (int *)(frame + L.pcnt);
    F.moved = (int *)(frame + L.moved);
    F.msg = uni(slot);
    F.n = n;
    F.np = L.np;
    F.W = L.W;
    F.T = T;
    F.qc = qc;
    F.qtab = nullptr;
    F.rowpos = nullptr;
    if (qc) {
        int *qt = (int *)(frame + L.qtab);
        const int words = uni(cd.q_bytes) >> 2;
        const int *src = uni(cd.q_tab);
        for (int i = tid; i < words; i += blockDim.x) qt[i] = src[i];
        F.qtab = qt;
        F.rowpos = uni(cd.q_rowpos);
        F.qdc = uni(cd.q_dc);
        F.qdv = uni(cd.q_dv);
        F.qvar = uni(cd.q_var_off);
        F.z = uni(cd.z);
        F.inv_z = uni(cd.q_inv_z);
    }
}

template <class Rule, int DCMAX, class M, bool kAcc>
struct GSearchDec {
    const SearchLaunch *a;
    GFrame F;
    unsigned long long *imask;
    int W;

    __device__ __forceinline__ void bind(const SearchJob &J, unsigned char *frame) {
        a = &J.a;
        unsigned char *slot = J.a.gscr + (size_t)blockIdx.x * J.a.slot_bytes;
        LdsG L;
        g_bind(J.cd, J.a.max_iter, frame, slot, F, L, kAcc);
        imask = (unsigned long long *)(frame + L.imask);
        W = L.W;
        F.imask = imask;
        F.fp_exit = uni(J.a.fp_exit);
        F.lam_g = nullptr;
        F.lam_base = base_lambda<Rule>(J.a);
        F.lam_imp = F.lam_base;
        F.hist = (unsigned long long *)(slot + J.a.hist_off);
    }

    __device__ __forceinline__ DecRes decode(int K) {
        const int B = blockDim.x, tid = threadIdx.x, n = F.n;
        F.lam_imp = impulse_lambda<Rule>(*a, K);
        __syncthreads();
        for (int v = tid; v < F.np; v += B) F.app[v] = v < n ? g_lambda(F, v) : Rule::kDummy;
        if constexpr (kAcc)
            for (int v = tid; v < F.np; v += B) F.acc[v] = 0;
        for (int i = tid; i < F.T + 2; i += B) {
            F.wsyn[i] = 0;
            F.pcnt[i] = 0;
            F.moved[i] = 0;
        }
        __syncthreads();
        return run_decode_g<Rule, DCMAX, M, kAcc>(F, a->offset);
    }
    __device__ __forceinline__ const unsigned long long *hist() const { return F.hist; }
};

// Workgroup bounds of the streamed kernels (the register budget follows).
// (the accumulating variant keeps the neighbour indices live across the
// update, so it takes at most 512 threads and twice the registers)
template <int DCMAX, bool kAcc = false> struct MaxBlockG {
    static constexpr int value = (DCMAX <= 16 && !kAcc) ? 1024 : 512;
};
template <int DCMAX, bool kAcc = false> struct MaxBlockGIs { static constexpr int value = MaxBlockG<DCMAX, kAcc>::value; };

// kAcc: the accumulating variant (APP sums by LDS atomics in the check pass;
// the variable pass reads no messages), for frames whose two LDS arrays fit.
template <class Rule, int DCMAX, bool kAcc>
__global__ __launch_bounds__((MaxBlockG<DCMAX, kAcc>::value)) void k_search_g(const SearchJob *jobs, int n_jobs,
                                                                       int *queue, long long n_items) {
    typedef typename std::conditional<Rule::kDummy == OmsRule::kDummy, signed char, int>::type M;
    extern __shared__ __align__(16) unsigned char smem[];
    GSearchDec<Rule, DCMAX, M, kAcc> dec;
    search_jobs(jobs, n_jobs, queue, n_items, dec, smem);
}

template <int DCMAX, bool kAcc>
struct GIsDec {
    IsChan a;
    GFrame F;
    int *lam;
    float *tn;
    int *tsl;

    __device__ __forceinline__ void bind(const IsJob &J, unsigned char *frame) {
        a = is_chan(J.a);
        unsigned char *slot = J.a.gscr + (size_t)blockIdx.x * J.a.slot_bytes;
        LdsG L;
        g_bind(J.cd, J.a.max_iter, frame, slot, F, L, kAcc);
        lam = uni((int *)(slot + J.a.lam_off));
        F.imask = nullptr;
        F.fp_exit = uni(J.a.fp_exit);
        F.lam_g = lam;
        F.lam_base = F.lam_imp = 0;
        F.hist = nullptr;
        tn = (float *)(frame + L.extra);
        tsl = (int *)(tn + kMaxWidth);
        const int tid = threadIdx.x;
        if (tid < kMaxWidth) tsl[tid] = tid < J.a.a ? J.a.ts[tid] : -1;
    }

    __device__ __forceinline__ DecRes decode_frame(int f) {
        const int B = blockDim.x, tid = threadIdx.x, n = F.n;
        int *lm = lam;
        int *app = F.app;
        is_channel(a, n, a.frame_base + (unsigned long long)f, frame_shift(a, f), tsl, tn, [&](int v, int l) {
            lm[v] = l;
            app[v] = l;
        });
        for (int v = n + tid; v < F.np; v += B) F.app[v] = SpaRule::kDummy;
        if constexpr (kAcc)
            for (int v = tid; v < F.np; v += B) F.acc[v] = 0;
        for (int i = tid; i < F.T + 2; i += B) {
            F.wsyn[i] = 0;
            F.pcnt[i] = 0;
            F.moved[i] = 0;
        }
        __syncthreads();
        return run_decode_g<SpaIsRule, DCMAX, int, kAcc>(F, 0);
    }
};

template <int DCMAX, bool kAcc>
__global__ __launch_bounds__((MaxBlockGIs<DCMAX, kAcc>::value)) void k_is_g(const IsJob *jobs, int n_jobs,
                                                                     int *queue, long long n_items) {
    extern __shared__ __align__(16) unsigned char smem[];
    GIsDec<DCMAX, kAcc> dec;
    is_jobs(jobs, n_jobs, queue, n_items, dec, smem);
}

// ---------------------------------------------------------------------------
// kernel table
// ---------------------------------------------------------------------------
typedef void (*SearchKernel)(const SearchJob *, int, int *, long long);
typedef void (*IsKernel)(const IsJob *, int, int *, long long);

struct KEntry {
    int dc, cpt, max_block, is_max_block;
    SearchKernel oms, spa, lnms;
    IsKernel is;
};

#define TSG_K(DC, CPT)                                                                \
    {DC, CPT, MaxBlock<DC, CPT>::value, MaxBlockIs<DC, CPT>::value, k_search<OmsRule, DC, CPT>, \
     k_search<SpaRule, DC, CPT>, k_search_l<DC, CPT>, k_is<DC, CPT>}
const KEntry kTable[] = {
    TSG_K(6, 1),  TSG_K(6, 2),  TSG_K(6, 4),  TSG_K(6, 8),  TSG_K(8, 1),  TSG_K(8, 2),
    TSG_K(8, 4),  TSG_K(8, 8),  TSG_K(12, 1), TSG_K(12, 2), TSG_K(12, 4), TSG_K(16, 1),
    TSG_K(16, 2), TSG_K(16, 4), TSG_K(24, 1), TSG_K(24, 2), TSG_K(32, 1), TSG_K(32, 2),
};
#undef TSG_K

// streamed-frame kernels, by largest check-degree class
struct GEntry {
    int dcmax, max_block[2], is_max_block[2];   // [0] gathering, [1] accumulating variant
    SearchKernel oms[2], spa[2];
    IsKernel is[2];
};
#define TSG_G(D)                                                                                 \
    {D, {MaxBlockG<D, false>::value, MaxBlockG<D, true>::value},                                 \
     {MaxBlockGIs<D, false>::value, MaxBlockGIs<D, true>::value},                                \
     {k_search_g<OmsRule, D, false>, k_search_g<OmsRule, D, true>},                              \
     {k_search_g<SpaRule, D, false>, k_search_g<SpaRule, D, true>}, {k_is_g<D, false>, k_is_g<D, true>}}
const GEntry kGTable[] = {TSG_G(8), TSG_G(16), TSG_G(24), TSG_G(32)};
#undef TSG_G

const KEntry *find_kernel(int dc, int cpt) {
    for (const KEntry &k : kTable)
        if (k.dc == dc && k.cpt == cpt) return &k;
    return nullptr;
}

const GEntry *find_g(int dcmax) {
    for (const GEntry &g : kGTable)
        if (g.dcmax == dcmax) return &g;
    return nullptr;
}

int padded_degree(const ts_code *c) {
    static const int dcs[] = {6, 8, 12, 16, 24, 32};
    for (int d : dcs)
        if (d >= c->dc_max) return d;
    set_error("check degree %d above the decoder's limit 32", c->dc_max);
    return 0;
}

// Largest check-degree class of the streamed kernel for a code: the kernel's
// registers are those of its widest class (8: 94-104 VGPRs for the SPA
// search, against 128-144 for 16).
int streamed_dcmax(const ts_code *c) {
    return c->dc_max <= 8 ? 8 : (c->dc_max <= 16 ? 16 : (c->dc_max <= 24 ? 24 : 32));
}

// Streamed plans: both variants (cpt 0 gathering, 1 accumulating) and every
// workgroup size up to the kernel's bound that fits.
int add_streamed_variant(ts_ctx *ctx, const ts_code *c, bool search, int decoder, int max_iter,
                         int var, std::vector<SearchPlan> *out) {
    const GEntry *g = find_g(streamed_dcmax(c));
    const size_t lds = kHdrLds + lds_layout_g(c->n, max_iter, c->dev.q_ok ? c->dev.q_bytes : 0, var == 1).total;
    if (!g || lds > ctx->lds_per_block) return TS_OK;
    size_t aux = 0;
    const size_t slot = streamed_slot_bytes(c, decoder, max_iter, search, &aux);
    const void *kern = search ? (const void *)(decoder == TS_DEC_OMS_I8 ? g->oms[var] : g->spa[var])
                              : (const void *)g->is[var];
    for (int block : {256, 512, 1024}) {
        if (block > (search ? g->max_block[var] : g->is_max_block[var])) continue;
        int per_cu = 0;
        TSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds));
        if (per_cu < 1) continue;
        SearchPlan p;
        p.kind = kPlanStreamed;
        p.decoder = decoder;
        p.block = block;
        p.cpt = var;
        p.dc = g->dcmax;
        p.lds = lds;
        p.grid = per_cu * ctx->num_cu;
        p.slot_bytes = slot;
        p.hist_off = aux;
        out->push_back(p);
    }
    return TS_OK;
}

int add_streamed_plans(ts_ctx *ctx, const ts_code *c, bool search, int decoder, int max_iter,
                       std::vector<SearchPlan> *out) {
    for (int var = 0; var < 2; ++var) {
        const int rc = add_streamed_variant(ctx, c, search, decoder, max_iter, var, out);
        if (rc) return rc;
    }
    return TS_OK;
}

}  // namespace

size_t streamed_slot_bytes(const ts_code *c, int decoder, int max_iter, bool search, size_t *aux_off) {
    const size_t msg = (size_t)c->dev.g_off[c->dev.g_ncls] * (decoder == TS_DEC_OMS_I8 ? 1 : 4);
    size_t o = (msg + 255) & ~(size_t)255;
    *aux_off = o;
    const LdsG L = lds_layout_g(c->n, max_iter, c->dev.q_ok ? c->dev.q_bytes : 0);
    o += search ? (size_t)max_iter * L.W * 8 : (size_t)L.np * 4;
    return (o + 255) & ~(size_t)255;
}

// Launch shapes of the impulse search, register-resident ones first (fewest
// checks per thread first), then streamed ones.
int plan_candidates(ts_ctx *ctx, const ts_code *c, int decoder, int max_iter,
                    std::vector<SearchPlan> *out) {
    out->clear();
    const int dc = padded_degree(c);
    if (!dc) return TS_E_INVAL;
    const size_t lds = kHdrLds + lds_layout(c->n, max_iter, true).total;
    if (lds <= ctx->lds_per_block) {
        for (int cp : {1, 2, 4, 8}) {
            const KEntry *ke = find_kernel(dc, cp);
            if (!ke) continue;
            const int block = ((c->m + cp - 1) / cp + 63) / 64 * 64;
            if (block > ke->max_block) continue;
            SearchKernel kern = decoder == TS_DEC_OMS_I8 ? ke->oms : (decoder == TS_DEC_SPA_F32 ? ke->spa : ke->lnms);
            int per_cu = 0;
            TSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, lds));
            if (per_cu < 1) continue;
            SearchPlan p;
            p.kind = kPlanRegister;
            p.decoder = decoder;
            p.block = block;
            p.cpt = cp;
            p.dc = dc;
            p.lds = lds;
            p.grid = per_cu * ctx->num_cu;
            // the layered decoder's fixed-point test saves the messages of a
            // verifying sweep (the flooding decoders see their changes directly)
            p.slot_bytes = decoder == TS_DEC_LNMS_Q4 ? (size_t)block * cp * dc * 4 : 0;
            p.hist_off = 0;
            out->push_back(p);
            if (!p.slot_bytes) continue;
            // the same shape with the save area in LDS, where it fits (the
            // autotuner weighs the lost occupancy against the global traffic)
            const size_t lds_s = lds + p.slot_bytes;
            int per_cu_s = 0;
            if (lds_s <= ctx->lds_per_block &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_s, (const void *)kern, block, lds_s) == hipSuccess &&
                per_cu_s >= 1) {
                p.lds = lds_s;
                p.grid = per_cu_s * ctx->num_cu;
                p.slot_bytes = 0;
                p.save_lds = 1;
                out->push_back(p);
            }
        }
    }
    if (decoder != TS_DEC_LNMS_Q4) {   // the layered decoder has the register layout only
        int rc = add_streamed_plans(ctx, c, true, decoder, max_iter, out);
        if (rc) return rc;
    }
    if (out->empty()) {
        set_error(decoder == TS_DEC_LNMS_Q4 ? "the layered decoder needs a register shape; none fits this code"
                                            : "code (n = %d) needs more LDS per workgroup than the device has",
                  c->n);
        return TS_E_INVAL;
    }
    return TS_OK;
}

int plan_search(ts_ctx *ctx, const ts_code *c, int decoder, int max_iter, SearchPlan *plan) {
    std::vector<SearchPlan> v;
    const int rc = plan_candidates(ctx, c, decoder, max_iter, &v);
    if (rc) return rc;
    *plan = v.front();
    return TS_OK;
}

static SearchKernel search_kernel(const SearchPlan &plan, int decoder) {
    if (plan.kind == kPlanRegister) {
        const KEntry *ke = find_kernel(plan.dc, plan.cpt);
        if (!ke) return nullptr;
        return decoder == TS_DEC_OMS_I8 ? ke->oms : (decoder == TS_DEC_SPA_F32 ? ke->spa : ke->lnms);
    }
    if (decoder == TS_DEC_LNMS_Q4 || plan.cpt < 0 || plan.cpt > 1) return nullptr;
    const GEntry *g = find_g(plan.dc);
    return g ? (decoder == TS_DEC_OMS_I8 ? g->oms[plan.cpt] : g->spa[plan.cpt]) : nullptr;
}

static IsKernel is_kernel(const SearchPlan &plan) {
    if (plan.kind == kPlanRegister) {
        const KEntry *k = find_kernel(plan.dc, plan.cpt);
        return k ? k->is : nullptr;
    }
    if (plan.cpt < 0 || plan.cpt > 1) return nullptr;
    const GEntry *g = find_g(plan.dc);
    return g ? g->is[plan.cpt] : nullptr;
}

int occupancy_grid(ts_ctx *ctx, const SearchPlan &plan, int decoder, bool search, int *grid) {
    const void *kern = search ? (const void *)search_kernel(plan, decoder) : (const void *)is_kernel(plan);
    if (!kern) {
        set_error("no kernel for kind %d dc %d cpt %d", plan.kind, plan.dc, plan.cpt);
        return TS_E_INVAL;
    }
    int per_cu = 0;
    TSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, plan.block, plan.lds));
    if (per_cu < 1) {
        set_error("kernel does not fit on a compute unit (block %d, %zu bytes of LDS)", plan.block, plan.lds);
        return TS_E_INVAL;
    }
    *grid = per_cu * ctx->num_cu;
    return TS_OK;
}

int launch_search_jobs(hipStream_t stream, const SearchPlan &plan, const SearchJob *d_jobs, int n_jobs,
                       int *queue, long long n_items) {
    if (n_items <= 0 || n_jobs <= 0) return TS_OK;
    if (n_items > INT_MAX) {
        set_error("too many items in one launch");
        return TS_E_INVAL;
    }
    SearchKernel kern = search_kernel(plan, plan.decoder);
    if (!kern) {
        set_error("no kernel for kind %d dc %d cpt %d", plan.kind, plan.dc, plan.cpt);
        return TS_E_INVAL;
    }
    const long long grid = n_items < plan.grid ? n_items : plan.grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(plan.block), plan.lds, stream, d_jobs, n_jobs,
                       queue, n_items);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

int launch_is_jobs(hipStream_t stream, const SearchPlan &plan, const IsJob *d_jobs, int n_jobs,
                   int *queue, long long n_items) {
    if (n_items <= 0 || n_jobs <= 0) return TS_OK;
    if (n_items > INT_MAX) {
        set_error("too many items in one launch");
        return TS_E_INVAL;
    }
    IsKernel kern = is_kernel(plan);
    if (!kern) {
        set_error("no IS kernel for kind %d dc %d cpt %d", plan.kind, plan.dc, plan.cpt);
        return TS_E_INVAL;
    }
    const long long grid = n_items < plan.grid ? n_items : plan.grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(plan.block), plan.lds, stream, d_jobs, n_jobs,
                       queue, n_items);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

// One job: its descriptor goes through the executor's staging ring.
int launch_search(ts_exec &ex, const SearchPlan &plan0, const SearchLaunch &a) {
    SearchPlan plan = plan0;
    plan.decoder = a.decoder;
    SearchJob j{};
    j.a = a;
    j.cd = *a.code;
    j.item0 = 0;
    if (plan.kind == kPlanStreamed && !a.gscr) {
        set_error("streamed launch without scratch");
        return TS_E_INVAL;
    }
    // register kind without scratch: no message save area (no fixed-point test)
    j.a.slot_bytes = (long long)plan.slot_bytes;
    j.a.save_lds = plan.save_lds;
    j.a.hist_off = (long long)plan.hist_off;
    if (a.n_patterns <= 0) return TS_OK;
    void *dj = nullptr;
    int slot = -1;
    int rc = ex.stage(&j, sizeof(j), &dj, &slot);
    if (rc) return rc;
    rc = launch_search_jobs(ex.stream, plan, (const SearchJob *)dj, 1, a.queue, a.n_patterns);
    ex.staged(slot);
    return rc;
}

int launch_fill(hipStream_t stream, int *p, int value, int64_t count) {
    if (count <= 0) return TS_OK;
    const int blk = 256;
    const long long grid = (count + blk - 1) / blk;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)grid), dim3(blk), 0, stream, p, value,
                       (long long)count);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

// IS launch shapes: every register-resident shape that fits (fewest checks per
// thread first), then the streamed kernel at each workgroup size; restricted to
// the requested layout.
int plan_is_candidates(ts_ctx *ctx, const ts_code *c, int max_iter, int layout,
                       std::vector<SearchPlan> *out) {
    out->clear();
    const int dc = padded_degree(c);
    if (!dc) return TS_E_INVAL;
    const size_t lds = kHdrLds + lds_layout(c->n, max_iter, false).total;
    if (lds <= ctx->lds_per_block && (layout == TS_LAYOUT_AUTO || layout == TS_LAYOUT_REGISTER)) {
        for (int cp : {1, 2, 4, 8}) {
            const KEntry *k = find_kernel(dc, cp);
            if (!k) continue;
            const int b = ((c->m + cp - 1) / cp + 63) / 64 * 64;
            if (b > k->is_max_block) continue;
            int per_cu = 0;
            TSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k->is, b, lds));
            if (per_cu < 1) continue;
            SearchPlan p;
            p.kind = kPlanRegister;
            p.decoder = TS_DEC_SPA_F32;
            p.block = b;
            p.cpt = cp;
            p.dc = dc;
            p.lds = lds;
            p.grid = per_cu * ctx->num_cu;
            p.slot_bytes = 0;
            p.hist_off = 0;
            out->push_back(p);
        }
    }
    if (layout != TS_LAYOUT_REGISTER) {
        const int rc = add_streamed_plans(ctx, c, false, TS_DEC_SPA_F32, max_iter, out);
        if (rc) return rc;
        out->erase(std::remove_if(out->begin(), out->end(),
                                  [&](const SearchPlan &p) { return !layout_accepts(layout, p); }),
                   out->end());
    }
    if (out->empty()) {
        set_error(layout == TS_LAYOUT_AUTO ? "code (n = %d) needs more LDS per workgroup than the device has"
                                           : "the requested decoder layout does not fit this code (n = %d)",
                  c->n);
        return TS_E_INVAL;
    }
    return TS_OK;
}

int plan_is(ts_ctx *ctx, const ts_code *c, int max_iter, int layout, SearchPlan *plan) {
    std::vector<SearchPlan> v;
    const int rc = plan_is_candidates(ctx, c, max_iter, layout, &v);
    if (rc) return rc;
    *plan = v.front();
    return TS_OK;
}

IsDev make_is_dev(const IsLaunch &a, const SearchPlan &plan) {
    IsDev d{};
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
    d.counters = a.counters;
    d.gscr = a.gscr;
    d.fp_exit = a.fp_exit;
    d.count_mode = a.count_mode;
    d.n_mix = a.n_mix;
    d.mix_s0 = a.mix_s0;
    d.mix_ds = a.mix_ds;
    d.slot_bytes = (long long)plan.slot_bytes;
    d.lam_off = (long long)plan.hist_off;
    return d;
}

int is_reduce_parts(int64_t n) { return (int)((n + kRedChunk - 1) / kRedChunk); }

RedJob make_red_job(const IsDev &d, const double *wf, const unsigned char *fail, int64_t n, double *out,
                    double *part) {
    RedJob j{};
    j.wf = wf;
    j.fail = fail;
    j.n = n;
    j.wconst = d.wconst;
    j.coef = d.shift / d.sigma;
    j.mix = MixW{d.n_mix, d.a, (long long)n, d.mix_s0, d.mix_ds, d.sigma};
    j.cmask = d.count_mode == TS_IS_COUNT_TS ? 2 : 1;
    j.part0 = 0;
    j.np = is_reduce_parts(n);
    j.part = part;
    j.out = out;
    return j;
}

int launch_is_reduce(hipStream_t stream, const RedJob &j, int mode) {
    if (j.np < 1) {
        set_error("empty reduction");
        return TS_E_INVAL;
    }
    hipLaunchKernelGGL(k_is_reduce, dim3(j.np), dim3(kRedThreads), 0, stream, j, mode);
    TSG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_is_reduce_final, dim3(1), dim3(kRedThreads), 0, stream, j, mode);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}

int launch_is_reduce_jobs(hipStream_t stream, const RedJob *d_jobs, int nj, int total_parts, int mode) {
    if (nj < 1) return TS_OK;
    if (total_parts < nj) {
        set_error("empty reduction");
        return TS_E_INVAL;
    }
    hipLaunchKernelGGL(k_is_reduce_jobs, dim3(total_parts), dim3(kRedThreads), 0, stream, d_jobs, nj, mode);
    TSG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_is_reduce_final_jobs, dim3(nj), dim3(kRedThreads), 0, stream, d_jobs, mode);
    TSG_HIP(hipGetLastError());
    return TS_OK;
}


}  // namespace tsg
