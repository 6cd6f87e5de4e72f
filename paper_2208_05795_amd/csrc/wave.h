// Wavefront (64-lane) helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace tsg {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Sum over the wavefront of values in [0, 2^B): one ballot and population
// count per bit, instead of the six shuffle steps of wave_sum.
template <int B>
__device__ __forceinline__ int wave_sum_bits(int x) {
    int s = 0;
#pragma unroll
    for (int b = 0; b < B; ++b) s += __popcll(__ballot((x >> b) & 1)) << b;
    return s;
}

// Bits that hold a count in [0, n].
constexpr int count_bits(int n) { return n < 2 ? 1 : 1 + count_bits(n >> 1); }

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
    return x;
}

__device__ __forceinline__ int wave_excl_scan(int x) {
    const int lane = lane_id();
    int incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    return incl - x;
}

// Orders the LDS accesses of one wavefront: every lane's earlier LDS writes are
// visible to every lane's later reads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace tsg
