// device_util.h -- wavefront-level helpers for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p3t {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ int count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive wave scan (Hillis-Steele over the 64 lanes).
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Common leading octal digits (tree levels) of two 63-bit Morton keys: 21 if equal.
__device__ __forceinline__ int common_levels(uint64_t a, uint64_t b) {
    uint64_t d = a ^ b;
    if (d == 0) return 21;
    int hb = 63 - __clzll((long long)d);   // highest differing bit, 0..62
    return 20 - hb / 3;
}

}  // namespace p3t
