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

// Exclusive wave prefix sum and total of small non-negative counts (< 2^BITS),
// bit-sliced through ballots: no cross-lane data movement.
template <int BITS>
__device__ __forceinline__ int wave_excl_small(int v, int &total) {
    int excl = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint64_t m = ballot((v >> b) & 1);
        excl += count_below(m) << b;
        tot += __popcll(m) << b;
    }
    total = tot;
    return excl;
}

// Exclusive wave prefix sum of any non-negative counts: bit-sliced when every
// count is below 32, shuffle scan otherwise.
__device__ __forceinline__ int wave_excl_count(int v, int &total) {
    if (!ballot(v >= 32)) return wave_excl_small<5>(v, total);
    const int incl = wave_incl_scan(v);
    total = __shfl(incl, kWave - 1, kWave);
    return incl - v;
}

// v from the lane that DPP control CTRL selects (0 where ROW_MASK disables
// the row); for float and double
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_src(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, true));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_src(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK,
                                                              0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL,
                                                              ROW_MASK, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each row of 16 lanes, in every lane of the row, by a fixed tree:
// pairs, quads, half rows, rows.
template <class T>
__device__ __forceinline__ T row_sum(T v) {
    v += dpp_src<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp_src<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp_src<0x141>(v);    // row_half_mirror
    v += dpp_src<0x140>(v);    // row_mirror
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Slices per wavefront for a group of n members: s slices of 64/s i-particles,
// V = ceil(n s / 64) virtual wavefronts, `per_round` per round;
// minimise issued lane work V * 64 / s, with a small charge per extra round.
__device__ __forceinline__ int choose_log2_slices(int n, int per_round) {
    int best = 0;
    float best_cost = 1e30f;
    for (int ls = 0; ls <= 6; ++ls) {
        const int nw = kWave >> ls;
        const int V = (n + nw - 1) / nw;
        const int rounds = (V + per_round - 1) / per_round;
        const float cost = (float)V * (float)nw * (1.0f + 0.05f * (float)(rounds - 1));
        if (cost < best_cost - 1e-3f) {
            best_cost = cost;
            best = ls;
        }
    }
    return best;
}

// Common leading octal digits (tree levels) of two 63-bit Morton keys: 21 if equal.
__device__ __forceinline__ int common_levels(uint64_t a, uint64_t b) {
    uint64_t d = a ^ b;
    if (d == 0) return 21;
    int hb = 63 - __clzll((long long)d);   // highest differing bit, 0..62
    return 20 - hb / 3;
}

}  // namespace p3t
