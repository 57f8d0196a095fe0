// scan_tiles.h -- two-launch exclusive scan of up to kScan2MaxTiles tiles of
// kScan2Tile elements: the tile sums, then every block adds up the sums of
// the tiles before its own and scans its tile from there, handing each
// element's exclusive prefix to a sink.
#pragma once

#include "device_util.h"

namespace p3t {

constexpr int kScan2Threads = 256;
constexpr int kScan2Items = 16;
constexpr int kScan2Tile = kScan2Threads * kScan2Items;
constexpr int64_t kScan2MaxTiles = 4096;

template <class T>
__global__ __launch_bounds__(kScan2Threads) void k_scan2_sums(const T *__restrict__ in, int64_t n,
                                                              T *__restrict__ tile_sums) {
    __shared__ T wsum[kScan2Threads / kWave];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScan2Tile;
    T run = 0;
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        const int64_t i = base + (int64_t)k * kScan2Threads + tid;   // coalesced
        if (i < n) run += in[i];
    }
    run = wave_sum(run);
    if (tid % kWave == 0) wsum[tid / kWave] = run;
    __syncthreads();
    if (tid == 0) {
        T s = 0;
        for (int k = 0; k < kScan2Threads / kWave; ++k) s += wsum[k];
        tile_sums[blockIdx.x] = s;
    }
}

// sink(i, prefix, value) for every i < n; *total (if given) = the sum of all
template <class T, class Sink>
__global__ __launch_bounds__(kScan2Threads) void k_scan2_tiles(const T *in, int64_t n,
                                                               const T *__restrict__ tile_sums,
                                                               T *total, Sink sink) {
    __shared__ T wsum[kScan2Threads / kWave];
    __shared__ T s_base;
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    // this tile's offset: the sum of the tiles before it
    T before = 0;
    for (int64_t b = tid; b < blockIdx.x; b += kScan2Threads) before += tile_sums[b];
    before = wave_sum(before);
    if (lane == 0) wsum[w] = before;
    __syncthreads();
    if (tid == 0) {
        T s = 0;
        for (int k = 0; k < kScan2Threads / kWave; ++k) s += wsum[k];
        s_base = s;
        if (total && blockIdx.x == gridDim.x - 1) *total = s + tile_sums[blockIdx.x];
    }
    __syncthreads();
    // the tile: each thread scans kScan2Items consecutive elements
    const int64_t base = (int64_t)blockIdx.x * kScan2Tile + (int64_t)tid * kScan2Items;
    T v[kScan2Items];
    T run = 0;
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        const int64_t i = base + k;
        v[k] = (i < n) ? in[i] : T(0);
        run += v[k];
    }
    const T incl = wave_incl_scan(run);
    __syncthreads();   // wsum is reused
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    T excl = s_base + incl - run;
    for (int k = 0; k < w; ++k) excl += wsum[k];
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        const int64_t i = base + k;
        if (i < n) sink(i, excl, v[k]);
        excl += v[k];
    }
}

template <class T>
struct StoreExclusive {
    T *out;
    __device__ __forceinline__ void operator()(int64_t i, T prefix, T) const { out[i] = prefix; }
};

}  // namespace p3t
