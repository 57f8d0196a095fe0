// scan.hip -- device-wide exclusive prefix sums (tile scan + recursive block
// sums), used for radix-sort digit offsets, tree node numbering, group
// compaction, list offsets and neighbour CSR offsets.
#include <vector>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const T *in, T *out, int64_t n,
                                                            T *block_sums, T *total) {
    __shared__ T wsum[kScanThreads / kWave];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    T v[kScanItems];
    T run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : T(0);
        run += v[k];
    }
    T incl = wave_incl_scan(run);
    const int w = tid / kWave, lane = tid % kWave;
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    T wbase = 0, btot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        if (k < w) wbase += wsum[k];
        btot += wsum[k];
    }
    T excl = wbase + incl - run;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = excl;
        excl += v[k];
    }
    if (tid == 0) {
        if (block_sums) block_sums[blockIdx.x] = btot;
        if (total) *total = btot;
    }
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T *out, int64_t n, const T *block_sums) {
    const T add = block_sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads) {
        int64_t i = base + k;
        if (i < n) out[i] += add;
    }
}

template <class T>
static int scan_rec(p3t_ctx *ctx, const T *in, T *out, int64_t n, T *total, T *tmp) {
    if (n <= 0) {
        if (total) return check_hip(ctx, hipMemsetAsync(total, 0, sizeof(T), ctx->stream), "scan");
        return P3T_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_scan_tile<T><<<1, kScanThreads, 0, ctx->stream>>>(in, out, n, nullptr, total);
        return check_hip(ctx, hipGetLastError(), "scan tile");
    }
    T *sums = tmp;
    k_scan_tile<T><<<(unsigned)nb, kScanThreads, 0, ctx->stream>>>(in, out, n, sums, nullptr);
    int rc = check_hip(ctx, hipGetLastError(), "scan tile");
    if (rc) return rc;
    rc = scan_rec<T>(ctx, sums, sums, nb, total, tmp + nb);
    if (rc) return rc;
    k_scan_add<T><<<(unsigned)nb, kScanThreads, 0, ctx->stream>>>(out, n, sums);
    return check_hip(ctx, hipGetLastError(), "scan add");
}

template <class T>
static int scan_any(p3t_ctx *ctx, const T *in, T *out, int64_t n, T *total) {
    // scratch: sum over recursion levels of the block counts
    int64_t need = 0, m = n;
    while (m > kScanTile) {
        m = (m + kScanTile - 1) / kScanTile;
        need += m;
    }
    int rc = ensure(ctx, ctx->scan_tmp, (size_t)(need + 1) * sizeof(int64_t));
    if (rc) return rc;
    return scan_rec<T>(ctx, in, out, n, total, ptr<T>(ctx->scan_tmp));
}

int scan_exclusive_i64(p3t_ctx *ctx, const int64_t *in, int64_t *out, int64_t n, int64_t *total) {
    return scan_any<int64_t>(ctx, in, out, n, total);
}

int scan_exclusive_i32(p3t_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *total) {
    return scan_any<int32_t>(ctx, in, out, n, total);
}

}  // namespace p3t
