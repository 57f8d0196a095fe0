// scan.hip -- device-wide exclusive prefix sums (tile scan + recursive block
// sums), used for radix-sort digit offsets, tree node numbering, group
// compaction, list offsets and neighbour CSR offsets.
#include <vector>

#include "device_util.h"
#include "internal.h"
#include "scan_tiles.h"

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
static int scan_rec(p3t_ctx *ctx, hipStream_t st, const T *in, T *out, int64_t n, T *total,
                    T *tmp) {
    if (n <= 0) {
        if (total) return check_hip(ctx, hipMemsetAsync(total, 0, sizeof(T), st), "scan");
        return P3T_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_scan_tile<T><<<1, kScanThreads, 0, st>>>(in, out, n, nullptr, total);
        return check_hip(ctx, hipGetLastError(), "scan tile");
    }
    T *sums = tmp;
    k_scan_tile<T><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, n, sums, nullptr);
    int rc = check_hip(ctx, hipGetLastError(), "scan tile");
    if (rc) return rc;
    rc = scan_rec<T>(ctx, st, sums, sums, nb, total, tmp + nb);
    if (rc) return rc;
    k_scan_add<T><<<(unsigned)nb, kScanThreads, 0, st>>>(out, n, sums);
    return check_hip(ctx, hipGetLastError(), "scan add");
}

static bool scan_two_pass(int64_t n) {
    return n > 0 && (n + kScan2Tile - 1) / kScan2Tile <= kScan2MaxTiles;
}

size_t scan_tmp_bytes(int64_t n) {
    if (scan_two_pass(n)) return (size_t)((n + kScan2Tile - 1) / kScan2Tile + 1) * sizeof(int64_t);
    // the recursive scan: sum over recursion levels of the block counts
    int64_t need = 0, m = n;
    while (m > kScanTile) {
        m = (m + kScanTile - 1) / kScanTile;
        need += m;
    }
    return (size_t)(need + 1) * sizeof(int64_t);
}

template <class T>
static int scan_any(p3t_ctx *ctx, hipStream_t st, DevBuf &tmp, const T *in, T *out, int64_t n,
                    T *total) {
    int rc = ensure(ctx, tmp, scan_tmp_bytes(n));
    if (rc) return rc;
    if (scan_two_pass(n)) {
        const unsigned tiles = (unsigned)((n + kScan2Tile - 1) / kScan2Tile);
        T *sums = ptr<T>(tmp);
        k_scan2_sums<T><<<tiles, kScanThreads, 0, st>>>(in, n, sums);
        k_scan2_tiles<T><<<tiles, kScanThreads, 0, st>>>(in, n, sums, total,
                                                         StoreExclusive<T>{out});
        return check_hip(ctx, hipGetLastError(), "scan");
    }
    return scan_rec<T>(ctx, st, in, out, n, total, ptr<T>(tmp));
}

// Block r: exclusive scan of row r in chunks of kScanThreads with a running carry.
__global__ __launch_bounds__(kScanThreads) void k_scan_rows(const int32_t *__restrict__ in,
                                                            int32_t *__restrict__ out,
                                                            int32_t *__restrict__ totals,
                                                            int64_t cols) {
    __shared__ int32_t s_wsum[kScanThreads / kWave];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int64_t row = (int64_t)blockIdx.x * cols;
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < cols; c0 += kScanThreads) {
        const int64_t c = c0 + tid;
        const int32_t v = c < cols ? in[row + c] : 0;
        const int32_t incl = wave_incl_scan(v);
        if (lane == kWave - 1) s_wsum[w] = incl;
        __syncthreads();
        int32_t wb = 0, tot = 0;
        for (int k = 0; k < kScanThreads / kWave; ++k) {
            wb += k < w ? s_wsum[k] : 0;
            tot += s_wsum[k];
        }
        if (c < cols) out[row + c] = carry + wb + incl - v;
        carry += tot;
        __syncthreads();   // s_wsum is rewritten by the next chunk
    }
    if (tid == 0) totals[blockIdx.x] = carry;
}

int scan_rows_i32(p3t_ctx *ctx, const int32_t *in, int32_t *out, int32_t *totals, int rows,
                  int64_t cols) {
    if (rows <= 0) return P3T_OK;
    k_scan_rows<<<rows, kScanThreads, 0, ctx->stream>>>(in, out, totals, cols);
    return check_hip(ctx, hipGetLastError(), "row scan");
}

int scan_exclusive_i64(p3t_ctx *ctx, const int64_t *in, int64_t *out, int64_t n, int64_t *total) {
    return scan_any<int64_t>(ctx, ctx->stream, ctx->scan_tmp, in, out, n, total);
}

int scan_exclusive_i32(p3t_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *total) {
    return scan_any<int32_t>(ctx, ctx->stream, ctx->scan_tmp, in, out, n, total);
}

int scan_exclusive_i64_on(p3t_ctx *ctx, hipStream_t st, DevBuf &tmp, const int64_t *in,
                          int64_t *out, int64_t n, int64_t *total) {
    return scan_any<int64_t>(ctx, st, tmp, in, out, n, total);
}

}  // namespace p3t
