// neighbors.hip -- per-particle neighbour lists (Section 2.2): for every
// particle i the particles j != i with |x_j - x_i| < h.  Only the near
// particles N_g of i's group can be neighbours (every other particle of the
// walk lies in a leaf whose box is at least h from the group's box, and
// rounding is monotone, so the FP64 test below fails for it); N_g is staged
// through LDS in tiles.  The test is dx*dx + dy*dy + dz*dz < h*h in FP64
// with dx = x_j - x_i, without fused multiply-adds (this file is compiled with
// -ffp-contract=off), which makes the lists exactly reproducible.
// Output: CSR in original particle order, each row ascending.
#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kNbrThreads = 256;

constexpr int kNbrTile = 256;

// One block per group; a lane is (i, slice) as in the interaction kernel: 64/s
// members times s slices of every staged tile of N_g.  The count pass reduces
// the slice counts per particle; the fill pass claims row slots with an atomic
// cursor per particle; a last kernel sorts each row.
template <bool FILL>
__global__ __launch_bounds__(kNbrThreads) void k_neighbors(
    const GroupInfo *__restrict__ grp, ListsDev L, const double *__restrict__ x,
    const double *__restrict__ y,
    const double *__restrict__ z, const int32_t *__restrict__ perm, double h2,
    int64_t *__restrict__ cnt, const int64_t *__restrict__ offsets, int32_t *__restrict__ cursor,
    int32_t *__restrict__ idx) {
    __shared__ double s_x[kNbrTile + kWave], s_y[kNbrTile + kWave], s_z[kNbrTile + kWave];
    __shared__ int32_t s_j[kNbrTile + kWave];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const GroupInfo gi = grp[blockIdx.x];
    const int64_t nb = L.beg[2][blockIdx.x], ne = L.end[2][blockIdx.x];   // near particles
    const int32_t *__restrict__ n_idx = L.idx[2];
    if (tid < kWave) {   // padding entries: never within h
        s_x[kNbrTile + tid] = s_y[kNbrTile + tid] = s_z[kNbrTile + tid] = INFINITY;
        s_j[kNbrTile + tid] = -2;
    }
    const int ls = choose_log2_slices(gi.count, 4);
    const int ns = 1 << ls, nw = kWave >> ls;
    const int il = lane & (nw - 1), slice = lane >> (6 - ls);
    const int V = (gi.count + nw - 1) / nw;
    for (int v0 = 0; v0 < V; v0 += 4) {
        const bool act = v0 + w < V;
        const int li = (v0 + w) * nw + il;
        const bool valid = act && li < gi.count;
        const int32_t i = gi.first + (valid ? li : 0);
        const double xi = x[i], yi = y[i], zi = z[i];
        const int64_t o = perm[i];
        const int64_t base = (FILL && valid) ? offsets[o] : 0;
        int k = 0;
        for (int64_t t0 = nb; t0 < ne; t0 += kNbrTile) {
            const int tl = (int)min<int64_t>(kNbrTile, ne - t0);
            __syncthreads();
            if (tid < tl) {
                const int32_t j = n_idx[t0 + tid];
                s_x[tid] = x[j];
                s_y[tid] = y[j];
                s_z[tid] = z[j];
                s_j[tid] = j;
            } else {
                s_x[tid] = s_y[tid] = s_z[tid] = INFINITY;
                s_j[tid] = -2;
            }
            __syncthreads();
            if (!valid) continue;
            const int iters = (tl + ns - 1) >> ls;
            for (int it = 0; it < iters; ++it) {
                const int e = slice + it * ns;
                const double dx = s_x[e] - xi, dy = s_y[e] - yi, dz = s_z[e] - zi;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const int32_t j = s_j[e];
                if (r2 < h2 && j != i) {
                    if (FILL) idx[base + atomicAdd(&cursor[o], 1)] = perm[j];
                    ++k;
                }
            }
        }
        if (!act || FILL) continue;
        for (int d = nw; d < kWave; d <<= 1) k += __shfl_xor(k, d, kWave);
        if (valid && slice == 0) cnt[o] = k;
    }
}

// Rows are short: insertion sort of each row into ascending original index.
__global__ void k_sort_rows(int64_t n, const int64_t *__restrict__ offsets, int32_t *__restrict__ idx) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int64_t b0 = offsets[o], len = offsets[o + 1] - b0;
    int32_t *row = idx + b0;
    for (int64_t a = 1; a < len; ++a) {
        const int32_t v = row[a];
        int64_t b = a - 1;
        while (b >= 0 && row[b] > v) {
            row[b + 1] = row[b];
            --b;
        }
        row[b + 1] = v;
    }
}

int launch_neighbors(p3t_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *nnz) {
    int rc;
    const int64_t n = ctx->n;
    if ((rc = ensure(ctx, ctx->nbr_cnt, (n + 1) * sizeof(int64_t)))) return rc;
    int64_t *cnt = ptr<int64_t>(ctx->nbr_cnt);
    int64_t *rb = ptr<int64_t>(ctx->readback);
    const ListsDev L = lists_dev(ctx);
    const double h2 = ctx->prm.r_search * ctx->prm.r_search;
    if ((rc = check_hip(ctx, hipMemsetAsync(cnt, 0, (n + 1) * sizeof(int64_t), ctx->stream), "memset")))
        return rc;
    const unsigned grid = (unsigned)ctx->n_groups;
    if (grid) {
        k_neighbors<false><<<grid, kNbrThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), L, ptr<double>(ctx->x),
            ptr<double>(ctx->y), ptr<double>(ctx->z), ptr<int32_t>(ctx->vals[0]), h2, cnt, nullptr,
            nullptr, nullptr);
        if ((rc = check_hip(ctx, hipGetLastError(), "neighbour count"))) return rc;
    }
    if ((rc = scan_exclusive_i64(ctx, cnt, cnt, n + 1, rb + 40))) return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + 40, rb + 40, sizeof(int64_t),
                                            hipMemcpyDeviceToHost, ctx->stream), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    const int64_t total = ctx->hpin[40];
    *nnz = total;
    ctx->nnz = total;
    if (total > cap)
        return set_error(ctx, P3T_ECAPACITY, "neighbour buffer holds %lld entries, %lld needed",
                         (long long)cap, (long long)total);
    if ((rc = check_hip(ctx, hipMemcpyAsync(offsets, cnt, (n + 1) * sizeof(int64_t),
                                            hipMemcpyDeviceToDevice, ctx->stream), "copy offsets")))
        return rc;
    if (grid && total > 0) {
        int32_t *cursor = ptr<int32_t>(ctx->gflag);   // free after the build: row cursors
        if ((rc = check_hip(ctx, hipMemsetAsync(cursor, 0, n * sizeof(int32_t), ctx->stream),
                            "memset")))
            return rc;
        k_neighbors<true><<<grid, kNbrThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), L, ptr<double>(ctx->x),
            ptr<double>(ctx->y), ptr<double>(ctx->z), ptr<int32_t>(ctx->vals[0]), h2, nullptr, cnt,
            cursor, idx);
        if ((rc = check_hip(ctx, hipGetLastError(), "neighbour fill"))) return rc;
        k_sort_rows<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, cnt, idx);
        if ((rc = check_hip(ctx, hipGetLastError(), "neighbour sort"))) return rc;
    }
    return P3T_OK;
}

}  // namespace p3t
