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

template <bool FILL>
__global__ __launch_bounds__(kNbrThreads) void k_neighbors(
    const GroupInfo *__restrict__ grp, const int64_t *__restrict__ n_off,
    const int32_t *__restrict__ n_idx, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const int32_t *__restrict__ perm, double h2,
    int64_t *__restrict__ cnt, const int64_t *__restrict__ offsets, int32_t *__restrict__ idx) {
    __shared__ double s_x[kNbrTile], s_y[kNbrTile], s_z[kNbrTile];
    __shared__ int32_t s_j[kNbrTile];
    const int tid = threadIdx.x;
    const GroupInfo gi = grp[blockIdx.x];
    const int64_t nb = n_off[blockIdx.x], ne = n_off[blockIdx.x + 1];
    for (int chunk = 0; chunk < gi.count; chunk += kNbrThreads) {
        const int li = chunk + tid;
        const bool valid = li < gi.count;
        const int32_t i = gi.first + (valid ? li : 0);
        const double xi = x[i], yi = y[i], zi = z[i];
        const int64_t o = perm[i];
        const int64_t base = (FILL && valid) ? offsets[o] : 0;
        int64_t k = 0;
        for (int64_t t0 = nb; t0 < ne; t0 += kNbrTile) {
            const int tl = (int)min<int64_t>(kNbrTile, ne - t0);
            __syncthreads();
            if (tid < tl) {
                const int32_t j = n_idx[t0 + tid];
                s_x[tid] = x[j];
                s_y[tid] = y[j];
                s_z[tid] = z[j];
                s_j[tid] = j;
            }
            __syncthreads();
            if (!valid) continue;
            for (int e = 0; e < tl; ++e) {
                const double dx = s_x[e] - xi, dy = s_y[e] - yi, dz = s_z[e] - zi;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const int32_t j = s_j[e];
                if (r2 < h2 && j != i) {
                    if (FILL) idx[base + k] = perm[j];
                    ++k;
                }
            }
        }
        if (!valid) continue;
        if (!FILL) {
            cnt[o] = k;
        } else {
            // rows are short: insertion sort into ascending original index
            int32_t *row = idx + base;
            for (int64_t a = 1; a < k; ++a) {
                const int32_t v = row[a];
                int64_t b = a - 1;
                while (b >= 0 && row[b] > v) {
                    row[b + 1] = row[b];
                    --b;
                }
                row[b + 1] = v;
            }
        }
    }
}

int launch_neighbors(p3t_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *nnz) {
    int rc;
    const int64_t n = ctx->n;
    if ((rc = ensure(ctx, ctx->nbr_cnt, (n + 1) * sizeof(int64_t)))) return rc;
    int64_t *cnt = ptr<int64_t>(ctx->nbr_cnt);
    int64_t *rb = ptr<int64_t>(ctx->readback);
    const int64_t stride = ctx->n_nodes + 1;
    const int64_t *n_off = ptr<int64_t>(ctx->off) + 2 * stride;   // near-particle lists
    const double h2 = ctx->prm.r_search * ctx->prm.r_search;
    if ((rc = check_hip(ctx, hipMemsetAsync(cnt, 0, (n + 1) * sizeof(int64_t), ctx->stream), "memset")))
        return rc;
    const unsigned grid = (unsigned)ctx->n_groups;
    if (grid) {
        k_neighbors<false><<<grid, kNbrThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), n_off, ptr<int32_t>(ctx->n_idx), ptr<double>(ctx->x),
            ptr<double>(ctx->y), ptr<double>(ctx->z), ptr<int32_t>(ctx->vals[0]), h2, cnt, nullptr,
            nullptr);
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
        k_neighbors<true><<<grid, kNbrThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), n_off, ptr<int32_t>(ctx->n_idx), ptr<double>(ctx->x),
            ptr<double>(ctx->y), ptr<double>(ctx->z), ptr<int32_t>(ctx->vals[0]), h2, nullptr, cnt,
            idx);
        if ((rc = check_hip(ctx, hipGetLastError(), "neighbour fill"))) return rc;
    }
    return P3T_OK;
}

}  // namespace p3t
