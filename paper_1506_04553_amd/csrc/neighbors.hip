// neighbors.hip -- per-particle neighbour lists (Section 2.2): for every
// particle i the particles j != i with |x_j - x_i| < h.  Only the near
// particles N_g of i's group can be neighbours (every other particle of the
// walk lies in a leaf whose box is at least h from the group's box, and
// rounding is monotone, so the FP64 test below fails for it).  The test is
// dx*dx + dy*dy + dz*dz < h*h in FP64 with dx = x_j - x_i, without fused
// multiply-adds (this file is compiled with -ffp-contract=off), which makes
// the lists exactly reproducible.
//
// One block per group.  N_g is staged through LDS in tiles; each staged
// particle is first tested against the group's bounding box, with the same
// FP64 expression on the per-axis gaps t = max(lo - x_j, 0, x_j - hi).  Since
// |dx| >= t for every member and rounding is monotone, a particle whose gap
// test fails cannot pass the pair test for any member, so only the survivors
// (usually a handful) are compacted and tested against every member.
//
// Rows are written in one pass into fixed-size slots (row o at o * cap, the
// slot size taken from the longest row of the previous call), then packed into
// the caller's CSR (original particle order, each row ascending).  A row
// longer than its slot raises a flag; the pass then runs again writing straight
// into the CSR at the offsets the first pass counted, and the rows are sorted
// in place.  Each row is written by the one thread that owns its particle.
#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kNbrThreads = 256;
constexpr int kNbrWaves = kNbrThreads / kWave;
constexpr int kNbrTile = kNbrThreads;
constexpr int32_t kNbrFirstCap = 32;

__device__ __forceinline__ double axis_gap(double v, double lo, double hi) {
    const double a = lo - v, b = v - hi;
    const double t = a > 0.0 ? a : 0.0;
    return b > t ? b : t;
}

// CSR = false: rows into slots of `cap` entries, counts into cnt (cnt[n] = 0
// for the scan), and, tagged with this call's number `tag` so that no word
// has to be cleared first: the longest row into *longest as
// max(tag << 32 | length), and *overflow = max(tag) if a row outgrew its slot.
// CSR = true: rows straight into out at the offsets off (cnt, cap unused).
template <bool CSR>
__global__ __launch_bounds__(kNbrThreads) void k_neighbors(
    const GroupInfo *__restrict__ grp, ListsDev L, const PosMass *__restrict__ xm,
    const int32_t *__restrict__ perm,
    double h2, int32_t cap, int32_t *__restrict__ out, const int64_t *__restrict__ off,
    int64_t *__restrict__ cnt, int64_t n, unsigned long long tag,
    unsigned long long *__restrict__ longest, unsigned long long *__restrict__ overflow) {
    __shared__ double s_x[kNbrTile], s_y[kNbrTile], s_z[kNbrTile];
    __shared__ int32_t s_j[kNbrTile];
    __shared__ int32_t s_wn[kNbrWaves];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int g = L.order[blockIdx.x];
    const GroupInfo gi = grp[g];
    const int64_t nb = L.beg[2][g], ne = L.end[2][g];   // near particles
    const int32_t *__restrict__ n_idx = L.idx[2];
    if (!CSR && blockIdx.x == 0 && tid == 0) cnt[n] = 0;
    int kmax = 0;

    for (int m0 = 0; m0 < gi.count; m0 += kNbrThreads) {
        const bool valid = m0 + tid < gi.count;
        const int32_t i = gi.first + (valid ? m0 + tid : 0);
        const PosMass pi = xm[i];
        const double xi = pi.x, yi = pi.y, zi = pi.z;
        const int64_t o = perm[i];
        int32_t *row = CSR ? out + (valid ? off[o] : 0) : out + o * (int64_t)cap;
        int k = 0;
        for (int64_t t0 = nb; t0 < ne; t0 += kNbrTile) {
            // stage: box prefilter, compacted survivors
            bool cand = false;
            int32_t j = 0;
            double xj = 0.0, yj = 0.0, zj = 0.0;
            if (t0 + tid < ne) {
                j = n_idx[t0 + tid];
                const PosMass pj = xm[j];
                xj = pj.x;
                yj = pj.y;
                zj = pj.z;
                const double tx = axis_gap(xj, gi.lo[0], gi.hi[0]);
                const double ty = axis_gap(yj, gi.lo[1], gi.hi[1]);
                const double tz = axis_gap(zj, gi.lo[2], gi.hi[2]);
                cand = tx * tx + ty * ty + tz * tz < h2;
            }
            const uint64_t mc = ballot(cand);
            __syncthreads();   // previous tile consumed
            if (lane == 0) s_wn[w] = __popcll(mc);
            __syncthreads();
            int base = 0, nc = 0;
            for (int q = 0; q < kNbrWaves; ++q) {
                base += q < w ? s_wn[q] : 0;
                nc += s_wn[q];
            }
            if (cand) {
                const int p = base + count_below(mc);
                s_x[p] = xj;
                s_y[p] = yj;
                s_z[p] = zj;
                s_j[p] = j;
            }
            __syncthreads();
            if (!valid) continue;
            for (int c = 0; c < nc; ++c) {
                const double dx = s_x[c] - xi, dy = s_y[c] - yi, dz = s_z[c] - zi;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const int32_t jj = s_j[c];
                if (r2 < h2 && jj != i) {
                    if (CSR || k < cap) row[k] = perm[jj];
                    ++k;
                }
            }
        }
        if (!CSR && valid) {
            cnt[o] = k;
            kmax = k > kmax ? k : kmax;
        }
    }
    if (CSR) return;
    // longest row of the block: one update per block
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int v = __shfl_xor(kmax, d, kWave);
        kmax = v > kmax ? v : kmax;
    }
    __syncthreads();   // s_wn is free: every wave is past its last tile
    if (lane == 0) s_wn[w] = kmax;
    __syncthreads();
    if (tid == 0) {
        for (int q = 1; q < kNbrWaves; ++q) kmax = s_wn[q] > kmax ? s_wn[q] : kmax;
        // one word for the whole grid: only blocks that would raise it update
        // it (most blocks' longest rows are below the maximum already seen)
        const unsigned long long v = (tag << 32) | (unsigned long long)kmax;
        if (v > __hip_atomic_load(longest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(longest, v);
        if (kmax > cap) atomicMax(overflow, tag);
    }
}

// Pack row o from its slot into the CSR, ascending (rows are short: insertion
// sort), and write the caller's offsets.
__global__ void k_pack_rows(int64_t n, int32_t cap, const int32_t *__restrict__ slots,
                            const int64_t *__restrict__ off, int64_t *__restrict__ offsets,
                            int32_t *__restrict__ idx) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o > n) return;
    offsets[o] = off[o];
    if (o == n) return;
    const int64_t b0 = off[o], len = off[o + 1] - b0;
    const int32_t *src = slots + o * (int64_t)cap;
    int32_t *row = idx + b0;
    for (int64_t a = 0; a < len; ++a) {
        const int32_t v = src[a];
        int64_t b = a - 1;
        while (b >= 0 && row[b] > v) {
            row[b + 1] = row[b];
            --b;
        }
        row[b + 1] = v;
    }
}

// Sort each CSR row in place and copy the offsets to the caller.
__global__ void k_sort_rows(int64_t n, const int64_t *__restrict__ off, int64_t *__restrict__ offsets,
                            int32_t *__restrict__ idx) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o > n) return;
    offsets[o] = off[o];
    if (o == n) return;
    const int64_t b0 = off[o], len = off[o + 1] - b0;
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

// readback slots (int64 units) used here: neighbour total, overflow flag, longest row
enum { RB_NNZ = 40, RB_NOVF = 41, RB_NMAX = 42 };

// The search, the scan of the row lengths and their readback run on a second
// stream (the hard part's first auxiliary stream, idle outside its calls) as
// soon as the walk's lists are complete, beside the interaction kernel or
// whatever else the context's stream runs meanwhile: it only reads the tree
// and the lists and writes workspaces of its own.  The host waits for that
// stream alone; the rows are then packed into the caller's arrays on the
// context's stream, after the search.
int launch_neighbors(p3t_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *nnz,
                     hipEvent_t t0, hipEvent_t t1) {
    int rc;
    const int64_t n = ctx->n;
    if ((rc = aux_streams(ctx))) return rc;
    hipStream_t st = ctx->stream, as = ctx->aux[0];
    const unsigned grid = (unsigned)ctx->n_groups;
    if (grid == 0) return set_error(ctx, P3T_ESTATE, "no groups");
    const int32_t row_cap = ctx->nbr_cap > 0 ? ctx->nbr_cap : kNbrFirstCap;
    // A workspace (re)allocated here may come from an allocator that hands out
    // memory which work still queued on the context's stream uses: the search
    // then also waits for that work.
    void *const had[3] = {ctx->nbr_cnt.p, ctx->nbr_slots.p, ctx->nbr_scan.p};
    if ((rc = ensure(ctx, ctx->nbr_cnt, (n + 1) * sizeof(int64_t)))) return rc;
    if ((rc = ensure(ctx, ctx->nbr_slots, (size_t)n * row_cap * sizeof(int32_t) + 4))) return rc;
    if ((rc = ensure(ctx, ctx->nbr_scan, scan_tmp_bytes(n + 1)))) return rc;
    const bool fresh = had[0] != ctx->nbr_cnt.p || had[1] != ctx->nbr_slots.p ||
                       had[2] != ctx->nbr_scan.p;
    int64_t *cnt = ptr<int64_t>(ctx->nbr_cnt);
    int64_t *rb = ptr<int64_t>(ctx->readback);
    const ListsDev L = lists_dev(ctx);
    const double h2 = ctx->prm.r_search * ctx->prm.r_search;
    // every particle's count is written (groups partition the particles), and
    // the entry past the last one, which takes part in the scan, is zeroed;
    // the longest row and the overflow flag carry this call's tag (the slots
    // were cleared once, when the readback area was allocated)
    const unsigned long long tag = ++ctx->nbr_tag;
    auto *rbu = reinterpret_cast<unsigned long long *>(rb);
    if ((rc = check_hip(ctx, hipStreamWaitEvent(as, ctx->ev_lists, 0), "wait"))) return rc;
    if (fresh) {
        if ((rc = check_hip(ctx, hipEventRecord(ctx->ev_sync[0], st), "event record"))) return rc;
        if ((rc = check_hip(ctx, hipStreamWaitEvent(as, ctx->ev_sync[0], 0), "wait"))) return rc;
    }
    if (t0 && (rc = check_hip(ctx, hipEventRecord(t0, as), "event record"))) return rc;
    k_neighbors<false><<<grid, kNbrThreads, 0, as>>>(
        ptr<GroupInfo>(ctx->grp), L, ptr<PosMass>(ctx->xm), ptr<int32_t>(ctx->vals[0]), h2, row_cap,
        ptr<int32_t>(ctx->nbr_slots), nullptr, cnt, n, tag, rbu + RB_NMAX, rbu + RB_NOVF);
    if ((rc = check_hip(ctx, hipGetLastError(), "neighbours"))) return rc;
    if ((rc = scan_exclusive_i64_on(ctx, as, ctx->nbr_scan, cnt, cnt, n + 1, rb + RB_NNZ)))
        return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_NNZ, rb + RB_NNZ, 3 * sizeof(int64_t),
                                            hipMemcpyDeviceToHost, as), "readback")))
        return rc;
    if (t1 && (rc = check_hip(ctx, hipEventRecord(t1, as), "event record"))) return rc;
    if ((rc = check_hip(ctx, hipEventRecord(ctx->ev_sync[1], as), "event record"))) return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(as), "sync"))) return rc;
    // what follows on the context's stream comes after the search
    if ((rc = check_hip(ctx, hipStreamWaitEvent(st, ctx->ev_sync[1], 0), "wait"))) return rc;
    const int64_t total = ctx->hpin[RB_NNZ];
    const auto *hu = reinterpret_cast<const unsigned long long *>(ctx->hpin);
    const bool over = hu[RB_NOVF] == tag;
    const int64_t longest = (hu[RB_NMAX] >> 32) == tag ? (int64_t)(hu[RB_NMAX] & 0xffffffffull) : 0;
    // next call: room for rows a little longer than the longest seen, within
    // a workspace of at most 1 GiB
    int64_t want = longest + longest / 4 + 8;
    const int64_t limit = n > 0 ? ((int64_t)1 << 28) / n : kNbrFirstCap;
    want = want < kNbrFirstCap ? kNbrFirstCap : want;
    want = want > limit ? limit : want;
    ctx->nbr_cap = (int32_t)(want > 1 ? want : 1);
    *nnz = total;
    ctx->nnz = total;
    if (total > cap)
        return set_error(ctx, P3T_ECAPACITY, "neighbour buffer holds %lld entries, %lld needed",
                         (long long)cap, (long long)total);
    if (!over) {
        k_pack_rows<<<blocks_for(n + 1, 256), 256, 0, st>>>(n, row_cap, ptr<int32_t>(ctx->nbr_slots),
                                                            cnt, offsets, idx);
        return check_hip(ctx, hipGetLastError(), "neighbour pack");
    }
    // some row did not fit its slot: write the rows straight into the CSR
    if (grid) {
        k_neighbors<true><<<grid, kNbrThreads, 0, st>>>(
            ptr<GroupInfo>(ctx->grp), L, ptr<PosMass>(ctx->xm), ptr<int32_t>(ctx->vals[0]), h2, 0,
            idx, cnt, nullptr, n, tag, nullptr, nullptr);
        if ((rc = check_hip(ctx, hipGetLastError(), "neighbours (CSR)"))) return rc;
    }
    k_sort_rows<<<blocks_for(n + 1, 256), 256, 0, st>>>(n, cnt, offsets, idx);
    return check_hip(ctx, hipGetLastError(), "neighbour sort");
}

}  // namespace p3t
