// walk.hip -- grouped tree walk (Section 2.2: Barnes-Hut with opening angle
// theta, walked once per group).  One wavefront walks the tree for one group
// and emits three lists:
//   C_g  accepted cells (multipole interactions),
//   F_g  particles of opened leaves whose box is at least h* = max(h, r_out)
//        away from the group box: for them K = W = 1 and j != i,
//   N_g  particles of the other opened leaves: the only candidates for
//        neighbours of the group's particles and for K, W < 1.
// The particle list P_g of the method is F_g + N_g.
// A cell c is accepted iff theta^2 * D^2(com_c, box_g) > side_c^2 and
// B^2(box_c, box_g) >= h^2, with D the point-to-box and B the box-to-box gap
// distance, each summed as (tx*tx + ty*ty) + tz*tz over per-axis gaps
// t = max(max(lo - p, 0), p - hi).  This file is compiled with
// -ffp-contract=off so these decisions are reproducible bit for bit.
//
// The walk is wavefront-cooperative: up to 64 pending nodes are popped from a
// stack, classified in parallel, and the children of opened internal nodes are
// pushed back.  Node levels never decrease towards the top of the stack and at
// most 8*64 entries of one level are pending at once, so 22*512 entries bound
// the stack; the walk runs with a small stack in LDS and falls back to a
// per-block stack of that bound in global memory if a group overflows it.
//
// The lists are produced in two passes: count, prefix-sum, then walk again
// writing at the exact offsets; the statistics (interaction counts, longest
// lists) are reductions over the per-group counts, so no two groups ever
// update the same memory word.
#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kWalkThreads = 64;        // one wavefront per block
constexpr int kLdsStack = 2048;
constexpr int kGlobalStack = kLevels * 8 * kWave + kWave;

enum WalkMode { kCount = 0, kEmit = 1 };

struct WalkParams {
    double th2, h2, hn2;   // theta^2, h^2, max(h, r_out)^2
};

// Device outputs of one walk launch.
struct WalkOut {
    int64_t *cnt;            // [3][stride] per-group counts (count pass)
    int64_t *beg, *end;      // [3][stride] segments (emit pass)
    int32_t *idx[3];         // final lists
    int32_t *stack_ovf;
    int64_t stride;
};

__device__ __forceinline__ double gap(double u, double v) {
    const double w = u > 0.0 ? u : 0.0;
    return v > w ? v : w;
}

template <int MODE>
__global__ __launch_bounds__(kWalkThreads) void k_walk(const GroupInfo *__restrict__ grp,
                                                        const int32_t *__restrict__ n_groups_dev,
                                                        const NodeWalk *__restrict__ nodes,
                                                        WalkParams wp, WalkOut wo,
                                                        int32_t *__restrict__ gstack, int use_global) {
    __shared__ int32_t lstack[kLdsStack];
    int32_t *stk = use_global ? gstack + (int64_t)blockIdx.x * kGlobalStack : lstack;
    const int cap = use_global ? kGlobalStack : kLdsStack;
    const int lane = threadIdx.x;
    const int G = *n_groups_dev;
    const int64_t S = wo.stride;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const GroupInfo gi = grp[g];
        int64_t run[3] = {0, 0, 0};
        int32_t *dst[3] = {nullptr, nullptr, nullptr};
        if (MODE == kEmit)
            for (int k = 0; k < 3; ++k) dst[k] = wo.idx[k] + wo.beg[k * S + g];
        int sp = 1;
        if (lane == 0) stk[0] = 0;
        __syncthreads();
        bool ovf = false;
        while (sp > 0) {
            const int k = sp < kWave ? sp : kWave;
            const int base = sp - k;
            const int32_t node = lane < k ? stk[base + lane] : -1;
            sp = base;
            __syncthreads();
            bool acc = false, leaf = false, near = false;
            int32_t first = 0, count = 0, cf = 0, ncld = 0;
            if (node >= 0) {
                const NodeWalk nd = nodes[node];
                const double t0 = gap(gi.lo[0] - nd.cx, nd.cx - gi.hi[0]);
                const double t1 = gap(gi.lo[1] - nd.cy, nd.cy - gi.hi[1]);
                const double t2 = gap(gi.lo[2] - nd.cz, nd.cz - gi.hi[2]);
                const double D2 = t0 * t0 + t1 * t1 + t2 * t2;
                const double b0 = gap(nd.lo[0] - gi.hi[0], gi.lo[0] - nd.hi[0]);
                const double b1 = gap(nd.lo[1] - gi.hi[1], gi.lo[1] - nd.hi[1]);
                const double b2 = gap(nd.lo[2] - gi.hi[2], gi.lo[2] - nd.hi[2]);
                const double B2 = b0 * b0 + b1 * b1 + b2 * b2;
                acc = (wp.th2 * D2 > nd.l2) && (B2 >= wp.h2);
                leaf = nd.n_child == 0;
                near = B2 < wp.hn2;
                first = nd.first;
                count = nd.count;
                cf = nd.child_first;
                ncld = nd.n_child;
            }
            const bool isC = node >= 0 && acc;
            const bool isO = node >= 0 && !acc && !leaf;
            const bool isF = node >= 0 && !acc && leaf && !near;
            const bool isN = node >= 0 && !acc && leaf && near;
            // accepted cells
            {
                const uint64_t mC = ballot(isC);
                if (MODE == kEmit && isC) dst[0][run[0] + count_below(mC)] = node;
                run[0] += __popcll(mC);
            }
            // particles of far, then near, opened leaves
#pragma unroll
            for (int kk = 1; kk < 3; ++kk) {
                const bool mine = kk == 1 ? isF : isN;
                const int c = mine ? count : 0;
                int tot;
                const int excl = wave_excl_count(c, tot);
                if (MODE == kEmit && mine) {
                    int32_t *d = dst[kk] + run[kk] + excl;
                    for (int t = 0; t < c; ++t) d[t] = first + t;
                }
                run[kk] += tot;
            }
            // children of opened internal nodes (at most 8 each)
            const int ocnt = isO ? ncld : 0;
            int otot;
            const int oexcl = wave_excl_small<4>(ocnt, otot);
            if (sp + otot > cap) {
                ovf = true;
                break;
            }
            if (isO) {
                int32_t *d = stk + sp + oexcl;
                for (int t = 0; t < ocnt; ++t) d[t] = cf + t;
            }
            sp += otot;
            __syncthreads();
        }
        __syncthreads();
        if (ovf) {
            if (lane == 0) atomicOr(wo.stack_ovf, 1);
            continue;
        }
        if (lane == 0) {
            for (int k = 0; k < 3; ++k) {
                if (MODE == kCount) wo.cnt[k * S + g] = run[k];
                else wo.end[k * S + g] = wo.beg[k * S + g] + run[k];
            }
        }
    }
}

// Statistics from the per-group counts: interactions sum_g n_g |C_g| and
// sum_g n_g (|F_g| + |N_g|), and the longest list of each kind.
__global__ __launch_bounds__(256) void k_walk_stats(const GroupInfo *__restrict__ grp,
                                                    const int32_t *__restrict__ n_groups_dev,
                                                    const int64_t *__restrict__ cnt, int64_t S,
                                                    unsigned long long *__restrict__ out) {
    const int G = *n_groups_dev;
    unsigned long long pc = 0, pp = 0, mx[3] = {0, 0, 0};
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
        const unsigned long long n = (unsigned long long)grp[g].count;
        const unsigned long long c0 = cnt[g], c1 = cnt[S + g], c2 = cnt[2 * S + g];
        pc += n * c0;
        pp += n * (c1 + c2);
        mx[0] = c0 > mx[0] ? c0 : mx[0];
        mx[1] = c1 > mx[1] ? c1 : mx[1];
        mx[2] = c2 > mx[2] ? c2 : mx[2];
    }
    pc = wave_sum(pc);
    pp = wave_sum(pp);
    for (int k = 0; k < 3; ++k)
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const unsigned long long o = __shfl_xor(mx[k], d, kWave);
            mx[k] = o > mx[k] ? o : mx[k];
        }
    if (lane_id() == 0) {   // one update per wavefront
        atomicAdd(&out[0], pc);
        atomicAdd(&out[1], pp);
        for (int k = 0; k < 3; ++k) atomicMax(&out[3 + k], mx[k]);
    }
}

static unsigned walk_grid(p3t_ctx *ctx) {
    int64_t g = ctx->n_nodes < 8192 ? ctx->n_nodes : 8192;
    return (unsigned)(g > 0 ? g : 1);
}

ListsDev lists_dev(const p3t_ctx *ctx) {
    ListsDev L;
    const int64_t stride = ctx->n_nodes + 1;
    const int64_t *beg = ptr<int64_t>(ctx->off), *end = ptr<int64_t>(ctx->seg_end);
    const DevBuf *bufs[3] = {&ctx->c_idx, &ctx->p_idx, &ctx->n_idx};
    for (int k = 0; k < 3; ++k) {
        L.beg[k] = beg + k * stride;
        L.end[k] = end + k * stride;
        L.idx[k] = ptr<int32_t>(*bufs[k]);
    }
    return L;
}

// read-back slots of the walk (int64 units of the readback area); slot 32 holds
// the leaf count written while marking groups
enum { RB_TOT = 24, RB_G = 28, RB_STACK = 29, RB_INTER = 30, RB_LEAVES = 32, RB_MAX = 33 };

int build_lists(p3t_ctx *ctx) {
    int rc;
    const int64_t nn = ctx->n_nodes;   // bound on the number of groups
    const int64_t stride = nn + 1;
    if ((rc = ensure(ctx, ctx->cnt, 3 * stride * sizeof(int64_t)))) return rc;
    if ((rc = ensure(ctx, ctx->off, 3 * stride * sizeof(int64_t)))) return rc;
    if ((rc = ensure(ctx, ctx->seg_end, 3 * stride * sizeof(int64_t)))) return rc;
    int64_t *cnt = ptr<int64_t>(ctx->cnt), *off = ptr<int64_t>(ctx->off);
    int64_t *end = ptr<int64_t>(ctx->seg_end);
    int64_t *rb = ptr<int64_t>(ctx->readback);
    int32_t *flags = ptr<int32_t>(ctx->dflags);
    const int32_t *G_dev = ptr<int32_t>(ctx->gscan) + ctx->n;
    const double hn = ctx->prm.r_search > ctx->prm.r_out ? ctx->prm.r_search : ctx->prm.r_out;
    const WalkParams wp{ctx->prm.theta * ctx->prm.theta, ctx->prm.r_search * ctx->prm.r_search,
                        hn * hn};
    const unsigned grid = walk_grid(ctx);
    hipStream_t st = ctx->stream;
    DevBuf *lbuf[3] = {&ctx->c_idx, &ctx->p_idx, &ctx->n_idx};
    WalkOut wo{};
    wo.cnt = cnt;
    wo.beg = off;
    wo.end = end;
    wo.stack_ovf = flags + 1;
    wo.stride = stride;

    for (int attempt = 0; attempt < 2; ++attempt) {
        const int use_global = attempt;
        if (use_global) {
            if ((rc = ensure(ctx, ctx->wstack, (size_t)grid * kGlobalStack * sizeof(int32_t))))
                return rc;
        }
        if ((rc = check_hip(ctx, hipMemsetAsync(flags + 1, 0, sizeof(int32_t), st), "memset")))
            return rc;
        // entries past the last group take part in the scans as zeros
        if ((rc = check_hip(ctx, hipMemsetAsync(cnt, 0, 3 * stride * sizeof(int64_t), st), "memset")))
            return rc;
        if ((rc = check_hip(ctx, hipMemsetAsync(rb + RB_INTER, 0, 2 * sizeof(int64_t), st), "memset")))
            return rc;
        if ((rc = check_hip(ctx, hipMemsetAsync(rb + RB_MAX, 0, 3 * sizeof(int64_t), st), "memset")))
            return rc;
        k_walk<kCount><<<grid, kWalkThreads, 0, st>>>(ptr<GroupInfo>(ctx->grp), G_dev,
                                                       ptr<NodeWalk>(ctx->node_walk), wp, wo,
                                                       ptr<int32_t>(ctx->wstack), use_global);
        if ((rc = check_hip(ctx, hipGetLastError(), "walk count"))) return rc;
        k_walk_stats<<<64, 256, 0, st>>>(ptr<GroupInfo>(ctx->grp), G_dev, cnt, stride,
                                         (unsigned long long *)(rb + RB_INTER));
        if ((rc = check_hip(ctx, hipGetLastError(), "walk stats"))) return rc;
        for (int k = 0; k < 3; ++k)
            if ((rc = scan_exclusive_i64(ctx, cnt + k * stride, off + k * stride, stride,
                                         rb + RB_TOT + k)))
                return rc;
        // read back: list totals, statistics, group count, stack overflow flag
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_TOT, rb + RB_TOT,
                                                (RB_MAX + 3 - RB_TOT) * sizeof(int64_t),
                                                hipMemcpyDeviceToHost, st), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_G, G_dev, sizeof(int32_t),
                                                hipMemcpyDeviceToHost, st), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_STACK, flags + 1, sizeof(int32_t),
                                                hipMemcpyDeviceToHost, st), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
        if (!*(int32_t *)(ctx->hpin + RB_STACK)) {
            ctx->walk_global = use_global;
            break;
        }
        if (use_global) return set_error(ctx, P3T_EINVAL, "tree walk stack overflow");
    }
    ctx->n_groups = *(int32_t *)(ctx->hpin + RB_G);
    ctx->n_cell_entries = ctx->hpin[RB_TOT];
    ctx->n_part_entries = ctx->hpin[RB_TOT + 1];
    ctx->n_near_entries = ctx->hpin[RB_TOT + 2];
    ctx->n_pc = ctx->hpin[RB_INTER];
    ctx->n_pp = ctx->hpin[RB_INTER + 1];
    ctx->n_leaves = ctx->hpin[RB_LEAVES];
    for (int k = 0; k < 3; ++k) {
        if ((rc = ensure(ctx, *lbuf[k], (ctx->hpin[RB_TOT + k] + 1) * sizeof(int32_t)))) return rc;
        wo.idx[k] = ptr<int32_t>(*lbuf[k]);
    }
    k_walk<kEmit><<<grid, kWalkThreads, 0, st>>>(ptr<GroupInfo>(ctx->grp), G_dev,
                                                  ptr<NodeWalk>(ctx->node_walk), wp, wo,
                                                  ptr<int32_t>(ctx->wstack), ctx->walk_global);
    return check_hip(ctx, hipGetLastError(), "walk emit");
}

}  // namespace p3t
