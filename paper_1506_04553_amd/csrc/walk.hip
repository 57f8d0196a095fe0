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
// the stack; the walk first runs with a small stack in LDS and falls back to a
// per-block stack of that bound in global memory if a group overflows it.
#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kWalkThreads = 64;        // one wavefront per block
constexpr int kLdsStack = 2048;
constexpr int kGlobalStack = kLevels * 8 * kWave + kWave;

struct WalkParams {
    double th2, h2, hn2;   // theta^2, h^2, max(h, r_out)^2
};

__device__ __forceinline__ double gap(double u, double v) {
    const double w = u > 0.0 ? u : 0.0;
    return v > w ? v : w;
}

template <bool EMIT>
__global__ __launch_bounds__(kWalkThreads) void k_walk(
    const GroupInfo *__restrict__ grp, const int32_t *__restrict__ n_groups_dev,
    const NodeWalk *__restrict__ nodes, WalkParams wp, int64_t *__restrict__ cnt_c,
    int64_t *__restrict__ cnt_p, int64_t *__restrict__ cnt_n, const int64_t *__restrict__ off_c,
    const int64_t *__restrict__ off_p, const int64_t *__restrict__ off_n, int32_t *__restrict__ c_idx,
    int32_t *__restrict__ p_idx, int32_t *__restrict__ n_idx, int32_t *__restrict__ gstack,
    int use_global, int32_t *__restrict__ overflow, unsigned long long *__restrict__ inter) {
    __shared__ int32_t lstack[kLdsStack];
    int32_t *stk = use_global ? gstack + (int64_t)blockIdx.x * kGlobalStack : lstack;
    const int cap = use_global ? kGlobalStack : kLdsStack;
    const int lane = threadIdx.x;
    const int G = *n_groups_dev;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const GroupInfo gi = grp[g];
        int64_t nc = 0, np = 0, nn = 0;
        const int64_t oc = EMIT ? off_c[g] : 0, op = EMIT ? off_p[g] : 0, on = EMIT ? off_n[g] : 0;
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
            const uint64_t mC = ballot(isC);
            if (EMIT && isC) c_idx[oc + nc + count_below(mC)] = node;
            nc += __popcll(mC);
            // particles of far opened leaves
            const int pcnt = isF ? count : 0;
            const int pincl = wave_incl_scan(pcnt);
            const int ptot = __shfl(pincl, kWave - 1, kWave);
            if (EMIT && isF) {
                int32_t *dst = p_idx + op + np + (pincl - pcnt);
                for (int t = 0; t < pcnt; ++t) dst[t] = first + t;
            }
            np += ptot;
            // particles of near opened leaves
            const int ncnt = isN ? count : 0;
            const int nincl = wave_incl_scan(ncnt);
            const int ntot = __shfl(nincl, kWave - 1, kWave);
            if (EMIT && isN) {
                int32_t *dst = n_idx + on + nn + (nincl - ncnt);
                for (int t = 0; t < ncnt; ++t) dst[t] = first + t;
            }
            nn += ntot;
            // children of opened internal nodes
            const int ocnt = isO ? ncld : 0;
            const int oincl = wave_incl_scan(ocnt);
            const int otot = __shfl(oincl, kWave - 1, kWave);
            if (sp + otot > cap) {
                ovf = true;
                break;
            }
            if (isO) {
                int32_t *dst = stk + sp + (oincl - ocnt);
                for (int t = 0; t < ocnt; ++t) dst[t] = cf + t;
            }
            sp += otot;
            __syncthreads();
        }
        __syncthreads();
        if (ovf) {
            if (lane == 0) atomicOr(overflow, 1);
            continue;
        }
        if (!EMIT && lane == 0) {
            cnt_c[g] = nc;
            cnt_p[g] = np;
            cnt_n[g] = nn;
            atomicAdd(&inter[0], (unsigned long long)(gi.count * nc));
            atomicAdd(&inter[1], (unsigned long long)(gi.count * (np + nn)));
        }
    }
}

static unsigned walk_grid(p3t_ctx *ctx) {
    int64_t g = ctx->n_nodes < 8192 ? ctx->n_nodes : 8192;
    return (unsigned)(g > 0 ? g : 1);
}

int build_lists(p3t_ctx *ctx) {
    int rc;
    const int64_t nn = ctx->n_nodes;   // bound on the number of groups
    const int64_t stride = nn + 1;
    if ((rc = ensure(ctx, ctx->cnt, 3 * stride * sizeof(int64_t)))) return rc;
    if ((rc = ensure(ctx, ctx->off, 3 * stride * sizeof(int64_t)))) return rc;
    int64_t *cnt = ptr<int64_t>(ctx->cnt), *off = ptr<int64_t>(ctx->off);
    int64_t *rb = ptr<int64_t>(ctx->readback);
    int32_t *flags = ptr<int32_t>(ctx->dflags);
    const int32_t *G_dev = ptr<int32_t>(ctx->gscan) + ctx->n;
    const double hn = ctx->prm.r_search > ctx->prm.r_out ? ctx->prm.r_search : ctx->prm.r_out;
    const WalkParams wp{ctx->prm.theta * ctx->prm.theta, ctx->prm.r_search * ctx->prm.r_search,
                        hn * hn};
    const unsigned grid = walk_grid(ctx);

    for (int attempt = 0; attempt < 2; ++attempt) {
        const int use_global = attempt;
        if (use_global) {
            if ((rc = ensure(ctx, ctx->wstack, (size_t)grid * kGlobalStack * sizeof(int32_t)))) return rc;
        }
        if ((rc = check_hip(ctx, hipMemsetAsync(cnt, 0, 3 * stride * sizeof(int64_t), ctx->stream),
                            "memset")))
            return rc;
        if ((rc = check_hip(ctx, hipMemsetAsync(flags + 1, 0, sizeof(int32_t), ctx->stream), "memset")))
            return rc;
        if ((rc = check_hip(ctx, hipMemsetAsync(rb + 30, 0, 2 * sizeof(int64_t), ctx->stream), "memset")))
            return rc;
        k_walk<false><<<grid, kWalkThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), G_dev, ptr<NodeWalk>(ctx->node_walk), wp, cnt, cnt + stride,
            cnt + 2 * stride, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
            ptr<int32_t>(ctx->wstack), use_global, flags + 1, (unsigned long long *)(rb + 30));
        if ((rc = check_hip(ctx, hipGetLastError(), "walk count"))) return rc;
        for (int k = 0; k < 3; ++k)
            if ((rc = scan_exclusive_i64(ctx, cnt + k * stride, off + k * stride, stride, rb + 24 + k)))
                return rc;
        // read back: groups, list totals, overflow flag
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + 24, rb + 24, 9 * sizeof(int64_t),
                                                hipMemcpyDeviceToHost, ctx->stream), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + 28, G_dev, sizeof(int32_t),
                                                hipMemcpyDeviceToHost, ctx->stream), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + 29, flags + 1, sizeof(int32_t),
                                                hipMemcpyDeviceToHost, ctx->stream), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
        const int32_t ovf = *(int32_t *)(ctx->hpin + 29);
        if (!ovf) {
            ctx->walk_global = use_global;
            break;
        }
        if (use_global) return set_error(ctx, P3T_EINVAL, "tree walk stack overflow");
    }
    ctx->n_groups = *(int32_t *)(ctx->hpin + 28);
    ctx->n_cell_entries = ctx->hpin[24];
    ctx->n_part_entries = ctx->hpin[25];
    ctx->n_near_entries = ctx->hpin[26];
    ctx->n_pc = ctx->hpin[30];
    ctx->n_pp = ctx->hpin[31];
    ctx->n_leaves = ctx->hpin[32];
    if ((rc = ensure(ctx, ctx->c_idx, (ctx->n_cell_entries + 1) * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->p_idx, (ctx->n_part_entries + 1) * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->n_idx, (ctx->n_near_entries + 1) * sizeof(int32_t)))) return rc;
    k_walk<true><<<grid, kWalkThreads, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), G_dev, ptr<NodeWalk>(ctx->node_walk), wp, nullptr, nullptr,
        nullptr, off, off + stride, off + 2 * stride, ptr<int32_t>(ctx->c_idx),
        ptr<int32_t>(ctx->p_idx), ptr<int32_t>(ctx->n_idx), ptr<int32_t>(ctx->wstack),
        ctx->walk_global, flags + 1, nullptr);
    return check_hip(ctx, hipGetLastError(), "walk emit");
}

}  // namespace p3t
