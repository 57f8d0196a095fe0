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
// Two ways to lay out the lists, both as one (begin, end) segment per group and
// list, with no two groups ever updating the same memory word:
//   fixed stride (when an earlier build gives the group count and the longest
//     lists): group g writes list k at g * cap_k in a single walk; a group
//     beyond the estimated count or a list longer than cap_k raises a flag and
//     the build falls back to
//   two passes: count, prefix-sum, then walk again writing at the exact
//     offsets (segments tile the arrays).
// The statistics (list totals, interaction counts, longest lists) are
// reductions over the per-group counts.
#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kWalkThreads = 64;        // one wavefront per block
constexpr int kWalkGrid = 8192;         // 32 resident wavefronts on each of 256 CUs
constexpr int kLdsStack = 1536;
constexpr int kGlobalStack = kLevels * 8 * kWave + kWave;

enum WalkMode { kCount = 0, kEmit = 1, kFixed = 2 };

struct WalkParams {
    double th2, h2, hn2;   // theta^2, h^2, max(h, r_out)^2
};

// Device outputs of one walk launch.
struct WalkOut {
    int64_t *cnt;            // [3][stride] per-group counts (count and fixed passes)
    int64_t *beg, *end;      // [3][stride] segments (emit and fixed passes)
    int32_t *idx[3];         // lists
    int64_t cap[3];          // fixed: entries reserved per group and list
    int64_t gcap;            // fixed: groups the lists have room for
    int32_t *stack_ovf;      // set if a group overflowed even the global stack
    int32_t *spilled;        // groups that walked on the global stack
    int32_t *cap_ovf;        // fixed: set if some group did not fit
    int64_t stride;
};

// the c consecutive indices first .. first + c - 1 at d, four to a store (the
// stores need only 4-byte alignment)
typedef int32_t int4u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ void write_range(int32_t *d, int32_t first, int c) {
    int t = 0;
    for (; t + 4 <= c; t += 4) {
        const int32_t f = first + t;
        *reinterpret_cast<int4u *>(d + t) = int4u{f, f + 1, f + 2, f + 3};
    }
    for (; t < c; ++t) d[t] = first + t;
}

__device__ __forceinline__ double gap(double u, double v) {
    const double w = u > 0.0 ? u : 0.0;
    return v > w ? v : w;
}

template <int MODE>
__global__ __launch_bounds__(kWalkThreads) void k_walk(const GroupInfo *__restrict__ grp,
                                                        const int32_t *__restrict__ n_groups_dev,
                                                        const NodeWalk *__restrict__ nodes,
                                                        WalkParams wp, WalkOut wo,
                                                        int32_t *__restrict__ gstack, int lds_cap) {
    __shared__ int32_t lstack[kLdsStack];
    int32_t *const gstk = gstack + (int64_t)blockIdx.x * kGlobalStack;
    const int lane = threadIdx.x;
    const int G = *n_groups_dev;
    const int64_t S = wo.stride;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const GroupInfo gi = grp[g];
        int64_t run[3] = {0, 0, 0};
        int32_t *dst[3] = {nullptr, nullptr, nullptr};
        if (MODE == kFixed && g >= wo.gcap) {
            if (lane == 0) atomicOr(wo.cap_ovf, 1);
            continue;
        }
        if (MODE == kEmit)
            for (int k = 0; k < 3; ++k) dst[k] = wo.idx[k] + wo.beg[k * S + g];
        if (MODE == kFixed)
            for (int k = 0; k < 3; ++k) dst[k] = wo.idx[k] + (int64_t)g * wo.cap[k];
        // the walk runs on the LDS stack; a group whose pending nodes outgrow
        // it walks again from the root on this block's stack in global memory
        bool ovf = false;
        for (int pass = 0; pass < 2; ++pass) {
            int32_t *const stk = pass ? gstk : lstack;
            const int cap = pass ? kGlobalStack : lds_cap;
            run[0] = run[1] = run[2] = 0;
            int sp = 1;
            ovf = false;
            if (lane == 0) stk[0] = 0;
            __syncthreads();
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
                    if (MODE != kCount && isC) {
                        const int64_t pos = run[0] + count_below(mC);
                        if (MODE == kEmit || pos < wo.cap[0]) dst[0][pos] = node;
                    }
                    run[0] += __popcll(mC);
                }
                // particles of far, then near, opened leaves
    #pragma unroll
                for (int kk = 1; kk < 3; ++kk) {
                    const bool mine = kk == 1 ? isF : isN;
                    const int c = mine ? count : 0;
                    int tot;
                    const int excl = wave_excl_count(c, tot);
                    if (MODE == kEmit && mine) write_range(dst[kk] + run[kk] + excl, first, c);
                    if (MODE == kFixed && mine) {
                        const int64_t pos = run[kk] + excl;
                        const int64_t lim = wo.cap[kk] - pos;
                        const int cc = lim < c ? (lim > 0 ? (int)lim : 0) : c;
                        write_range(dst[kk] + pos, first, cc);
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
            if (!ovf) break;
            if (lane == 0) atomicAdd(pass ? wo.stack_ovf : wo.spilled, 1);
        }
        if (ovf) continue;   // cannot happen: the global stack holds the bound
        if (lane == 0) {
            bool over = false;
            for (int k = 0; k < 3; ++k) {
                if (MODE == kCount) wo.cnt[k * S + g] = run[k];
                if (MODE == kEmit) wo.end[k * S + g] = wo.beg[k * S + g] + run[k];
                if (MODE == kFixed) {
                    const int64_t b = (int64_t)g * wo.cap[k];
                    over = over || run[k] > wo.cap[k];
                    wo.cnt[k * S + g] = run[k];
                    wo.beg[k * S + g] = b;
                    wo.end[k * S + g] = b + (run[k] < wo.cap[k] ? run[k] : wo.cap[k]);
                }
            }
            if (over) atomicOr(wo.cap_ovf, 1);
        }
    }
}

// Walk results read back by the host (int64 slots).
struct WalkStats {
    unsigned long long total[3];   // sum over groups of |C_g|, |F_g|, |N_g|
    unsigned long long n_groups;
    unsigned long long pc, pp;     // sum_g n_g |C_g|, sum_g n_g (|F_g| + |N_g|)
    unsigned long long pp_near;    // sum_g n_g |N_g|
    unsigned long long n_leaves;
    unsigned long long maxlen[3];  // longest list of each kind
    int32_t stack_ovf, cap_ovf;    // flags written by the walk
    int32_t spilled, pad;          // groups that needed the global stack
};

static_assert(sizeof(WalkStats) == kRbWalkWords * 8, "walk statistics slots");

constexpr int kOrderBins = 128;   // launch-order buckets (see below)

// Statistics from the per-group counts, and the leaf count of the tree; also
// clears the launch-order bucket counts.
__global__ __launch_bounds__(1024) void k_walk_stats(const GroupInfo *__restrict__ grp,
                                                    const int32_t *__restrict__ n_groups_dev,
                                                    const int64_t *__restrict__ cnt, int64_t S,
                                                    const int32_t *__restrict__ nchild,
                                                    int64_t n_nodes, WalkStats *__restrict__ out,
                                                    uint32_t *__restrict__ order_hist) {
    const int G = *n_groups_dev;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 < kOrderBins) order_hist[t0] = 0;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    unsigned long long tot[3] = {0, 0, 0}, mx[3] = {0, 0, 0}, pc = 0, pp = 0, ppn = 0, lv = 0;
    for (int64_t g = t0; g < G; g += nt) {
        const unsigned long long n = (unsigned long long)grp[g].count;
        for (int k = 0; k < 3; ++k) {
            const unsigned long long c = cnt[k * S + g];
            tot[k] += c;
            mx[k] = c > mx[k] ? c : mx[k];
        }
        pc += n * cnt[g];
        pp += n * (cnt[S + g] + cnt[2 * S + g]);
        ppn += n * cnt[2 * S + g];
    }
    for (int64_t i = t0; i < n_nodes; i += nt) lv += nchild[i] == 0;
    // wave reductions, then one set of updates per block
    __shared__ unsigned long long s_red[16][10];
    unsigned long long v[10] = {pc, pp, ppn, lv, tot[0], tot[1], tot[2], mx[0], mx[1], mx[2]};
    for (int k = 0; k < 7; ++k) v[k] = wave_sum(v[k]);
    for (int k = 7; k < 10; ++k)
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const unsigned long long o = __shfl_xor(v[k], d, kWave);
            v[k] = o > v[k] ? o : v[k];
        }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0)
        for (int k = 0; k < 10; ++k) s_red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x / kWave); ++q) {
            for (int k = 0; k < 7; ++k) v[k] += s_red[q][k];
            for (int k = 7; k < 10; ++k) v[k] = s_red[q][k] > v[k] ? s_red[q][k] : v[k];
        }
        atomicAdd(&out->pc, v[0]);
        atomicAdd(&out->pp, v[1]);
        atomicAdd(&out->pp_near, v[2]);
        atomicAdd(&out->n_leaves, v[3]);
        for (int k = 0; k < 3; ++k) {
            atomicAdd(&out->total[k], v[4 + k]);
            atomicMax(&out->maxlen[k], v[7 + k]);
        }
    }
    if (t0 == 0) out->n_groups = (unsigned long long)G;
}

static unsigned walk_grid(p3t_ctx *ctx) {
    int64_t g = ctx->n_nodes < kWalkGrid ? ctx->n_nodes : kWalkGrid;
    return (unsigned)(g > 0 ? g : 1);
}

ListsDev lists_dev(const p3t_ctx *ctx) {
    ListsDev L;
    L.order = ptr<int32_t>(ctx->gorder);
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

// ---------------------------------------------------------------------------
// Launch order of the per-group kernels: groups in buckets of estimated work
// (quarter octaves of n_g (35 |C_g| + 15 |P_g|), the interaction kernel's
// instruction count), largest first; the order inside a bucket is arbitrary
// (it decides only which block runs which group).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int order_bin(const GroupInfo &gi, const int64_t *cnt, int64_t S, int g) {
    const float cost = (float)gi.count * (35.0f * (float)cnt[g] +
                                          15.0f * (float)(cnt[S + g] + cnt[2 * S + g]));
    int b = (int)(4.0f * log2f(cost + 1.0f));
    b = b < 0 ? 0 : (b > kOrderBins - 1 ? kOrderBins - 1 : b);
    return kOrderBins - 1 - b;
}

// bucket counts (one atomic per bucket and wavefront) and each group's rank in its bucket
__global__ __launch_bounds__(256) void k_order_count(const GroupInfo *__restrict__ grp, int64_t G,
                                                     const int64_t *__restrict__ cnt, int64_t S,
                                                     uint32_t *__restrict__ hist,
                                                     int32_t *__restrict__ rank) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = g < G;
    const int b = valid ? order_bin(grp[g], cnt, S, (int)g) : 0;
    uint64_t same = ballot(valid);
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const bool bit = (b >> k) & 1;
        const uint64_t bb = ballot(bit);
        same &= bit ? bb : ~bb;
    }
    const int leader = valid ? __ffsll((long long)same) - 1 : 0;
    uint32_t base = 0;
    if (valid && lane_id() == leader) base = atomicAdd(&hist[b], (uint32_t)__popcll(same));
    base = __shfl(base, leader, kWave);
    if (valid) rank[g] = (b << 24) | (int32_t)(base + count_below(same));
}

// each block takes the bucket starts (exclusive scan of the counts) itself
__global__ __launch_bounds__(256) void k_order_place(int64_t G, const int32_t *__restrict__ rank,
                                                     const uint32_t *__restrict__ hist,
                                                     int32_t *__restrict__ order) {
    static_assert(kOrderBins <= 256, "one thread per bucket");
    __shared__ uint32_t s_cnt[kOrderBins], s_start[kOrderBins];
    const int t = threadIdx.x;
    if (t < kOrderBins) s_cnt[t] = hist[t];
    __syncthreads();
    if (t < kOrderBins) {
        uint32_t e = 0;
        for (int k = 0; k < t; ++k) e += s_cnt[k];
        s_start[t] = e;
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + t;
    if (g >= G) return;
    const int32_t r = rank[g];
    order[s_start[r >> 24] + (r & 0xffffff)] = (int32_t)g;
}

__global__ void k_order_identity(int64_t G, int32_t *__restrict__ order) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G) order[g] = (int32_t)g;
}

static int build_order(p3t_ctx *ctx, int64_t stride) {
    int rc;
    const int64_t G = ctx->n_groups;
    if ((rc = ensure(ctx, ctx->gorder, (G + 1) * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->grank, (G + 1) * sizeof(int32_t)))) return rc;
    if (G <= 0) return P3T_OK;
    if (G >= (1 << 24)) {   // ranks are packed in 24 bits: keep the group order
        k_order_identity<<<blocks_for(G, 256), 256, 0, ctx->stream>>>(G, ptr<int32_t>(ctx->gorder));
        return check_hip(ctx, hipGetLastError(), "group order");
    }
    // the bucket counts were cleared by the walk statistics
    uint32_t *hist = ptr<uint32_t>(ctx->ghist);
    k_order_count<<<blocks_for(G, 256), 256, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), G, ptr<int64_t>(ctx->cnt), stride, hist, ptr<int32_t>(ctx->grank));
    k_order_place<<<blocks_for(G, 256), 256, 0, ctx->stream>>>(G, ptr<int32_t>(ctx->grank), hist,
                                                              ptr<int32_t>(ctx->gorder));
    return check_hip(ctx, hipGetLastError(), "group order");
}

static int run_walk_stats(p3t_ctx *ctx, const int32_t *G_dev, int64_t stride, WalkStats *ws) {
    // few large blocks: the block results meet in same-address atomics
    k_walk_stats<<<32, 1024, 0, ctx->stream>>>(ptr<GroupInfo>(ctx->grp), G_dev,
                                              ptr<int64_t>(ctx->cnt), stride,
                                              ptr<int32_t>(ctx->node_nchild), ctx->n_nodes, ws,
                                              ptr<uint32_t>(ctx->ghist));
    int rc = check_hip(ctx, hipGetLastError(), "walk stats");
    if (rc) return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + kRbWalk, ws, sizeof(WalkStats),
                                            hipMemcpyDeviceToHost, ctx->stream), "readback")))
        return rc;
    return check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync");
}

// the lists and their launch order are complete at this point of the
// context's stream: work on other streams that reads them waits for ev_lists
static int lists_done(p3t_ctx *ctx, int rc) {
    if (rc) return rc;
    return check_hip(ctx, hipEventRecord(ctx->ev_lists, ctx->stream), "event record");
}

int build_lists(p3t_ctx *ctx, bool stats_cleared) {
    static_assert(kRbWalk * 8 + sizeof(WalkStats) <= 40 * 8, "walk readback overlaps other slots");
    int rc;
    const int64_t nn = ctx->n_nodes;   // bound on the number of groups
    const int64_t stride = nn + 1;
    if ((rc = ensure(ctx, ctx->cnt, 3 * stride * sizeof(int64_t)))) return rc;
    if ((rc = ensure(ctx, ctx->off, 3 * stride * sizeof(int64_t)))) return rc;
    if ((rc = ensure(ctx, ctx->seg_end, 3 * stride * sizeof(int64_t)))) return rc;
    // launch-order bucket counts, cleared by the walk statistics
    if ((rc = ensure(ctx, ctx->ghist, kOrderBins * sizeof(uint32_t)))) return rc;
    int64_t *cnt = ptr<int64_t>(ctx->cnt), *off = ptr<int64_t>(ctx->off);
    int64_t *end = ptr<int64_t>(ctx->seg_end);
    WalkStats *ws = reinterpret_cast<WalkStats *>(ptr<int64_t>(ctx->readback) + kRbWalk);
    const WalkStats *hs = reinterpret_cast<const WalkStats *>(ctx->hpin + kRbWalk);
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
    wo.stack_ovf = &ws->stack_ovf;
    wo.cap_ovf = &ws->cap_ovf;
    wo.spilled = &ws->spilled;
    wo.stride = stride;
    // every block has a global-memory stack for groups that outgrow the LDS one
    if ((rc = ensure(ctx, ctx->wstack, (size_t)grid * kGlobalStack * sizeof(int32_t)))) return rc;
    int32_t *gstack = ptr<int32_t>(ctx->wstack);
    const int lds_cap = (ctx->walk_lds_cap >= 64 && ctx->walk_lds_cap < kLdsStack) ? ctx->walk_lds_cap
                                                                              : kLdsStack;

    auto reset = [&]() {
        return check_hip(ctx, hipMemsetAsync(ws, 0, sizeof(WalkStats), st), "memset");
    };
    auto finish = [&](bool fixed) {
        ctx->n_groups = (int64_t)hs->n_groups;
        for (int k = 0; k < 3; ++k) {
            ctx->list_total[k] = (int64_t)hs->total[k];
            ctx->list_extent[k] = fixed ? ctx->n_groups * wo.cap[k] : ctx->list_total[k];
            ctx->hint_max[k] = (int64_t)hs->maxlen[k];
        }
        ctx->hint_groups = ctx->n_groups;
        ctx->n_pc = (int64_t)hs->pc;
        ctx->n_pp = (int64_t)hs->pp;
        ctx->n_pp_near = (int64_t)hs->pp_near;
        ctx->n_leaves = (int64_t)hs->n_leaves;
        ctx->walk_fixed = fixed ? 1 : 0;
        ctx->walk_global = hs->spilled > 0 ? 1 : 0;
    };
    auto stack_error = [&]() {
        return set_error(ctx, P3T_EINVAL, "tree walk stack overflow");
    };

    // ---- single walk into fixed-stride segments, sized from the last build ----
    if (ctx->hint_groups > 0 && ctx->prm.n_crit == ctx->hint_n_crit) {
        const int64_t gcap = ctx->hint_groups + ctx->hint_groups / 8 + 64;
        bool ok = gcap <= stride;
        for (int k = 0; k < 3 && ok; ++k) {
            const int64_t m = ctx->hint_max[k];
            wo.cap[k] = (m + m / 4 + 64 + 63) / 64 * 64;
            // keep the reserved room within a few times the last build's lists
            ok = gcap * wo.cap[k] <= 8 * ctx->list_total[k] + (1 << 22);
        }
        if (ok) {
            wo.gcap = gcap;
            for (int k = 0; k < 3; ++k) {
                if ((rc = ensure(ctx, *lbuf[k], (gcap * wo.cap[k] + 1) * sizeof(int32_t)))) return rc;
                wo.idx[k] = ptr<int32_t>(*lbuf[k]);
            }
            if (!stats_cleared && (rc = reset())) return rc;
            k_walk<kFixed><<<grid, kWalkThreads, 0, st>>>(ptr<GroupInfo>(ctx->grp), G_dev,
                                                           ptr<NodeWalk>(ctx->node_walk), wp, wo,
                                                           gstack, lds_cap);
            if ((rc = check_hip(ctx, hipGetLastError(), "walk"))) return rc;
            if ((rc = run_walk_stats(ctx, G_dev, stride, ws))) return rc;
            if (hs->stack_ovf) return stack_error();
            if (!hs->cap_ovf) {
                finish(true);
                return lists_done(ctx, build_order(ctx, stride));
            }
        }
    }

    // ---- two passes: count, prefix sums, emit at exact offsets ----
    if ((rc = reset())) return rc;
    // entries past the last group take part in the scans as zeros
    if ((rc = check_hip(ctx, hipMemsetAsync(cnt, 0, 3 * stride * sizeof(int64_t), st), "memset")))
        return rc;
    k_walk<kCount><<<grid, kWalkThreads, 0, st>>>(ptr<GroupInfo>(ctx->grp), G_dev,
                                                   ptr<NodeWalk>(ctx->node_walk), wp, wo, gstack,
                                                   lds_cap);
    if ((rc = check_hip(ctx, hipGetLastError(), "walk count"))) return rc;
    for (int k = 0; k < 3; ++k)
        if ((rc = scan_exclusive_i64(ctx, cnt + k * stride, off + k * stride, stride, nullptr)))
            return rc;
    if ((rc = run_walk_stats(ctx, G_dev, stride, ws))) return rc;
    if (hs->stack_ovf) return stack_error();
    for (int k = 0; k < 3; ++k) {
        if ((rc = ensure(ctx, *lbuf[k], ((int64_t)hs->total[k] + 1) * sizeof(int32_t)))) return rc;
        wo.idx[k] = ptr<int32_t>(*lbuf[k]);
        wo.cap[k] = 0;
    }
    finish(false);
    ctx->hint_n_crit = ctx->prm.n_crit;
    k_walk<kEmit><<<grid, kWalkThreads, 0, st>>>(ptr<GroupInfo>(ctx->grp), G_dev,
                                                  ptr<NodeWalk>(ctx->node_walk), wp, wo, gstack,
                                                  lds_cap);
    if ((rc = check_hip(ctx, hipGetLastError(), "walk emit"))) return rc;
    return lists_done(ctx, build_order(ctx, stride));
}

}  // namespace p3t
