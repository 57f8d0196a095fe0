// tree.hip -- octree construction on the GPU: root cube, Morton keys, LSD
// radix sort (its last pass writes the sorted particle records),
// particle-parallel octree topology, bottom-up moments (monopole + quadrupole,
// Section 2.2 "up to the quadrupole moment") and group selection.
//
// Every quantity that feeds a discrete decision (keys, node boundaries,
// centre of mass, boxes) is a fixed IEEE FP64 operation sequence: this file is
// compiled with -ffp-contract=off, so no multiply-add is fused.
//
// Conventions (the method leaves them open):
//   root cube  lo_a = min_i x_ia, L = 2^ceil(log2(max_a extent_a)), L = 1 if 0;
//   key        q_a = min(floor((x_a - lo_a) * (2^21 / L)), 2^21 - 1) interleaved
//              x,y,z from the most significant bit of each 3-bit level digit;
//   order      ascending key, ties by original index (stable sort of 0..n-1);
//   node       (level l, key prefix) range; split into its non-empty octants
//              iff count > n_leaf and l < 21; numbered breadth first;
//   moments    M, S = sum m x folded in member order (leaves) or child order
//              (internal), com = S / M; box = member min/max;
//   groups     nodes with (count <= n_crit or leaf) whose ancestors all have
//              count > n_crit, ordered by first particle.
#include <math.h>

#include "device_util.h"
#include "internal.h"
#include "scan_tiles.h"

namespace p3t {

// ---------------------------------------------------------------------------
// Root cube
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

// per block: lo xyz, hi xyz, and 1 if some input of the block is invalid
constexpr int kBboxRec = 7;
constexpr int kBboxUnroll = 4;
// at most one record per thread of a keys block, which reduces them all
constexpr int kBboxMaxBlocks = 256;

// Bounding box and input check: every block reduces its share of the
// particles to a record (lo xyz, hi xyz, invalid-input flag).  The keys
// kernel reduces the records to the root cube (root_cube below).
__global__ __launch_bounds__(kRedThreads) void k_bbox(const double *__restrict__ pos,
                                                      const double *__restrict__ mass, int64_t n,
                                                      double *__restrict__ partial) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int flag = 0;
    // kBboxUnroll particles per thread and round, loaded together
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n;
         i0 += kBboxUnroll * stride) {
        PosMass r[kBboxUnroll];
#pragma unroll
        for (int j = 0; j < kBboxUnroll; ++j) {
            const int64_t i = i0 + j * stride;
            if (i < n) r[j] = PosMass{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], mass[i]};
        }
#pragma unroll
        for (int j = 0; j < kBboxUnroll; ++j) {
            const int64_t i = i0 + j * stride;
            if (i >= n) continue;
            const double v[3] = {r[j].x, r[j].y, r[j].z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                flag |= !isfinite(v[a]);
                lo[a] = fmin(lo[a], v[a]);
                hi[a] = fmax(hi[a], v[a]);
            }
            flag |= !(isfinite(r[j].m) && r[j].m > 0.0);
        }
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], d, kWave));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], d, kWave));
        }
        flag |= __shfl_xor(flag, d, kWave);
    }
    __shared__ double s[kRedThreads / kWave][6];
    __shared__ int sf[kRedThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        for (int a = 0; a < 3; ++a) { s[w][a] = lo[a]; s[w][3 + a] = hi[a]; }
        sf[w] = flag;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kRedThreads / kWave; ++k) {
            for (int a = 0; a < 3; ++a) {
                s[0][a] = fmin(s[0][a], s[k][a]);
                s[0][3 + a] = fmax(s[0][3 + a], s[k][3 + a]);
            }
            sf[0] |= sf[k];
        }
        for (int a = 0; a < 6; ++a) partial[kBboxRec * blockIdx.x + a] = s[0][a];
        partial[kBboxRec * blockIdx.x + 6] = sf[0] ? 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Morton keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread_bits3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, index): kRsPasses passes of kRsBits bits.
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 8;
constexpr int kRsTile = kRsThreads * kRsRounds;   // 2048 keys per block
constexpr int kRsWaves = kRsThreads / kWave;
constexpr int kRsBits = 8;                         // digit width: 8 passes cover the 63 key bits
constexpr int kRsBins = 1 << kRsBits;
constexpr int kRsPasses = (3 * kMaxLevel + kRsBits - 1) / kRsBits;
constexpr int kRsPer = kRsBins / kRsThreads;       // digits per thread in the bookkeeping
static_assert(kRsBins % kRsThreads == 0, "whole digits per thread");

__device__ __forceinline__ int rs_digit(uint64_t key, int shift) {
    return (int)((key >> shift) & (kRsBins - 1));
}

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                        int shift, int32_t *__restrict__ counts,
                                                        int nb) {
    __shared__ int32_t h[kRsBins];
    for (int d = threadIdx.x; d < kRsBins; d += kRsThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    uint64_t k[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t i = base + r * kRsThreads + threadIdx.x;
        k[r] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r)
        if (base + r * kRsThreads + threadIdx.x < n) atomicAdd(&h[rs_digit(k[r], shift)], 1);
    __syncthreads();
    for (int d = threadIdx.x; d < kRsBins; d += kRsThreads)
        counts[(int64_t)d * nb + blockIdx.x] = h[d];
}

// Morton keys of the tile of kRsTile particles of this block, their indices,
// the tile's histogram of the first radix digit (the keys' low bits), and each
// particle's position and mass packed in one 32-byte record (xm_in, input
// order) for the sort's final gather
// The root cube from the bounding box's nbb (<= kRsThreads) block records, by
// every thread of the block alike (min and max are exact in any order): the
// smallest power-of-two side that holds the box, from its low corner.  Block
// 0 stores it, and the input check, for the kernels that follow.
struct RootCube {
    double lo[3], L, scale;
    int bad;
};

__device__ __forceinline__ RootCube root_cube(const double *__restrict__ partial, int nbb,
                                              RootInfo *__restrict__ root,
                                              int64_t *__restrict__ bad_rb) {
    static_assert(kBboxMaxBlocks <= kRsThreads, "a record per thread");
    __shared__ double s7[kRsThreads / kWave][kBboxRec];
    double v[kBboxRec] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    if ((int)threadIdx.x < nbb)
        for (int a = 0; a < kBboxRec; ++a) v[a] = partial[kBboxRec * threadIdx.x + a];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], __shfl_xor(v[a], d, kWave));
            v[3 + a] = fmax(v[3 + a], __shfl_xor(v[3 + a], d, kWave));
        }
        v[6] = fmax(v[6], __shfl_xor(v[6], d, kWave));
    }
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0)
        for (int a = 0; a < kBboxRec; ++a) s7[w][a] = v[a];
    __syncthreads();
    for (int k = 0; k < kRsThreads / kWave; ++k) {
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], s7[k][a]);
            v[3 + a] = fmax(v[3 + a], s7[k][3 + a]);
        }
        v[6] = fmax(v[6], s7[k][6]);
    }
    RootCube c;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        c.lo[a] = v[a];
        const double e = v[3 + a] - v[a];
        if (e > ext) ext = e;
    }
    c.L = 1.0;
    if (ext > 0.0) {
        int e;
        const double f = frexp(ext, &e);
        c.L = (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
    }
    c.scale = ldexp(1.0, kMaxLevel) / c.L;
    c.bad = v[6] != 0.0 ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) root->lo[a] = c.lo[a];
        root->L = c.L;
        root->scale = c.scale;
        root->bad_input = c.bad;
        *bad_rb = c.bad;
    }
    return c;
}

__global__ __launch_bounds__(kRsThreads) void k_keys_hist(const double *__restrict__ pos,
                                                          const double *__restrict__ mass, int64_t n,
                                                          const double *__restrict__ partial,
                                                          int nbb, RootInfo *__restrict__ root,
                                                          int64_t *__restrict__ bad_rb,
                                                          uint64_t *__restrict__ keys,
                                                          int32_t *__restrict__ idx,
                                                          PosMass *__restrict__ xm_in,
                                                          int32_t *__restrict__ counts, int nb) {
    __shared__ int32_t h[kRsBins];
    for (int d = threadIdx.x; d < kRsBins; d += kRsThreads) h[d] = 0;
    // the tile's particles are on their way while the root cube is reduced
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    PosMass r[kRsRounds];
#pragma unroll
    for (int k = 0; k < kRsRounds; ++k) {
        const int64_t i = base + k * kRsThreads + threadIdx.x;
        if (i < n) r[k] = PosMass{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], mass[i]};
    }
    const RootCube cube = root_cube(partial, nbb, root, bad_rb);   // its barrier also covers h
    const double scale = cube.scale;
    const double lo[3] = {cube.lo[0], cube.lo[1], cube.lo[2]};
#pragma unroll
    for (int k = 0; k < kRsRounds; ++k) {
        const int64_t i = base + k * kRsThreads + threadIdx.x;
        if (i >= n) break;
        const double x[3] = {r[k].x, r[k].y, r[k].z};
        uint64_t q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double t = floor((x[a] - lo[a]) * scale);
            const uint64_t v = (uint64_t)t;
            q[a] = v > 0x1fffffull ? 0x1fffffull : v;
        }
        const uint64_t key = (spread_bits3(q[0]) << 2) | (spread_bits3(q[1]) << 1) | spread_bits3(q[2]);
        keys[i] = key;
        idx[i] = (int32_t)i;
        xm_in[i] = r[k];
        atomicAdd(&h[rs_digit(key, 0)], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRsBins; d += kRsThreads)
        counts[(int64_t)d * nb + blockIdx.x] = h[d];
}

// exclusive scan over the kRsBins digits, thread t holding digits
// kRsPer t .. kRsPer t + kRsPer - 1 in v
__device__ __forceinline__ void block_excl_scan_bins(int v[kRsPer], int32_t *s_wsum) {
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    int local = 0;
#pragma unroll
    for (int k = 0; k < kRsPer; ++k) local += v[k];
    const int incl = wave_incl_scan(local);
    if (lane == kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    int run = incl - local;
    for (int k = 0; k < w; ++k) run += s_wsum[k];
#pragma unroll
    for (int k = 0; k < kRsPer; ++k) {
        const int c = v[k];
        v[k] = run;
        run += c;
    }
}

// LAST: the final pass also writes the sorted particle records xm (gathered
// from the packed input records) and clears the n + 1 group-start flags.
struct SortedOut {
    const PosMass *xm_in;
    PosMass *xm;
    int32_t *gflag;
};

template <bool LAST>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t n, int shift, const int32_t *__restrict__ offsets,
    const int32_t *__restrict__ totals, int nb, SortedOut so) {
    __shared__ uint64_t s_key[kRsTile];
    __shared__ int32_t s_val[kRsTile];
    __shared__ int32_t s_start[kRsBins], s_gbase[kRsBins];
    __shared__ int32_t s_wcnt[kRsWaves][kRsBins];
    __shared__ int32_t s_wsum[kRsWaves], s_wsum2[kRsWaves];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    const int64_t tile_n = std::min<int64_t>(kRsTile, n - base);
    // wavefront w ranks the kRsRounds * 64 consecutive keys from wbase; its
    // per-digit running counts live in its own row of s_wcnt
    constexpr int kPerWave = kRsRounds * kWave;
    const int64_t wbase = base + (int64_t)w * kPerWave;
    for (int d = lane; d < kRsBins; d += kWave) s_wcnt[w][d] = 0;
    uint64_t key[kRsRounds];
    int32_t val[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t i = wbase + r * kWave + lane;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0;
    }
    int dig[kRsRounds], rank[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const bool valid = wbase + r * kWave + lane < n;
        const int d = rs_digit(key[r], shift);
        uint64_t same = ballot(valid);
#pragma unroll
        for (int b = 0; b < kRsBits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const int below = count_below(same);
        // earlier keys of this digit in the wavefront's chunk, then this round's
        // (the row is this wavefront's alone, and its LDS accesses are in order)
        const int prior = s_wcnt[w][d];
        if (valid && below == 0) s_wcnt[w][d] = prior + __popcll(same);
        dig[r] = d;
        rank[r] = prior + below;
    }
    __syncthreads();
    // per digit: the wavefronts' offsets inside the digit, the digit's start
    // in the tile, and its first output position
    {
        int c[kRsPer], t[kRsPer];
#pragma unroll
        for (int k = 0; k < kRsPer; ++k) {
            const int d = kRsPer * tid + k;
            int run = 0;
#pragma unroll
            for (int v = 0; v < kRsWaves; ++v) {
                const int x = s_wcnt[v][d];
                s_wcnt[v][d] = run;
                run += x;
            }
            c[k] = run;
            t[k] = totals[d];
        }
        block_excl_scan_bins(c, s_wsum);
        block_excl_scan_bins(t, s_wsum2);
#pragma unroll
        for (int k = 0; k < kRsPer; ++k) {
            const int d = kRsPer * tid + k;
            s_start[d] = c[k];
            s_gbase[d] = t[k] + offsets[(int64_t)d * nb + blockIdx.x] - c[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        if (wbase + r * kWave + lane < n) {
            const int d = dig[r];
            const int p = s_start[d] + s_wcnt[w][d] + rank[r];
            s_key[p] = key[r];
            s_val[p] = val[r];
        }
    }
    __syncthreads();
    for (int p = tid; p < tile_n; p += kRsThreads) {
        const uint64_t k = s_key[p];
        const int64_t o = (int64_t)s_gbase[rs_digit(k, shift)] + p;
        const int32_t v = s_val[p];
        kout[o] = k;
        vout[o] = v;
        if (LAST) {
            so.xm[o] = so.xm_in[v];
            so.gflag[o] = 0;
        }
    }
    if (LAST && blockIdx.x == 0 && tid == 0) so.gflag[n] = 0;
}

// The moments folds count the groups per particle tile for the group scan when
// the particles fit kScan2MaxTiles tiles (n + 1 flags).
static bool group_tiles_counted(const p3t_ctx *ctx, int64_t n) {
    return !ctx->groups_generic && (n + 1 + kScan2Tile - 1) / kScan2Tile <= kScan2MaxTiles;
}

// Root cube, keys, the kRsPasses radix passes, and the sorted particle
// records: the first digit's histogram comes with the keys, the records with
// the last pass.
int build_sorted(p3t_ctx *ctx, const double *pos, const double *mass, int64_t n) {
    int rc;
    const int nbb = (int)std::min<int64_t>(
        kBboxMaxBlocks, (n + (int64_t)kRedThreads * kBboxUnroll - 1) / ((int64_t)kRedThreads * kBboxUnroll));
    const int nb = (int)((n + kRsTile - 1) / kRsTile);
    if ((rc = ensure(ctx, ctx->root, sizeof(RootInfo)))) return rc;
    if ((rc = ensure(ctx, ctx->bbox, kBboxRec * nbb * sizeof(double)))) return rc;
    for (p3t::DevBuf *b : {&ctx->keys[0], &ctx->keys[1]})
        if ((rc = ensure(ctx, *b, n * sizeof(uint64_t)))) return rc;
    for (p3t::DevBuf *b : {&ctx->vals[0], &ctx->vals[1]})
        if ((rc = ensure(ctx, *b, n * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->hist, (size_t)kRsBins * nb * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->histc, (size_t)kRsBins * nb * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->rs_tot, kRsBins * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->xm, n * sizeof(PosMass)))) return rc;
    if ((rc = ensure(ctx, ctx->xm_in, n * sizeof(PosMass)))) return rc;
    if ((rc = ensure(ctx, ctx->gflag, (n + 1) * sizeof(int32_t)))) return rc;
    double *partial = ptr<double>(ctx->bbox);
    k_bbox<<<nbb, kRedThreads, 0, ctx->stream>>>(pos, mass, n, partial);
    int32_t *cnt = ptr<int32_t>(ctx->histc), *off = ptr<int32_t>(ctx->hist);
    int32_t *tot = ptr<int32_t>(ctx->rs_tot);
    // the input check goes straight to the pinned host words (read after the
    // topology's synchronisation)
    k_keys_hist<<<nb, kRsThreads, 0, ctx->stream>>>(pos, mass, n, partial, nbb,
                                                     ptr<RootInfo>(ctx->root),
                                                     ctx->hpin + kRbTopoBad,
                                                     ptr<uint64_t>(ctx->keys[0]),
                                                     ptr<int32_t>(ctx->vals[0]),
                                                     ptr<PosMass>(ctx->xm_in), cnt, nb);
    if ((rc = check_hip(ctx, hipGetLastError(), "root/keys"))) return rc;
    const SortedOut so{ptr<PosMass>(ctx->xm_in), ptr<PosMass>(ctx->xm), ptr<int32_t>(ctx->gflag)};
    int src = 0;
    for (int pass = 0; pass < kRsPasses; ++pass) {
        const int shift = kRsBits * pass;
        uint64_t *kin = ptr<uint64_t>(ctx->keys[src]), *kout = ptr<uint64_t>(ctx->keys[1 - src]);
        int32_t *vin = ptr<int32_t>(ctx->vals[src]), *vout = ptr<int32_t>(ctx->vals[1 - src]);
        if (pass > 0) {
            k_rs_hist<<<nb, kRsThreads, 0, ctx->stream>>>(kin, n, shift, cnt, nb);
            if ((rc = check_hip(ctx, hipGetLastError(), "radix hist"))) return rc;
        }
        if ((rc = scan_rows_i32(ctx, cnt, off, tot, kRsBins, nb))) return rc;
        auto scatter = pass == kRsPasses - 1 ? k_rs_scatter<true> : k_rs_scatter<false>;
        scatter<<<nb, kRsThreads, 0, ctx->stream>>>(kin, vin, kout, vout, n, shift, off, tot, nb,
                                                     so);
        if ((rc = check_hip(ctx, hipGetLastError(), "radix scatter"))) return rc;
        src = 1 - src;
    }
    // the passes alternate between the two buffers: an odd count ends in the second
    if (src == 1) {
        std::swap(ctx->keys[0], ctx->keys[1]);
        std::swap(ctx->vals[0], ctx->vals[1]);
    }
    return P3T_OK;  // the sorted keys and permutation are in keys[0] / vals[0]
}

// ---------------------------------------------------------------------------
// Octree topology from sorted keys, in parallel over particles.
//
// With c(a) = common levels of keys a-1 and a, position a starts the nodes of
// levels c(a)+1 .. e(a) (all levels 0.. for a = 0), provided the level-c(a)
// node containing a has more than n_leaf particles; e(a) is the first of those
// levels whose node does not split.  A node starting at a at level l has more
// than n_leaf particles iff key a+n_leaf shares its level-l prefix.  Breadth
// first ids follow from per-level ranks of the start positions.
// ---------------------------------------------------------------------------
constexpr int kTopoThreads = 256;
constexpr int kTopoWaves = kTopoThreads / kWave;

__device__ __forceinline__ int64_t lower_bound_key(const uint64_t *keys, int64_t lo, int64_t hi,
                                                   uint64_t v) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// first index in [lo, hi) whose key exceeds v, searching outwards from lo
// (doubling steps, then bisection): cost grows with the distance found, and
// most nodes are small
__device__ __forceinline__ int64_t gallop_upper_key(const uint64_t *keys, int64_t lo, int64_t hi,
                                                    uint64_t v) {
    int64_t step = 1, prev = lo;
    int64_t probe = lo;
    while (probe < hi && keys[probe] <= v) {
        prev = probe + 1;
        probe = lo + step;
        step <<= 1;
    }
    int64_t a = prev, b = probe < hi ? probe : hi;
    while (a < b) {
        const int64_t mid = a + ((b - a) >> 1);
        if (keys[mid] <= v) a = mid + 1; else b = mid;
    }
    return a;
}

// range code: lo | hi << 8, or -1 when no node starts at a
// Up to this leaf size the topology kernels read their keys from an on-chip
// window (the block's keys and n_leaf on either side) instead of searching.
constexpr int kTopoWin = 64;
// stands for positions outside [0, n): its prefix at every level differs from
// that of every key (keys have 63 bits)
constexpr uint64_t kNoKey = ~0ull;

// keys base - before .. base + kTopoThreads + after - 1 of the block into s_k
__device__ __forceinline__ void load_key_window(uint64_t *s_k, const uint64_t *keys, int64_t n,
                                                int64_t base, int before, int after) {
    for (int t = threadIdx.x; t < kTopoThreads + before + after; t += kTopoThreads) {
        const int64_t i = base - before + t;
        s_k[t] = (i >= 0 && i < n) ? keys[i] : kNoKey;
    }
}

// (block 0 also clears the n_gtile group counters of the moments folds)
__global__ __launch_bounds__(kTopoThreads) void k_topo_ranges(const uint64_t *__restrict__ keys,
                                                              int64_t n, int n_leaf,
                                                              int32_t *__restrict__ range,
                                                              int32_t *__restrict__ blk, int nb,
                                                              int32_t *__restrict__ gtile,
                                                              int n_gtile) {
    __shared__ int32_t cnt[kLevels];
    __shared__ uint64_t s_k[kTopoThreads + 2 * kTopoWin];
    if (threadIdx.x < kLevels) cnt[threadIdx.x] = 0;
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < n_gtile; t += kTopoThreads) gtile[t] = 0;
    const int64_t base = (int64_t)blockIdx.x * kTopoThreads;
    const bool win = n_leaf <= kTopoWin;
    if (win) load_key_window(s_k, keys, n, base, n_leaf, n_leaf);
    __syncthreads();
    const int64_t a = base + threadIdx.x;
    const int o = threadIdx.x + n_leaf;   // a's slot in the window
    int lo = 1, hi = 0;
    if (a < n) {
        const uint64_t ka = win ? s_k[o] : keys[a];
        const int c = (a == 0) ? -1 : common_levels(win ? s_k[o - 1] : keys[a - 1], ka);
        const int m = (a + n_leaf < n)
                          ? common_levels(ka, win ? s_k[o + n_leaf] : keys[a + n_leaf])
                          : -1;
        bool exists;
        if (a == 0) {
            exists = true;
        } else if (c >= kMaxLevel) {
            exists = false;   // duplicate key: no node starts here
        } else if (win) {
            // the level-c node holding a (a contiguous run of keys) has more
            // than n_leaf members iff at least n_leaf of the n_leaf keys on
            // either side of a share a's level-c prefix
            const int sh = 3 * (kMaxLevel - c);
            const uint64_t P = ka >> sh;
            int same = 0;
            for (int k = 1; k <= n_leaf; ++k)
                same += (int)((s_k[o - k] >> sh) == P) + (int)((s_k[o + k] >> sh) == P);
            exists = same >= n_leaf;
        } else {
            // the level-c node containing a must have more than n_leaf particles
            const int sh = 3 * (kMaxLevel - c);
            const uint64_t base = (sh >= 64) ? 0ull : ((ka >> sh) << sh);
            const int64_t p = lower_bound_key(keys, 0, a, base);
            exists = (p + n_leaf < n) && common_levels(keys[p], keys[p + n_leaf]) >= c;
        }
        if (exists) {
            lo = c + 1;
            const int msplit = m < 20 ? m : 20;
            hi = (msplit + 1 > lo) ? msplit + 1 : lo;
        }
        range[a] = exists ? (lo | (hi << 8)) : -1;
        for (int l = lo; l <= hi; ++l) atomicAdd(&cnt[l], 1);
    }
    __syncthreads();
    if (threadIdx.x < kLevels) blk[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// first node id of every level, and the node count at [kLevels] (computed on
// the host from the per-level node counts, passed by value)
struct LevelStarts {
    int64_t s[kLevels + 1];
};

// blk_off: per level, the exclusive scan of the node starts over the blocks
__global__ __launch_bounds__(kTopoThreads) void k_topo_emit(
    const uint64_t *__restrict__ keys, int64_t n, int n_leaf, const int32_t *__restrict__ range,
    const int32_t *__restrict__ blk_off, const LevelStarts level_start, int nb,
    int32_t *__restrict__ level, int32_t *__restrict__ first,
    int32_t *__restrict__ count, int32_t *__restrict__ child, int32_t *__restrict__ nchild,
    uint64_t *__restrict__ prefix) {
    __shared__ uint64_t s_ball[kLevels][kTopoWaves];
    __shared__ int32_t s_wc[kLevels][kTopoWaves];
    __shared__ uint64_t s_k[kTopoThreads + kTopoWin];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int64_t a = (int64_t)blockIdx.x * kTopoThreads + tid;
    const bool win = n_leaf <= kTopoWin;
    if (win) load_key_window(s_k, keys, n, (int64_t)blockIdx.x * kTopoThreads, 0, n_leaf);
    const int32_t code = (a < n) ? range[a] : -1;
    const int lo = code < 0 ? 1 : (code & 255), hi = code < 0 ? 0 : (code >> 8);
    // all lanes: per-level membership masks of this wave
    for (int l = 0; l < kLevels; ++l) {
        const uint64_t b = ballot(l >= lo && l <= hi);
        if (lane == 0) {
            s_ball[l][w] = b;
            s_wc[l][w] = __popcll(b);
        }
    }
    __syncthreads();
    if (code < 0) return;
    const uint64_t ka = win ? s_k[tid] : keys[a];
    // number of level-l starts before position a, plus the level's first id
    auto rank_at = [&](int l) -> int32_t {
        int base = (int)level_start.s[l] + blk_off[(int64_t)l * nb + blockIdx.x];
        for (int k = 0; k < w; ++k) base += s_wc[l][k];
        return base + count_below(s_ball[l][w]);
    };
    int32_t id = rank_at(lo);
    for (int l = lo; l <= hi; ++l) {
        const int32_t next = (l < kMaxLevel) ? rank_at(l + 1) : 0;
        const int sh = 3 * (kMaxLevel - l);
        if (l == hi) {
            // a leaf: at most n_leaf members unless at the deepest level
            // (equal keys); internal nodes are counted by the moments fold
            int cnt = n_leaf + 1;
            if (win) {
                const uint64_t P = ka >> sh;
                cnt = 1;
                for (int k = 1; k <= n_leaf; ++k) cnt += (int)((s_k[tid + k] >> sh) == P);
            }
            if (cnt > n_leaf) {
                const uint64_t kmax = ka | ((sh >= 64) ? ~0ull : ((1ull << sh) - 1ull));
                cnt = (int)(gallop_upper_key(keys, a + 1, n, kmax) - a);
            }
            count[id] = cnt;
        }
        level[id] = l;
        first[id] = (int32_t)a;
        child[id] = next;
        nchild[id] = (l == hi) ? 0 : -1;
        prefix[id] = (sh >= 64) ? 0ull : (ka >> sh);
        id = next;
    }
}

// children are contiguous: n_child = (first child of the next node at this level)
// - (own first child); parents from the children ranges.  Run by the leaf
// moments kernel for the internal nodes.
__device__ __forceinline__ void topo_links(int64_t id, const int32_t *__restrict__ level,
                                           const int32_t *__restrict__ child,
                                           int32_t *__restrict__ nchild,
                                           int32_t *__restrict__ parent,
                                           const LevelStarts &level_start) {
    const int l = level[id];
    const int64_t next = (id + 1 < level_start.s[l + 1]) ? child[id + 1] : level_start.s[l + 2];
    const int32_t cf = child[id];
    const int32_t nc = (int32_t)(next - cf);
    nchild[id] = nc;
    for (int k = 0; k < nc; ++k) parent[cf + k] = (int32_t)id;
}

int build_topology(p3t_ctx *ctx, int64_t n) {
    int rc;
    const int nb = (int)((n + kTopoThreads - 1) / kTopoThreads);
    // n + 1: the array later holds the groups' node_at
    if ((rc = ensure(ctx, ctx->lvlrange, (n + 1) * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->tblk, (size_t)kLevels * nb * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->tblk_off, (size_t)kLevels * nb * sizeof(int32_t)))) return rc;
    if ((rc = ensure_readback(ctx))) return rc;
    const uint64_t *keys = ptr<uint64_t>(ctx->keys[0]);
    int32_t *blk = ptr<int32_t>(ctx->tblk), *blk_off = ptr<int32_t>(ctx->tblk_off);
    // the groups' per-tile counts (for the compaction's scan), when it fits one
    const int64_t n_gtile = (n + 1 + kScan2Tile - 1) / kScan2Tile;
    const bool gcount = group_tiles_counted(ctx, n);
    if (gcount && (rc = ensure(ctx, ctx->gtile, n_gtile * sizeof(int32_t)))) return rc;
    k_topo_ranges<<<nb, kTopoThreads, 0, ctx->stream>>>(
        keys, n, ctx->prm.n_leaf, ptr<int32_t>(ctx->lvlrange), blk, nb,
        gcount ? ptr<int32_t>(ctx->gtile) : nullptr, gcount ? (int)n_gtile : 0);
    if ((rc = check_hip(ctx, hipGetLastError(), "topology ranges"))) return rc;
    // the per-level node counts (int32, in the words before the input check) go
    // straight to the pinned host words; one synchronisation makes them and the
    // input check visible
    static_assert(kLevels * sizeof(int32_t) <= kRbTopoBad * sizeof(int64_t), "readback layout");
    int32_t *level_total = reinterpret_cast<int32_t *>(ctx->hpin);
    if ((rc = scan_rows_i32(ctx, blk, blk_off, level_total, kLevels, nb))) return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    if (ctx->hpin[kRbTopoBad])
        return set_error(ctx, P3T_EINVAL, "non-finite position or non-positive/non-finite mass");
    LevelStarts ls;
    const int32_t *hl = reinterpret_cast<const int32_t *>(ctx->hpin);
    int64_t run = 0;
    for (int l = 0; l < kLevels; ++l) {
        ls.s[l] = ctx->level_start[l] = run;
        run += hl[l];
    }
    ls.s[kLevels] = ctx->level_start[kLevels] = run;
    ctx->n_nodes = run;
    ctx->depth = 0;
    for (int l = 0; l < kLevels; ++l)
        if (ctx->level_start[l + 1] > ctx->level_start[l]) ctx->depth = l;
    const int64_t nn = ctx->n_nodes;
    for (p3t::DevBuf *b : {&ctx->node_level, &ctx->node_first, &ctx->node_count, &ctx->node_child,
                           &ctx->node_nchild, &ctx->node_parent})
        if ((rc = ensure(ctx, *b, nn * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->node_prefix, nn * sizeof(uint64_t)))) return rc;
    k_topo_emit<<<nb, kTopoThreads, 0, ctx->stream>>>(
        keys, n, ctx->prm.n_leaf, ptr<int32_t>(ctx->lvlrange), blk_off, ls, nb, ptr<int32_t>(ctx->node_level),
        ptr<int32_t>(ctx->node_first), ptr<int32_t>(ctx->node_count), ptr<int32_t>(ctx->node_child),
        ptr<int32_t>(ctx->node_nchild), ptr<uint64_t>(ctx->node_prefix));
    return check_hip(ctx, hipGetLastError(), "topology emit");
}

// ---------------------------------------------------------------------------
// Moments, bottom up: every leaf in one launch (a thread per node), then the
// internal nodes level by level from the deepest, one launch per level.  The
// folds are the same IEEE operation sequences in the same order (members in
// sorted order, children in octant order) whichever thread performs them.
// ---------------------------------------------------------------------------
struct MomentArrays {
    const int32_t *level, *first, *child, *nchild, *parent;
    int32_t *count;                 // leaves' counts in; internal nodes' counts out
    const RootInfo *root;
    const PosMass *xm;
    double *S;
    NodeWalk *nw;
    NodeMP *mp;
    int64_t n_nodes;
    // groups: the highest nodes with at most n_crit members, or leaves; each
    // flags its first particle (gflag) and is recorded there (node_at)
    int n_crit;
    int32_t *gflag, *node_at;
    int32_t *gtile;                 // groups per kScan2Tile particles (null: not counted)
    int64_t *walk_zero;             // the walk's statistics words, cleared here
};

// Group counts per particle tile, gathered per lane (one open tile) and added
// to gtile per wavefront and tile.
struct TileCount {
    int32_t tile = -1, count = 0;
};

__device__ __forceinline__ void mark_group(const MomentArrays &A, int32_t node, int32_t first,
                                           TileCount &tc) {
    A.gflag[first] = 1;
    A.node_at[first] = node;
    if (!A.gtile) return;
    const int32_t t = first / kScan2Tile;
    if (tc.count == 0 || tc.tile == t) {
        tc.tile = t;
        ++tc.count;
    } else {
        atomicAdd(&A.gtile[t], 1);   // the lane's groups straddle a tile boundary
    }
}

// all lanes of the wavefront: one atomic add per distinct open tile
__device__ __forceinline__ void flush_tile_counts(const MomentArrays &A, const TileCount &tc) {
    if (!A.gtile) return;
    const bool has = tc.count > 0;
    uint64_t todo = ballot(has);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int32_t t = __shfl(tc.tile, lead, kWave);
        const bool same = has && tc.tile == t;
        const int32_t sum = wave_sum(same ? tc.count : 0);
        if (lane_id() == lead) atomicAdd(&A.gtile[t], sum);
        todo &= ~ballot(same);
    }
}

// L: the root cell's side
__device__ __forceinline__ void store_node(const MomentArrays &A, double L, int64_t id, int lev,
                                           int nc, int32_t child_first, int32_t f, int32_t cnt,
                                           double M, double Sx, double Sy, double Sz,
                                           const double lo[3], const double hi[3],
                                           const double q[6]) {
    const double cx = Sx / M, cy = Sy / M, cz = Sz / M;
    A.S[id] = Sx;
    A.S[A.n_nodes + id] = Sy;
    A.S[2 * A.n_nodes + id] = Sz;
    const double side = ldexp(L, -lev);
    NodeWalk o;
    o.cx = cx; o.cy = cy; o.cz = cz;
    o.l2 = side * side;
    for (int a = 0; a < 3; ++a) { o.lo[a] = lo[a]; o.hi[a] = hi[a]; }
    o.child_first = nc ? child_first : -1;
    o.n_child = nc;
    o.first = f;
    o.count = cnt;
    A.nw[id] = o;
    NodeMP p;
    p.cx = cx; p.cy = cy; p.cz = cz; p.M = M;
    for (int a = 0; a < 6; ++a) p.q[a] = q[a];
    A.mp[id] = p;
}

// fold of a leaf's members in sorted order: M, S = sum m x (left folds),
// box, and the quadrupole about com = S / M
__device__ __forceinline__ void leaf_moments(const MomentArrays &A, int64_t id) {
    constexpr int kChunk = 8;    // members held in registers at once
    const int32_t f = A.first[id], cnt = A.count[id], e = f + cnt;
    double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double q[6] = {0, 0, 0, 0, 0, 0};
    PosMass pk[kChunk];
    // the members, loaded together (clamped to the last member) kChunk at a
    // time; a leaf of at most kChunk members is read once for both folds
    auto load = [&](int32_t k0) {
#pragma unroll
        for (int c = 0; c < kChunk; ++c) pk[c] = A.xm[k0 + c < e ? k0 + c : e - 1];
    };
    for (int32_t k0 = f; k0 < e; k0 += kChunk) {
        load(k0);
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            if (k0 + c >= e) continue;
            const double mk = pk[c].m, xk = pk[c].x, yk = pk[c].y, zk = pk[c].z;
            M = M + mk;
            Sx = Sx + mk * xk;
            Sy = Sy + mk * yk;
            Sz = Sz + mk * zk;
            lo[0] = fmin(lo[0], xk); lo[1] = fmin(lo[1], yk); lo[2] = fmin(lo[2], zk);
            hi[0] = fmax(hi[0], xk); hi[1] = fmax(hi[1], yk); hi[2] = fmax(hi[2], zk);
        }
    }
    const double cx = Sx / M, cy = Sy / M, cz = Sz / M;
    for (int32_t k0 = f; k0 < e; k0 += kChunk) {
        if (cnt > kChunk) load(k0);
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            if (k0 + c >= e) continue;
            const double mk = pk[c].m;
            const double dx = pk[c].x - cx, dy = pk[c].y - cy, dz = pk[c].z - cz;
            const double r2 = dx * dx + dy * dy + dz * dz;
            q[0] += mk * (3.0 * dx * dx - r2);
            q[1] += mk * (3.0 * dy * dy - r2);
            q[2] += mk * (3.0 * dz * dz - r2);
            q[3] += mk * 3.0 * dx * dy;
            q[4] += mk * 3.0 * dx * dz;
            q[5] += mk * 3.0 * dy * dz;
        }
    }
    store_node(A, A.root->L, id, A.level[id], 0, -1, f, cnt, M, Sx, Sy, Sz, lo, hi, q);
}

// Internal nodes are folded from their children staged in LDS in chunks of
// kMomChunk children (see fold_chunk).
constexpr int kMomChunk = 256;
constexpr int kMomChildMax = 8;
constexpr int kMomStage = kMomChunk + kMomChildMax - 1;
constexpr int kMomThreads = 320;   // >= kMomStage: one staging round
static_assert(kMomThreads >= kMomStage, "one staging round");

// What a parent's fold reads of each child, staged in LDS.
struct ChildRec {
    double M, Sx, Sy, Sz, cx, cy, cz;
    double q[6];
    double lo[3], hi[3];
    int32_t count, first, n_child, pad;
};

__device__ __forceinline__ ChildRec load_child(const MomentArrays &A, int64_t k) {
    const NodeMP m = A.mp[k];
    const NodeWalk &w = A.nw[k];
    ChildRec r;
    r.M = m.M;
    r.Sx = A.S[k];
    r.Sy = A.S[A.n_nodes + k];
    r.Sz = A.S[2 * A.n_nodes + k];
    r.cx = m.cx; r.cy = m.cy; r.cz = m.cz;
    for (int a = 0; a < 6; ++a) r.q[a] = m.q[a];
    for (int a = 0; a < 3; ++a) {
        r.lo[a] = w.lo[a];
        r.hi[a] = w.hi[a];
    }
    r.count = w.count;
    r.first = w.first;
    r.n_child = w.n_child;
    r.pad = 0;
    return r;
}

// fold of an internal node's nc (at most 8) children child(0 .. nc-1) in octant
// order, the children's quadrupoles shifted to the node's centre of mass; the
// node's count is the sum of its children's
template <class Child>
__device__ __forceinline__ void internal_moments(const MomentArrays &A, double L, int64_t id, int lev,
                                                 int32_t first_child, const Child &child, int nc,
                                                 TileCount &tc) {
    double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double q[6] = {0, 0, 0, 0, 0, 0};
    int32_t cnt = 0;
    for (int k = 0; k < nc; ++k) {
        const ChildRec c = child(k);
        cnt += c.count;
        M = M + c.M;
        Sx = Sx + c.Sx;
        Sy = Sy + c.Sy;
        Sz = Sz + c.Sz;
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], c.lo[a]);
            hi[a] = fmax(hi[a], c.hi[a]);
        }
    }
    const double cx = Sx / M, cy = Sy / M, cz = Sz / M;
    for (int k = 0; k < nc; ++k) {
        const ChildRec c = child(k);
        const double dx = c.cx - cx, dy = c.cy - cy, dz = c.cz - cz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double Mk = c.M;
        q[0] += c.q[0] + Mk * (3.0 * dx * dx - r2);
        q[1] += c.q[1] + Mk * (3.0 * dy * dy - r2);
        q[2] += c.q[2] + Mk * (3.0 * dz * dz - r2);
        q[3] += c.q[3] + Mk * 3.0 * dx * dy;
        q[4] += c.q[4] + Mk * 3.0 * dx * dz;
        q[5] += c.q[5] + Mk * 3.0 * dy * dz;
    }
    A.count[id] = cnt;
    const int32_t f = child(0).first;   // the node's first particle is its first child's
    store_node(A, L, id, lev, nc, first_child, f, cnt, M, Sx, Sy, Sz, lo, hi, q);
    // groups among the children (this node has more than n_crit members), or
    // the root itself
    if (cnt > A.n_crit) {
        for (int k = 0; k < nc; ++k) {
            const ChildRec c = child(k);
            if (c.count <= A.n_crit || c.n_child == 0) mark_group(A, first_child + k, c.first, tc);
        }
    } else if (lev == 0) {
        mark_group(A, (int32_t)id, f, tc);
    }
}

// every leaf's moments; every internal node's child count and its children's
// parent links (the topology's last step)
__global__ __launch_bounds__(128) void k_moments_leaves(MomentArrays A, int32_t *__restrict__ nchild,
                                                        int32_t *__restrict__ parent,
                                                        LevelStarts ls) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < kRbWalkWords) A.walk_zero[id] = 0;
    if (id >= A.n_nodes) return;
    if (id == 0) parent[0] = -1;
    if (nchild[id] != 0) {
        topo_links(id, A.level, A.child, nchild, parent, ls);
    } else {
        leaf_moments(A, id);
        if (id == 0) {   // a root that is a leaf: the only group
            TileCount tc;
            mark_group(A, 0, 0, tc);
            if (A.gtile) atomicAdd(&A.gtile[0], tc.count);
        }
    }
}

// The internal nodes of level lev whose first child lies in the chunk of
// children [k0, k0 + kMomChunk) of the children level [cb, ce): a thread per
// child stages that child's record in LDS (consecutive threads, consecutive
// records), with the kMomChildMax - 1 children past the chunk so that every
// parent whose first child is in the chunk has all its children on chip; the
// thread of each parent's first child folds the parent.

struct MomStage {
    ChildRec c[kMomStage];
    int32_t par[kMomStage];
    int32_t before;   // parent of the child before the chunk (-1 at the level's start)
};

__device__ __forceinline__ void fold_chunk(const MomentArrays &A, MomStage &st, int lev, int64_t cb,
                                           int64_t ce, int64_t k0) {
    const int t = threadIdx.x;
    const double L = A.root->L;   // read while the stage fills
    if (t < kMomStage) {
        const int64_t k = k0 + t;
        if (k < ce) {
            st.c[t] = load_child(A, k);
            st.par[t] = A.parent[k];
        } else {
            st.par[t] = -1;
        }
    }
    if (t == kMomStage) st.before = k0 > cb ? A.parent[k0 - 1] : -1;
    __syncthreads();
    TileCount tc;
    if (t < kMomChunk && k0 + t < ce) {
        const int32_t p = st.par[t];
        // a parent's children are consecutive
        const int32_t before = t > 0 ? st.par[t - 1] : st.before;
        if (before != p) {
            int nc = 1;
            while (nc < kMomChildMax && st.par[t + nc] == p) ++nc;
            const ChildRec *c = st.c + t;
            internal_moments(A, L, p, lev, (int32_t)(k0 + t), [c](int j) { return c[j]; }, nc,
                             tc);
        }
    }
    flush_tile_counts(A, tc);
    __syncthreads();   // the stage is reused
}

// one chunk per block
__global__ __launch_bounds__(kMomThreads) void k_moments_level(MomentArrays A, int lev, int64_t cb,
                                                               int64_t ce) {
    __shared__ MomStage st;
    fold_chunk(A, st, lev, cb, ce, cb + (int64_t)blockIdx.x * kMomChunk);
}

// The top levels top .. 0 (children levels of at most kMomTopChildren nodes)
// in one block, chunk after chunk; the block's barriers order each level after
// the one below it (one compute unit: the block sees its own writes).
constexpr int64_t kMomTopChildren = 4 * kMomChunk;
__global__ __launch_bounds__(kMomThreads) void k_moments_top(MomentArrays A, int top,
                                                            LevelStarts ls) {
    __shared__ MomStage st;
    for (int l = top; l >= 0; --l) {
        const int64_t cb = ls.s[l + 1], ce = ls.s[l + 2];
        for (int64_t k0 = cb; k0 < ce; k0 += kMomChunk) fold_chunk(A, st, l, cb, ce, k0);
    }
}

int build_moments(p3t_ctx *ctx) {
    int rc;
    const int64_t nn = ctx->n_nodes;
    if ((rc = ensure(ctx, ctx->node_S, 3 * nn * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->node_walk, nn * sizeof(NodeWalk)))) return rc;
    if ((rc = ensure(ctx, ctx->node_mp, nn * sizeof(NodeMP)))) return rc;
    MomentArrays A;
    A.level = ptr<int32_t>(ctx->node_level);
    A.first = ptr<int32_t>(ctx->node_first);
    A.count = ptr<int32_t>(ctx->node_count);
    A.child = ptr<int32_t>(ctx->node_child);
    A.nchild = ptr<int32_t>(ctx->node_nchild);
    A.parent = ptr<int32_t>(ctx->node_parent);
    A.root = ptr<RootInfo>(ctx->root);
    A.xm = ptr<PosMass>(ctx->xm);
    A.S = ptr<double>(ctx->node_S);
    A.nw = ptr<NodeWalk>(ctx->node_walk);
    A.mp = ptr<NodeMP>(ctx->node_mp);
    A.n_nodes = nn;
    A.n_crit = ctx->prm.n_crit;
    // the group flags were cleared by the last radix pass; the topology's
    // per-particle range codes are dead and their array holds node_at
    A.gflag = ptr<int32_t>(ctx->gflag);
    A.node_at = ptr<int32_t>(ctx->lvlrange);
    A.gtile = group_tiles_counted(ctx, ctx->n) ? ptr<int32_t>(ctx->gtile) : nullptr;
    A.walk_zero = ptr<int64_t>(ctx->readback) + kRbWalk;
    LevelStarts ls;
    for (int l = 0; l <= kLevels; ++l) ls.s[l] = ctx->level_start[l];
    k_moments_leaves<<<blocks_for(nn, 128), 128, 0, ctx->stream>>>(
        A, ptr<int32_t>(ctx->node_nchild), ptr<int32_t>(ctx->node_parent), ls);
    if ((rc = check_hip(ctx, hipGetLastError(), "moments (leaves)"))) return rc;
    // the levels 0 .. top whose children levels hold at most kMomTopChildren
    // nodes go to one block
    int top = -1;
    while (top + 1 <= (int)ctx->depth - 1 &&
           ctx->level_start[top + 3] - ctx->level_start[top + 2] <= kMomTopChildren)
        ++top;
    for (int l = (int)ctx->depth - 1; l > top; --l) {   // the deepest level holds leaves only
        const int64_t cb = ctx->level_start[l + 1], ce = ctx->level_start[l + 2];
        k_moments_level<<<blocks_for(ce - cb, kMomChunk), kMomThreads, 0, ctx->stream>>>(
            A, l, cb, ce);
        if ((rc = check_hip(ctx, hipGetLastError(), "moments (level)"))) return rc;
    }
    if (top >= 0) {
        k_moments_top<<<1, kMomThreads, 0, ctx->stream>>>(A, top, ls);
        if ((rc = check_hip(ctx, hipGetLastError(), "moments (top levels)"))) return rc;
    }
    return P3T_OK;
}

// ---------------------------------------------------------------------------
// Groups: the moments folds flag the first particle of every group node; the
// flagged particles are compacted in particle order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ GroupInfo group_info(const NodeWalk &nd, int32_t id) {
    GroupInfo g;
    for (int k = 0; k < 3; ++k) {
        g.lo[k] = nd.lo[k];
        g.hi[k] = nd.hi[k];
        g.c[k] = (nd.lo[k] + nd.hi[k]) * 0.5;
    }
    g.first = nd.first;
    g.count = nd.count;
    g.node = id;
    g.pad = 0;
    return g;
}

// the group record of a flagged particle, at its rank among the flags
struct GroupSink {
    const int32_t *node_at;
    const NodeWalk *nw;
    GroupInfo *grp;
    __device__ __forceinline__ void operator()(int64_t a, int32_t slot, int32_t flag) const {
        if (!flag) return;
        const int32_t id = node_at[a];
        grp[slot] = group_info(nw[id], id);
    }
};

// (more than kScan2MaxTiles tiles of particles) also clears the walk's
// statistics words (zero, nz of them)
__global__ void k_group_compact(int64_t n, const int32_t *__restrict__ flag,
                                const int32_t *__restrict__ slot, const int32_t *__restrict__ node_at,
                                const NodeWalk *__restrict__ nw, GroupInfo *__restrict__ grp,
                                int64_t *__restrict__ zero, int nz) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < nz) zero[a] = 0;
    if (a >= n || !flag[a]) return;
    const int32_t id = node_at[a];
    grp[slot[a]] = group_info(nw[id], id);
}

int build_groups(p3t_ctx *ctx) {
    int rc;
    const int64_t n = ctx->n, nn = ctx->n_nodes;
    if ((rc = ensure(ctx, ctx->gflag, (n + 1) * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->gscan, (n + 1) * sizeof(int32_t)))) return rc;
    if ((rc = ensure(ctx, ctx->lvlrange, (n + 1) * sizeof(int32_t)))) return rc;   // reused: node_at
    if ((rc = ensure(ctx, ctx->grp, (nn + 1) * sizeof(GroupInfo)))) return rc;
    int32_t *flag = ptr<int32_t>(ctx->gflag), *slot = ptr<int32_t>(ctx->gscan);
    int32_t *node_at = ptr<int32_t>(ctx->lvlrange);
    // the group nodes were flagged by the moments folds; slot[n] = number of
    // groups (device), read back together with the list sizes
    const int64_t tiles = (n + 1 + kScan2Tile - 1) / kScan2Tile;
    if (group_tiles_counted(ctx, n)) {
        // the folds counted the groups per tile; the scan places the group
        // records itself
        k_scan2_tiles<int32_t><<<(unsigned)tiles, kScan2Threads, 0, ctx->stream>>>(
            flag, n + 1, ptr<int32_t>(ctx->gtile), slot + n,
            GroupSink{node_at, ptr<NodeWalk>(ctx->node_walk), ptr<GroupInfo>(ctx->grp)});
        return check_hip(ctx, hipGetLastError(), "groups");
    }
    if ((rc = scan_exclusive_i32(ctx, flag, slot, n + 1, nullptr))) return rc;
    k_group_compact<<<blocks_for(n > kRbWalkWords ? n : kRbWalkWords, 256), 256, 0, ctx->stream>>>(
        n, flag, slot, node_at, ptr<NodeWalk>(ctx->node_walk), ptr<GroupInfo>(ctx->grp),
        ptr<int64_t>(ctx->readback) + kRbWalk, kRbWalkWords);
    return check_hip(ctx, hipGetLastError(), "group compact");
}

}  // namespace p3t
