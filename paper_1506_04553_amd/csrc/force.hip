// force.hip -- long-range (soft) interaction kernels.
//
// For every particle i of group g (Section 2.1 soft force, Section 2.2 tree):
//   particle terms over P_g, j != i:   a_i += m_j K(y) d / s^3,  phi_i -= m_j W(y) / s
//   cell terms over C_g (r = x_i - com): a_i += K(y_c) [-M r/s^3 + Q r/s^5 - 5/2 (r.Q.r) r/s^7]
//                                        phi_i += W(y_c) [-M/s - (r.Q.r) / (2 s^5)]
// with s the softened distance, y = s / r_out, K and W the changeover functions
// of Section 2.1 (denominator of G read as (gamma - 1)^7).
//
// Kernel design (one block of four wavefronts per group):
//  * a lane is (i, slice): 64/s group members times s slices, each slice
//    taking every s-th entry of a list tile; s (a power of two) is chosen per
//    group to minimise padded lane work, so groups of any size keep the lanes
//    busy.  Each lane carries two i-particles (two "virtual wavefronts") that
//    share every LDS read; a group of V virtual wavefronts takes ceil(V/8)
//    rounds over its lists.  Slice partial sums are reduced in FP64 with
//    cross-lane shuffles in a fixed order;
//  * list entries are staged through LDS tiles of 256 loaded by the whole
//    block, the next tile being fetched into registers while the current one
//    is consumed; loop trip counts are wave-uniform (lanes past the end of a
//    tile read zero-mass padding entries);
//    positions are shifted to the group's box centre in FP64 while staging (the
//    mixed path then rounds the offsets to FP32);
//  * K and W differ from 1 only when s < r_out.  The walk splits the particle
//    list into far particles (leaf box at least max(h, r_out) from the group
//    box: K = W = 1, never i itself), evaluated as plain softened terms with no
//    test at all, and near particles, where a wave-uniform branch taken only
//    when some lane has s < r_out evaluates K, W and the j == i exclusion.  W's
//    middle branch is evaluated in FP64 in both paths (its monomial form
//    cancels by two orders of magnitude).  Accepted cells lie at least h from
//    the group, so their K = W = 1 is tested only when h < r_out;
//  * the mixed path accumulates each tile in FP32 and adds tile partials to a
//    compensated (Kahan) FP32 sum per particle and component.
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kForceWaves = 4;      // wavefronts per group (block)
constexpr int kForceThreads = kForceWaves * kWave;
constexpr int kTile = kForceThreads;

struct ForceParams {
    double eps2, rout2, inv_rout, gamma, inv_1mg, C_over_rout;
    double w[7];
    double wl, wm;
    int use_quad;
};

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: the hardware estimate y, then one step of the series
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 with e = 1 - x y^2.  The arguments are
// softened squared distances, finite and positive, so no special values are
// screened (a zero argument only arises for a particle with itself at zero
// softening, and that pair is discarded by index).
__device__ __forceinline__ double rsq(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// W(y)/y on gamma <= y < 1 (FP64)
__device__ __forceinline__ double w_over_y_band(double y, const ForceParams &fp) {
    double p = fp.w[6];
    for (int k = 5; k >= 0; --k) p = p * y + fp.w[k];
    return p + fp.wl * log(y) + fp.wm / y;
}

// K(y) and W(y)/s for one pair; self pair gives (0, 0).
template <class R>
__device__ __forceinline__ void changeover(R r2, R rinv, const ForceParams &fp, R &K, R &Ws) {
    const R s = r2 * rinv;
    const R y = s * (R)fp.inv_rout;
    if (y >= R(1)) {
        K = R(1);
        Ws = rinv;
    } else if (y < (R)fp.gamma) {
        K = R(0);
        Ws = (R)fp.C_over_rout;
    } else {
        const R x = (y - (R)fp.gamma) * (R)fp.inv_1mg;
        const R x2 = x * x;
        K = x2 * x2 * fmaR(x, fmaR(x, fmaR(x, R(-20), R(70)), R(-84)), R(35));
        Ws = (R)(w_over_y_band((double)y, fp) * fp.inv_rout);
    }
}

// compensated accumulation of tile partials (FP32); FP64 adds directly
template <class R>
struct Sum {
    R s = 0, c = 0;
    __device__ __forceinline__ void add(R v) {
        const R y = v - c;
        const R t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};
template <>
struct Sum<double> {
    double s = 0;
    __device__ __forceinline__ void add(double v) { s += v; }
    __device__ __forceinline__ double value() const { return s; }
};

// LDS records: one 128-bit (float) or 2x128-bit (double) read per particle,
// three / five per cell (16-byte aligned: a cell is 48 bytes in float, 80 in
// double, which keeps the double kernel's LDS within four blocks per CU).
template <class R>
struct alignas(4 * sizeof(R)) PJ {
    R x, y, z, m;
};
template <class R>
struct alignas(16) CJ {
    R x, y, z, M, qxx, qyy, qzz, qxy, qxz, qyz;
};

// i-particle slot: position offset, tile partials and compensated sums
template <class R>
struct Slot {
    R x, y, z;
    R ax, ay, az, ph;
    Sum<R> sx, sy, sz, sp;
    int32_t i;
    // FP32: fold the tile partials into the compensated sums; FP64: the
    // partials are the sums (no second set of registers)
    __device__ __forceinline__ void flush() {
        if (sizeof(R) == 8) return;
        sx.add(ax); sy.add(ay); sz.add(az); sp.add(ph);
        ax = ay = az = ph = R(0);
    }
    __device__ __forceinline__ double total(int c) const {
        if (sizeof(R) == 8)
            return c == 0 ? (double)ax : c == 1 ? (double)ay : c == 2 ? (double)az : (double)ph;
        return c == 0 ? sx.value() : c == 1 ? sy.value() : c == 2 ? sz.value() : sp.value();
    }
};

template <class R>
__device__ __forceinline__ void pp_fast(Slot<R> &q, const PJ<R> &j, R eps2) {
    const R dx = j.x - q.x, dy = j.y - q.y, dz = j.z - q.z;
    const R r2 = fmaR(dx, dx, fmaR(dy, dy, fmaR(dz, dz, eps2)));
    const R rinv = rsq(r2);
    const R mr = j.m * rinv;
    const R f = mr * (rinv * rinv);
    q.ax = fmaR(f, dx, q.ax);
    q.ay = fmaR(f, dy, q.ay);
    q.az = fmaR(f, dz, q.az);
    q.ph -= mr;
}

template <class R>
__device__ __forceinline__ void pp_full(Slot<R> &q, const PJ<R> &j, int32_t jid, R eps2,
                                        const ForceParams &fp) {
    const R dx = j.x - q.x, dy = j.y - q.y, dz = j.z - q.z;
    const R r2 = fmaR(dx, dx, fmaR(dy, dy, fmaR(dz, dz, eps2)));
    const R rinv = rsq(r2);
    R K, Ws;
    changeover<R>(r2, rinv, fp, K, Ws);
    // the pair of a particle with itself is discarded by selection, not by a
    // zero factor: at zero softening its 1/s is infinite
    const bool self = jid == q.i;
    const R f = self ? R(0) : j.m * K * (rinv * rinv * rinv);
    q.ax = fmaR(f, dx, q.ax);
    q.ay = fmaR(f, dy, q.ay);
    q.az = fmaR(f, dz, q.az);
    q.ph = fmaR(-j.m, self ? R(0) : Ws, q.ph);
}

// cell term; with B = (r.Q.r)/s^4:
//   phi += -(M + B/2)/s,  a += -(M + 5B/2) r/s^3 + Q r/s^5
// Where K = W = 1 for every cell (CHECK_K false) the potential is accumulated
// as two FMAs and the radial factor as -M/s^3 - 5/2 (r.Q.r)/s^7, one operation
// fewer than scaling a combined factor.
template <class R, bool QUAD, bool CHECK_K>
__device__ __forceinline__ void pc_term(Slot<R> &q, const CJ<R> &c, R eps2, R rout2,
                                        const ForceParams &fp) {
    const R rx = q.x - c.x, ry = q.y - c.y, rz = q.z - c.z;
    const R r2 = fmaR(rx, rx, fmaR(ry, ry, fmaR(rz, rz, eps2)));
    const R rinv = rsq(r2);
    const R u = rinv * rinv;
    const R rinv3 = rinv * u;
    if (QUAD && !CHECK_K) {
        const R Qx = fmaR(c.qxx, rx, fmaR(c.qxy, ry, c.qxz * rz));
        const R Qy = fmaR(c.qxy, rx, fmaR(c.qyy, ry, c.qyz * rz));
        const R Qz = fmaR(c.qxz, rx, fmaR(c.qyz, ry, c.qzz * rz));
        const R rQr = fmaR(rx, Qx, fmaR(ry, Qy, rz * Qz));
        const R rinv5 = rinv3 * u;
        const R Bs = rQr * rinv5;   // (r.Q.r)/s^5
        q.ph = fmaR(-c.M, rinv, q.ph);
        q.ph = fmaR(Bs, R(-0.5), q.ph);
        const R cr = fmaR(Bs * u, R(-2.5), -c.M * rinv3);
        q.ax = fmaR(cr, rx, fmaR(rinv5, Qx, q.ax));
        q.ay = fmaR(cr, ry, fmaR(rinv5, Qy, q.ay));
        q.az = fmaR(cr, rz, fmaR(rinv5, Qz, q.az));
        return;
    }
    R cr, cq = R(0), pot;
    R Qx = R(0), Qy = R(0), Qz = R(0);
    if (QUAD) {
        Qx = fmaR(c.qxx, rx, fmaR(c.qxy, ry, c.qxz * rz));
        Qy = fmaR(c.qxy, rx, fmaR(c.qyy, ry, c.qyz * rz));
        Qz = fmaR(c.qxz, rx, fmaR(c.qyz, ry, c.qzz * rz));
        const R rQr = fmaR(rx, Qx, fmaR(ry, Qy, rz * Qz));
        const R B = rQr * (u * u);
        pot = fmaR(B, R(-0.5), -c.M) * rinv;
        cr = fmaR(B, R(2.5), c.M) * (-rinv3);
        cq = rinv3 * u;
    } else {
        pot = -c.M * rinv;
        cr = -c.M * rinv3;
    }
    if (CHECK_K) {
        if (ballot(r2 < rout2)) {
            R K, Ws;
            changeover<R>(r2, rinv, fp, K, Ws);
            const R W = Ws * r2 * rinv;   // W(y) = (W/s) s
            cr *= K;
            cq *= K;
            pot *= W;
        }
    }
    if (QUAD) {
        q.ax = fmaR(cr, rx, fmaR(cq, Qx, q.ax));
        q.ay = fmaR(cr, ry, fmaR(cq, Qy, q.ay));
        q.az = fmaR(cr, rz, fmaR(cq, Qz, q.az));
    } else {
        q.ax = fmaR(cr, rx, q.ax);
        q.ay = fmaR(cr, ry, q.ay);
        q.az = fmaR(cr, rz, q.az);
    }
    q.ph += pot;
}

// Per-tile loops of one wavefront over its slice of the staged entries, for
// one or two active i-slots (TWO), so that the loop bodies carry no branch on
// the slot count.  The FP64 loops are unrolled deeper (four entries): their
// pipe otherwise waits on FP64 latencies.
// A slice's entries are consecutive in LDS (the tile is stored slice by
// slice), so unrolled iterations read at immediate offsets from one address.
// Trip counts are wave-uniform: lanes past the end of a tile read the padding
// entries (zero mass, far away), whose terms are exactly zero.
template <class R, bool TWO>
__device__ __forceinline__ void far_tile(Slot<R> *q, const PJ<R> *sp, int iters, R eps2) {
#pragma unroll(sizeof(R) == 8 ? 4 : 2)
    for (int it = 0; it < iters; ++it, ++sp) {
        const PJ<R> pj = *sp;
        pp_fast<R>(q[0], pj, eps2);
        if (TWO) pp_fast<R>(q[1], pj, eps2);
    }
}

template <class R, bool TWO>
__device__ __forceinline__ void near_tile(Slot<R> *q, const PJ<R> *sp, const int32_t *sj, int iters,
                                          R eps2, R rout2, const ForceParams &fp) {
    for (int it = 0; it < iters; ++it, ++sp, ++sj) {
        const PJ<R> pj = *sp;
        // the changeover path where s < r_out, and for a particle's own pair
        // (zero offset: s^2 = eps^2 exactly), which only that path discards, also
        // when the softening reaches beyond r_out
        const R dx0 = pj.x - q[0].x, dy0 = pj.y - q[0].y, dz0 = pj.z - q[0].z;
        const R r20 = fmaR(dx0, dx0, fmaR(dy0, dy0, fmaR(dz0, dz0, eps2)));
        bool nr = (r20 < rout2) | (r20 == eps2);
        if (TWO) {
            const R dx1 = pj.x - q[1].x, dy1 = pj.y - q[1].y, dz1 = pj.z - q[1].z;
            const R r21 = fmaR(dx1, dx1, fmaR(dy1, dy1, fmaR(dz1, dz1, eps2)));
            nr = nr | (r21 < rout2) | (r21 == eps2);
        }
        if (ballot(nr)) {
            const int32_t jid = *sj;
            pp_full<R>(q[0], pj, jid, eps2, fp);
            if (TWO) pp_full<R>(q[1], pj, jid, eps2, fp);
        } else {
            pp_fast<R>(q[0], pj, eps2);
            if (TWO) pp_fast<R>(q[1], pj, eps2);
        }
    }
}

template <class R, bool QUAD, bool CHECK_K, bool TWO>
__device__ __forceinline__ void cell_tile(Slot<R> *q, const CJ<R> *sc, int iters, R eps2, R rout2,
                                          const ForceParams &fp) {
#pragma unroll(sizeof(R) == 8 ? 4 : 2)
    for (int it = 0; it < iters; ++it, ++sc) {
        const CJ<R> cj = *sc;
        pc_term<R, QUAD, CHECK_K>(q[0], cj, eps2, rout2, fp);
        if (TWO) pc_term<R, QUAD, CHECK_K>(q[1], cj, eps2, rout2, fp);
    }
}

// Occupancy: FP32, five wavefronts per SIMD (96 VGPRs; the hot loops keep
// their registers, a few values of the near path and of the tile loop go to
// scratch), which hides more latency than four of 118 VGPRs; FP64, four (128
// VGPRs).
template <class R, bool QUAD, bool CHECK_K>
__global__ __launch_bounds__(kForceThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 4 : 5))) void k_force(
    const GroupInfo *__restrict__ grp, ListsDev L, const PosMass *__restrict__ xm,
    const NodeMP *__restrict__ mp, const int32_t *__restrict__ perm, ForceParams fp,
    double *__restrict__ acc, double *__restrict__ pot) {
    // one tile, stored slice by slice (see below)
    __shared__ PJ<R> s_p[kTile + kWave];
    __shared__ int32_t s_jid[kTile + kWave];
    __shared__ CJ<R> s_c[kTile + kWave];
    const PJ<R> zero_p{R(-1e18), R(-1e18), R(-1e18), R(0)};
    CJ<R> zero_c;
    zero_c.x = zero_c.y = zero_c.z = R(-1e18);
    zero_c.M = zero_c.qxx = zero_c.qyy = zero_c.qzz = zero_c.qxy = zero_c.qxz = zero_c.qyz = R(0);

    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int g = L.order[blockIdx.x];
    const GroupInfo gi = grp[g];
    const double gcx = gi.c[0], gcy = gi.c[1], gcz = gi.c[2];
    const int64_t cb = L.beg[0][g], ce = L.end[0][g];
    const int64_t pb = L.beg[1][g], pe = L.end[1][g];
    const int64_t nb = L.beg[2][g], ne = L.end[2][g];
    const int32_t *__restrict__ c_idx = L.idx[0];
    const int32_t *__restrict__ p_idx = L.idx[1];
    const int32_t *__restrict__ n_idx = L.idx[2];
    const R eps2 = (R)fp.eps2, rout2 = (R)fp.rout2;

    const int ls = choose_log2_slices(gi.count, 2 * kForceWaves);
    const int ns = 1 << ls;
    const int nw = kWave >> ls;                 // i-particles per virtual wavefront
    const int il = lane & (nw - 1), slice = lane >> (6 - ls);
    const int V = (gi.count + nw - 1) / nw;
    // Tile entry e belongs to slice e mod ns, as its (e / ns)-th entry; it is
    // stored at (e mod ns) S + e / ns, S = kTile / ns + 1, so each slice's
    // entries are consecutive (one spare slot per slice staggers the slices
    // over the LDS banks).  Entries past a tile's end are staged as padding,
    // and no slice reads beyond kTile / ns entries, so every slot read holds
    // an entry or padding; ns S <= kTile + kWave.
    const int S = (kTile >> ls) + 1;
    const int spos = (tid & (ns - 1)) * S + (tid >> ls);   // this thread's staging slot
    const int sbase = slice * S;                            // this lane's slice

    for (int v0 = 0; v0 < V; v0 += 2 * kForceWaves) {
        // this wavefront's two virtual wavefronts (i-slots) in this round
        const bool act0 = v0 + w < V, act1 = v0 + kForceWaves + w < V;
        Slot<R> q[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int li = (v0 + kForceWaves * k + w) * nw + il;
            const bool valid = (k == 0 ? act0 : act1) && li < gi.count;
            const int32_t i = gi.first + (valid ? li : 0);
            const PosMass pi = xm[i];
            q[k].i = valid ? i : -1;
            // padding lanes sit far away: every term stays finite and is discarded
            q[k].x = valid ? (R)(pi.x - gcx) : R(1e18);
            q[k].y = valid ? (R)(pi.y - gcy) : R(1e18);
            q[k].z = valid ? (R)(pi.z - gcz) : R(1e18);
            q[k].ax = q[k].ay = q[k].az = q[k].ph = R(0);
        }
        // FP32 partials are folded into the compensated sums every >= 64 iterations
        int since = 0;
        auto fold = [&](int iters, bool last) {
            since += iters;
            if (since >= 64 || last) {
                if (act0) q[0].flush();
                if (act1) q[1].flush();
                since = 0;
            }
        };

        // ---- particle-particle terms: tiles staged through LDS by the whole
        //      block, the next tile fetched into registers while the current one
        //      is consumed ----
        // a list particle shifted to the group centre (FP64), then rounded to R
        auto stage = [&](const PosMass &pj) {
            return PJ<R>{(R)(pj.x - gcx), (R)(pj.y - gcy), (R)(pj.z - gcz), (R)pj.m};
        };
        auto stream_particles = [&](const int32_t *list, int64_t b, int64_t e, auto &&consume) {
            PJ<R> pre = zero_p;
            int32_t prej = -2;
            if (b + tid < e) {
                prej = list[b + tid];
                pre = stage(xm[prej]);
            }
            for (int64_t t0 = b; t0 < e; t0 += kTile) {
                const int tl = (int)min<int64_t>(kTile, e - t0);
                __syncthreads();
                s_p[spos] = pre;
                s_jid[spos] = prej;
                __syncthreads();
                if (t0 + kTile + tid < e) {
                    prej = list[t0 + kTile + tid];
                    pre = stage(xm[prej]);
                } else {
                    pre = zero_p;
                    prej = -2;
                }
                const int iters = (tl + ns - 1) >> ls;
                consume(iters);
                fold(iters, t0 + kTile >= e);
            }
        };
        // far particles: K = W = 1 and j != i, plain softened terms
        stream_particles(p_idx, pb, pe, [&](int iters) {
            if (act1) far_tile<R, true>(q, s_p + sbase, iters, eps2);
            else if (act0) far_tile<R, false>(q, s_p + sbase, iters, eps2);
        });
        // near particles: changeover and self exclusion where s < r_out
        stream_particles(n_idx, nb, ne, [&](int iters) {
            if (act1) near_tile<R, true>(q, s_p + sbase, s_jid + sbase, iters, eps2, rout2, fp);
            else if (act0)
                near_tile<R, false>(q, s_p + sbase, s_jid + sbase, iters, eps2, rout2, fp);
        });

        // ---- particle-cell terms ----
        {
            auto load_cell = [&](int64_t e) {
                const NodeMP c = mp[c_idx[e]];
                CJ<R> r;
                r.x = (R)(c.cx - gcx); r.y = (R)(c.cy - gcy); r.z = (R)(c.cz - gcz); r.M = (R)c.M;
                r.qxx = (R)c.q[0]; r.qyy = (R)c.q[1]; r.qzz = (R)c.q[2];
                r.qxy = (R)c.q[3]; r.qxz = (R)c.q[4]; r.qyz = (R)c.q[5];
                return r;
            };
            CJ<R> pre = (cb + tid < ce) ? load_cell(cb + tid) : zero_c;
            for (int64_t t0 = cb; t0 < ce; t0 += kTile) {
                const int tl = (int)min<int64_t>(kTile, ce - t0);
                __syncthreads();
                s_c[spos] = pre;
                __syncthreads();
                pre = (t0 + kTile + tid < ce) ? load_cell(t0 + kTile + tid) : zero_c;
                const int iters = (tl + ns - 1) >> ls;
                if (act1)
                    cell_tile<R, QUAD, CHECK_K, true>(q, s_c + sbase, iters, eps2, rout2, fp);
                else if (act0)
                    cell_tile<R, QUAD, CHECK_K, false>(q, s_c + sbase, iters, eps2, rout2, fp);
                fold(iters, t0 + kTile >= ce);
            }
        }

        // ---- reduce the slices of each particle in FP64 (fixed order), write ----
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (!(k == 0 ? act0 : act1)) continue;
            double r0 = q[k].total(0), r1 = q[k].total(1), r2 = q[k].total(2),
                   r3 = q[k].total(3);
            for (int d = nw; d < kWave; d <<= 1) {
                r0 += __shfl_xor(r0, d, kWave);
                r1 += __shfl_xor(r1, d, kWave);
                r2 += __shfl_xor(r2, d, kWave);
                r3 += __shfl_xor(r3, d, kWave);
            }
            if (slice == 0 && q[k].i >= 0) {
                const int64_t o = perm[q[k].i];
                acc[3 * o] = r0;
                acc[3 * o + 1] = r1;
                acc[3 * o + 2] = r2;
                if (pot) pot[o] = r3;
            }
        }
    }
}

static ForceParams force_params(const p3t_ctx *ctx) {
    ForceParams fp{};
    fp.eps2 = ctx->prm.eps * ctx->prm.eps;
    fp.rout2 = ctx->prm.r_out * ctx->prm.r_out;
    fp.inv_rout = 1.0 / ctx->prm.r_out;
    fp.gamma = ctx->chg.gamma;
    fp.inv_1mg = ctx->chg.inv_1mg;
    fp.C_over_rout = ctx->chg.C / ctx->prm.r_out;
    for (int k = 0; k < 7; ++k) fp.w[k] = ctx->chg.w[k];
    fp.wl = ctx->chg.wl;
    fp.wm = ctx->chg.wm;
    fp.use_quad = ctx->prm.use_quadrupole ? 1 : 0;
    return fp;
}

template <class R, bool QUAD, bool CHECK_K>
static void launch_force_t(p3t_ctx *ctx, const ForceParams &fp, double *acc, double *pot) {
    k_force<R, QUAD, CHECK_K><<<(unsigned)ctx->n_groups, kForceThreads, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), lists_dev(ctx), ptr<PosMass>(ctx->xm), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), fp, acc, pot);
}

template <class R>
static void launch_force_r(p3t_ctx *ctx, const ForceParams &fp, double *acc, double *pot) {
    // accepted cells lie at least h away from every group member, so K = W = 1
    // on every cell term whenever h >= r_out
    const bool check_k = ctx->prm.r_search < ctx->prm.r_out;
    const bool quad = ctx->prm.use_quadrupole != 0;
    if (quad && !check_k) launch_force_t<R, true, false>(ctx, fp, acc, pot);
    else if (quad) launch_force_t<R, true, true>(ctx, fp, acc, pot);
    else if (!check_k) launch_force_t<R, false, false>(ctx, fp, acc, pot);
    else launch_force_t<R, false, true>(ctx, fp, acc, pot);
}

int launch_force(p3t_ctx *ctx, double *acc, double *pot) {
    const ForceParams fp = force_params(ctx);
    if (ctx->n_groups <= 0) return P3T_OK;
    if (ctx->prm.precision == P3T_PREC_MIXED) launch_force_r<float>(ctx, fp, acc, pot);
    else launch_force_r<double>(ctx, fp, acc, pot);
    return check_hip(ctx, hipGetLastError(), "force");
}

// ---------------------------------------------------------------------------
// Leapfrog: v += dt_kick * a; x += dt_drift * v
// ---------------------------------------------------------------------------
__global__ void k_kick_drift(int64_t n3, double *__restrict__ pos, double *__restrict__ vel,
                             const double *__restrict__ acc, double dk, double dd) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n3) return;
    const double v = vel[k] + dk * acc[k];
    vel[k] = v;
    pos[k] = pos[k] + dd * v;
}

int launch_kick_drift(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *acc,
                      double dt_kick, double dt_drift) {
    if (n <= 0) return P3T_OK;
    k_kick_drift<<<blocks_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, pos, vel, acc, dt_kick,
                                                                   dt_drift);
    return check_hip(ctx, hipGetLastError(), "kick/drift");
}

}  // namespace p3t
