// force.hip -- long-range (soft) interaction kernels.
//
// For every particle i of group g (Section 2.1 soft force, Section 2.2 tree):
//   particle terms over P_g, j != i:   a_i += m_j K(y) d / s^3,  phi_i -= m_j W(y) / s
//   cell terms over C_g (r = x_i - com): a_i += K(y_c) [-M r/s^3 + Q r/s^5 - 5/2 (r.Q.r) r/s^7]
//                                        phi_i += W(y_c) [-M/s - (r.Q.r) / (2 s^5)]
// with s the softened distance, y = s / r_out, K and W the changeover functions
// of Section 2.1 (denominator of G read as (gamma - 1)^7).
//
// Kernel design (one 256-thread block per group):
//  * group members are split over the block as (i, slice): a group of n_g
//    members padded to the next power of two p uses 256/p slices, each slice
//    walking every (256/p)-th entry of a list tile, so small groups still fill
//    the block; slice partial sums are reduced in FP64 at the end;
//  * list entries are staged through LDS in tiles of 256, each entry fetched
//    from HBM once per group; positions are shifted to the group's box centre
//    in FP64 while staging (the mixed path then rounds the offsets to FP32);
//  * K and W differ from 1 only when s < r_out.  The common case evaluates the
//    plain softened term; a wave-uniform branch, taken only when some lane of
//    the wave has s < r_out, evaluates K, W and the j == i exclusion.  W's
//    middle branch is evaluated in FP64 in both paths (its monomial form
//    cancels by two orders of magnitude);
//  * the mixed path accumulates each tile in FP32 and adds tile partials to a
//    compensated (Kahan) FP32 sum per particle and component.
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kForceThreads = 256;
constexpr int kTile = 256;

struct ForceParams {
    double eps2, rout2, inv_rout, gamma, inv_1mg, C_over_rout;
    double w[7];
    double wl, wm;
    int use_quad;
};

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
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

template <class R>
struct Acc4 {
    R ax = 0, ay = 0, az = 0, ph = 0;
};

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

template <class R>
__global__ __launch_bounds__(kForceThreads) void k_force(
    const GroupInfo *__restrict__ grp, const int64_t *__restrict__ p_off,
    const int32_t *__restrict__ p_idx, const int64_t *__restrict__ c_off,
    const int32_t *__restrict__ c_idx, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ m, const NodeMP *__restrict__ mp,
    const int32_t *__restrict__ perm, ForceParams fp, double *__restrict__ acc,
    double *__restrict__ pot) {
    __shared__ R s_px[kTile], s_py[kTile], s_pz[kTile], s_pm[kTile];
    __shared__ int32_t s_jid[kTile];
    __shared__ R s_c[10][kTile];
    __shared__ double s_red[4][kForceThreads];

    const int tid = threadIdx.x;
    const GroupInfo gi = grp[blockIdx.x];
    const double gcx = gi.c[0], gcy = gi.c[1], gcz = gi.c[2];
    const int64_t pb = p_off[blockIdx.x], pe = p_off[blockIdx.x + 1];
    const int64_t cb = c_off[blockIdx.x], ce = c_off[blockIdx.x + 1];
    const R eps2 = (R)fp.eps2, rout2 = (R)fp.rout2;

    for (int chunk = 0; chunk < gi.count; chunk += kForceThreads) {
        const int nc = min(kForceThreads, gi.count - chunk);
        int lg = 0;
        while ((1 << lg) < nc) ++lg;
        const int pad = 1 << lg;
        const int nslice = kForceThreads >> lg;
        const int li = tid & (pad - 1), slice = tid >> lg;
        const bool ivalid = li < nc;
        const int32_t i = gi.first + chunk + (ivalid ? li : 0);
        // far-away dummy position for padding lanes: every term is ~0 and stays finite
        const R xi = ivalid ? (R)(x[i] - gcx) : R(1e18), yi = ivalid ? (R)(y[i] - gcy) : R(1e18),
                zi = ivalid ? (R)(z[i] - gcz) : R(1e18);
        Sum<R> sx, sy, sz, sp;

        // ---- particle-particle terms ----
        for (int64_t t0 = pb; t0 < pe; t0 += kTile) {
            const int tl = (int)min<int64_t>(kTile, pe - t0);
            __syncthreads();
            if (tid < tl) {
                const int32_t j = p_idx[t0 + tid];
                s_px[tid] = (R)(x[j] - gcx);
                s_py[tid] = (R)(y[j] - gcy);
                s_pz[tid] = (R)(z[j] - gcz);
                s_pm[tid] = (R)m[j];
                s_jid[tid] = j;
            }
            __syncthreads();
            Acc4<R> a;
            for (int k = slice; k < tl; k += nslice) {
                const R dx = s_px[k] - xi, dy = s_py[k] - yi, dz = s_pz[k] - zi;
                const R mj = s_pm[k];
                const R r2 = fmaR(dx, dx, fmaR(dy, dy, fmaR(dz, dz, eps2)));
                const R rinv = rsq(r2);
                if (ballot(r2 < rout2)) {
                    R K, Ws;
                    changeover<R>(r2, rinv, fp, K, Ws);
                    if (s_jid[k] == i) { K = R(0); Ws = R(0); }
                    const R f = mj * K * rinv * rinv * rinv;
                    a.ax = fmaR(f, dx, a.ax);
                    a.ay = fmaR(f, dy, a.ay);
                    a.az = fmaR(f, dz, a.az);
                    a.ph = fmaR(-mj, Ws, a.ph);
                } else {
                    const R mr = mj * rinv;
                    const R f = mr * rinv * rinv;
                    a.ax = fmaR(f, dx, a.ax);
                    a.ay = fmaR(f, dy, a.ay);
                    a.az = fmaR(f, dz, a.az);
                    a.ph -= mr;
                }
            }
            sx.add(a.ax); sy.add(a.ay); sz.add(a.az); sp.add(a.ph);
        }

        // ---- particle-cell terms ----
        for (int64_t t0 = cb; t0 < ce; t0 += kTile) {
            const int tl = (int)min<int64_t>(kTile, ce - t0);
            __syncthreads();
            if (tid < tl) {
                const NodeMP c = mp[c_idx[t0 + tid]];
                s_c[0][tid] = (R)(c.cx - gcx);
                s_c[1][tid] = (R)(c.cy - gcy);
                s_c[2][tid] = (R)(c.cz - gcz);
                s_c[3][tid] = (R)c.M;
                for (int q = 0; q < 6; ++q) s_c[4 + q][tid] = fp.use_quad ? (R)c.q[q] : R(0);
            }
            __syncthreads();
            Acc4<R> a;
            for (int k = slice; k < tl; k += nslice) {
                const R rx = xi - s_c[0][k], ry = yi - s_c[1][k], rz = zi - s_c[2][k];
                const R M = s_c[3][k];
                const R r2 = fmaR(rx, rx, fmaR(ry, ry, fmaR(rz, rz, eps2)));
                const R rinv = rsq(r2);
                const R rinv2 = rinv * rinv;
                const R rinv3 = rinv * rinv2;
                const R qxx = s_c[4][k], qyy = s_c[5][k], qzz = s_c[6][k];
                const R qxy = s_c[7][k], qxz = s_c[8][k], qyz = s_c[9][k];
                const R Qx = fmaR(qxx, rx, fmaR(qxy, ry, qxz * rz));
                const R Qy = fmaR(qxy, rx, fmaR(qyy, ry, qyz * rz));
                const R Qz = fmaR(qxz, rx, fmaR(qyz, ry, qzz * rz));
                const R rQr = fmaR(rx, Qx, fmaR(ry, Qy, rz * Qz));
                const R rinv5 = rinv3 * rinv2;
                const R rinv7 = rinv5 * rinv2;
                R fa = fmaR(R(-2.5) * rQr, rinv7, -M * rinv3);   // coefficient of r
                R fq = rinv5;                                     // coefficient of Q r
                R pp = fmaR(R(-0.5) * rQr, rinv5, -M * rinv);
                if (ballot(r2 < rout2)) {
                    R K, Ws;
                    changeover<R>(r2, rinv, fp, K, Ws);
                    const R W = Ws * r2 * rinv;            // W(y) = (W/s) s
                    fa *= K;
                    fq *= K;
                    pp *= W;
                }
                a.ax = fmaR(fa, rx, fmaR(fq, Qx, a.ax));
                a.ay = fmaR(fa, ry, fmaR(fq, Qy, a.ay));
                a.az = fmaR(fa, rz, fmaR(fq, Qz, a.az));
                a.ph += pp;
            }
            sx.add(a.ax); sy.add(a.ay); sz.add(a.az); sp.add(a.ph);
        }

        // ---- reduce the slices of each particle in FP64, fixed order ----
        __syncthreads();
        s_red[0][tid] = sx.value();
        s_red[1][tid] = sy.value();
        s_red[2][tid] = sz.value();
        s_red[3][tid] = sp.value();
        __syncthreads();
        if (slice == 0 && ivalid) {
            double r[4] = {0, 0, 0, 0};
            for (int s = 0; s < nslice; ++s)
                for (int q = 0; q < 4; ++q) r[q] += s_red[q][s * pad + li];
            const int64_t o = perm[i];
            acc[3 * o] = r[0];
            acc[3 * o + 1] = r[1];
            acc[3 * o + 2] = r[2];
            if (pot) pot[o] = r[3];
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

int launch_force(p3t_ctx *ctx, double *acc, double *pot) {
    const ForceParams fp = force_params(ctx);
    if (ctx->n_groups <= 0) return P3T_OK;
    const unsigned grid = (unsigned)ctx->n_groups;
    const int64_t stride = ctx->n_nodes + 1;
    const int64_t *off = ptr<int64_t>(ctx->off);
    if (ctx->prm.precision == P3T_PREC_MIXED) {
        k_force<float><<<grid, kForceThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), off + stride, ptr<int32_t>(ctx->p_idx), off,
            ptr<int32_t>(ctx->c_idx), ptr<double>(ctx->x), ptr<double>(ctx->y), ptr<double>(ctx->z),
            ptr<double>(ctx->m), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), fp, acc, pot);
    } else {
        k_force<double><<<grid, kForceThreads, 0, ctx->stream>>>(
            ptr<GroupInfo>(ctx->grp), off + stride, ptr<int32_t>(ctx->p_idx), off,
            ptr<int32_t>(ctx->c_idx), ptr<double>(ctx->x), ptr<double>(ctx->y), ptr<double>(ctx->z),
            ptr<double>(ctx->m), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), fp, acc, pot);
    }
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
