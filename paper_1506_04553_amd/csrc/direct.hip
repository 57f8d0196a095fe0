// direct.hip -- O(N^2) direct summation of the softened force and potential
// over every pair, for energies and diagnostics (the exact sums the tree
// approximates; Section 2.1):
//   NEWTON  a_i = sum_{j != i} m_j d / s^3,            phi_i = -sum m_j / s
//   SOFT    a_i = sum m_j K(s) d / s^3,                 phi_i = -sum m_j W(s) / s
//   HARD    a_i = sum m_j (1 - K(s)) d / s^3,           phi_i = -sum m_j (1 - W(s)) / s
// with d = x_j - x_i, s^2 = |d|^2 + eps^2 and y = s / r_out.  FP64 throughout.
//
// Layout: a block of 256 threads owns 512 i-particles (two per thread, two
// independent accumulation chains); j-particles stream through LDS in tiles of
// 256 as 32-byte records.  Every block reads all of the positions, which stay
// in L2, so the kernel is bound by FP64 issue, not by HBM.  Beyond r_out
// (almost every pair) K = W = 1: SOFT is the NEWTON pair, HARD contributes
// nothing, and the changeover polynomials run only inside r_out.
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kDirThreads = 256;
constexpr int kDirPerThread = 2;
constexpr int kDirTile = 256;

struct DirectConsts {
    double eps2, rout2, inv_rout, gamma, inv_1mg, C_over_rout;
    double w[7];
    double wl, wm;
};

struct alignas(32) DJ {
    double x, y, z, m;
};

// 1/sqrt(x), x > 0: the hardware estimate r and one step of the series
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8, e = 1 - x r^2, which cubes the estimate's
// relative error (~2^-22) to below the FP64 rounding level
__device__ __forceinline__ double rsq_nr(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * r, r, 1.0);
    return __builtin_fma(r * e, __builtin_fma(e, 0.375, 0.5), r);
}

// K(y) and W(y)/s on y < 1
__device__ __forceinline__ void changeover_in(double s, double rinv, const DirectConsts &dc,
                                              double &K, double &Ws) {
    const double y = s * dc.inv_rout;
    if (y < dc.gamma) {
        K = 0.0;
        Ws = dc.C_over_rout;
        return;
    }
    const double x = (y - dc.gamma) * dc.inv_1mg;
    const double x2 = x * x;
    K = x2 * x2 * __builtin_fma(x, __builtin_fma(x, __builtin_fma(x, -20.0, 70.0), -84.0), 35.0);
    double p = dc.w[6];
    for (int k = 5; k >= 0; --k) p = __builtin_fma(p, y, dc.w[k]);
    Ws = (p + dc.wl * log(y) + dc.wm / y) * dc.inv_rout;
    (void)rinv;
}

// SELF: the tile may hold particle i itself, whose pair is excluded (and kept
// finite when eps = 0)
template <int MODE, bool SELF>
__device__ __forceinline__ void pair(double xi, double yi, double zi, int64_t i, const DJ &j,
                                     int64_t jid, const DirectConsts &dc, double a[4]) {
    const double dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
    double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, dc.eps2)));
    double mf = j.m;
    if (SELF && jid == i) {
        mf = 0.0;
        r2 = 1.0;
    }
    const double rinv = rsq_nr(r2);
    if (MODE == P3T_DIRECT_NEWTON) {
        const double mr = mf * rinv;
        const double mr3 = mr * rinv * rinv;
        a[0] = __builtin_fma(mr3, dx, a[0]);
        a[1] = __builtin_fma(mr3, dy, a[1]);
        a[2] = __builtin_fma(mr3, dz, a[2]);
        a[3] -= mr;
        return;
    }
    if (r2 >= dc.rout2) {                  // K = W = 1
        if (MODE == P3T_DIRECT_SOFT) {
            const double mr = mf * rinv;
            const double mr3 = mr * rinv * rinv;
            a[0] = __builtin_fma(mr3, dx, a[0]);
            a[1] = __builtin_fma(mr3, dy, a[1]);
            a[2] = __builtin_fma(mr3, dz, a[2]);
            a[3] -= mr;
        }
        return;
    }
    double K, Ws;
    changeover_in(r2 * rinv, rinv, dc, K, Ws);
    const double kf = MODE == P3T_DIRECT_SOFT ? K : 1.0 - K;
    const double wf = MODE == P3T_DIRECT_SOFT ? Ws : rinv - Ws;
    const double f = mf * kf * rinv * rinv * rinv;
    a[0] = __builtin_fma(f, dx, a[0]);
    a[1] = __builtin_fma(f, dy, a[1]);
    a[2] = __builtin_fma(f, dz, a[2]);
    a[3] -= mf * wf;
}

template <int MODE>
__global__ __launch_bounds__(kDirThreads) void k_direct(int64_t n, const double *__restrict__ pos,
                                                       const double *__restrict__ mass,
                                                       DirectConsts dc, double *__restrict__ acc,
                                                       double *__restrict__ pot) {
    __shared__ DJ s_j[kDirTile];
    const int tid = threadIdx.x;
    int64_t ii[kDirPerThread];
    double xi[kDirPerThread], yi[kDirPerThread], zi[kDirPerThread];
    double a[kDirPerThread][4];
#pragma unroll
    for (int q = 0; q < kDirPerThread; ++q) {
        const int64_t i = (int64_t)blockIdx.x * (kDirThreads * kDirPerThread) + q * kDirThreads + tid;
        ii[q] = i;
        const int64_t ic = i < n ? i : n - 1;
        xi[q] = pos[3 * ic];
        yi[q] = pos[3 * ic + 1];
        zi[q] = pos[3 * ic + 2];
        a[q][0] = a[q][1] = a[q][2] = a[q][3] = 0.0;
    }
    for (int64_t t0 = 0; t0 < n; t0 += kDirTile) {
        const int tl = (int)min<int64_t>(kDirTile, n - t0);
        __syncthreads();
        if (tid < tl) {
            const int64_t j = t0 + tid;
            s_j[tid] = DJ{pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], mass[j]};
        }
        __syncthreads();
        // only the tiles that overlap the block's own particles can hold i
        const int64_t i0 = (int64_t)blockIdx.x * (kDirThreads * kDirPerThread);
        if (t0 + tl > i0 && t0 < i0 + kDirThreads * kDirPerThread) {
            for (int k = 0; k < tl; ++k) {
                const DJ jj = s_j[k];
#pragma unroll
                for (int q = 0; q < kDirPerThread; ++q)
                    pair<MODE, true>(xi[q], yi[q], zi[q], ii[q], jj, t0 + k, dc, a[q]);
            }
        } else {
            for (int k = 0; k < tl; ++k) {
                const DJ jj = s_j[k];
#pragma unroll
                for (int q = 0; q < kDirPerThread; ++q)
                    pair<MODE, false>(xi[q], yi[q], zi[q], ii[q], jj, t0 + k, dc, a[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kDirPerThread; ++q) {
        const int64_t i = ii[q];
        if (i >= n) continue;
        acc[3 * i] = a[q][0];
        acc[3 * i + 1] = a[q][1];
        acc[3 * i + 2] = a[q][2];
        if (pot) pot[i] = a[q][3];
    }
}

int launch_direct(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                  const p3t_params *p, int mode, double *acc, double *pot) {
    const Changeover c = make_changeover(p->r_in, p->r_out);
    DirectConsts dc{};
    dc.eps2 = p->eps * p->eps;
    dc.rout2 = p->r_out * p->r_out;
    dc.inv_rout = c.inv_rout;
    dc.gamma = c.gamma;
    dc.inv_1mg = c.inv_1mg;
    dc.C_over_rout = c.C * c.inv_rout;
    for (int k = 0; k < 7; ++k) dc.w[k] = c.w[k];
    dc.wl = c.wl;
    dc.wm = c.wm;
    const unsigned blocks = blocks_for(n, kDirThreads * kDirPerThread);
    if (mode == P3T_DIRECT_NEWTON)
        k_direct<P3T_DIRECT_NEWTON><<<blocks, kDirThreads, 0, ctx->stream>>>(n, pos, mass, dc, acc, pot);
    else if (mode == P3T_DIRECT_SOFT)
        k_direct<P3T_DIRECT_SOFT><<<blocks, kDirThreads, 0, ctx->stream>>>(n, pos, mass, dc, acc, pot);
    else
        k_direct<P3T_DIRECT_HARD><<<blocks, kDirThreads, 0, ctx->stream>>>(n, pos, mass, dc, acc, pot);
    return check_hip(ctx, hipGetLastError(), "direct");
}

}  // namespace p3t
