// vjp.hip -- vector-Jacobian product of the long-range force and potential:
// for L = sum_i w_i . a_i + c_i phi_i, the gradients dL/dx_k and dL/dm_k with
// the tree, groups and interaction lists of the last build held fixed.
//
// Pair term (j in P_g, j != i), d = x_j - x_i, s^2 = |d|^2 + eps^2 and
// g(s) = K/s^3:  a_i += m_j g d,  phi_i -= m_j W/s (Section 2.1).  With
// K = W - s dW/ds one has d(W/s)/ds = -K/s^2, so
//   dl/dd = m_j [ g w + g'(s) (w.d) d/s + c K d/s^3 ],   dl/dm_j = g (w.d) - c W/s,
// added to x_j and subtracted from x_i.
// Cell term, r = x_i - com: A = -M r/s^3 + Q r/s^5 - 5/2 (r.Q.r) r/s^7 = -grad Phi,
// Phi = -M/s - (r.Q.r)/(2 s^5); l = K (w.A) + c W Phi, so
//   dl/dr = (K'(w.A) + c W' Phi) r/s - K H w - c W A   (H = Hessian of Phi),
//   dl/dcom = -dl/dr,  dl/dM = -K (w.r)/s^3 - c W/s,
//   dl/dQ (symmetric part) = K [(w r^T + r w^T)/(2 s^5) - 5/2 (w.r) r r^T/s^7] - c W r r^T/(2 s^5).
// Cell adjoints reach the member particles through com = S/M, M = sum m and
// Q = sum m (3 d d^T - |d|^2 I), d = x - com (sum m d = 0): each cell's
// contribution is the quadratic form f(x) = d^T B d + beta.d + gamma with
// B = 3 S - tr(S) I, beta = dl/dcom / M, gamma = dl/dM, and
//   dL/dm_k += f(x_k),   dL/dx_k += m_k (2 B d_k + beta).
// The forms of a leaf's ancestors are summed top-down, each re-centred at the
// child's centre of mass, so every particle needs only its leaf's form.
//
// The adjoint arithmetic takes no decisions (the lists are frozen), so unlike
// the rest of the library it lets the compiler fuse multiply-adds.  Runs of at
// most 32 terms are summed in R before each run's sum joins an FP64 sum; a
// member's cell and far-particle terms are summed in R over the 64 entries of
// a wavefront (a fixed tree) before joining an FP64 sum.
//
// Two passes over each group's lists: the first sums the near-particle terms
// of each member; the second sums, for each list entry, the terms of all
// members and scatters them, and evaluates each (member, cell) and (member,
// far particle) term only once, for both sides.
//
// The pair and cell terms are evaluated in the precision of the forward pass
// (R = double, or R = float on offsets from the group's centre taken in FP64,
// as in the interaction kernel; K and W themselves are evaluated in FP64) and
// summed in FP64.  Scatter to list entries uses FP64 atomic adds, one per
// (group, entry, component) after reduction over the group's members, so the
// result is reproducible up to the order of those atomic additions.  The cell
// adjoints are held component-major ([10][n_nodes]): the ten adds of one entry
// then fall on ten different cache lines, where in cell-major order they
// would queue on one line.  The push-down of the cell adjoints is FP64.
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kVjpThreads = 256;
constexpr int kVjpTile = 256;

struct VjpParams {
    double eps2, rout2, inv_rout, gamma, inv_1mg, C;
    double w[7];
    double wl, wm;
    int use_quad;
    int has_c;
};

// K, dK/ds, W, dW/ds at softened distance s.
struct Chg {
    double K, Ks, W, Ws;
};

__device__ __forceinline__ Chg changeover_ds(double s, const VjpParams &vp) {
#pragma clang fp contract(fast)
    Chg c;
    const double y = s * vp.inv_rout;
    if (y >= 1.0) {
        c.K = 1.0; c.Ks = 0.0; c.W = 1.0; c.Ws = 0.0;
    } else if (y < vp.gamma) {
        c.K = 0.0; c.Ks = 0.0; c.W = vp.C * y; c.Ws = vp.C * vp.inv_rout;
    } else {
        const double x = (y - vp.gamma) * vp.inv_1mg;
        const double x2 = x * x;
        c.K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
        const double u = x * (1.0 - x);
        const double dKdy = 140.0 * u * u * u * vp.inv_1mg;
        double p = vp.w[6];
        for (int k = 5; k >= 0; --k) p = p * y + vp.w[k];
        c.W = y * (p + vp.wl * log(y) + vp.wm / y);
        const double dWdy = (c.W - c.K) / y;
        c.Ks = dKdy * vp.inv_rout;
        c.Ws = dWdy * vp.inv_rout;
    }
    return c;
}

// K = W = 1 and dK/ds = dW/ds = 0 (pairs and cells at least r_out apart)
__device__ __forceinline__ Chg changeover_unit() { return Chg{1.0, 0.0, 1.0, 0.0}; }

__device__ __forceinline__ float vrsq(float v) { return __builtin_amdgcn_rsqf(v); }
// FP64: hardware estimate y and one step of (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8,
// e = 1 - v y^2; v is a softened squared distance of two different particles,
// finite and positive, so no special values are screened
__device__ __forceinline__ double vrsq(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    const double e = __builtin_fma(-v * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

// d(l_ij)/dd and d(l_ij)/dm_j for one pair; CHG false: K = W = 1 known.
template <class R, bool CHG>
__device__ __forceinline__ void pair_grad(R dx, R dy, R dz, R mj, R wx, R wy, R wz, R ci,
                                          const VjpParams &vp, R gd[3], R &gm) {
#pragma clang fp contract(fast)
    const R s2 = dx * dx + dy * dy + dz * dz + (R)vp.eps2;
    const R inv = vrsq(s2);
    const R s = s2 * inv;
    const R inv2 = inv * inv, inv3 = inv2 * inv;
    const Chg c = CHG ? changeover_ds((double)s, vp) : changeover_unit();
    const R K = (R)c.K, Ks = (R)c.Ks, W = (R)c.W;
    const R g = K * inv3;
    const R gp = Ks * inv3 - R(3) * K * inv2 * inv2;
    const R wd = wx * dx + wy * dy + wz * dz;
    const R t = gp * wd * inv + ci * K * inv3;
    gd[0] = mj * (g * wx + t * dx);
    gd[1] = mj * (g * wy + t * dy);
    gd[2] = mj * (g * wz + t * dz);
    gm = g * wd - ci * W * inv;
}

template <class R>
struct CellGrad {
    R gr[3];    // dl/dr (r = x_i - com)
    R gM;       // dl/dM
    R S[6];     // symmetric dl/dQ: xx yy zz xy xz yz
};

// a cell as staged for the adjoint kernels: centre of mass (shifted), M, Q
template <class R>
struct VjpCell {
    R x, y, z, M, q[6];
};

template <class R, bool CHG, bool QUAD>
__device__ __forceinline__ void cell_grad(R rx, R ry, R rz, R M, const R q[6], R wx, R wy, R wz,
                                          R ci, const VjpParams &vp, CellGrad<R> &o) {
#pragma clang fp contract(fast)
    const R s2 = rx * rx + ry * ry + rz * rz + (R)vp.eps2;
    const R inv = vrsq(s2);
    const R s = s2 * inv;
    const R inv2 = inv * inv, inv3 = inv2 * inv, inv5 = inv3 * inv2, inv7 = inv5 * inv2,
            inv9 = inv7 * inv2;
    const Chg c = CHG ? changeover_ds((double)s, vp) : changeover_unit();
    const R K = (R)c.K, Ks = (R)c.Ks, W = (R)c.W, Ws = (R)c.Ws;
    R Qr[3] = {0, 0, 0}, Qw[3] = {0, 0, 0}, qq = 0;
    if (QUAD) {
        Qr[0] = q[0] * rx + q[3] * ry + q[4] * rz;
        Qr[1] = q[3] * rx + q[1] * ry + q[5] * rz;
        Qr[2] = q[4] * rx + q[5] * ry + q[2] * rz;
        Qw[0] = q[0] * wx + q[3] * wy + q[4] * wz;
        Qw[1] = q[3] * wx + q[1] * wy + q[5] * wz;
        Qw[2] = q[4] * wx + q[5] * wy + q[2] * wz;
        qq = rx * Qr[0] + ry * Qr[1] + rz * Qr[2];
    }
    const R r[3] = {rx, ry, rz}, w[3] = {wx, wy, wz};
    const R rw = rx * wx + ry * wy + rz * wz;
    const R Qrw = Qr[0] * wx + Qr[1] * wy + Qr[2] * wz;
    R A[3], Hw[3];
    const R cw = M * inv3 + R(2.5) * qq * inv7;
    const R cr = R(-3) * M * rw * inv5 + R(5) * Qrw * inv7 - R(17.5) * qq * rw * inv9;
    const R cq = R(5) * rw * inv7;
    for (int a = 0; a < 3; ++a) {
        A[a] = -M * r[a] * inv3 + Qr[a] * inv5 - R(2.5) * qq * r[a] * inv7;
        Hw[a] = w[a] * cw - Qw[a] * inv5 + r[a] * cr + Qr[a] * cq;
    }
    const R Phi = -M * inv - R(0.5) * qq * inv5;
    const R wA = wx * A[0] + wy * A[1] + wz * A[2];
    const R radial = (Ks * wA + ci * Ws * Phi) * inv;
    for (int a = 0; a < 3; ++a) o.gr[a] = radial * r[a] - K * Hw[a] - ci * W * A[a];
    o.gM = -K * rw * inv3 - ci * W * inv;
    if (QUAD) {
        const R k5 = R(0.5) * K * inv5, k7 = R(-2.5) * K * rw * inv7, cwq = R(-0.5) * ci * W * inv5;
        const R rr = k7 + cwq;
        o.S[0] = R(2) * k5 * wx * rx + rr * rx * rx;
        o.S[1] = R(2) * k5 * wy * ry + rr * ry * ry;
        o.S[2] = R(2) * k5 * wz * rz + rr * rz * rz;
        o.S[3] = k5 * (wx * ry + wy * rx) + rr * rx * ry;
        o.S[4] = k5 * (wx * rz + wz * rx) + rr * rx * rz;
        o.S[5] = k5 * (wy * rz + wz * ry) + rr * ry * rz;
    } else {
        for (int a = 0; a < 6; ++a) o.S[a] = R(0);
    }
}

// The same terms for a cell at least r_out from the member (K = W = 1, dK/ds =
// dW/ds = 0), rearranged: with cw = M/s^3 + 5/2 qq/s^7 (qq = r.Q.r),
//   dl/dr = -cw w + Q w/s^5 + (c cw - cr) r - (cq + c/s^5) Q r,
//   cr = -3 M (r.w)/s^5 + 5 (r.Q.w)/s^7 - 35/2 qq (r.w)/s^9,  cq = 5 (r.w)/s^7,
// and dl/dQ = (w r^T + r w^T)/(2 s^5) + rr r r^T, rr = -5/2 (r.w)/s^7 - c/(2 s^5).
// Outputs: g = dl/dr, gM = dl/dM, S = dl/dQ (xx yy zz xy xz yz; zero without
// the quadrupole).
template <class R, bool QUAD>
__device__ __forceinline__ void cell_grad_far(R rx, R ry, R rz, R M, const R q[6], R wx, R wy,
                                              R wz, R ci, R eps2, R g[3], R &gM, R S[6]) {
#pragma clang fp contract(fast)
    const R s2 = rx * rx + ry * ry + rz * rz + eps2;
    const R inv = vrsq(s2);
    const R inv2 = inv * inv, inv3 = inv2 * inv, inv5 = inv3 * inv2;
    const R rw = rx * wx + ry * wy + rz * wz;
    gM = -rw * inv3 - ci * inv;
    if (!QUAD) {
        const R cw = M * inv3;
        const R b = ci * cw + R(3) * M * rw * inv5;   // c cw - cr, cr = -3 M (r.w)/s^5
        g[0] = b * rx - cw * wx;
        g[1] = b * ry - cw * wy;
        g[2] = b * rz - cw * wz;
        for (int a = 0; a < 6; ++a) S[a] = R(0);
        return;
    }
    const R inv7 = inv5 * inv2, inv9 = inv7 * inv2;
    const R Qr0 = q[0] * rx + q[3] * ry + q[4] * rz;
    const R Qr1 = q[3] * rx + q[1] * ry + q[5] * rz;
    const R Qr2 = q[4] * rx + q[5] * ry + q[2] * rz;
    const R Qw0 = q[0] * wx + q[3] * wy + q[4] * wz;
    const R Qw1 = q[3] * wx + q[1] * wy + q[5] * wz;
    const R Qw2 = q[4] * wx + q[5] * wy + q[2] * wz;
    const R qq = rx * Qr0 + ry * Qr1 + rz * Qr2;
    const R Qrw = Qr0 * wx + Qr1 * wy + Qr2 * wz;
    const R cw = M * inv3 + R(2.5) * qq * inv7;
    const R cr = R(-3) * M * rw * inv5 + R(5) * Qrw * inv7 - R(17.5) * qq * rw * inv9;
    const R b = ci * cw - cr;
    const R gq = -(R(5) * rw * inv7 + ci * inv5);
    g[0] = b * rx - cw * wx + inv5 * Qw0 + gq * Qr0;
    g[1] = b * ry - cw * wy + inv5 * Qw1 + gq * Qr1;
    g[2] = b * rz - cw * wz + inv5 * Qw2 + gq * Qr2;
    const R rr = R(-2.5) * rw * inv7 - R(0.5) * ci * inv5;
    const R k5 = R(0.5) * inv5;
    const R ux = k5 * wx, uy = k5 * wy, uz = k5 * wz;
    const R vx = rr * rx, vy = rr * ry, vz = rr * rz;
    S[0] = rx * (R(2) * ux + vx);
    S[1] = ry * (R(2) * uy + vy);
    S[2] = rz * (R(2) * uz + vz);
    S[3] = ry * (ux + vx) + rx * uy;
    S[4] = rz * (ux + vx) + rx * uz;
    S[5] = rz * (uy + vy) + ry * uz;
}

// coordinates are taken relative to `shift` in FP64 before rounding to R: the
// group's centre for R = float, the origin (no change) for R = double
template <class R>
__device__ __forceinline__ void group_shift(const GroupInfo &gi, double sh[3]) {
    for (int a = 0; a < 3; ++a) sh[a] = sizeof(R) == 4 ? gi.c[a] : 0.0;
}

template <class R>
__device__ __forceinline__ VjpCell<R> stage_cell(const NodeMP &c, const double sh[3]) {
    VjpCell<R> v;
    v.x = (R)(c.cx - sh[0]);
    v.y = (R)(c.cy - sh[1]);
    v.z = (R)(c.cz - sh[2]);
    v.M = (R)c.M;
    for (int a = 0; a < 6; ++a) v.q[a] = (R)c.q[a];
    return v;
}

// ---------------------------------------------------------------------------
// Pass 1: per particle i (one group per block), the i-side near-particle terms.
// ---------------------------------------------------------------------------
// Terms are summed in R over runs of at most kFold and each run's sum is added
// to an FP64 accumulator.
constexpr int kFold = 32;
// a run of member terms is parked one lane per member and row, half a run at a time
static_assert(kFold == 32, "two halves of 16 members");

// a list particle as staged in LDS: position (shifted) and mass
template <class R>
struct alignas(4 * sizeof(R)) VjpPart {
    R x, y, z, m;
};

// one tile of particle-list entries against member i (NEAR: the list may hold
// i itself, which is skipped)
template <class R, bool NEAR>
__device__ __forceinline__ void vjp_i_pp_tile(const VjpPart<R> *sp, const int32_t *sj, int tl,
                                              int slice, int nslice, int32_t i, R xi, R yi, R zi,
                                              R wx, R wy, R wz, R ci, const VjpParams &vp,
                                              double &g0, double &g1, double &g2) {
    for (int k0 = slice; k0 < tl; k0 += kFold * nslice) {
        const int k1 = min(tl, k0 + kFold * nslice);
        R p0 = 0, p1 = 0, p2 = 0;
        for (int k = k0; k < k1; k += nslice) {
            if (NEAR && sj[k] == i) continue;
            const VjpPart<R> q = sp[k];
            R gd[3], gmj;
            pair_grad<R, NEAR>(q.x - xi, q.y - yi, q.z - zi, q.m, wx, wy, wz, ci, vp, gd, gmj);
            p0 -= gd[0]; p1 -= gd[1]; p2 -= gd[2];
        }
        g0 += (double)p0; g1 += (double)p1; g2 += (double)p2;
    }
}

template <class R>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_i(
    const GroupInfo *__restrict__ grp, ListsDev L, const PosMass *__restrict__ xm,
    const NodeMP *__restrict__ mp,
    const int32_t *__restrict__ perm, const double *__restrict__ wv, const double *__restrict__ cv,
    VjpParams vp, double *__restrict__ gx, double *__restrict__ gm, int64_t n) {
    __shared__ VjpPart<R> s_p[kVjpTile];
    __shared__ int32_t s_j[kVjpTile];
    __shared__ double s_red[3][kVjpThreads];
    const int tid = threadIdx.x;
    const int g = L.order[blockIdx.x];
    const GroupInfo gi = grp[g];
    double sh[3];
    group_shift<R>(gi, sh);
    // members in chunks of the largest power of two that fits (at most 256),
    // so that a chunk fills its lanes: 74 members run as 64 + 8 + 2
    for (int chunk = 0, nc = 0; chunk < gi.count; chunk += nc) {
        const int rem = gi.count - chunk;
        int lg = 0;
        while (lg < 8 && (2 << lg) <= rem) ++lg;
        nc = 1 << lg;
        const int pad = nc, nslice = kVjpThreads >> lg;
        const int li = tid & (pad - 1), slice = tid >> lg;
        const int32_t i = gi.first + chunk + li;
        const int64_t o = perm[i];
        const PosMass pi = xm[i];
        const R xi = (R)(pi.x - sh[0]), yi = (R)(pi.y - sh[1]), zi = (R)(pi.z - sh[2]);
        const R wx = (R)wv[3 * o], wy = (R)wv[3 * o + 1], wz = (R)wv[3 * o + 2];
        const R ci = vp.has_c ? (R)cv[o] : R(0);
        double g0 = 0, g1 = 0, g2 = 0;
        {   // near particles (the far ones are summed by the list-entry pass)
            const int32_t *idxs = L.idx[2];
            const int64_t pb = L.beg[2][g];
            const int64_t pe = L.end[2][g];
            for (int64_t t0 = pb; t0 < pe; t0 += kVjpTile) {
                const int tl = (int)min<int64_t>(kVjpTile, pe - t0);
                __syncthreads();
                if (tid < tl) {
                    const int32_t j = idxs[t0 + tid];
                    const PosMass pj = xm[j];
                    s_p[tid] = VjpPart<R>{(R)(pj.x - sh[0]), (R)(pj.y - sh[1]), (R)(pj.z - sh[2]),
                                          (R)pj.m};
                    s_j[tid] = j;
                }
                __syncthreads();
                vjp_i_pp_tile<R, true>(s_p, s_j, tl, slice, nslice, i, xi, yi, zi, wx, wy, wz, ci,
                                       vp, g0, g1, g2);
            }
        }
        __syncthreads();
        s_red[0][tid] = g0; s_red[1][tid] = g1; s_red[2][tid] = g2;
        __syncthreads();
        if (slice == 0) {
            double r[3] = {0, 0, 0};
            for (int sidx = 0; sidx < nslice; ++sidx)
                for (int a = 0; a < 3; ++a) r[a] += s_red[a][sidx * pad + li];
            gx[i] = r[0];
            gx[n + i] = r[1];
            gx[2 * n + i] = r[2];
            gm[i] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 2: per list entry (particle j or cell c), the sum over the group's
// members, scattered with one atomic add per component; the cell terms also
// give the members their i-side cell terms.  Cell adjoints are
// component-major: component a of cell c at cadj[a * n_nodes + c].
// ---------------------------------------------------------------------------
// a group member as staged in LDS: position (shifted), w and c
template <class R>
struct alignas(4 * sizeof(R)) VjpMember {
    R x, y, z, c, wx, wy, wz, pad;
};

// list particle j against members [0, nc); NEAR: j may be a member, skipped
template <class R, bool NEAR>
__device__ __forceinline__ void vjp_scatter_pp(const VjpMember<R> *si, const int32_t *sid, int nc,
                                               int32_t j, R xj, R yj, R zj, R mj,
                                               const VjpParams &vp, double acc[4]) {
    for (int k0 = 0; k0 < nc; k0 += kFold) {
        const int k1 = min(nc, k0 + kFold);
        R p0 = 0, p1 = 0, p2 = 0, pm = 0;
        for (int k = k0; k < k1; ++k) {
            if (NEAR && sid[k] == j) continue;
            const VjpMember<R> q = si[k];
            R gd[3], gmj;
            pair_grad<R, NEAR>(xj - q.x, yj - q.y, zj - q.z, mj, q.wx, q.wy, q.wz, q.c, vp, gd,
                               gmj);
            p0 += gd[0]; p1 += gd[1]; p2 += gd[2]; pm += gmj;
        }
        acc[0] += (double)p0; acc[1] += (double)p1; acc[2] += (double)p2; acc[3] += (double)pm;
    }
}

template <class R, bool CELL_K, bool QUAD>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_scatter(
    const GroupInfo *__restrict__ grp, ListsDev L, const PosMass *__restrict__ xm,
    const NodeMP *__restrict__ mp,
    const int32_t *__restrict__ perm, const double *__restrict__ wv, const double *__restrict__ cv,
    VjpParams vp, double *__restrict__ gx, double *__restrict__ gm, double *__restrict__ cadj,
    int64_t n, int64_t n_nodes) {
    __shared__ VjpMember<R> s_i[kVjpThreads];
    __shared__ int32_t s_id[kVjpThreads];
    // per wavefront and member: the member's cell terms dl/dr (FP64 partials)
    __shared__ double s_gr[kVjpThreads / kWave][kVjpThreads][3];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int g = L.order[blockIdx.x];
    const GroupInfo gi = grp[g];
    double sh[3];
    group_shift<R>(gi, sh);
    const int64_t cb = L.beg[0][g], ce = L.end[0][g];
    const int64_t fb = L.beg[1][g], fe = L.end[1][g];
    const int64_t nb = L.beg[2][g], ne = L.end[2][g];
    const int32_t *__restrict__ c_idx = L.idx[0];
    const int32_t *__restrict__ p_idx = L.idx[1];
    const int32_t *__restrict__ n_idx = L.idx[2];
    const int64_t nf = fe - fb, np = nf + (ne - nb);   // far entries first, then near
    for (int chunk = 0; chunk < gi.count; chunk += kVjpThreads) {
        const int nc = min(kVjpThreads, gi.count - chunk);
        __syncthreads();
        if (tid < nc) {
            const int32_t i = gi.first + chunk + tid;
            const int64_t o = perm[i];
            const PosMass pi = xm[i];
            s_i[tid] = VjpMember<R>{(R)(pi.x - sh[0]), (R)(pi.y - sh[1]), (R)(pi.z - sh[2]),
                                    vp.has_c ? (R)cv[o] : R(0), (R)wv[3 * o], (R)wv[3 * o + 1],
                                    (R)wv[3 * o + 2], R(0)};
            s_id[tid] = i;
        }
        __syncthreads();
        for (int k = lane; k < nc; k += kWave) s_gr[w][k][0] = s_gr[w][k][1] = s_gr[w][k][2] = 0.0;
        // far particles (K = W = 1, never a member): a lane per entry, the
        // members from LDS; each pair's term counts for both sides, the
        // members' parts gathered as for the cells below.  Lanes past the end
        // hold a massless particle far away, whose terms are exactly zero.
        for (int64_t e0 = (int64_t)w * kWave; e0 < nf; e0 += kVjpThreads) {
            const bool valid = e0 + lane < nf;
            const int32_t j = valid ? p_idx[fb + e0 + lane] : 0;
            const PosMass pj = xm[j];
            const R xj = valid ? (R)(pj.x - sh[0]) : R(1e18), yj = valid ? (R)(pj.y - sh[1]) : R(1e18),
                    zj = valid ? (R)(pj.z - sh[2]) : R(1e18);
            const R mj = valid ? (R)pj.m : R(0);
            double acc[4] = {0, 0, 0, 0};
            for (int k0 = 0; k0 < nc; k0 += kFold) {
                const int k1 = min(nc, k0 + kFold);
                R p[4] = {0, 0, 0, 0};
                R mg[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int kh = min(k1, k0 + 16 * (h + 1));
                    for (int k = k0 + 16 * h; k < kh; ++k) {
                        const VjpMember<R> q = s_i[k];
                        R gd[3], gmj;
                        pair_grad<R, false>(xj - q.x, yj - q.y, zj - q.z, mj, q.wx, q.wy, q.wz, q.c,
                                            vp, gd, gmj);
                        p[0] += gd[0]; p[1] += gd[1]; p[2] += gd[2]; p[3] += gmj;
                        const bool mine = (lane & 15) == ((k - k0) & 15);
                        for (int a = 0; a < 3; ++a) {
                            const R t = row_sum(gd[a]);
                            mg[h][a] = mine ? t : mg[h][a];
                        }
                    }
                }
                for (int a = 0; a < 4; ++a) acc[a] += (double)p[a];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    for (int a = 0; a < 3; ++a) {
                        R t = mg[h][a];
                        t += __shfl_xor(t, 16, kWave);
                        t += __shfl_xor(t, 32, kWave);
                        mg[h][a] = t;
                    }
                    if (lane < 16 && k0 + 16 * h + lane < k1)   // the member's part: -dl/dd
                        for (int a = 0; a < 3; ++a)
                            s_gr[w][k0 + 16 * h + lane][a] -= (double)mg[h][a];
                }
            }
            if (valid) {
                atomicAdd(&gx[j], acc[0]);
                atomicAdd(&gx[n + j], acc[1]);
                atomicAdd(&gx[2 * n + j], acc[2]);
                atomicAdd(&gm[j], acc[3]);
            }
        }
        // near particles (the list may hold a member): a lane per entry, this
        // side only
        for (int64_t e = nf + tid; e < np; e += kVjpThreads) {
            const int32_t j = n_idx[nb + (e - nf)];
            const PosMass pj = xm[j];
            const R xj = (R)(pj.x - sh[0]), yj = (R)(pj.y - sh[1]), zj = (R)(pj.z - sh[2]);
            const R mj = (R)pj.m;
            double acc[4] = {0, 0, 0, 0};
            vjp_scatter_pp<R, true>(s_i, s_id, nc, j, xj, yj, zj, mj, vp, acc);
            atomicAdd(&gx[j], acc[0]);
            atomicAdd(&gx[n + j], acc[1]);
            atomicAdd(&gx[2 * n + j], acc[2]);
            atomicAdd(&gm[j], acc[3]);
        }
        // cells: a lane per entry, the members from LDS.  Each pair's dl/dr
        // counts for both sides: the cell's sums stay in the lane; the
        // member's are summed over each row of 16 entries (a fixed tree) and
        // parked in the row's lane (k - k0) mod 16 of mg[half] for the run of
        // members k0 .. k1 - 1; after the run a butterfly over the four rows
        // completes each member's sum, which joins the wavefront's FP64
        // partials in s_gr.  Lanes past the end hold a massless cell far away
        // and add zero.
        const int64_t ncell = ce - cb;
        for (int64_t e0 = (int64_t)w * kWave; e0 < ncell; e0 += kVjpThreads) {
            const bool valid = e0 + lane < ncell;
            const int32_t cid = valid ? c_idx[cb + e0 + lane] : 0;
            VjpCell<R> c = stage_cell<R>(mp[cid], sh);
            if (!valid) {
                c.x = c.y = c.z = R(1e18);
                c.M = R(0);
                for (int a = 0; a < 6; ++a) c.q[a] = R(0);
            }
            double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int k0 = 0; k0 < nc; k0 += kFold) {
                const int k1 = min(nc, k0 + kFold);
                R p[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                R mg[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int kh = min(k1, k0 + 16 * (h + 1));
                    for (int k = k0 + 16 * h; k < kh; ++k) {
                        const VjpMember<R> q = s_i[k];
                        R gr[3], gM, S[6];
                        if (CELL_K) {
                            CellGrad<R> cg;
                            cell_grad<R, true, QUAD>(q.x - c.x, q.y - c.y, q.z - c.z, c.M, c.q,
                                                     q.wx, q.wy, q.wz, q.c, vp, cg);
                            for (int a = 0; a < 3; ++a) gr[a] = cg.gr[a];
                            gM = cg.gM;
                            for (int a = 0; a < 6; ++a) S[a] = cg.S[a];
                        } else {
                            cell_grad_far<R, QUAD>(q.x - c.x, q.y - c.y, q.z - c.z, c.M, c.q, q.wx,
                                                   q.wy, q.wz, q.c, (R)vp.eps2, gr, gM, S);
                        }
                        p[0] -= gr[0]; p[1] -= gr[1]; p[2] -= gr[2];
                        p[3] += gM;
                        if (QUAD)
                            for (int a = 0; a < 6; ++a) p[4 + a] += S[a];
                        // (a massless padding cell gives dl/dr = 0 exactly)
                        const bool mine = (lane & 15) == ((k - k0) & 15);
                        for (int a = 0; a < 3; ++a) {
                            const R t = row_sum(gr[a]);
                            mg[h][a] = mine ? t : mg[h][a];
                        }
                    }
                }
                for (int a = 0; a < 10; ++a) acc[a] += (double)p[a];
                // the four rows' parts of each member's sum: lane j of row 0
                // then holds member k0 + 16 h + j's
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    for (int a = 0; a < 3; ++a) {
                        R t = mg[h][a];
                        t += __shfl_xor(t, 16, kWave);
                        t += __shfl_xor(t, 32, kWave);
                        mg[h][a] = t;
                    }
                    if (lane < 16 && k0 + 16 * h + lane < k1)
                        for (int a = 0; a < 3; ++a)
                            s_gr[w][k0 + 16 * h + lane][a] += (double)mg[h][a];
                }
            }
            if (valid)
                for (int a = 0; a < 10; ++a)
                    if (acc[a] != 0.0) atomicAdd(&cadj[a * n_nodes + cid], acc[a]);
        }
        __syncthreads();
        // the members' cell terms, wavefront partials in a fixed order (another
        // group may be adding to the same particle as a list entry)
        if (tid < nc) {
            const int32_t i = s_id[tid];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double r = 0.0;
                for (int v = 0; v < kVjpThreads / kWave; ++v) r += s_gr[v][tid][a];
                atomicAdd(&gx[a * n + i], r);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 3: per leaf, sum the quadratic forms of its ancestors (re-centred at
// each child's centre of mass) and apply them to the leaf's members.
// ---------------------------------------------------------------------------
struct Form {
    double B[6];     // symmetric xx yy zz xy xz yz
    double b[3];
    double g;
};

// adj: component a at adj[a * stride]
__device__ __forceinline__ void form_add_own(Form &f, const double *adj, int64_t stride, double M) {
    double v[10];
    for (int a = 0; a < 10; ++a) v[a] = adj[a * stride];
    const double tr = v[4] + v[5] + v[6];
    f.B[0] += 3.0 * v[4] - tr;
    f.B[1] += 3.0 * v[5] - tr;
    f.B[2] += 3.0 * v[6] - tr;
    f.B[3] += 3.0 * v[7];
    f.B[4] += 3.0 * v[8];
    f.B[5] += 3.0 * v[9];
    f.b[0] += v[0] / M;
    f.b[1] += v[1] / M;
    f.b[2] += v[2] / M;
    f.g += v[3];
}

__device__ __forceinline__ void Bmul(const double B[6], const double v[3], double o[3]) {
    o[0] = B[0] * v[0] + B[3] * v[1] + B[4] * v[2];
    o[1] = B[3] * v[0] + B[1] * v[1] + B[5] * v[2];
    o[2] = B[4] * v[0] + B[5] * v[1] + B[2] * v[2];
}

// re-centre f from point p to point p + e
__device__ __forceinline__ void form_shift(Form &f, const double e[3]) {
    double Be[3];
    Bmul(f.B, e, Be);
    f.g += e[0] * Be[0] + e[1] * Be[1] + e[2] * Be[2] + f.b[0] * e[0] + f.b[1] * e[1] + f.b[2] * e[2];
    for (int a = 0; a < 3; ++a) f.b[a] += 2.0 * Be[a];
}

__global__ void k_vjp_down(int64_t n_nodes, const int32_t *__restrict__ nchild,
                           const int32_t *__restrict__ parent, const NodeMP *__restrict__ mp,
                           const NodeWalk *__restrict__ nw, const double *__restrict__ cadj,
                           const PosMass *__restrict__ xm,
                           double *__restrict__ gx, double *__restrict__ gm, int64_t n) {
    const int64_t leaf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= n_nodes || nchild[leaf] != 0) return;
    int32_t chain[kLevels + 1];
    int depth = 0;
    for (int32_t c = (int32_t)leaf; c >= 0 && depth <= kLevels; c = parent[c]) chain[depth++] = c;
    Form f{};
    for (int k = depth - 1; k >= 0; --k) {
        const int32_t c = chain[k];
        if (k < depth - 1) {
            const int32_t p = chain[k + 1];
            const double e[3] = {mp[c].cx - mp[p].cx, mp[c].cy - mp[p].cy, mp[c].cz - mp[p].cz};
            form_shift(f, e);
        }
        form_add_own(f, cadj + c, n_nodes, mp[c].M);
    }
    const double cx = mp[leaf].cx, cy = mp[leaf].cy, cz = mp[leaf].cz;
    const int32_t first = nw[leaf].first, cnt = nw[leaf].count;
    for (int32_t k = first; k < first + cnt; ++k) {
        const PosMass pk = xm[k];
        const double d[3] = {pk.x - cx, pk.y - cy, pk.z - cz};
        double Bd[3];
        Bmul(f.B, d, Bd);
        gm[k] += d[0] * Bd[0] + d[1] * Bd[1] + d[2] * Bd[2] + f.b[0] * d[0] + f.b[1] * d[1] +
                 f.b[2] * d[2] + f.g;
        const double mk = pk.m;
        gx[k] += mk * (2.0 * Bd[0] + f.b[0]);
        gx[n + k] += mk * (2.0 * Bd[1] + f.b[1]);
        gx[2 * n + k] += mk * (2.0 * Bd[2] + f.b[2]);
    }
}

__global__ void k_vjp_unpermute(int64_t n, const int32_t *__restrict__ perm,
                                const double *__restrict__ gx, const double *__restrict__ gm,
                                double *__restrict__ gpos, double *__restrict__ gmass) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = perm[s];
    gpos[3 * o] = gx[s];
    gpos[3 * o + 1] = gx[n + s];
    gpos[3 * o + 2] = gx[2 * n + s];
    gmass[o] = gm[s];
}

__global__ void k_vjp_zero(int64_t count, double *__restrict__ a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) a[k] = 0.0;
}

int launch_vjp(p3t_ctx *ctx, const double *w, const double *c, double *gpos, double *gmass) {
    int rc;
    const int64_t n = ctx->n, nn = ctx->n_nodes;
    if ((rc = ensure(ctx, ctx->vjp_gx, 3 * n * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->vjp_gm, n * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->vjp_cell, 10 * nn * sizeof(double)))) return rc;
    return launch_vjp_ws(ctx, w, c, gpos, gmass, ptr<double>(ctx->vjp_gx), ptr<double>(ctx->vjp_gm),
                         ptr<double>(ctx->vjp_cell));
}

int launch_vjp_ws(p3t_ctx *ctx, const double *w, const double *c, double *gpos, double *gmass,
                  double *gx, double *gm, double *cadj) {
    int rc;
    const int64_t n = ctx->n, nn = ctx->n_nodes;
    VjpParams vp{};
    vp.eps2 = ctx->prm.eps * ctx->prm.eps;
    vp.rout2 = ctx->prm.r_out * ctx->prm.r_out;
    vp.inv_rout = 1.0 / ctx->prm.r_out;
    vp.gamma = ctx->chg.gamma;
    vp.inv_1mg = ctx->chg.inv_1mg;
    vp.C = ctx->chg.C;
    for (int k = 0; k < 7; ++k) vp.w[k] = ctx->chg.w[k];
    vp.wl = ctx->chg.wl;
    vp.wm = ctx->chg.wm;
    vp.use_quad = ctx->prm.use_quadrupole ? 1 : 0;
    vp.has_c = c != nullptr;
    const ListsDev L = lists_dev(ctx);
    // the cell adjoints are accumulated: clear them (a fill kernel, which a
    // caller's graph capture records as an ordinary kernel node)
    k_vjp_zero<<<blocks_for(10 * nn, 256), 256, 0, ctx->stream>>>(10 * nn, cadj);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp clear"))) return rc;
    const unsigned G = (unsigned)ctx->n_groups;
    // accepted cells lie at least h from every member: K = W = 1 on them when h >= r_out
    const bool cell_k = ctx->prm.r_search < ctx->prm.r_out;
    // the adjoint terms follow the forward pass's precision
    const bool mixed = ctx->prm.precision == P3T_PREC_MIXED;
    auto ki = mixed ? k_vjp_i<float> : k_vjp_i<double>;
    const bool quad = vp.use_quad != 0;
    auto ks = mixed ? (cell_k ? (quad ? k_vjp_scatter<float, true, true>
                                      : k_vjp_scatter<float, true, false>)
                              : (quad ? k_vjp_scatter<float, false, true>
                                      : k_vjp_scatter<float, false, false>))
                    : (cell_k ? (quad ? k_vjp_scatter<double, true, true>
                                      : k_vjp_scatter<double, true, false>)
                              : (quad ? k_vjp_scatter<double, false, true>
                                      : k_vjp_scatter<double, false, false>));
    ki<<<G, kVjpThreads, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), L, ptr<PosMass>(ctx->xm), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), w, c, vp, gx, gm,
        n);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp i-side"))) return rc;
    ks<<<G, kVjpThreads, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), L, ptr<PosMass>(ctx->xm), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), w, c, vp, gx, gm,
        cadj, n, nn);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp scatter"))) return rc;
    k_vjp_down<<<blocks_for(nn, 128), 128, 0, ctx->stream>>>(
        nn, ptr<int32_t>(ctx->node_nchild), ptr<int32_t>(ctx->node_parent), ptr<NodeMP>(ctx->node_mp),
        ptr<NodeWalk>(ctx->node_walk), cadj, ptr<PosMass>(ctx->xm), gx, gm, n);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp push-down"))) return rc;
    k_vjp_unpermute<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ptr<int32_t>(ctx->vals[0]), gx,
                                                                 gm, gpos, gmass);
    return check_hip(ctx, hipGetLastError(), "vjp unpermute");
}

}  // namespace p3t
