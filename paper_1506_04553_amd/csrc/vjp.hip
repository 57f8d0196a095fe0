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
// Everything is FP64.  Scatter to list entries uses FP64 atomic adds, one per
// (group, entry, component) after reduction over the group's members, so the
// result is reproducible up to the order of those atomic additions.
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

// d(l_ij)/dd and d(l_ij)/dm_j for one pair; CHG false: K = W = 1 known.
template <bool CHG>
__device__ __forceinline__ void pair_grad(double dx, double dy, double dz, double mj, double wx,
                                          double wy, double wz, double ci, const VjpParams &vp,
                                          double gd[3], double &gm) {
    const double s2 = dx * dx + dy * dy + dz * dz + vp.eps2;
    const double inv = rsqrt(s2);
    const double s = s2 * inv;
    const double inv2 = inv * inv, inv3 = inv2 * inv;
    const Chg c = CHG ? changeover_ds(s, vp) : changeover_unit();
    const double g = c.K * inv3;
    const double gp = c.Ks * inv3 - 3.0 * c.K * inv2 * inv2;
    const double wd = wx * dx + wy * dy + wz * dz;
    const double t = gp * wd * inv + ci * c.K * inv3;
    gd[0] = mj * (g * wx + t * dx);
    gd[1] = mj * (g * wy + t * dy);
    gd[2] = mj * (g * wz + t * dz);
    gm = g * wd - ci * c.W * inv;
}

struct CellGrad {
    double gr[3];    // dl/dr (r = x_i - com)
    double gM;       // dl/dM
    double S[6];     // symmetric dl/dQ: xx yy zz xy xz yz
};

template <bool CHG>
__device__ __forceinline__ void cell_grad(double rx, double ry, double rz, double M, const double q[6],
                                          double wx, double wy, double wz, double ci,
                                          const VjpParams &vp, CellGrad &o) {
    const double s2 = rx * rx + ry * ry + rz * rz + vp.eps2;
    const double inv = rsqrt(s2);
    const double s = s2 * inv;
    const double inv2 = inv * inv, inv3 = inv2 * inv, inv5 = inv3 * inv2, inv7 = inv5 * inv2,
                 inv9 = inv7 * inv2;
    const Chg c = CHG ? changeover_ds(s, vp) : changeover_unit();
    double Qr[3] = {0, 0, 0}, Qw[3] = {0, 0, 0}, qq = 0.0;
    if (vp.use_quad) {
        Qr[0] = q[0] * rx + q[3] * ry + q[4] * rz;
        Qr[1] = q[3] * rx + q[1] * ry + q[5] * rz;
        Qr[2] = q[4] * rx + q[5] * ry + q[2] * rz;
        Qw[0] = q[0] * wx + q[3] * wy + q[4] * wz;
        Qw[1] = q[3] * wx + q[1] * wy + q[5] * wz;
        Qw[2] = q[4] * wx + q[5] * wy + q[2] * wz;
        qq = rx * Qr[0] + ry * Qr[1] + rz * Qr[2];
    }
    const double r[3] = {rx, ry, rz}, w[3] = {wx, wy, wz};
    const double rw = rx * wx + ry * wy + rz * wz;
    const double Qrw = Qr[0] * wx + Qr[1] * wy + Qr[2] * wz;
    double A[3], Hw[3];
    const double cw = M * inv3 + 2.5 * qq * inv7;
    const double cr = -3.0 * M * rw * inv5 + 5.0 * Qrw * inv7 - 17.5 * qq * rw * inv9;
    const double cq = 5.0 * rw * inv7;
    for (int a = 0; a < 3; ++a) {
        A[a] = -M * r[a] * inv3 + Qr[a] * inv5 - 2.5 * qq * r[a] * inv7;
        Hw[a] = w[a] * cw - Qw[a] * inv5 + r[a] * cr + Qr[a] * cq;
    }
    const double Phi = -M * inv - 0.5 * qq * inv5;
    const double wA = wx * A[0] + wy * A[1] + wz * A[2];
    const double radial = (c.Ks * wA + ci * c.Ws * Phi) * inv;
    for (int a = 0; a < 3; ++a) o.gr[a] = radial * r[a] - c.K * Hw[a] - ci * c.W * A[a];
    o.gM = -c.K * rw * inv3 - ci * c.W * inv;
    if (vp.use_quad) {
        const double k5 = 0.5 * c.K * inv5, k7 = -2.5 * c.K * rw * inv7, cwq = -0.5 * ci * c.W * inv5;
        const double rr = k7 + cwq;
        o.S[0] = 2.0 * k5 * wx * rx + rr * rx * rx;
        o.S[1] = 2.0 * k5 * wy * ry + rr * ry * ry;
        o.S[2] = 2.0 * k5 * wz * rz + rr * rz * rz;
        o.S[3] = k5 * (wx * ry + wy * rx) + rr * rx * ry;
        o.S[4] = k5 * (wx * rz + wz * rx) + rr * rx * rz;
        o.S[5] = k5 * (wy * rz + wz * ry) + rr * ry * rz;
    } else {
        for (int a = 0; a < 6; ++a) o.S[a] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Pass 1: per particle i (one group per block), the i-side terms.
// ---------------------------------------------------------------------------
// CELL_K: accepted cells may lie within r_out of a member (h < r_out)
template <bool CELL_K>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_i(
    const GroupInfo *__restrict__ grp, ListsDev L, const double *__restrict__ x,
    const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ m, const NodeMP *__restrict__ mp,
    const int32_t *__restrict__ perm, const double *__restrict__ wv, const double *__restrict__ cv,
    VjpParams vp, double *__restrict__ gx, double *__restrict__ gm, int64_t n) {
    __shared__ double s_p[4][kVjpTile];
    __shared__ int32_t s_j[kVjpTile];
    __shared__ NodeMP s_c[kVjpTile];
    __shared__ double s_red[3][kVjpThreads];
    const int tid = threadIdx.x;
    const int g = L.order[blockIdx.x];
    const GroupInfo gi = grp[g];
    const int64_t cb = L.beg[0][g], ce = L.end[0][g];
    const int32_t *__restrict__ c_idx = L.idx[0];
    // members in chunks of the largest power of two that fits (at most 256),
    // so that a chunk fills its lanes: 74 members run as 64 + 8 + 2
    for (int chunk = 0, nc = 0; chunk < gi.count; chunk += nc) {
        const int rem = gi.count - chunk;
        int lg = 0;
        while (lg < 8 && (2 << lg) <= rem) ++lg;
        nc = 1 << lg;
        const int pad = nc, nslice = kVjpThreads >> lg;
        const int li = tid & (pad - 1), slice = tid >> lg;
        const bool valid = li < nc;
        const int32_t i = gi.first + chunk + (valid ? li : 0);
        const int64_t o = perm[i];
        const double xi = x[i], yi = y[i], zi = z[i];
        const double wx = wv[3 * o], wy = wv[3 * o + 1], wz = wv[3 * o + 2];
        const double ci = vp.has_c ? cv[o] : 0.0;
        double g0 = 0, g1 = 0, g2 = 0;
        for (int list = 0; list < 2; ++list) {        // far and near particles
            const int32_t *idxs = L.idx[1 + list];
            const int64_t pb = L.beg[1 + list][g];
            const int64_t pe = L.end[1 + list][g];
            for (int64_t t0 = pb; t0 < pe; t0 += kVjpTile) {
                const int tl = (int)min<int64_t>(kVjpTile, pe - t0);
                __syncthreads();
                if (tid < tl) {
                    const int32_t j = idxs[t0 + tid];
                    s_p[0][tid] = x[j]; s_p[1][tid] = y[j]; s_p[2][tid] = z[j]; s_p[3][tid] = m[j];
                    s_j[tid] = j;
                }
                __syncthreads();
                for (int k = slice; k < tl; k += nslice) {
                    if (s_j[k] == i) continue;
                    double gd[3], gmj;
                    if (list == 0)   // far particles: K = W = 1
                        pair_grad<false>(s_p[0][k] - xi, s_p[1][k] - yi, s_p[2][k] - zi, s_p[3][k],
                                         wx, wy, wz, ci, vp, gd, gmj);
                    else
                        pair_grad<true>(s_p[0][k] - xi, s_p[1][k] - yi, s_p[2][k] - zi, s_p[3][k],
                                        wx, wy, wz, ci, vp, gd, gmj);
                    g0 -= gd[0]; g1 -= gd[1]; g2 -= gd[2];
                }
            }
        }
        for (int64_t t0 = cb; t0 < ce; t0 += kVjpTile) {
            const int tl = (int)min<int64_t>(kVjpTile, ce - t0);
            __syncthreads();
            if (tid < tl) s_c[tid] = mp[c_idx[t0 + tid]];
            __syncthreads();
            for (int k = slice; k < tl; k += nslice) {
                const NodeMP c = s_c[k];
                CellGrad cg;
                cell_grad<CELL_K>(xi - c.cx, yi - c.cy, zi - c.cz, c.M, c.q, wx, wy, wz, ci, vp, cg);
                g0 += cg.gr[0]; g1 += cg.gr[1]; g2 += cg.gr[2];
            }
        }
        __syncthreads();
        s_red[0][tid] = g0; s_red[1][tid] = g1; s_red[2][tid] = g2;
        __syncthreads();
        if (slice == 0 && valid) {
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
// members, scattered with one atomic add per component.
// ---------------------------------------------------------------------------
template <bool CELL_K>
__global__ __launch_bounds__(kVjpThreads) void k_vjp_scatter(
    const GroupInfo *__restrict__ grp, ListsDev L, const double *__restrict__ x,
    const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ m, const NodeMP *__restrict__ mp,
    const int32_t *__restrict__ perm, const double *__restrict__ wv, const double *__restrict__ cv,
    VjpParams vp, double *__restrict__ gx, double *__restrict__ gm, double *__restrict__ cadj,
    int64_t n) {
    __shared__ double s_i[7][kVjpThreads];   // x y z w(3) c of the group's members
    __shared__ int32_t s_id[kVjpThreads];
    const int tid = threadIdx.x;
    const int g = L.order[blockIdx.x];
    const GroupInfo gi = grp[g];
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
            s_i[0][tid] = x[i]; s_i[1][tid] = y[i]; s_i[2][tid] = z[i];
            s_i[3][tid] = wv[3 * o]; s_i[4][tid] = wv[3 * o + 1]; s_i[5][tid] = wv[3 * o + 2];
            s_i[6][tid] = vp.has_c ? cv[o] : 0.0;
            s_id[tid] = i;
        }
        __syncthreads();
        for (int64_t e = tid; e < np; e += kVjpThreads) {
            const bool far = e < nf;
            const int32_t j = far ? p_idx[fb + e] : n_idx[nb + (e - nf)];
            const double xj = x[j], yj = y[j], zj = z[j], mj = m[j];
            double a0 = 0, a1 = 0, a2 = 0, am = 0;
            for (int k = 0; k < nc; ++k) {
                if (s_id[k] == j) continue;
                double gd[3], gmj;
                if (far)   // K = W = 1
                    pair_grad<false>(xj - s_i[0][k], yj - s_i[1][k], zj - s_i[2][k], mj, s_i[3][k],
                                     s_i[4][k], s_i[5][k], s_i[6][k], vp, gd, gmj);
                else
                    pair_grad<true>(xj - s_i[0][k], yj - s_i[1][k], zj - s_i[2][k], mj, s_i[3][k],
                                    s_i[4][k], s_i[5][k], s_i[6][k], vp, gd, gmj);
                a0 += gd[0]; a1 += gd[1]; a2 += gd[2]; am += gmj;
            }
            atomicAdd(&gx[j], a0);
            atomicAdd(&gx[n + j], a1);
            atomicAdd(&gx[2 * n + j], a2);
            atomicAdd(&gm[j], am);
        }
        for (int64_t e = cb + tid; e < ce; e += kVjpThreads) {
            const int32_t cid = c_idx[e];
            const NodeMP c = mp[cid];
            double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int k = 0; k < nc; ++k) {
                CellGrad cg;
                cell_grad<CELL_K>(s_i[0][k] - c.cx, s_i[1][k] - c.cy, s_i[2][k] - c.cz, c.M, c.q, s_i[3][k],
                          s_i[4][k], s_i[5][k], s_i[6][k], vp, cg);
                acc[0] -= cg.gr[0]; acc[1] -= cg.gr[1]; acc[2] -= cg.gr[2];
                acc[3] += cg.gM;
                for (int a = 0; a < 6; ++a) acc[4 + a] += cg.S[a];
            }
            double *dst = cadj + 10 * (int64_t)cid;
            for (int a = 0; a < 10; ++a)
                if (acc[a] != 0.0) atomicAdd(&dst[a], acc[a]);
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

__device__ __forceinline__ void form_add_own(Form &f, const double *adj, double M) {
    const double tr = adj[4] + adj[5] + adj[6];
    f.B[0] += 3.0 * adj[4] - tr;
    f.B[1] += 3.0 * adj[5] - tr;
    f.B[2] += 3.0 * adj[6] - tr;
    f.B[3] += 3.0 * adj[7];
    f.B[4] += 3.0 * adj[8];
    f.B[5] += 3.0 * adj[9];
    f.b[0] += adj[0] / M;
    f.b[1] += adj[1] / M;
    f.b[2] += adj[2] / M;
    f.g += adj[3];
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
                           const double *__restrict__ x, const double *__restrict__ y,
                           const double *__restrict__ z, const double *__restrict__ m,
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
        form_add_own(f, cadj + 10 * (int64_t)c, mp[c].M);
    }
    const double cx = mp[leaf].cx, cy = mp[leaf].cy, cz = mp[leaf].cz;
    const int32_t first = nw[leaf].first, cnt = nw[leaf].count;
    for (int32_t k = first; k < first + cnt; ++k) {
        const double d[3] = {x[k] - cx, y[k] - cy, z[k] - cz};
        double Bd[3];
        Bmul(f.B, d, Bd);
        gm[k] += d[0] * Bd[0] + d[1] * Bd[1] + d[2] * Bd[2] + f.b[0] * d[0] + f.b[1] * d[1] +
                 f.b[2] * d[2] + f.g;
        const double mk = m[k];
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

int launch_vjp(p3t_ctx *ctx, const double *w, const double *c, double *gpos, double *gmass) {
    int rc;
    const int64_t n = ctx->n, nn = ctx->n_nodes;
    if ((rc = ensure(ctx, ctx->vjp_gx, 3 * n * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->vjp_gm, n * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->vjp_cell, 10 * nn * sizeof(double)))) return rc;
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
    double *gx = ptr<double>(ctx->vjp_gx), *gm = ptr<double>(ctx->vjp_gm);
    double *cadj = ptr<double>(ctx->vjp_cell);
    const ListsDev L = lists_dev(ctx);
    if ((rc = check_hip(ctx, hipMemsetAsync(cadj, 0, 10 * nn * sizeof(double), ctx->stream), "memset")))
        return rc;
    const unsigned G = (unsigned)ctx->n_groups;
    // accepted cells lie at least h from every member: K = W = 1 on them when h >= r_out
    const bool cell_k = ctx->prm.r_search < ctx->prm.r_out;
    auto ki = cell_k ? k_vjp_i<true> : k_vjp_i<false>;
    auto ks = cell_k ? k_vjp_scatter<true> : k_vjp_scatter<false>;
    ki<<<G, kVjpThreads, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), L, ptr<double>(ctx->x), ptr<double>(ctx->y), ptr<double>(ctx->z),
        ptr<double>(ctx->m), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), w, c, vp, gx, gm,
        n);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp i-side"))) return rc;
    ks<<<G, kVjpThreads, 0, ctx->stream>>>(
        ptr<GroupInfo>(ctx->grp), L, ptr<double>(ctx->x), ptr<double>(ctx->y), ptr<double>(ctx->z),
        ptr<double>(ctx->m), ptr<NodeMP>(ctx->node_mp), ptr<int32_t>(ctx->vals[0]), w, c, vp, gx, gm,
        cadj, n);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp scatter"))) return rc;
    k_vjp_down<<<blocks_for(nn, 128), 128, 0, ctx->stream>>>(
        nn, ptr<int32_t>(ctx->node_nchild), ptr<int32_t>(ctx->node_parent), ptr<NodeMP>(ctx->node_mp),
        ptr<NodeWalk>(ctx->node_walk), cadj, ptr<double>(ctx->x), ptr<double>(ctx->y),
        ptr<double>(ctx->z), ptr<double>(ctx->m), gx, gm, n);
    if ((rc = check_hip(ctx, hipGetLastError(), "vjp push-down"))) return rc;
    k_vjp_unpermute<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ptr<int32_t>(ctx->vals[0]), gx,
                                                                 gm, gpos, gmass);
    return check_hip(ctx, hipGetLastError(), "vjp unpermute");
}

}  // namespace p3t
