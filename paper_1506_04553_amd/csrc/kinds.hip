// kinds.hip -- particle kinds for the SMBH runs (Section 3.2.2): the last
// n_special particles of the arrays are special; a pair of a normal and a
// special particle takes its own cutoff radii, softening and neighbour radius,
// and a pair of two special particles its own softening and, when it is not
// split, no soft part at all (the pair is integrated wholly by Hermite).
//
// The tree and its lists cover the normal particles only.  Here:
//   * the soft force and potential of every pair that involves a special
//     particle (O(N n_special) direct sums): added to the normal particles'
//     rows, written to the special particles' rows;
//   * the neighbour lists of all particles: a normal particle's tree row
//     followed by the special particles within the normal-special radius; a
//     special particle's row by the normal particles within that radius and
//     the other special particles (all of them when their pair is not split),
//     every row ascending.
// Special particles are few (the paper uses two), so one block per special
// particle sweeps the normal particles.
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kKindThreads = 256;

// constants of one kind of pair for the soft sums
struct SoftPair {
    double eps2, inv_rout, gamma, inv_1mg, C_over_rout;
    double w[7];
    double wl, wm;
    int split;
};

struct KindsConsts {
    SoftPair ns, ss;
    int64_t first_sp, n;
};

static SoftPair soft_pair(double eps, double r_in, double r_out, int split) {
    SoftPair q{};
    q.eps2 = eps * eps;
    q.split = split;
    if (!split) return q;
    const Changeover c = make_changeover(r_in, r_out);
    q.inv_rout = c.inv_rout;
    q.gamma = c.gamma;
    q.inv_1mg = c.inv_1mg;
    q.C_over_rout = c.C * c.inv_rout;
    for (int k = 0; k < 7; ++k) q.w[k] = c.w[k];
    q.wl = c.wl;
    q.wm = c.wm;
    return q;
}

// soft pull of j on i: a += m_j K d / s^3, phi -= m_j W / s (FP64)
__device__ inline void soft_pull(const double *xi, const double *xj, double mj, const SoftPair &q,
                                 double a[3], double &ph) {
    if (!q.split) return;
    const double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
    const double s2 = dx * dx + dy * dy + dz * dz + q.eps2;
    const double s = sqrt(s2);
    const double y = s * q.inv_rout;
    double K, Ws;
    if (y >= 1.0) {
        K = 1.0;
        Ws = 1.0 / s;
    } else if (y < q.gamma) {
        K = 0.0;
        Ws = q.C_over_rout;
    } else {
        const double x = (y - q.gamma) * q.inv_1mg;
        const double x2 = x * x;
        K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
        double p = q.w[6];
        for (int k = 5; k >= 0; --k) p = p * y + q.w[k];
        Ws = (p + q.wl * log(y) + q.wm / y) * q.inv_rout;
    }
    const double f = mj * K / (s2 * s);
    a[0] += f * dx;
    a[1] += f * dy;
    a[2] += f * dz;
    ph -= mj * Ws;
}

// normal particles: add the pulls of the special particles
__global__ __launch_bounds__(kKindThreads) void k_kinds_soft_normal(
    const double *__restrict__ pos, const double *__restrict__ mass, KindsConsts kc,
    double *__restrict__ acc, double *__restrict__ pot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.first_sp) return;
    double a[3] = {0.0, 0.0, 0.0}, ph = 0.0;
    for (int64_t b = kc.first_sp; b < kc.n; ++b) soft_pull(pos + 3 * i, pos + 3 * b, mass[b], kc.ns, a, ph);
    for (int q = 0; q < 3; ++q) acc[3 * i + q] += a[q];
    if (pot) pot[i] += ph;
}

// special particle first_sp + blockIdx.x: the pulls of every other particle
__global__ __launch_bounds__(kKindThreads) void k_kinds_soft_special(
    const double *__restrict__ pos, const double *__restrict__ mass, KindsConsts kc,
    double *__restrict__ acc, double *__restrict__ pot) {
    __shared__ double s_r[4][kKindThreads];
    const int64_t b = kc.first_sp + blockIdx.x;
    double a[3] = {0.0, 0.0, 0.0}, ph = 0.0;
    for (int64_t j = threadIdx.x; j < kc.n; j += kKindThreads) {
        if (j == b) continue;
        soft_pull(pos + 3 * b, pos + 3 * j, mass[j], j >= kc.first_sp ? kc.ss : kc.ns, a, ph);
    }
    s_r[0][threadIdx.x] = a[0];
    s_r[1][threadIdx.x] = a[1];
    s_r[2][threadIdx.x] = a[2];
    s_r[3][threadIdx.x] = ph;
    __syncthreads();
    for (int w = kKindThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) s_r[q][threadIdx.x] += s_r[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q) acc[3 * b + q] = s_r[q][0];
        if (pot) pot[b] = s_r[3][0];
    }
}

// ---------------------------------------------------------------------------
// Neighbour lists with a radius per kind of pair.
// ---------------------------------------------------------------------------
struct KindsNbr {
    double h2_ns, h2_ss;
    int split_ss;
    int64_t first_sp, n;
};

__device__ inline bool within(const double *xi, const double *xj, double h2) {
    const double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
    return dx * dx + dy * dy + dz * dz < h2;
}

// the special particles on special particle b's row
__device__ inline bool ss_listed(const double *pos, int64_t b, int64_t c, const KindsNbr &kn) {
    return c != b && (!kn.split_ss || within(pos + 3 * b, pos + 3 * c, kn.h2_ss));
}

__global__ __launch_bounds__(kKindThreads) void k_kn_count_normal(
    const double *__restrict__ pos, const int64_t *__restrict__ nn_off, KindsNbr kn,
    int64_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kn.first_sp) return;
    int64_t c = nn_off[i + 1] - nn_off[i];
    for (int64_t b = kn.first_sp; b < kn.n; ++b) c += within(pos + 3 * i, pos + 3 * b, kn.h2_ns);
    cnt[i] = c;
}

__global__ __launch_bounds__(kKindThreads) void k_kn_count_special(const double *__restrict__ pos,
                                                                   KindsNbr kn,
                                                                   int64_t *__restrict__ cnt) {
    __shared__ int64_t s_c[kKindThreads];
    const int64_t b = kn.first_sp + blockIdx.x;
    int64_t c = 0;
    for (int64_t j = threadIdx.x; j < kn.first_sp; j += kKindThreads)
        c += within(pos + 3 * b, pos + 3 * j, kn.h2_ns);
    for (int64_t j = kn.first_sp + threadIdx.x; j < kn.n; j += kKindThreads) c += ss_listed(pos, b, j, kn);
    s_c[threadIdx.x] = c;
    __syncthreads();
    for (int w = kKindThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_c[threadIdx.x] += s_c[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[b] = s_c[0];
}

__global__ __launch_bounds__(kKindThreads) void k_kn_fill_normal(
    const double *__restrict__ pos, const int64_t *__restrict__ nn_off,
    const int32_t *__restrict__ nn_idx, KindsNbr kn, const int64_t *__restrict__ off,
    int32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kn.first_sp) return;
    int64_t o = off[i];
    for (int64_t e = nn_off[i]; e < nn_off[i + 1]; ++e) idx[o++] = nn_idx[e];
    for (int64_t b = kn.first_sp; b < kn.n; ++b)
        if (within(pos + 3 * i, pos + 3 * b, kn.h2_ns)) idx[o++] = (int32_t)b;
}

// special particle b's row, ascending: an ordered compaction of the hits over
// chunks of the block
__global__ __launch_bounds__(kKindThreads) void k_kn_fill_special(const double *__restrict__ pos,
                                                                  KindsNbr kn,
                                                                  const int64_t *__restrict__ off,
                                                                  int32_t *__restrict__ idx) {
    __shared__ int s_scan[kKindThreads];
    const int64_t b = kn.first_sp + blockIdx.x;
    int64_t o = off[b];
    for (int64_t j0 = 0; j0 < kn.n; j0 += kKindThreads) {
        const int64_t j = j0 + threadIdx.x;
        int hit = 0;
        if (j < kn.first_sp) hit = within(pos + 3 * b, pos + 3 * j, kn.h2_ns);
        else if (j < kn.n) hit = ss_listed(pos, b, j, kn);
        s_scan[threadIdx.x] = hit;
        __syncthreads();
        for (int w = 1; w < kKindThreads; w <<= 1) {   // inclusive scan
            const int v = (int)threadIdx.x >= w ? s_scan[threadIdx.x - w] : 0;
            __syncthreads();
            s_scan[threadIdx.x] += v;
            __syncthreads();
        }
        if (hit) idx[o + s_scan[threadIdx.x] - 1] = (int32_t)j;
        o += s_scan[kKindThreads - 1];
        __syncthreads();
    }
}

static KindsConsts kinds_consts(int64_t n, const p3t_kinds *kd) {
    KindsConsts kc;
    kc.ns = soft_pair(kd->eps_ns, kd->r_in_ns, kd->r_out_ns, 1);
    kc.ss = soft_pair(kd->eps_ss, kd->r_in_ss, kd->r_out_ss, kd->split_ss);
    kc.first_sp = n - kd->n_special;
    kc.n = n;
    return kc;
}

int launch_kinds_soft(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                      const p3t_params *p, const p3t_kinds *kd, double *acc, double *pot) {
    (void)p;
    if (!kd || kd->n_special == 0) return P3T_OK;
    const KindsConsts kc = kinds_consts(n, kd);
    if (kc.first_sp > 0)
        k_kinds_soft_normal<<<blocks_for(kc.first_sp, kKindThreads), kKindThreads, 0, ctx->stream>>>(
            pos, mass, kc, acc, pot);
    k_kinds_soft_special<<<(unsigned)kd->n_special, kKindThreads, 0, ctx->stream>>>(pos, mass, kc,
                                                                                  acc, pot);
    return check_hip(ctx, hipGetLastError(), "kinds soft");
}

// readback slot (int64 units) used here: the merged lists' total
enum { RB_KNNZ = 60 };

int launch_kinds_neighbors(p3t_ctx *ctx, int64_t n, const double *pos, const p3t_kinds *kd,
                           const int64_t *nn_off, const int32_t *nn_idx, int64_t *off,
                           int32_t *idx, int64_t cap, int64_t *nnz) {
    int rc;
    hipStream_t st = ctx->stream;
    if ((rc = ensure_readback(ctx))) return rc;
    if ((rc = ensure(ctx, ctx->kinds_cnt, (size_t)(n + 1) * sizeof(int64_t)))) return rc;
    int64_t *cnt = ptr<int64_t>(ctx->kinds_cnt), *rb = ptr<int64_t>(ctx->readback);
    KindsNbr kn;
    kn.h2_ns = kd->r_search_ns * kd->r_search_ns;
    kn.h2_ss = kd->r_search_ss * kd->r_search_ss;
    kn.split_ss = kd->split_ss;
    kn.first_sp = n - kd->n_special;
    kn.n = n;
    if (kn.first_sp > 0)
        k_kn_count_normal<<<blocks_for(kn.first_sp, kKindThreads), kKindThreads, 0, st>>>(
            pos, nn_off, kn, cnt);
    if (kd->n_special > 0)
        k_kn_count_special<<<(unsigned)kd->n_special, kKindThreads, 0, st>>>(pos, kn, cnt);
    if ((rc = check_hip(ctx, hipGetLastError(), "kinds count"))) return rc;
    if ((rc = check_hip(ctx, hipMemsetAsync(cnt + n, 0, sizeof(int64_t), st), "memset"))) return rc;
    if ((rc = scan_exclusive_i64(ctx, cnt, cnt, n + 1, rb + RB_KNNZ))) return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_KNNZ, rb + RB_KNNZ, sizeof(int64_t),
                                            hipMemcpyDeviceToHost, st), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
    const int64_t total = ctx->hpin[RB_KNNZ];
    *nnz = total;
    if (total > cap)
        return set_error(ctx, P3T_ECAPACITY, "neighbour capacity %lld < %lld", (long long)cap,
                         (long long)total);
    if ((rc = check_hip(ctx, hipMemcpyAsync(off, cnt, (size_t)(n + 1) * sizeof(int64_t),
                                            hipMemcpyDeviceToDevice, st), "copy")))
        return rc;
    if (kn.first_sp > 0)
        k_kn_fill_normal<<<blocks_for(kn.first_sp, kKindThreads), kKindThreads, 0, st>>>(
            pos, nn_off, nn_idx, kn, cnt, idx);
    if (kd->n_special > 0)
        k_kn_fill_special<<<(unsigned)kd->n_special, kKindThreads, 0, st>>>(pos, kn, cnt, idx);
    return check_hip(ctx, hipGetLastError(), "kinds fill");
}

}  // namespace p3t
