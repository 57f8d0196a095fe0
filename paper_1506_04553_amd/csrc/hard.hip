// hard.hip -- the hard part of the P3T split (Section 2.1) on the GPU: the
// (1 - K) force, its jerk and the (1 - W) potential over neighbour lists, and
// the fourth-order Hermite integration of H_hard with block timesteps over one
// soft step.
//
// Pair term, d = x_j - x_i, v = v_j - v_i, s^2 = |d|^2 + eps^2, y = s / r_out:
//   a_i   += m_j (1 - K) d / s^3
//   jerk_i += m_j [ (1 - K) (v - 3 (d.v) d / s^2) / s^3 - K'(s) ((d.v)/s) d / s^3 ]
//   phi_i -= m_j (1 - W) / s
// summed over i's list in list order, each quantity by the same IEEE operation
// sequence as the definition (the library builds with contraction off), so the
// force and jerk of a given list are reproducible bit for bit.
//
// Integration.  Particles with an empty list are isolated and drift.  The
// others form clusters: connected components of the neighbour graph.  No force
// crosses a component boundary during the soft step, so every component is
// integrated by one workgroup on its own, with its own block steps, and no
// grid-wide synchronisation is needed.  Per block step of a component:
// t_next = min (t_i + dt_i); every member is predicted to t_next; members with
// t_i + dt_i = t_next are active; their force and jerk are evaluated from the
// predicted states, then they are corrected (Hermite interpolation of the
// second and third derivatives from a and jerk at both ends) and given their
// next timestep:
//   first step  dt <= eta_s sqrt((|a|^2 + a0^2) / |a'|^2)
//   later       dt <= eta sqrt((sqrt(|a|^2 + a0^2) |a''| + |a'|^2) / (|a'| |a'''| + |a''|^2))
// with dt = dt_max / 2^k; the step doubles when twice the step fits, stays
// within dt_max and the particle's time is a multiple of it, else it halves
// until it fits.  A particle's trajectory depends only on its own component,
// so this equals one global block-step loop over all particles.
//
// Components come from a lock-free union-find over the list edges (a root is
// always linked under a smaller root, so every chain decreases and the final
// root of a component is its smallest index), members are gathered into
// contiguous slots, and components are launched largest first.  A component of
// fewer than 1024 members runs from LDS: each thread keeps its members' state
// in registers, the predicted positions and velocities that neighbours read
// live in LDS, and so do the component's list entries as local indices (they
// fall back to a global copy when they outgrow their LDS area).  Three size
// classes (< 64, < 256, < 1024 members) have their own block shapes and run
// concurrently on forked streams; components of 1024 members or more advance
// together on the context stream, one grid-wide launch per phase of a block
// step, so that a large component is spread over the whole device.
#include <math.h>
#include <string.h>

#include <vector>

#include "device_util.h"
#include "internal.h"

namespace p3t {

constexpr int kHardThreads = 256;
constexpr int kGiantThreads = 256;   // grid-wide step kernels for components of >= 1024
constexpr int kGiantBatch = 32;     // block steps launched between host checks
constexpr int kMaxDtLevel = 40;
constexpr int kUnionTries = 1 << 20;

// parameters of one kind of pair: 0 normal-normal, 1 normal-special,
// 2 special-special (the last particles of the arrays may be special)
struct PairKind {
    double eps, r_in, r_out, gam;
    double C, G1;          // W/y below r_in, G(1) of the changeover region
    int split;             // 0: the pair is wholly hard (K = W = 0)
};

struct HardConsts {
    PairKind k[3];
    int64_t first_sp;      // particles from here on are special (n when there are none)
};

__device__ inline PairKind pair_kind(const HardConsts &hc, bool si, bool sj) {
    return (si && sj) ? hc.k[2] : (si || sj) ? hc.k[1] : hc.k[0];
}

struct HermConsts {
    double t_end, dt_max, dt_min, eta, eta_s, a0;
    double eta_sp, eta_s_sp;   // accuracy parameters of special particles
    int64_t max_block_steps;
};

// readback slots (int64 units) used here
enum { RB_HBAD = 48, RB_HNHARD = 49, RB_HNCL = 50, RB_HMAXCL = 51, RB_HLIMIT = 52,
       RB_HSTEPS = 53, RB_HMAXBLK = 54, RB_HNNZ = 55, RB_HCLASS = 56 /* 4 int32 class sizes */,
       RB_HGIANT = 58, RB_HSUB = 61 /* 5 int32 sub-class sizes of the < 64 class */ };

// size classes by floor(log2(members)): < 64, < 256, < 1024, the rest
constexpr int kClassBucket[3] = {5, 7, 9};
constexpr int kNumClasses = 4;
constexpr int kAux = 3;         // streams beside the context stream, one per LDS class

// ---------------------------------------------------------------------------
// Changeover functions, written as the formulas of Section 2.1 (G with the
// denominator (gamma - 1)^7).
// ---------------------------------------------------------------------------
__host__ __device__ inline double hk_K(double y, double gam) {
    if (y < gam) return 0.0;
    if (y >= 1.0) return 1.0;
    const double x = (y - gam) / (1.0 - gam);
    const double x2 = x * x;
    return x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
}

__host__ __device__ inline double hk_dK(double y, double gam) {   // dK/dy
    if (y < gam || y >= 1.0) return 0.0;
    const double x = (y - gam) / (1.0 - gam);
    const double u = x * (1.0 - x);
    return 140.0 * u * u * u / (1.0 - gam);
}

__host__ __device__ inline double hk_G(double y, double g) {
    const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g, g7 = g6 * g;
    const double y2 = y * y, y3 = y2 * y, y4 = y3 * y, y5 = y4 * y, y6 = y5 * y, y7 = y6 * y;
    const double gm1 = g - 1.0;
    const double gm7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
    const double num = -(10.0 / 3.0) * y7 + 14.0 * (g + 1.0) * y6 - 21.0 * (g2 + 3.0 * g + 1.0) * y5 +
                       (35.0 * (g3 + 9.0 * g2 + 9.0 * g + 1.0) / 3.0) * y4 -
                       70.0 * (g3 + 3.0 * g2 + g) * y3 + 210.0 * (g3 + g2) * y2 -
                       140.0 * g3 * y * log(y) + (g7 - 7.0 * g6 + 21.0 * g5 - 35.0 * g4);
    return num / gm7;
}

static double hk_C(double g) {
    const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g;
    const double gm1 = g - 1.0;
    const double gm7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
    return 7.0 * (g6 - 9.0 * g5 + 45.0 * g4 - 60.0 * g3 * log(g) - 45.0 * g2 + 9.0 * g - 1.0) /
           (3.0 * gm7);
}

__device__ inline double hk_W(double y, const PairKind &q) {
    if (y < q.gam) return q.C * y;
    if (y >= 1.0) return 1.0;
    return hk_G(y, q.gam) + (1.0 - q.G1) * y;
}

// Hard force, jerk (and potential if POT) on i from its list at positions x and
// velocities v, indexed through `map` (identity for caller arrays, particle ->
// slot for the integrator's state).
template <bool POT, bool MAP>
__device__ inline void hard_sum(int64_t i, int64_t si, const double *__restrict__ x,
                                const double *__restrict__ v, const double *__restrict__ mass,
                                const int64_t *__restrict__ off, const int32_t *__restrict__ idx,
                                const int32_t *__restrict__ map, const HardConsts &hc,
                                double a[3], double jk[3], double *phi) {
    a[0] = a[1] = a[2] = 0.0;
    jk[0] = jk[1] = jk[2] = 0.0;
    double p = 0.0;
    const double xi = x[3 * si], yi = x[3 * si + 1], zi = x[3 * si + 2];
    const double ui = v[3 * si], vi = v[3 * si + 1], wi = v[3 * si + 2];
    const bool spi = i >= hc.first_sp;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        const int32_t j = idx[e];
        const PairKind q = pair_kind(hc, spi, j >= hc.first_sp);
        const int64_t sj = MAP ? map[j] : j;
        const double dx = x[3 * sj] - xi;
        const double dy = x[3 * sj + 1] - yi;
        const double dz = x[3 * sj + 2] - zi;
        const double vx = v[3 * sj] - ui;
        const double vy = v[3 * sj + 1] - vi;
        const double vz = v[3 * sj + 2] - wi;
        const double s2 = dx * dx + dy * dy + dz * dz + q.eps * q.eps;
        const double s = sqrt(s2);
        const double y = s / q.r_out;
        const double K = q.split ? hk_K(y, q.gam) : 0.0;
        const double Ks = q.split ? hk_dK(y, q.gam) / q.r_out : 0.0;
        const double mj = mass[j];
        const double inv_s3 = 1.0 / (s2 * s);
        const double rv = dx * vx + dy * vy + dz * vz;
        const double f = mj * (1.0 - K) * inv_s3;
        const double c = 3.0 * rv / s2;
        const double g = mj * Ks * rv / s * inv_s3;
        a[0] += f * dx;
        a[1] += f * dy;
        a[2] += f * dz;
        jk[0] += f * (vx - c * dx) - g * dx;
        jk[1] += f * (vy - c * dy) - g * dy;
        jk[2] += f * (vz - c * dz) - g * dz;
        if (POT) p -= mj * (1.0 - (q.split ? hk_W(y, q) : 0.0)) / s;
    }
    if (POT) *phi = p;
}

// Rows must be well formed before any kernel walks them: offsets non-decreasing
// from a non-negative start, entries in [0, n), not the row's own particle, and
// symmetric (i is on the row of every j on i's row; the components of the
// neighbour graph are joined from one end of each edge, and the integrators
// index a neighbour inside its component).  Without an index array (HAS_IDX
// false) every row must be empty and nothing else is read.
template <bool HAS_IDX>
__global__ void k_hard_validate(int64_t n, const int64_t *__restrict__ off,
                                const int32_t *__restrict__ idx, int64_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t b = off[i], e = off[i + 1];
    if (b < 0 || e < b || (!HAS_IDX && e != b)) { atomicOr((unsigned long long *)bad, 1ull); return; }
    if (!HAS_IDX) return;
    for (int64_t k = b; k < e; ++k) {
        const int32_t j = idx[k];
        if (j < 0 || j >= n || j == i) { atomicOr((unsigned long long *)bad, 1ull); return; }
        const int64_t jb = off[j], je = off[j + 1];
        if (jb < 0 || je < jb) { atomicOr((unsigned long long *)bad, 1ull); return; }
        bool back = false;   // rows need not be sorted: a linear search of j's row
        for (int64_t t = jb; t < je && !back; ++t) back = idx[t] == (int32_t)i;
        if (!back) { atomicOr((unsigned long long *)bad, 1ull); return; }
    }
}

__global__ __launch_bounds__(kHardThreads) void k_hard_force(
    int64_t n, const double *__restrict__ pos, const double *__restrict__ vel,
    const double *__restrict__ mass, const int64_t *__restrict__ off,
    const int32_t *__restrict__ idx, HardConsts hc, double *__restrict__ acc,
    double *__restrict__ jerk, double *__restrict__ pot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[3], jk[3], p = 0.0;
    if (pot)
        hard_sum<true, false>(i, i, pos, vel, mass, off, idx, nullptr, hc, a, jk, &p);
    else
        hard_sum<false, false>(i, i, pos, vel, mass, off, idx, nullptr, hc, a, jk, &p);
    for (int k = 0; k < 3; ++k) {
        acc[3 * i + k] = a[k];
        jerk[3 * i + k] = jk[k];
    }
    if (pot) pot[i] = p;
}

// ---------------------------------------------------------------------------
// Components of the neighbour graph.
// ---------------------------------------------------------------------------
__device__ inline int32_t ld_par(const int32_t *par, int32_t x) {
    return __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Parents only ever decrease, so the chain is finite; path halving
// by compare-and-swap keeps that invariant.
__device__ int32_t uf_find(int32_t *par, int32_t x) {
    for (;;) {
        int32_t p = ld_par(par, x);
        if (p == x) return x;
        const int32_t gp = ld_par(par, p);
        if (gp != p) atomicCAS(&par[x], p, gp);
        x = gp;
    }
}

__global__ void k_cc_init(int64_t n, int32_t *__restrict__ par, int32_t *__restrict__ ccount,
                          int32_t *__restrict__ cfill) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    par[i] = (int32_t)i;
    ccount[i] = 0;
    cfill[i] = 0;
}

__global__ void k_cc_union(int64_t n, const int64_t *__restrict__ off,
                           const int32_t *__restrict__ idx, int32_t *par, int64_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        const int32_t j = idx[e];
        if (j <= i) continue;            // each edge once
        int32_t a = (int32_t)i, b = j;
        int t = 0;
        for (; t < kUnionTries; ++t) {
            a = uf_find(par, a);
            b = uf_find(par, b);
            if (a == b) break;
            if (a < b) { const int32_t s = a; a = b; b = s; }
            if (atomicCAS(&par[a], a, b) == a) break;   // a was still a root
        }
        if (t == kUnionTries) atomicOr((unsigned long long *)bad, 2ull);
    }
}

// label = root; count members per root
__global__ void k_cc_count(int64_t n, const int64_t *__restrict__ off, int32_t *par,
                           int32_t *__restrict__ label, int32_t *__restrict__ ccount) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (off[i + 1] == off[i]) { label[i] = -1; return; }
    const int32_t r = uf_find(par, (int32_t)i);
    label[i] = r;
    atomicAdd(&ccount[r], 1);
}

__global__ void k_cc_rootflag(int64_t n, const int32_t *__restrict__ ccount,
                              int32_t *__restrict__ rflag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rflag[i] = ccount[i] > 0 ? 1 : 0;
}

// members into slots cstart[root] + k; isolated particles drift
__global__ void k_cc_place(int64_t n, const int32_t *__restrict__ label,
                           const int32_t *__restrict__ cstart, int32_t *__restrict__ cfill,
                           int32_t *__restrict__ mem, int32_t *__restrict__ slot,
                           double *__restrict__ pos, const double *__restrict__ vel,
                           double dt_soft) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = label[i];
    if (r < 0) {
        slot[i] = -1;
        for (int k = 0; k < 3; ++k) pos[3 * i + k] += dt_soft * vel[3 * i + k];
        return;
    }
    const int32_t s = cstart[r] + atomicAdd(&cfill[r], 1);
    mem[s] = (int32_t)i;
    slot[i] = s;
}

__device__ inline int size_bucket(int32_t size) { return 31 - __clz(size); }

// cluster ranges and a histogram of floor(log2(size)); counts gather in LDS
// first, so that the few global counters see one atomic per block
__global__ __launch_bounds__(256) void k_cc_clusters(
    int64_t n, const int32_t *__restrict__ ccount, const int32_t *__restrict__ cstart,
    const int32_t *__restrict__ cid, int32_t *__restrict__ cl_beg, int32_t *__restrict__ cl_end,
    int32_t *__restrict__ bhist, unsigned long long *maxsize) {
    __shared__ int32_t s_h[32];
    __shared__ unsigned int s_max;
    if (threadIdx.x < 32) s_h[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t c = r < n ? ccount[r] : 0;
    if (c > 0) {
        const int32_t k = cid[r];
        cl_beg[k] = cstart[r];
        cl_end[k] = cstart[r] + c;
        atomicAdd(&s_h[size_bucket(c)], 1);
        atomicMax(&s_max, (unsigned int)c);
    }
    __syncthreads();
    if (threadIdx.x < 32 && s_h[threadIdx.x]) atomicAdd(&bhist[threadIdx.x], s_h[threadIdx.x]);
    if (threadIdx.x == 0 && s_max) atomicMax(maxsize, (unsigned long long)s_max);
}

// exclusive offsets of the size buckets, largest sizes first (one thread)
__global__ void k_cc_bucket_scan(int32_t *bhist) {
    int32_t acc = 0;
    for (int b = 31; b >= 0; --b) {
        const int32_t c = bhist[b];
        bhist[b] = acc;
        acc += c;
    }
}

// clusters into `order` by bucket, largest buckets first; each block reserves
// its run of every bucket with one global atomic
__global__ __launch_bounds__(256) void k_cc_order(int64_t n_cl, const int32_t *__restrict__ cl_beg,
                                                  const int32_t *__restrict__ cl_end,
                                                  int32_t *__restrict__ bfill,
                                                  const int32_t *__restrict__ boff,
                                                  int32_t *__restrict__ order) {
    __shared__ int32_t s_cnt[32], s_base[32];
    if (threadIdx.x < 32) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int b = -1, rank = 0;
    if (c < n_cl) {
        b = size_bucket(cl_end[c] - cl_beg[c]);
        rank = atomicAdd(&s_cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < 32 && s_cnt[threadIdx.x])
        s_base[threadIdx.x] = boff[threadIdx.x] + atomicAdd(&bfill[threadIdx.x], s_cnt[threadIdx.x]);
    __syncthreads();
    if (b >= 0) order[s_base[b] + rank] = (int32_t)c;
}

// ---------------------------------------------------------------------------
// Hermite integration, one workgroup per component.
// ---------------------------------------------------------------------------
struct HermState {
    double *x, *v, *a, *j, *a2, *a3, *xp, *vp, *a1, *j1;   // [slots][3]
    double *t, *dt;                                        // [slots]
    int32_t *ns;                                           // [slots]
};

__device__ inline double norm3(const double *v) {
    return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

__device__ inline double crit_first(const double *a, const double *j, const HermConsts &hp,
                                    double eta_s) {
    const double na = norm3(a), nj = norm3(j);
    if (nj == 0.0) return hp.dt_max;
    return eta_s * sqrt((na * na + hp.a0 * hp.a0) / (nj * nj));
}

// the denominator's first term is |a'| |a'''| (the form with matching units)
__device__ inline double crit_full(const double *a, const double *j, const double *a2,
                                   const double *a3, const HermConsts &hp, double eta) {
    const double na = norm3(a), nj = norm3(j), n2 = norm3(a2), n3 = norm3(a3);
    const double num = sqrt(na * na + hp.a0 * hp.a0) * n2 + nj * nj;
    const double den = nj * n3 + n2 * n2;
    if (den == 0.0) return hp.dt_max;
    return eta * sqrt(num / den);
}

// Components of kGiant members or more run as a sequence of grid-wide launches
// per block step over all of their members (flattened: member k belongs to
// component g with gpre[g] <= k < gpre[g + 1], slot gbeg[g] + k - gpre[g]):
// the minimum of t + dt per component, the prediction, then force and
// correction of the active members.  Two buffers of per-component minima
// alternate between steps; the step that reads one resets the other.  A
// component past t_end does nothing, so the host can run steps in batches
// and stop when every component is done.
struct GiantView {
    const int32_t *gbeg, *gpre;   // [n_giant], [n_giant + 1]
    int32_t n_giant, n_members;
};

__device__ inline void giant_member(const GiantView &gv, int32_t k, int32_t &g, int32_t &s) {
    int lo = 0, hi = gv.n_giant - 1;
    while (lo < hi) {            // last g with gpre[g] <= k
        const int mid = (lo + hi + 1) >> 1;
        if (gv.gpre[mid] <= k) lo = mid; else hi = mid - 1;
    }
    g = lo;
    s = gv.gbeg[lo] + (k - gv.gpre[lo]);
}

__global__ void k_giant_load(GiantView gv, const int32_t *__restrict__ mem,
                             const double *__restrict__ pos, const double *__restrict__ vel,
                             HermState S, unsigned long long *tmin) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < gv.n_giant) {
        tmin[k] = __double_as_longlong(INFINITY);
        tmin[gv.n_giant + k] = __double_as_longlong(INFINITY);
    }
    if (k >= gv.n_members) return;
    int32_t g, s;
    giant_member(gv, k, g, s);
    const int32_t i = mem[s];
    for (int q = 0; q < 3; ++q) {
        S.x[3 * s + q] = pos[3 * i + q];
        S.v[3 * s + q] = vel[3 * i + q];
    }
    S.t[s] = 0.0;
    S.ns[s] = 0;
}

__global__ void k_giant_first(GiantView gv, const int32_t *__restrict__ mem,
                              const int32_t *__restrict__ slot, const int64_t *__restrict__ off,
                              const int32_t *__restrict__ idx, const double *__restrict__ mass,
                              HardConsts hc, HermConsts hp, HermState S) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= gv.n_members) return;
    int32_t g, s;
    giant_member(gv, k, g, s);
    double dummy;
    hard_sum<false, true>(mem[s], s, S.x, S.v, mass, off, idx, slot, hc, S.a + 3 * s, S.j + 3 * s,
                          &dummy);
    const double cr = crit_first(S.a + 3 * s, S.j + 3 * s, hp,
                                 mem[s] >= hc.first_sp ? hp.eta_s_sp : hp.eta_s);
    double d = hp.dt_max;
    while (d > cr && d > hp.dt_min) d *= 0.5;
    S.dt[s] = d;
}

// step parity b: minima go to tmin[b * n_giant + g]
__global__ void k_giant_min(GiantView gv, HermState S, unsigned long long *tmin, int b) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= gv.n_members) return;
    int32_t g, s;
    giant_member(gv, k, g, s);
    atomicMin(&tmin[b * gv.n_giant + g],
              (unsigned long long)__double_as_longlong(S.t[s] + S.dt[s]));
}

__global__ void k_giant_predict(GiantView gv, HermConsts hp, HermState S,
                                unsigned long long *tmin, int b, int32_t *gsteps) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < gv.n_giant) tmin[(1 - b) * gv.n_giant + k] = __double_as_longlong(INFINITY);
    if (k >= gv.n_members) return;
    int32_t g, s;
    giant_member(gv, k, g, s);
    const double t_next = __longlong_as_double((long long)tmin[b * gv.n_giant + g]);
    if (!(t_next <= hp.t_end)) return;
    if (k == gv.gpre[g]) gsteps[g] += 1;   // block steps of component g
    const double h = t_next - S.t[s];
    for (int q = 0; q < 3; ++q) {
        const int i3 = 3 * s + q;
        S.xp[i3] = S.x[i3] + S.v[i3] * h + S.a[i3] * (h * h / 2.0) + S.j[i3] * (h * h * h / 6.0);
        S.vp[i3] = S.v[i3] + S.a[i3] * h + S.j[i3] * (h * h / 2.0);
    }
}

// The summands one list entry adds to a and jerk (the operations of hard_sum),
// for particle i at slot si and neighbour j at slot sj of the predicted state.
__device__ inline void pair_terms_g(int64_t i, int64_t si, int32_t j, int64_t sj,
                                    const double *__restrict__ x, const double *__restrict__ v,
                                    const double *__restrict__ mass, const HardConsts &hc,
                                    double o[6]) {
    const PairKind q = pair_kind(hc, i >= hc.first_sp, j >= hc.first_sp);
    const double dx = x[3 * sj] - x[3 * si];
    const double dy = x[3 * sj + 1] - x[3 * si + 1];
    const double dz = x[3 * sj + 2] - x[3 * si + 2];
    const double vx = v[3 * sj] - v[3 * si];
    const double vy = v[3 * sj + 1] - v[3 * si + 1];
    const double vz = v[3 * sj + 2] - v[3 * si + 2];
    const double s2 = dx * dx + dy * dy + dz * dz + q.eps * q.eps;
    const double s = sqrt(s2);
    const double y = s / q.r_out;
    const double K = q.split ? hk_K(y, q.gam) : 0.0;
    const double Ks = q.split ? hk_dK(y, q.gam) / q.r_out : 0.0;
    const double mj = mass[j];
    const double inv_s3 = 1.0 / (s2 * s);
    const double rv = dx * vx + dy * vy + dz * vz;
    const double f = mj * (1.0 - K) * inv_s3;
    const double c = 3.0 * rv / s2;
    const double g = mj * Ks * rv / s * inv_s3;
    o[0] = f * dx;
    o[1] = f * dy;
    o[2] = f * dz;
    o[3] = f * (vx - c * dx) - g * dx;
    o[4] = f * (vy - c * dy) - g * dy;
    o[5] = f * (vz - c * dz) - g * dz;
}

// one wavefront per member: the lanes evaluate the row's summands 64 at a time
// and lane 0 adds them in list order, then corrects the member
__global__ __launch_bounds__(kGiantThreads) void k_giant_correct(
    GiantView gv, const int32_t *__restrict__ mem, const int32_t *__restrict__ slot,
    const int64_t *__restrict__ off, const int32_t *__restrict__ idx,
    const double *__restrict__ mass, HardConsts hc, HermConsts hp, HermState S,
    const unsigned long long *tmin, int b) {
    const int lane = threadIdx.x & 63;
    const int32_t k = blockIdx.x * (kGiantThreads / 64) + (threadIdx.x >> 6);
    if (k >= gv.n_members) return;                   // whole wavefront
    int32_t g, s;
    giant_member(gv, k, g, s);
    const double t_next = __longlong_as_double((long long)tmin[b * gv.n_giant + g]);
    if (!(t_next <= hp.t_end) || S.t[s] + S.dt[s] != t_next) return;   // whole wavefront
    const int32_t i = mem[s];
    const int64_t rb = off[i], re = off[i + 1];
    double sum[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t e0 = rb; e0 < re; e0 += 64) {
        double o[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const int64_t e = e0 + lane;
        if (e < re) {
            const int32_t j = idx[e];
            pair_terms_g(i, s, j, slot[j], S.xp, S.vp, mass, hc, o);
        }
        const int cnt = (int)min<int64_t>(64, re - e0);
        for (int src = 0; src < cnt; ++src)
            for (int q = 0; q < 6; ++q) {
                const double w = __shfl(o[q], src);
                if (lane == 0) sum[q] += w;
            }
    }
    if (lane != 0) return;
    const double h = S.dt[s];
    double a2[3], a3[3];
    for (int q = 0; q < 3; ++q) {
        const int i3 = 3 * s + q;
        const double a1 = sum[q], j1 = sum[3 + q];
        const double s2 = (-6.0 * (S.a[i3] - a1) - h * (4.0 * S.j[i3] + 2.0 * j1)) / (h * h);
        const double s3 = (12.0 * (S.a[i3] - a1) + 6.0 * h * (S.j[i3] + j1)) / (h * h * h);
        S.x[i3] = S.xp[i3] + s2 * (h * h * h * h / 24.0) + s3 * (h * h * h * h * h / 120.0);
        S.v[i3] = S.vp[i3] + s2 * (h * h * h / 6.0) + s3 * (h * h * h * h / 24.0);
        S.a[i3] = a1;
        S.j[i3] = j1;
        a2[q] = s2 + s3 * h;
        a3[q] = s3;
    }
    S.t[s] = t_next;
    S.ns[s] += 1;
    const double cr = crit_full(S.a + 3 * s, S.j + 3 * s, a2, a3, hp,
                                i >= hc.first_sp ? hp.eta_sp : hp.eta);
    double d = h;
    if (2.0 * d <= cr && 2.0 * d <= hp.dt_max && fmod(S.t[s], 2.0 * d) == 0.0)
        d = 2.0 * d;
    else
        while (d > cr && d > hp.dt_min) d *= 0.5;
    S.dt[s] = d;
}

__global__ void k_giant_store(GiantView gv, const int32_t *__restrict__ mem, HermState S,
                              double *__restrict__ pos, double *__restrict__ vel,
                              int32_t *__restrict__ nsteps_out, unsigned long long *rb) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long my = 0;
    if (k < gv.n_members) {
        int32_t g, s;
        giant_member(gv, k, g, s);
        const int32_t i = mem[s];
        for (int q = 0; q < 3; ++q) {
            pos[3 * i + q] = S.x[3 * s + q];
            vel[3 * i + q] = S.v[3 * s + q];
        }
        if (nsteps_out) nsteps_out[i] = S.ns[s];
        my = (unsigned long long)S.ns[s];
    }
    for (int o = 32; o > 0; o >>= 1) my += __shfl_xor(my, o);
    if ((threadIdx.x & 63) == 0 && my) atomicAdd(rb + (RB_HSTEPS - RB_HBAD), my);
}

// giant components' ranges (order[0 .. n_giant) are the largest components);
// one thread: there are few of them
__global__ void k_giant_ranges(const int32_t *__restrict__ order, const int32_t *__restrict__ cl_beg,
                               const int32_t *__restrict__ cl_end, int32_t n_giant,
                               int32_t *__restrict__ gbeg, int32_t *__restrict__ gpre,
                               int32_t *__restrict__ gsteps) {
    int32_t acc = 0;
    for (int32_t g = 0; g < n_giant; ++g) {
        const int32_t c = order[g];
        gbeg[g] = cl_beg[c];
        gpre[g] = acc;
        gsteps[g] = 0;
        acc += cl_end[c] - cl_beg[c];
    }
    gpre[n_giant] = acc;
}

__global__ void k_giant_maxsteps(const int32_t *__restrict__ gsteps, int32_t n_giant,
                                 unsigned long long *rb) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n_giant) atomicMax(rb + (RB_HMAXBLK - RB_HBAD), (unsigned long long)gsteps[g]);
}

// cluster counts of the size classes, largest class first: [>= 1024, < 1024,
// < 256, < 64] members (from the bucket histogram, before it is scanned)
// and the < 64 class split by lanes per component, in the same (largest first)
// order: [32, 64) members on 64 lanes, [16, 32) on 32, [8, 16) on 16, [4, 8) on
// 8, [1, 4) on 4
__global__ void k_cc_classes(const int32_t *bhist, int32_t *cls, int32_t *sub) {
    int32_t c[kNumClasses] = {0, 0, 0, 0};
    for (int b = 0; b < 32; ++b) {
        int k = 0;
        for (int q = 0; q < 3; ++q)
            if (b <= kClassBucket[q]) { k = 3 - q; break; }
        c[k] += bhist[b];
    }
    for (int k = 0; k < kNumClasses; ++k) cls[k] = c[k];
    sub[0] = bhist[5];
    sub[1] = bhist[4];
    sub[2] = bhist[3];
    sub[3] = bhist[2];
    sub[4] = bhist[0] + bhist[1];
}

// local index of every list entry: the neighbour's slot minus the first slot of
// the entry's component
__global__ void k_hard_local(int64_t n, const int64_t *__restrict__ off,
                             const int32_t *__restrict__ idx, const int32_t *__restrict__ label,
                             const int32_t *__restrict__ cid, const int32_t *__restrict__ cl_beg,
                             const int32_t *__restrict__ slot, int32_t *__restrict__ lidx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = label[i];
    if (r < 0) return;
    const int32_t base = cl_beg[cid[r]];
    for (int64_t e = off[i]; e < off[i + 1]; ++e) lidx[e] = slot[idx[e]] - base;
}

// The six summands one list entry adds to a and jerk, by the operations of
// hard_sum: member k's predicted state against neighbour jl, both local.
__device__ inline void pair_terms(int k, int jl, const double *xs, const double *vs,
                                  const double *sm, const int8_t *ssp, const HardConsts &hc,
                                  double o[6]) {
    const PairKind q = pair_kind(hc, ssp[k] != 0, ssp[jl] != 0);
    const double dx = xs[3 * jl] - xs[3 * k];
    const double dy = xs[3 * jl + 1] - xs[3 * k + 1];
    const double dz = xs[3 * jl + 2] - xs[3 * k + 2];
    const double vx = vs[3 * jl] - vs[3 * k];
    const double vy = vs[3 * jl + 1] - vs[3 * k + 1];
    const double vz = vs[3 * jl + 2] - vs[3 * k + 2];
    const double s2 = dx * dx + dy * dy + dz * dz + q.eps * q.eps;
    const double s = sqrt(s2);
    const double y = s / q.r_out;
    const double K = q.split ? hk_K(y, q.gam) : 0.0;
    const double Ks = q.split ? hk_dK(y, q.gam) / q.r_out : 0.0;
    const double mj = sm[jl];
    const double inv_s3 = 1.0 / (s2 * s);
    const double rv = dx * vx + dy * vy + dz * vz;
    const double f = mj * (1.0 - K) * inv_s3;
    const double c = 3.0 * rv / s2;
    const double g = mj * Ks * rv / s * inv_s3;
    o[0] = f * dx;
    o[1] = f * dy;
    o[2] = f * dz;
    o[3] = f * (vx - c * dx) - g * dx;
    o[4] = f * (vy - c * dy) - g * dy;
    o[5] = f * (vz - c * dz) - g * dz;
}

// hard_sum on a component held in LDS: member k's predicted state, neighbours
// through local indices nb[rb .. re), masses from sm, summed in list order.
__device__ inline void hard_sum_local(int k, const double *xs, const double *vs, const double *sm,
                                      const int8_t *ssp, const int32_t *nb, int64_t rb,
                                      int64_t re, const HardConsts &hc, double a[3],
                                      double jk[3]) {
    a[0] = a[1] = a[2] = 0.0;
    jk[0] = jk[1] = jk[2] = 0.0;
    for (int64_t e = rb; e < re; ++e) {
        double o[6];
        pair_terms(k, nb[e], xs, vs, sm, ssp, hc, o);
        a[0] += o[0];
        a[1] += o[1];
        a[2] += o[2];
        jk[0] += o[3];
        jk[1] += o[4];
        jk[2] += o[5];
    }
}

template <int T>
__device__ inline double block_min_t(double v, double *s_red) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    if (T == 64) return v;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_red[w] = v;
    __syncthreads();
    double r = s_red[0];
    for (int k = 1; k < T / 64; ++k) r = fmin(r, s_red[k]);
    return r;
}

// Exclusive prefix sum of one int per thread over a block of T threads; the
// block total in `total`.  Every thread of the block must call it.
template <int T>
__device__ inline int block_scan_excl(int v, int *s_ws, int &total) {
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if ((int)(threadIdx.x & 63) >= o) incl += y;
    }
    if (T == 64) {
        total = __shfl(incl, 63);
        return incl - v;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) s_ws[w] = incl;
    __syncthreads();
    int before = 0, tot = 0;
    for (int q = 0; q < T / 64; ++q) {
        const int x = s_ws[q];
        if (q < w) before += x;
        tot += x;
    }
    total = tot;
    __syncthreads();
    return before + incl - v;
}

// One component of fewer than T * R members per block; member k is owned by
// thread k % T, slot r = k / T of its registers.  With C > 0 and the lists in
// LDS, a block step gathers the list entries of its active members, evaluates
// their pair terms across the whole block, C entries at a time, into LDS, and
// each owner then adds its row's terms in list order -- the same sums as the
// sequential loop.
template <int T, int R, int ECAP, int C>
__global__ __launch_bounds__(T) void k_hermite_lds(
    const int32_t *__restrict__ cl_beg, const int32_t *__restrict__ cl_end,
    const int32_t *__restrict__ order, int32_t order_base, const int32_t *__restrict__ mem,
    const int64_t *__restrict__ off, const int32_t *__restrict__ lidx,
    const double *__restrict__ mass, double *__restrict__ pos, double *__restrict__ vel,
    HardConsts hc, HermConsts hp, int32_t *__restrict__ nsteps_out, unsigned long long *rb) {
    constexpr int M = T * R;
    __shared__ double s_xp[3 * M], s_vp[3 * M], s_m[M];
    __shared__ int32_t s_row[M + 1];
    __shared__ int32_t s_nb[ECAP];
    __shared__ int16_t s_ae[C > 0 ? ECAP : 1];      // active entries of a step ...
    __shared__ int16_t s_aown[C > 0 ? ECAP : 1];    // ... and their members
    __shared__ double s_term[C > 0 ? 6 * C : 1];
    __shared__ int s_ws[T / 64];
    __shared__ double s_red[T / 64];
    __shared__ int8_t s_sp[M];   // 1: special particle
    const int c = order[order_base + blockIdx.x];
    const int b = cl_beg[c], nm = cl_end[c] - b;
    const int tid = threadIdx.x;
    for (int k = tid; k < nm; k += T) {
        const int32_t i = mem[b + k];
        s_row[k + 1] = (int32_t)(off[i + 1] - off[i]);
        s_m[k] = mass[i];
        s_sp[k] = i >= hc.first_sp;
    }
    __syncthreads();
    if (tid == 0) {
        s_row[0] = 0;
        for (int k = 1; k <= nm; ++k) s_row[k] += s_row[k - 1];
    }
    __syncthreads();
    const int n_edges = s_row[nm];
    const bool in_lds = n_edges <= ECAP;
    // list entries as local indices, row by row, in LDS if they fit
    if (in_lds)
        for (int k = tid; k < nm; k += T) {
            const int32_t i = mem[b + k];
            const int64_t e0 = off[i];
            for (int q = s_row[k]; q < s_row[k + 1]; ++q) s_nb[q] = lidx[e0 + (q - s_row[k])];
        }
    const bool rowpar = C > 0 && in_lds;
    double x[R][3], v[R][3], a[R][3], jk[R][3], t[R], dt[R];
    int ns[R];
    int64_t e0[R];   // first global list entry of the member's row (global fallback)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = tid + r * T;
        t[r] = 0.0;
        dt[r] = INFINITY;
        ns[r] = 0;
        e0[r] = 0;
        if (k < nm) {
            const int32_t i = mem[b + k];
            e0[r] = off[i];
            for (int q = 0; q < 3; ++q) {
                x[r][q] = pos[3 * i + q];
                v[r][q] = vel[3 * i + q];
                s_xp[3 * k + q] = x[r][q];
                s_vp[3 * k + q] = v[r][q];
            }
        }
    }
    __syncthreads();
    // neighbours of member k: local indices at nbp + rowb
    const int32_t *nbp = in_lds ? s_nb : lidx;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = tid + r * T;
        if (k >= nm) continue;
        const int64_t rowb = in_lds ? (int64_t)s_row[k] : e0[r];
        const int64_t rowe = rowb + (s_row[k + 1] - s_row[k]);
        hard_sum_local(k, s_xp, s_vp, s_m, s_sp, nbp, rowb, rowe, hc, a[r], jk[r]);
        const double cr = crit_first(a[r], jk[r], hp, s_sp[k] ? hp.eta_s_sp : hp.eta_s);
        double d = hp.dt_max;
        while (d > cr && d > hp.dt_min) d *= 0.5;
        dt[r] = d;
    }
    int64_t steps = 0;
    for (;;) {
        double lmin = INFINITY;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double tn = t[r] + dt[r];
            if (tn < lmin) lmin = tn;
        }
        const double t_next = block_min_t<T>(lmin, s_red);
        if (!(t_next <= hp.t_end)) break;
        if (steps == hp.max_block_steps) {
            if (tid == 0) atomicOr(rb + (RB_HLIMIT - RB_HBAD), 1ull);
            break;
        }
        ++steps;
        if (T == 64) __syncthreads();   // the previous step's reads of s_xp are done
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = tid + r * T;
            if (k >= nm) continue;
            const double h = t_next - t[r];
            for (int q = 0; q < 3; ++q) {
                s_xp[3 * k + q] = x[r][q] + v[r][q] * h + a[r][q] * (h * h / 2.0) +
                                  jk[r][q] * (h * h * h / 6.0);
                s_vp[3 * k + q] = v[r][q] + a[r][q] * h + jk[r][q] * (h * h / 2.0);
            }
        }
        __syncthreads();
        double a1[R][3], j1[R][3];
        if (rowpar) {
            // the active members' list entries, gathered in row order
            int lens[R], abase[R], L = 0, n_act = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = tid + r * T;
                lens[r] = (k < nm && t[r] + dt[r] == t_next) ? s_row[k + 1] - s_row[k] : 0;
                L += lens[r];
                for (int q = 0; q < 3; ++q) a1[r][q] = j1[r][q] = 0.0;
            }
            int o0 = block_scan_excl<T>(L, s_ws, n_act);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                abase[r] = o0;
                const int k = tid + r * T;
                for (int q = 0; q < lens[r]; ++q) {
                    s_ae[o0 + q] = (int16_t)(s_row[k] + q);
                    s_aown[o0 + q] = (int16_t)k;
                }
                o0 += lens[r];
            }
            __syncthreads();
            for (int c0 = 0; c0 < n_act; c0 += (C > 0 ? C : 1)) {
                const int c1 = min(c0 + C, n_act);
                for (int e = c0 + tid; e < c1; e += T) {
                    double o[6];
                    pair_terms(s_aown[e], s_nb[s_ae[e]], s_xp, s_vp, s_m, s_sp, hc, o);
                    for (int q = 0; q < 6; ++q) s_term[6 * (e - c0) + q] = o[q];
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!lens[r]) continue;
                    const int rb = max(abase[r], c0), re = min(abase[r] + lens[r], c1);
                    for (int e = rb; e < re; ++e) {
                        const double *o = s_term + 6 * (e - c0);
                        a1[r][0] += o[0];
                        a1[r][1] += o[1];
                        a1[r][2] += o[2];
                        j1[r][0] += o[3];
                        j1[r][1] += o[4];
                        j1[r][2] += o[5];
                    }
                }
                __syncthreads();
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = tid + r * T;
                if (k >= nm || t[r] + dt[r] != t_next) continue;
                const int64_t rowb = in_lds ? (int64_t)s_row[k] : e0[r];
                const int64_t rowe = rowb + (s_row[k + 1] - s_row[k]);
                hard_sum_local(k, s_xp, s_vp, s_m, s_sp, nbp, rowb, rowe, hc, a1[r], j1[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = tid + r * T;
            if (k >= nm || t[r] + dt[r] != t_next) continue;
            double a2[3], a3[3];
            const double h = dt[r];
            for (int q = 0; q < 3; ++q) {
                const double s2 =
                    (-6.0 * (a[r][q] - a1[r][q]) - h * (4.0 * jk[r][q] + 2.0 * j1[r][q])) / (h * h);
                const double s3 =
                    (12.0 * (a[r][q] - a1[r][q]) + 6.0 * h * (jk[r][q] + j1[r][q])) / (h * h * h);
                x[r][q] = s_xp[3 * k + q] + s2 * (h * h * h * h / 24.0) +
                          s3 * (h * h * h * h * h / 120.0);
                v[r][q] = s_vp[3 * k + q] + s2 * (h * h * h / 6.0) + s3 * (h * h * h * h / 24.0);
                a[r][q] = a1[r][q];
                jk[r][q] = j1[r][q];
                a2[q] = s2 + s3 * h;
                a3[q] = s3;
            }
            t[r] = t_next;
            ns[r] += 1;
            const double cr = crit_full(a[r], jk[r], a2, a3, hp, s_sp[k] ? hp.eta_sp : hp.eta);
            double d = h;
            if (2.0 * d <= cr && 2.0 * d <= hp.dt_max && fmod(t[r], 2.0 * d) == 0.0)
                d = 2.0 * d;
            else
                while (d > cr && d > hp.dt_min) d *= 0.5;
            dt[r] = d;
        }
    }
    unsigned long long my_steps = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = tid + r * T;
        if (k >= nm) continue;
        const int32_t i = mem[b + k];
        for (int q = 0; q < 3; ++q) {
            pos[3 * i + q] = x[r][q];
            vel[3 * i + q] = v[r][q];
        }
        if (nsteps_out) nsteps_out[i] = ns[r];
        my_steps += (unsigned long long)ns[r];
    }
    for (int o = 32; o > 0; o >>= 1) my_steps += __shfl_xor(my_steps, o);
    if ((tid & 63) == 0 && my_steps) atomicAdd(rb + (RB_HSTEPS - RB_HBAD), my_steps);
    if (tid == 0) atomicMax(rb + (RB_HMAXBLK - RB_HBAD), (unsigned long long)steps);
}

// Components of fewer than 64 members, several to a wavefront: SUB lanes per
// component (4, 8, 16, 32 or 64), member k on lane k of its sub-group.  Every
// sub-group runs its own block-step loop with the operations of k_hermite_lds
// (its minimum of t + dt by shuffles inside the sub-group); the wavefront loops
// until every sub-group is past t_end.  The list entries of a component with
// fewer than 32 members always fit its share of the LDS area.  With RP, a
// block step spreads the active members' list entries over the sub-group's
// lanes, SUB at a time, and each owner then adds its row's terms in list order
// (the same sums as the loop over its own row), so that a member with many
// neighbours no longer sets the length of the step alone.
constexpr int kPackEdges = 2048;

template <bool RP>
struct PackLds {
    double xp[3 * kWave], vp[3 * kWave], m[kWave];
    int32_t row[kWave + 16];
    int32_t nb[kPackEdges];
    int16_t ae[RP ? kPackEdges : 1];     // active entries of a step ...
    int16_t aown[RP ? kPackEdges : 1];   // ... and their members
    double term[RP ? 6 * kWave : 1];     // one chunk of terms per sub-group
    int8_t sp[kWave];
};

template <int SUB, bool RP>
__device__ __forceinline__ void hermite_sub(
    int slot, int32_t n_slots, const int32_t *__restrict__ cl_beg,
    const int32_t *__restrict__ cl_end, const int32_t *__restrict__ order, int32_t order_base,
    const int32_t *__restrict__ mem, const int64_t *__restrict__ off,
    const int32_t *__restrict__ lidx, const double *__restrict__ mass, double *__restrict__ pos,
    double *__restrict__ vel, const HardConsts &hc, const HermConsts &hp,
    int32_t *__restrict__ nsteps_out, unsigned long long *rb, PackLds<RP> &L) {
    constexpr int P = kWave / SUB;           // components per wavefront
    constexpr int NBCAP = kPackEdges / P;    // list entries in LDS per component
    static_assert(SUB == kWave || SUB * (SUB - 1) <= NBCAP, "lists must fit");
    const int tid = threadIdx.x, sub = tid / SUB, lt = tid % SUB;
    const int cs = slot * P + sub;           // this sub-group's component, in launch order
    const bool has = cs < n_slots;
    const int c = has ? order[order_base + cs] : 0;
    const int b = has ? cl_beg[c] : 0;
    const int nm = has ? cl_end[c] - b : 0;
    double *xs = L.xp + 3 * SUB * sub, *vs = L.vp + 3 * SUB * sub, *sm = L.m + SUB * sub;
    int8_t *ssp = L.sp + SUB * sub;
    int32_t *row = L.row + (SUB + 1) * sub, *nb = L.nb + NBCAP * sub;
    const bool mine = lt < nm;               // this lane owns member lt
    int32_t i = 0;
    if (mine) {
        i = mem[b + lt];
        row[lt + 1] = (int32_t)(off[i + 1] - off[i]);
        sm[lt] = mass[i];
        ssp[lt] = i >= hc.first_sp;
    }
    __syncthreads();
    if (lt == 0 && has) {
        row[0] = 0;
        for (int k = 1; k <= nm; ++k) row[k] += row[k - 1];
    }
    __syncthreads();
    const int n_edges = has ? row[nm] : 0;
    const bool in_lds = n_edges <= NBCAP;
    const int64_t e0 = mine ? off[i] : 0;
    if (in_lds && mine)
        for (int q = row[lt]; q < row[lt + 1]; ++q) nb[q] = lidx[e0 + (q - row[lt])];
    double x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, a[3], jk[3];
    double t = 0.0, dt = INFINITY;
    int ns = 0;
    if (mine)
        for (int q = 0; q < 3; ++q) {
            x[q] = pos[3 * i + q];
            v[q] = vel[3 * i + q];
            xs[3 * lt + q] = x[q];
            vs[3 * lt + q] = v[q];
        }
    __syncthreads();
    // neighbours of the member: local indices at nbp + rowb
    const int32_t *nbp = in_lds ? nb : lidx;
    const int64_t rowb = mine ? (in_lds ? (int64_t)row[lt] : e0) : 0;
    const int64_t rowe = mine ? rowb + (row[lt + 1] - row[lt]) : 0;
    if (mine) {
        hard_sum_local(lt, xs, vs, sm, ssp, nbp, rowb, rowe, hc, a, jk);
        const double cr = crit_first(a, jk, hp, ssp[lt] ? hp.eta_s_sp : hp.eta_s);
        double d = hp.dt_max;
        while (d > cr && d > hp.dt_min) d *= 0.5;
        dt = d;
    }
    int64_t steps = 0;
    bool live = has;
    for (;;) {
        double tn = mine ? t + dt : INFINITY;
        for (int o = SUB / 2; o > 0; o >>= 1) tn = fmin(tn, __shfl_xor(tn, o));
        const double t_next = tn;
        if (live && !(t_next <= hp.t_end)) live = false;
        if (live && steps == hp.max_block_steps) {
            if (lt == 0) atomicOr(rb + (RB_HLIMIT - RB_HBAD), 1ull);
            live = false;
        }
        if (!__any(live)) break;
        if (live) ++steps;
        __syncthreads();   // the previous step's reads of xs and vs are done
        if (live && mine) {
            const double h = t_next - t;
            for (int q = 0; q < 3; ++q) {
                xs[3 * lt + q] = x[q] + v[q] * h + a[q] * (h * h / 2.0) + jk[q] * (h * h * h / 6.0);
                vs[3 * lt + q] = v[q] + a[q] * h + jk[q] * (h * h / 2.0);
            }
        }
        __syncthreads();
        const bool act = live && mine && t + dt == t_next;
        double a1[3] = {0.0, 0.0, 0.0}, j1[3] = {0.0, 0.0, 0.0};
        if (RP) {
            // the active members' entries of this sub-group, gathered in row order
            const bool par = in_lds;                 // the same on every lane of the sub-group
            const int len = (act && par) ? row[lt + 1] - row[lt] : 0;
            int incl = len;
            for (int o = 1; o < SUB; o <<= 1) {
                const int y = __shfl_up(incl, o, SUB);
                if (lt >= o) incl += y;
            }
            const int base = incl - len;
            const int n_act = __shfl(incl, SUB - 1, SUB);
            int16_t *ae = L.ae + NBCAP * sub, *aown = L.aown + NBCAP * sub;
            for (int q = 0; q < len; ++q) {
                ae[base + q] = (int16_t)(row[lt] + q);
                aown[base + q] = (int16_t)lt;
            }
            // chunks: as many as the longest sub-group of the wavefront needs
            int chunks = (n_act + SUB - 1) / SUB;
            for (int o = kWave / 2; o >= SUB; o >>= 1) chunks = max(chunks, __shfl_xor(chunks, o));
            __syncthreads();
            double *term = L.term + 6 * SUB * sub;
            for (int k = 0; k < chunks; ++k) {
                const int c0 = k * SUB, e = c0 + lt;
                if (e < n_act) {
                    double o[6];
                    pair_terms(aown[e], nb[ae[e]], xs, vs, sm, ssp, hc, o);
                    for (int q = 0; q < 6; ++q) term[6 * lt + q] = o[q];
                }
                __syncthreads();
                const int r0 = max(base, c0), r1 = min(base + len, c0 + SUB);
                for (int q = r0; q < r1; ++q) {
                    const double *o = term + 6 * (q - c0);
                    a1[0] += o[0];
                    a1[1] += o[1];
                    a1[2] += o[2];
                    j1[0] += o[3];
                    j1[1] += o[4];
                    j1[2] += o[5];
                }
                __syncthreads();
            }
            if (act && !par) hard_sum_local(lt, xs, vs, sm, ssp, nbp, rowb, rowe, hc, a1, j1);
        } else if (act) {
            hard_sum_local(lt, xs, vs, sm, ssp, nbp, rowb, rowe, hc, a1, j1);
        }
        if (act) {
            double a2[3], a3[3];
            const double h = dt;
            for (int q = 0; q < 3; ++q) {
                const double s2 = (-6.0 * (a[q] - a1[q]) - h * (4.0 * jk[q] + 2.0 * j1[q])) / (h * h);
                const double s3 = (12.0 * (a[q] - a1[q]) + 6.0 * h * (jk[q] + j1[q])) / (h * h * h);
                x[q] = xs[3 * lt + q] + s2 * (h * h * h * h / 24.0) + s3 * (h * h * h * h * h / 120.0);
                v[q] = vs[3 * lt + q] + s2 * (h * h * h / 6.0) + s3 * (h * h * h * h / 24.0);
                a[q] = a1[q];
                jk[q] = j1[q];
                a2[q] = s2 + s3 * h;
                a3[q] = s3;
            }
            t = t_next;
            ns += 1;
            const double cr = crit_full(a, jk, a2, a3, hp, ssp[lt] ? hp.eta_sp : hp.eta);
            double d = h;
            if (2.0 * d <= cr && 2.0 * d <= hp.dt_max && fmod(t, 2.0 * d) == 0.0)
                d = 2.0 * d;
            else
                while (d > cr && d > hp.dt_min) d *= 0.5;
            dt = d;
        }
    }
    unsigned long long my = 0;
    if (mine) {
        for (int q = 0; q < 3; ++q) {
            pos[3 * i + q] = x[q];
            vel[3 * i + q] = v[q];
        }
        if (nsteps_out) nsteps_out[i] = ns;
        my = (unsigned long long)ns;
    }
    unsigned long long mx = (unsigned long long)steps;
    for (int o = kWave / 2; o > 0; o >>= 1) {
        my += __shfl_xor(my, o);
        const unsigned long long y = __shfl_xor(mx, o);
        mx = y > mx ? y : mx;
    }
    if (tid == 0 && my) atomicAdd(rb + (RB_HSTEPS - RB_HBAD), my);
    if (tid == 0 && mx) atomicMax(rb + (RB_HMAXBLK - RB_HBAD), mx);
}

// The packings of one launch: n[k] components on 64 >> k lanes each, taken
// from `order` at ob[k]; blocks [bs[k - 1], bs[k]) run packing k (bs[-1] = 0).
constexpr int kPacks = 5;
struct PackPlan {
    int32_t n[kPacks];
    int32_t ob[kPacks];
    int32_t bs[kPacks];
};

template <bool RP>
__global__ __launch_bounds__(kWave) void k_hermite_pack(
    PackPlan pp, const int32_t *__restrict__ cl_beg, const int32_t *__restrict__ cl_end,
    const int32_t *__restrict__ order, const int32_t *__restrict__ mem,
    const int64_t *__restrict__ off, const int32_t *__restrict__ lidx,
    const double *__restrict__ mass, double *__restrict__ pos, double *__restrict__ vel,
    HardConsts hc, HermConsts hp, int32_t *__restrict__ nsteps_out, unsigned long long *rb) {
    __shared__ PackLds<RP> L;
    const int bx = blockIdx.x;
#define P3T_PACK_ARGS cl_beg, cl_end, order, pp.ob[K], mem, off, lidx, mass, pos, vel, hc, hp, \
                      nsteps_out, rb, L
    if (bx < pp.bs[0]) {
        constexpr int K = 0;
        hermite_sub<64, RP>(bx, pp.n[K], P3T_PACK_ARGS);
    } else if (bx < pp.bs[1]) {
        constexpr int K = 1;
        hermite_sub<32, RP>(bx - pp.bs[0], pp.n[K], P3T_PACK_ARGS);
    } else if (bx < pp.bs[2]) {
        constexpr int K = 2;
        hermite_sub<16, RP>(bx - pp.bs[1], pp.n[K], P3T_PACK_ARGS);
    } else if (bx < pp.bs[3]) {
        constexpr int K = 3;
        hermite_sub<8, RP>(bx - pp.bs[2], pp.n[K], P3T_PACK_ARGS);
    } else {
        constexpr int K = 4;
        hermite_sub<4, RP>(bx - pp.bs[3], pp.n[K], P3T_PACK_ARGS);
    }
#undef P3T_PACK_ARGS
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static PairKind pair_kind_of(double eps, double r_in, double r_out, int split) {
    PairKind q;
    q.eps = eps;
    q.r_in = r_in;
    q.r_out = r_out;
    q.gam = r_in / r_out;
    q.C = q.gam > 0.0 ? hk_C(q.gam) : 7.0 / 3.0;
    q.G1 = hk_G(1.0, q.gam);
    q.split = split;
    return q;
}

static HardConsts hard_consts(const p3t_params *p, const p3t_kinds *kd, int64_t n) {
    HardConsts hc;
    hc.k[0] = pair_kind_of(p->eps, p->r_in, p->r_out, 1);
    if (kd && kd->n_special > 0) {
        hc.k[1] = pair_kind_of(kd->eps_ns, kd->r_in_ns, kd->r_out_ns, 1);
        hc.k[2] = pair_kind_of(kd->eps_ss, kd->r_in_ss, kd->r_out_ss, kd->split_ss);
        hc.first_sp = n - kd->n_special;
    } else {
        hc.k[1] = hc.k[2] = hc.k[0];
        hc.first_sp = n;
    }
    return hc;
}

int validate_csr(p3t_ctx *ctx, int64_t n, const int64_t *off, const int32_t *idx) {
    int rc;
    if ((rc = ensure_readback(ctx))) return rc;
    int64_t *rb = ptr<int64_t>(ctx->readback);
    if ((rc = check_hip(ctx, hipMemsetAsync(rb + RB_HBAD, 0, sizeof(int64_t), ctx->stream), "memset")))
        return rc;
    if (idx)
        k_hard_validate<true><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, off, idx, rb + RB_HBAD);
    else
        k_hard_validate<false><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, off, idx, rb + RB_HBAD);
    if ((rc = check_hip(ctx, hipGetLastError(), "list check"))) return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_HBAD, rb + RB_HBAD, sizeof(int64_t),
                                            hipMemcpyDeviceToHost, ctx->stream), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    if (ctx->hpin[RB_HBAD])
        return set_error(ctx, P3T_EINVAL,
                         "neighbour lists malformed (bad offsets, index out of range, self entry, "
                         "not symmetric, or entries without an index array)");
    return P3T_OK;
}

// kAux streams (default priority) and kAux + 1 events for the concurrent
// classes, made on first use
int aux_streams(p3t_ctx *ctx) {
    if (ctx->aux_ready) return P3T_OK;
    int rc;
    for (int k = 0; k < kAux; ++k)
        if (!ctx->aux[k] &&
            (rc = check_hip(ctx, hipStreamCreateWithFlags(&ctx->aux[k], hipStreamNonBlocking),
                            "stream")))
            return rc;
    for (int k = 0; k < kAux + 1; ++k)
        if (!ctx->aev[k] &&
            (rc = check_hip(ctx, hipEventCreateWithFlags(&ctx->aev[k], hipEventDisableTiming),
                            "event")))
            return rc;
    ctx->aux_ready = 1;
    return P3T_OK;
}

// The components of >= 1024 members, on the context stream: block steps in
// batches of grid-wide launches until every component has reached t_end (or
// the block-step bound is reached, which ends the call with ELIMIT).
static int run_giant(p3t_ctx *ctx, int32_t n_giant, const int32_t *order, const int32_t *cl_beg,
                     const int32_t *cl_end, const int32_t *mem, const int32_t *slot,
                     const int64_t *off, const int32_t *idx, const double *mass, double *pos,
                     double *vel, const HardConsts &hc, const HermConsts &hp, const HermState &S,
                     int32_t *nsteps, unsigned long long *rbh) {
    int rc;
    hipStream_t st = ctx->stream;
    const size_t ints = 3 * (size_t)n_giant + 1, words = 2 * (size_t)n_giant;
    if ((rc = ensure(ctx, ctx->hard_giant, words * 8 + ints * 4 + 64))) return rc;
    unsigned long long *tmin = ptr<unsigned long long>(ctx->hard_giant);
    int32_t *gbeg = reinterpret_cast<int32_t *>(tmin + words), *gpre = gbeg + n_giant,
            *gsteps = gpre + n_giant + 1;
    k_giant_ranges<<<1, 1, 0, st>>>(order, cl_beg, cl_end, n_giant, gbeg, gpre, gsteps);
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_HGIANT, gpre + n_giant, sizeof(int32_t),
                                            hipMemcpyDeviceToHost, st), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
    GiantView gv{gbeg, gpre, n_giant, *reinterpret_cast<const int32_t *>(ctx->hpin + RB_HGIANT)};
    const unsigned blocks = blocks_for(gv.n_members > n_giant ? gv.n_members : n_giant, kGiantThreads);
    const unsigned wave_blocks = blocks_for(gv.n_members, kGiantThreads / 64);   // a wave per member
    k_giant_load<<<blocks, kGiantThreads, 0, st>>>(gv, mem, pos, vel, S, tmin);
    k_giant_first<<<blocks, kGiantThreads, 0, st>>>(gv, mem, slot, off, idx, mass, hc, hp, S);
    if ((rc = check_hip(ctx, hipGetLastError(), "giant components"))) return rc;
    std::vector<unsigned long long> last((size_t)n_giant);
    for (int64_t step = 0;;) {
        for (int q = 0; q < kGiantBatch; ++q, ++step) {
            const int b = (int)(step & 1);
            k_giant_min<<<blocks, kGiantThreads, 0, st>>>(gv, S, tmin, b);
            k_giant_predict<<<blocks, kGiantThreads, 0, st>>>(gv, hp, S, tmin, b, gsteps);
            k_giant_correct<<<wave_blocks, kGiantThreads, 0, st>>>(gv, mem, slot, off, idx, mass,
                                                                  hc, hp, S, tmin, b);
        }
        if ((rc = check_hip(ctx, hipGetLastError(), "giant step"))) return rc;
        // the minima of the batch's last step: every component done when all exceed t_end
        const int b = (int)((step - 1) & 1);
        if ((rc = check_hip(ctx, hipMemcpyAsync(last.data(), tmin + (size_t)b * n_giant,
                                                (size_t)n_giant * 8, hipMemcpyDeviceToHost, st),
                            "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
        bool done = true;
        for (unsigned long long w : last) {
            double t;
            memcpy(&t, &w, sizeof(t));
            if (t <= hp.t_end) done = false;
        }
        if (done) break;
        if (step >= hp.max_block_steps) {
            k_giant_store<<<blocks, kGiantThreads, 0, st>>>(gv, mem, S, pos, vel, nsteps, rbh);
            return set_error(ctx, P3T_ELIMIT, "a component reached the block-step limit");
        }
    }
    k_giant_store<<<blocks, kGiantThreads, 0, st>>>(gv, mem, S, pos, vel, nsteps, rbh);
    k_giant_maxsteps<<<blocks_for(n_giant, 256), 256, 0, st>>>(gsteps, n_giant, rbh);
    return check_hip(ctx, hipGetLastError(), "giant store");
}

int launch_hard_force(p3t_ctx *ctx, int64_t n, const double *pos, const double *vel,
                      const double *mass, const int64_t *off, const int32_t *idx,
                      const p3t_params *p, const p3t_kinds *kd, double *acc, double *jerk,
                      double *pot) {
    int rc;
    if ((rc = ensure_readback(ctx))) return rc;
    if ((rc = validate_csr(ctx, n, off, idx))) return rc;
    const HardConsts hc = hard_consts(p, kd, n);
    k_hard_force<<<blocks_for(n, kHardThreads), kHardThreads, 0, ctx->stream>>>(
        n, pos, vel, mass, off, idx, hc, acc, jerk, pot);
    return check_hip(ctx, hipGetLastError(), "hard force");
}

int launch_hermite(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass,
                   const int64_t *off, const int32_t *idx, const p3t_params *p,
                   const p3t_kinds *kd, const p3t_hermite_params *hpar, int32_t *nsteps,
                   p3t_hermite_stats *stats) {
    int rc;
    hipStream_t st = ctx->stream;
    if ((rc = ensure_readback(ctx))) return rc;
    if ((rc = aux_streams(ctx))) return rc;
    if ((rc = check_hip(ctx, hipEventRecord(ctx->ev[10], st), "event"))) return rc;
    if ((rc = validate_csr(ctx, n, off, idx))) return rc;
    // workspace: 7 per-particle int32 arrays, then per-slot state
    if ((rc = ensure(ctx, ctx->hard_ix, 7 * (size_t)(n + 1) * sizeof(int32_t)))) return rc;
    int32_t *par = ptr<int32_t>(ctx->hard_ix), *label = par + (n + 1), *ccount = label + (n + 1),
            *cfill = ccount + (n + 1), *cstart = cfill + (n + 1), *cid = cstart + (n + 1),
            *slotv = cid + (n + 1);
    int64_t *rb = ptr<int64_t>(ctx->readback);
    if ((rc = check_hip(ctx, hipMemsetAsync(rb + RB_HBAD, 0, 8 * sizeof(int64_t), st), "memset")))
        return rc;
    const unsigned nb = blocks_for(n, 256);
    k_cc_init<<<nb, 256, 0, st>>>(n, par, ccount, cfill);
    k_cc_union<<<nb, 256, 0, st>>>(n, off, idx, par, rb + RB_HBAD);
    k_cc_count<<<nb, 256, 0, st>>>(n, off, par, label, ccount);
    if ((rc = check_hip(ctx, hipGetLastError(), "components"))) return rc;
    if ((rc = scan_exclusive_i32(ctx, ccount, cstart, n, reinterpret_cast<int32_t *>(rb + RB_HNHARD))))
        return rc;
    k_cc_rootflag<<<nb, 256, 0, st>>>(n, ccount, cid);
    if ((rc = scan_exclusive_i32(ctx, cid, cid, n, reinterpret_cast<int32_t *>(rb + RB_HNCL))))
        return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_HBAD, rb + RB_HBAD, 3 * sizeof(int64_t),
                                            hipMemcpyDeviceToHost, st), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_HNNZ, off + n, sizeof(int64_t),
                                            hipMemcpyDeviceToHost, st), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
    if (ctx->hpin[RB_HBAD]) return set_error(ctx, P3T_ELIMIT, "component search did not settle");
    const int64_t n_hard = *reinterpret_cast<const int32_t *>(ctx->hpin + RB_HNHARD);
    const int64_t n_cl = *reinterpret_cast<const int32_t *>(ctx->hpin + RB_HNCL);
    const int64_t nnz = ctx->hpin[RB_HNNZ];
    // per-slot state: ten [m][3] and two [m] FP64 arrays; then int32 arrays:
    // steps [m], members [m], cluster begin/end/order [c], size buckets [64],
    // local list indices [nnz]
    const int64_t m = n_hard > 0 ? n_hard : 1, c = n_cl > 0 ? n_cl : 1;
    const size_t dbl = (size_t)m * 32;
    const size_t i32 = 2 * (size_t)m + 3 * (size_t)c + 64 + (size_t)(nnz > 0 ? nnz : 1);
    if ((rc = ensure(ctx, ctx->hard_state, dbl * sizeof(double) + i32 * sizeof(int32_t)))) return rc;
    double *base = ptr<double>(ctx->hard_state);
    HermState S;
    double **arr[10] = {&S.x, &S.v, &S.a, &S.j, &S.a2, &S.a3, &S.xp, &S.vp, &S.a1, &S.j1};
    for (int k = 0; k < 10; ++k) *arr[k] = base + (size_t)k * 3 * m;
    S.t = base + 30 * (size_t)m;
    S.dt = S.t + m;
    S.ns = reinterpret_cast<int32_t *>(base + dbl);
    int32_t *mem = S.ns + m, *cl_beg = mem + m, *cl_end = cl_beg + c, *order = cl_end + c;
    int32_t *bhist = order + c, *bfill = bhist + 32, *lidx = bfill + 32;
    if ((rc = check_hip(ctx, hipMemsetAsync(bhist, 0, 64 * sizeof(int32_t), st), "memset")))
        return rc;
    k_cc_place<<<nb, 256, 0, st>>>(n, label, cstart, cfill, mem, slotv, pos, vel, hpar->dt_soft);
    k_cc_clusters<<<nb, 256, 0, st>>>(n, ccount, cstart, cid, cl_beg, cl_end, bhist,
                                      reinterpret_cast<unsigned long long *>(rb + RB_HMAXCL));
    k_cc_classes<<<1, 1, 0, st>>>(bhist, reinterpret_cast<int32_t *>(rb + RB_HCLASS),
                                  reinterpret_cast<int32_t *>(rb + RB_HSUB));
    k_cc_bucket_scan<<<1, 1, 0, st>>>(bhist);
    if (nsteps) {
        // isolated particles take no Hermite step
        if ((rc = check_hip(ctx, hipMemsetAsync(nsteps, 0, n * sizeof(int32_t), st), "memset")))
            return rc;
    }
    if (n_cl > 0) {
        k_cc_order<<<blocks_for(n_cl, 256), 256, 0, st>>>(n_cl, cl_beg, cl_end, bfill, bhist, order);
        k_hard_local<<<nb, 256, 0, st>>>(n, off, idx, label, cid, cl_beg, slotv, lidx);
        if ((rc = check_hip(ctx, hipGetLastError(), "components"))) return rc;
        if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_HCLASS, rb + RB_HCLASS,
                                                (RB_HSUB + 3 - RB_HCLASS) * sizeof(int64_t),
                                                hipMemcpyDeviceToHost, st), "readback")))
            return rc;
        if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
        int32_t cls[kNumClasses], sub[kPacks];
        memcpy(cls, ctx->hpin + RB_HCLASS, sizeof(cls));
        memcpy(sub, ctx->hpin + RB_HSUB, sizeof(sub));
        if (sub[0] + sub[1] + sub[2] + sub[3] + sub[4] != cls[3])
            return set_error(ctx, P3T_EHIP, "component classes do not add up");
        HermConsts hc2;
        hc2.t_end = hpar->dt_soft;
        hc2.dt_max = hpar->dt_max;
        hc2.dt_min = ldexp(hpar->dt_max, -kMaxDtLevel);
        hc2.eta = hpar->eta;
        hc2.eta_s = hpar->eta_s;
        hc2.a0 = hpar->a0;
        const bool sp = kd && kd->n_special > 0;
        hc2.eta_sp = sp ? kd->eta_sp : hpar->eta;
        hc2.eta_s_sp = sp ? kd->eta_s_sp : hpar->eta_s;
        hc2.max_block_steps = hpar->max_block_steps > 0 ? hpar->max_block_steps : (1LL << 22);
        const HardConsts hk = hard_consts(p, kd, n);
        unsigned long long *rbh = reinterpret_cast<unsigned long long *>(rb + RB_HBAD);
        // fork: the three LDS classes on their own streams, the largest
        // components on the context stream
        if ((rc = check_hip(ctx, hipEventRecord(ctx->aev[0], st), "event"))) return rc;
        for (int k = 0; k < kAux; ++k)
            if ((rc = check_hip(ctx, hipStreamWaitEvent(ctx->aux[k], ctx->aev[0], 0), "wait")))
                return rc;
        int32_t base_k = cls[0];
        if (cls[1] > 0)
            k_hermite_lds<512, 2, 8192, 512><<<(unsigned)cls[1], 512, 0, ctx->aux[0]>>>(
                cl_beg, cl_end, order, base_k, mem, off, lidx, mass, pos, vel, hk, hc2, nsteps, rbh);
        base_k += cls[1];
        if (cls[2] > 0)
            k_hermite_lds<256, 1, 4096, 512><<<(unsigned)cls[2], 256, 0, ctx->aux[1]>>>(
                cl_beg, cl_end, order, base_k, mem, off, lidx, mass, pos, vel, hk, hc2, nsteps, rbh);
        base_k += cls[2];
        if (cls[3] > 0) {
            // the packings of 16 to 64 lanes (components of 8 to 63 members) with
            // their terms spread over the lanes, on the context stream; those of
            // 4 and 8 lanes on their own stream
            PackPlan wide{}, narrow{};
            int32_t ob = base_k, nw = 0, nn = 0;
            for (int k = 0; k < kPacks; ++k) {
                const int per = 1 << k;   // components per block: 1, 2, 4, 8, 16
                const int32_t blocks = (sub[k] + per - 1) / per;
                PackPlan &pl = k < 3 ? wide : narrow;
                int32_t &nb = k < 3 ? nw : nn;
                pl.n[k] = sub[k];
                pl.ob[k] = ob;
                nb += blocks;
                ob += sub[k];
                for (int q = k; q < kPacks; ++q) pl.bs[q] = nb;
            }
            if (nn > 0)
                k_hermite_pack<false><<<(unsigned)nn, kWave, 0, ctx->aux[2]>>>(
                    narrow, cl_beg, cl_end, order, mem, off, lidx, mass, pos, vel, hk, hc2, nsteps, rbh);
            if (nw > 0)
                k_hermite_pack<true><<<(unsigned)nw, kWave, 0, st>>>(
                    wide, cl_beg, cl_end, order, mem, off, lidx, mass, pos, vel, hk, hc2, nsteps, rbh);
        }

        if ((rc = check_hip(ctx, hipGetLastError(), "hermite"))) return rc;
        if (cls[0] > 0 && (rc = run_giant(ctx, cls[0], order, cl_beg, cl_end, mem, slotv, off, idx,
                                          mass, pos, vel, hk, hc2, S, nsteps, rbh)))
            return rc;
        for (int k = 0; k < kAux; ++k) {
            if ((rc = check_hip(ctx, hipEventRecord(ctx->aev[1 + k], ctx->aux[k]), "event"))) return rc;
            if ((rc = check_hip(ctx, hipStreamWaitEvent(st, ctx->aev[1 + k], 0), "wait"))) return rc;
        }
    }
    if ((rc = check_hip(ctx, hipGetLastError(), "hermite"))) return rc;
    if ((rc = check_hip(ctx, hipEventRecord(ctx->ev[11], st), "event"))) return rc;
    if ((rc = check_hip(ctx, hipMemcpyAsync(ctx->hpin + RB_HMAXCL, rb + RB_HMAXCL, 4 * sizeof(int64_t),
                                            hipMemcpyDeviceToHost, st), "readback")))
        return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(st), "sync"))) return rc;
    if (stats) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev[10], ctx->ev[11]);
        stats->n_hard = n_hard;
        stats->n_clusters = n_cl;
        stats->max_cluster = ctx->hpin[RB_HMAXCL];
        stats->steps = ctx->hpin[RB_HSTEPS];
        stats->max_block_steps = ctx->hpin[RB_HMAXBLK];
        stats->ms = ms;
    }
    if (ctx->hpin[RB_HLIMIT])
        return set_error(ctx, P3T_ELIMIT, "a component reached the block-step limit");
    return P3T_OK;
}

}  // namespace p3t
