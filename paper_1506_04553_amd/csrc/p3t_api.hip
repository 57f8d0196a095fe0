// p3t_api.hip -- the C ABI (include/p3t.h): context, workspaces, parameter
// validation, stage sequencing, statistics and inspection.
#include <math.h>
#include <stdlib.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "internal.h"

using namespace p3t;

// Static workspace of p3t_long_force_vjp_noalloc: one array per device, part
// of the library's code object, so that call allocates nothing.  Host code
// never uses the array's name as an address: p3t_create resolves its device
// address once per device (with that device current) and every use goes
// through that pointer.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

namespace p3t {

int set_error(p3t_ctx *ctx, int status, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return status;
}

int check_hip(p3t_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return P3T_OK;
    return set_error(ctx, P3T_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int ensure(p3t_ctx *ctx, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.p && b.bytes >= bytes) return P3T_OK;
    release(ctx, b);
    size_t cap = bytes + bytes / 8;   // headroom: sizes drift from step to step
    cap = (cap + 255) & ~(size_t)255;
    void *p = nullptr;
    if (ctx->alloc) {
        p = ctx->alloc(cap, ctx->user);
        if (!p) return set_error(ctx, P3T_ENOMEM, "allocator returned NULL for %zu bytes", cap);
    } else {
        hipError_t e = hipMalloc(&p, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ctx, P3T_ENOMEM, "hipMalloc(%zu): %s", cap, hipGetErrorString(e));
        }
    }
    b.p = p;
    b.bytes = cap;
    return P3T_OK;
}

int ensure_readback(p3t_ctx *ctx) {
    if (ctx->readback.p) return P3T_OK;
    int rc = ensure(ctx, ctx->readback, kReadbackWords * sizeof(int64_t));
    if (rc) return rc;
    // cleared once, when allocated: the neighbour search's tagged words rely on it
    return check_hip(ctx, hipMemsetAsync(ctx->readback.p, 0, ctx->readback.bytes, ctx->stream),
                     "memset");
}

void release(p3t_ctx *ctx, DevBuf &b) {
    if (!b.p) return;
    if (ctx->free_) ctx->free_(b.p, ctx->user);
    else (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

// Constants of K and W for gamma = r_in / r_out (Section 2.1, G with
// denominator (gamma - 1)^7).
Changeover make_changeover(double r_in, double r_out) {
    Changeover c{};
    const double g = r_in / r_out;
    c.r_out = r_out;
    c.inv_rout = 1.0 / r_out;
    c.gamma = g;
    c.inv_1mg = 1.0 / (1.0 - g);
    const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g, g7 = g6 * g;
    const double D = pow(g - 1.0, 7);
    const double glog = (g > 0.0) ? g3 * log(g) : 0.0;
    c.C = 7.0 * (g6 - 9.0 * g5 + 45.0 * g4 - 60.0 * glog - 45.0 * g2 + 9.0 * g - 1.0) / (3.0 * D);
    const double a7 = -10.0 / 3.0, a6 = 14.0 * (g + 1.0), a5 = -21.0 * (g2 + 3.0 * g + 1.0),
                 a4 = 35.0 * (g3 + 9.0 * g2 + 9.0 * g + 1.0) / 3.0,
                 a3 = -70.0 * (g3 + 3.0 * g2 + g), a2 = 210.0 * (g3 + g2), al = -140.0 * g3,
                 a0 = g7 - 7.0 * g6 + 21.0 * g5 - 35.0 * g4;
    const double G1 = (a7 + a6 + a5 + a4 + a3 + a2 + a0) / D;
    // W/y = G(y)/y + 1 - G(1)
    c.w[6] = a7 / D;
    c.w[5] = a6 / D;
    c.w[4] = a5 / D;
    c.w[3] = a4 / D;
    c.w[2] = a3 / D;
    c.w[1] = a2 / D;
    c.w[0] = 1.0 - G1;
    c.wl = al / D;
    c.wm = a0 / D;
    return c;
}

}  // namespace p3t

static const char *kStatus[] = {"ok", "invalid argument", "out of device memory",
                                "capacity exceeded", "call out of order", "HIP error",
                                "iteration limit reached"};

extern "C" const char *p3t_status_string(int s) {
    if (s <= 0 && s >= -6) return kStatus[-s];
    return "unknown status";
}

extern "C" const char *p3t_last_error(p3t_ctx *ctx) { return ctx ? ctx->err : "null context"; }

extern "C" int p3t_check_params(const p3t_params *p) {
    if (!p) return P3T_EINVAL;
    const double v[5] = {p->eps, p->r_in, p->r_out, p->theta, p->r_search};
    for (double d : v)
        if (!isfinite(d)) return P3T_EINVAL;
    if (p->eps < 0.0 || !(p->r_out > 0.0) || p->r_in < 0.0 || !(p->r_in < p->r_out)) return P3T_EINVAL;
    if (p->theta < 0.0 || !(p->r_search > 0.0)) return P3T_EINVAL;
    if (p->n_leaf < 1 || p->n_crit < p->n_leaf) return P3T_EINVAL;
    if (p->use_quadrupole != 0 && p->use_quadrupole != 1) return P3T_EINVAL;
    if (p->precision != P3T_PREC_FP64 && p->precision != P3T_PREC_MIXED) return P3T_EINVAL;
    return P3T_OK;
}

extern "C" int p3t_create(p3t_ctx **out, int device, void *hip_stream, p3t_alloc_fn alloc,
                          p3t_free_fn free_, void *alloc_user) {
    if (!out) return P3T_EINVAL;
    *out = nullptr;
    if ((alloc == nullptr) != (free_ == nullptr)) return P3T_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return P3T_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) return P3T_EHIP;
    p3t_ctx *ctx = new (std::nothrow) p3t_ctx();
    if (!ctx) return P3T_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->alloc = alloc;
    ctx->free_ = free_;
    ctx->user = alloc_user;
    // P3T_WALK_LDS_STACK=k (k >= 64) caps the walk's on-chip stack at k entries
    if (const char *ev = getenv("P3T_WALK_LDS_STACK")) ctx->walk_lds_cap = atoi(ev);
    // P3T_GROUPS_GENERIC=1 takes the group compaction of the largest inputs
    // (a plain scan of the flags, then the records) at any size
    if (const char *ev = getenv("P3T_GROUPS_GENERIC")) ctx->groups_generic = atoi(ev) > 0;
    if (device >= kMaxDevices) {
        delete ctx;
        return P3T_EINVAL;
    }
    {
        // the static workspace's address on this device (the device is current)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *sp = nullptr;
            if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
                (void)hipGetLastError();
                delete ctx;
                return P3T_EHIP;
            }
            g_scratch_ptr[device] = sp;
        }
        ctx->scratch = g_scratch_ptr[device];
    }
    // coherent: some kernels write their few result words straight into it,
    // read by the host after the stream's synchronisation
    hipError_t e = hipHostMalloc((void **)&ctx->hpin, 64 * sizeof(int64_t), hipHostMallocCoherent);
    for (int k = 0; k < 12 && e == hipSuccess; ++k) e = hipEventCreate(&ctx->ev[k]);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_lists, hipEventDisableTiming);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&ctx->ev_sync[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        p3t_destroy(ctx);
        return P3T_EHIP;
    }
    *out = ctx;
    return P3T_OK;
}

extern "C" void p3t_destroy(p3t_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    DevBuf *bufs[] = {&ctx->root, &ctx->keys[0], &ctx->keys[1], &ctx->vals[0], &ctx->vals[1],
                      &ctx->hist, &ctx->histc, &ctx->rs_tot, &ctx->xm, &ctx->xm_in, &ctx->lvlrange,
                      &ctx->tblk, &ctx->tblk_off, &ctx->gtile, &ctx->node_level, &ctx->node_first,
                      &ctx->node_count, &ctx->node_child, &ctx->node_nchild, &ctx->node_parent,
                      &ctx->node_prefix, &ctx->node_S, &ctx->node_walk, &ctx->node_mp, &ctx->gflag,
                      &ctx->gscan, &ctx->grp, &ctx->cnt, &ctx->off, &ctx->c_idx, &ctx->p_idx,
                      &ctx->n_idx, &ctx->wstack, &ctx->readback, &ctx->scan_tmp,
                      &ctx->nbr_cnt, &ctx->nbr_slots, &ctx->nbr_scan, &ctx->vjp_gx, &ctx->vjp_gm, &ctx->vjp_cell, &ctx->bbox,
                      &ctx->seg_end, &ctx->gorder, &ctx->grank, &ctx->ghist, &ctx->hard_ix,
                      &ctx->hard_state, &ctx->step_off, &ctx->step_idx, &ctx->step_off2,
                      &ctx->step_idx2, &ctx->kinds_cnt, &ctx->hard_giant};
    for (DevBuf *b : bufs) release(ctx, *b);
    if (ctx->hpin) (void)hipHostFree(ctx->hpin);
    for (int k = 0; k < 12; ++k)
        if (ctx->ev[k]) (void)hipEventDestroy(ctx->ev[k]);
    for (int k = 0; k < 4; ++k)
        if (ctx->aux[k]) {
            (void)hipStreamSynchronize(ctx->aux[k]);
            (void)hipStreamDestroy(ctx->aux[k]);
        }
    for (int k = 0; k < 5; ++k)
        if (ctx->aev[k]) (void)hipEventDestroy(ctx->aev[k]);
    if (ctx->ev_lists) (void)hipEventDestroy(ctx->ev_lists);
    for (int k = 0; k < 2; ++k)
        if (ctx->ev_sync[k]) (void)hipEventDestroy(ctx->ev_sync[k]);
    delete ctx;
}

enum { EV_BUILD = 0, EV_FORCE = 2, EV_NBR = 4, EV_VJP = 6, EV_WALK = 8 };

static int mark(p3t_ctx *ctx, int ev) {
    return check_hip(ctx, hipEventRecord(ctx->ev[ev], ctx->stream), "event record");
}

static int elapsed_ms(p3t_ctx *ctx, int pair, double *out) {
    float ms = 0.f;
    int rc = check_hip(ctx, hipEventSynchronize(ctx->ev[pair + 1]), "event sync");
    if (rc) return rc;
    rc = check_hip(ctx, hipEventElapsedTime(&ms, ctx->ev[pair], ctx->ev[pair + 1]), "event time");
    if (rc) return rc;
    *out = ms;
    return P3T_OK;
}

extern "C" int p3t_build_tree(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                              const p3t_params *p) {
    if (!ctx) return P3T_EINVAL;
    if (n < 1 || n > (int64_t)INT32_MAX - 1 || !pos || !mass)
        return set_error(ctx, P3T_EINVAL, "bad particle arrays (n = %lld)", (long long)n);
    if (p3t_check_params(p) != P3T_OK) return set_error(ctx, P3T_EINVAL, "invalid parameters");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    ctx->built = 0;
    ctx->lists_released = 0;
    ctx->n = n;
    ctx->prm = *p;
    ctx->chg = make_changeover(p->r_in, p->r_out);
    if ((rc = ensure_readback(ctx))) return rc;
    if ((rc = mark(ctx, EV_BUILD))) return rc;
    if ((rc = build_sorted(ctx, pos, mass, n))) return rc;
    if ((rc = build_topology(ctx, n))) return rc;
    if ((rc = build_moments(ctx))) return rc;
    if ((rc = build_groups(ctx))) return rc;
    if ((rc = mark(ctx, EV_WALK))) return rc;
    if ((rc = build_lists(ctx, true))) return rc;
    if ((rc = mark(ctx, EV_WALK + 1))) return rc;
    if ((rc = mark(ctx, EV_BUILD + 1))) return rc;
    ctx->ms_build = ctx->ms_walk = -1.0;   // resolved lazily by p3t_get_stats
    ctx->ms_force = ctx->ms_nbr = ctx->ms_vjp = 0.0;
    ctx->built = 1;
    return P3T_OK;
}

// the lists of the current build, walked again if they were released
static int ensure_lists(p3t_ctx *ctx) {
    if (!ctx->lists_released) return P3T_OK;
    const int rc = build_lists(ctx, false);
    if (rc == P3T_OK) ctx->lists_released = 0;
    return rc;
}

extern "C" int p3t_release_lists(p3t_ctx *ctx) {
    if (!ctx) return P3T_EINVAL;
    if (!ctx->built) return set_error(ctx, P3T_ESTATE, "p3t_release_lists before p3t_build_tree");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    // the stream's work may still read the lists: free only after it drains
    if ((rc = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    release(ctx, ctx->c_idx);
    release(ctx, ctx->p_idx);
    release(ctx, ctx->n_idx);
    ctx->lists_released = 1;
    return P3T_OK;
}

extern "C" int p3t_long_force(p3t_ctx *ctx, double *acc, double *pot) {
    if (!ctx) return P3T_EINVAL;
    if (!ctx->built) return set_error(ctx, P3T_ESTATE, "p3t_long_force before p3t_build_tree");
    if (!acc) return set_error(ctx, P3T_EINVAL, "acc is NULL");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    if ((rc = ensure_lists(ctx))) return rc;
    if ((rc = mark(ctx, EV_FORCE))) return rc;
    if ((rc = launch_force(ctx, acc, pot))) return rc;
    if ((rc = mark(ctx, EV_FORCE + 1))) return rc;
    ctx->ms_force = -1.0;   // resolved lazily by p3t_get_stats
    return P3T_OK;
}

extern "C" int p3t_neighbors(p3t_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *nnz) {
    if (!ctx) return P3T_EINVAL;
    if (!ctx->built) return set_error(ctx, P3T_ESTATE, "p3t_neighbors before p3t_build_tree");
    if (!offsets || !nnz || cap < 0 || (cap > 0 && !idx))
        return set_error(ctx, P3T_EINVAL, "bad neighbour buffers");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    if ((rc = ensure_lists(ctx))) return rc;
    // timed on the search's own stream (the packing into the caller's arrays,
    // on the context's stream, is not included)
    if ((rc = launch_neighbors(ctx, offsets, idx, cap, nnz, ctx->ev[EV_NBR], ctx->ev[EV_NBR + 1])))
        return rc;
    ctx->ms_nbr = -1.0;
    return P3T_OK;
}

extern "C" int p3t_long_force_vjp(p3t_ctx *ctx, const double *w, const double *c, double *gpos,
                                  double *gmass) {
    if (!ctx) return P3T_EINVAL;
    if (!ctx->built) return set_error(ctx, P3T_ESTATE, "p3t_long_force_vjp before p3t_build_tree");
    if (!w || !gpos || !gmass) return set_error(ctx, P3T_EINVAL, "bad VJP buffers");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    if ((rc = ensure_lists(ctx))) return rc;
    if ((rc = mark(ctx, EV_VJP))) return rc;
    if ((rc = launch_vjp(ctx, w, c, gpos, gmass))) return rc;
    if ((rc = mark(ctx, EV_VJP + 1))) return rc;
    ctx->ms_vjp = -1.0;
    return P3T_OK;
}

extern "C" int p3t_long_force_vjp_noalloc(p3t_ctx *ctx, const double *w, const double *c,
                                          double *gpos, double *gmass) {
    if (!ctx) return P3T_EINVAL;
    if (!ctx->built)
        return set_error(ctx, P3T_ESTATE, "p3t_long_force_vjp_noalloc before p3t_build_tree");
    // walking the tree again would allocate the lists
    if (ctx->lists_released)
        return set_error(ctx, P3T_ESTATE,
                         "p3t_long_force_vjp_noalloc needs the build's lists; they were released");
    if (!w || !gpos || !gmass) return set_error(ctx, P3T_EINVAL, "bad VJP buffers");
    const int64_t n = ctx->n, nn = ctx->n_nodes;
    // gx [3 n], gm [n], cell adjoints [10 n_nodes], each 256-byte aligned
    const size_t a = 256 / sizeof(double);
    const size_t ngx = (3 * (size_t)n + a - 1) / a * a, ngm = ((size_t)n + a - 1) / a * a;
    const size_t need = (ngx + ngm + 10 * (size_t)nn) * sizeof(double);
    if (need > kScratchBytes)
        return set_error(ctx, P3T_ECAPACITY,
                         "p3t_long_force_vjp_noalloc needs %zu bytes of workspace for n = %lld and "
                         "%lld nodes (4 n + 10 n_nodes doubles); its static workspace holds %zu",
                         need, (long long)n, (long long)nn, kScratchBytes);
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    double *gx = static_cast<double *>(ctx->scratch), *gm = gx + ngx, *cadj = gm + ngm;
    if ((rc = mark(ctx, EV_VJP))) return rc;
    if ((rc = launch_vjp_ws(ctx, w, c, gpos, gmass, gx, gm, cadj))) return rc;
    if ((rc = mark(ctx, EV_VJP + 1))) return rc;
    ctx->ms_vjp = -1.0;
    return P3T_OK;
}

extern "C" int p3t_kick_drift(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *acc,
                              double dt_kick, double dt_drift) {
    if (!ctx || n < 0 || (n > 0 && (!pos || !vel || !acc)) || !isfinite(dt_kick) || !isfinite(dt_drift))
        return ctx ? set_error(ctx, P3T_EINVAL, "bad kick/drift arguments") : P3T_EINVAL;
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    return launch_kick_drift(ctx, n, pos, vel, acc, dt_kick, dt_drift);
}

static bool hermite_params_ok(const p3t_hermite_params *hp) {
    if (!hp) return false;
    const double v[5] = {hp->dt_soft, hp->dt_max, hp->eta, hp->eta_s, hp->a0};
    for (double d : v)
        if (!isfinite(d)) return false;
    if (!(hp->dt_soft > 0.0) || !(hp->dt_max > 0.0) || hp->dt_max > hp->dt_soft) return false;
    if (fmod(hp->dt_soft, hp->dt_max) != 0.0) return false;
    return hp->eta > 0.0 && hp->eta_s > 0.0 && hp->a0 >= 0.0 && hp->max_block_steps >= 0;
}

// particle kinds: NULL or n_special = 0 mean one kind
static bool kinds_ok(const p3t_kinds *kd, int64_t n) {
    if (!kd) return true;
    if (kd->n_special < 0 || kd->n_special > n) return false;
    if (kd->n_special == 0) return true;
    const double v[10] = {kd->r_in_ns, kd->r_out_ns, kd->r_search_ns, kd->eps_ns, kd->r_in_ss,
                          kd->r_out_ss, kd->r_search_ss, kd->eps_ss, kd->eta_sp, kd->eta_s_sp};
    for (double d : v)
        if (!isfinite(d)) return false;
    if (kd->r_in_ns < 0.0 || !(kd->r_in_ns < kd->r_out_ns) || !(kd->r_search_ns > 0.0) ||
        kd->eps_ns < 0.0 || kd->eps_ss < 0.0)
        return false;
    if (kd->split_ss != 0 && kd->split_ss != 1) return false;
    if (kd->split_ss &&
        (kd->r_in_ss < 0.0 || !(kd->r_in_ss < kd->r_out_ss) || !(kd->r_search_ss > 0.0)))
        return false;
    return kd->eta_sp > 0.0 && kd->eta_s_sp > 0.0;
}

static bool has_special(const p3t_kinds *kd) { return kd && kd->n_special > 0; }

extern "C" int p3t_hard_force(p3t_ctx *ctx, int64_t n, const double *pos, const double *vel,
                              const double *mass, const int64_t *offsets, const int32_t *idx,
                              const p3t_params *p, const p3t_kinds *kinds, double *acc,
                              double *jerk, double *pot) {
    if (!ctx) return P3T_EINVAL;
    if (n < 1 || n > INT32_MAX || !pos || !vel || !mass || !offsets || !acc || !jerk ||
        p3t_check_params(p) != P3T_OK || !kinds_ok(kinds, n))
        return set_error(ctx, P3T_EINVAL, "bad hard-force arguments");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    return launch_hard_force(ctx, n, pos, vel, mass, offsets, idx, p, kinds, acc, jerk, pot);
}

extern "C" int p3t_hermite_hard(p3t_ctx *ctx, int64_t n, double *pos, double *vel,
                                const double *mass, const int64_t *offsets, const int32_t *idx,
                                const p3t_params *p, const p3t_kinds *kinds,
                                const p3t_hermite_params *hp, int32_t *nsteps,
                                p3t_hermite_stats *stats) {
    if (!ctx) return P3T_EINVAL;
    if (n < 1 || n > INT32_MAX || !pos || !vel || !mass || !offsets ||
        p3t_check_params(p) != P3T_OK || !hermite_params_ok(hp) || !kinds_ok(kinds, n))
        return set_error(ctx, P3T_EINVAL, "bad Hermite arguments");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    return launch_hermite(ctx, n, pos, vel, mass, offsets, idx, p, kinds, hp, nsteps, stats);
}

extern "C" int p3t_kinds_soft(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                              const p3t_params *p, const p3t_kinds *kinds, double *acc,
                              double *pot) {
    if (!ctx) return P3T_EINVAL;
    if (n < 1 || !pos || !mass || !acc || p3t_check_params(p) != P3T_OK || !kinds_ok(kinds, n))
        return set_error(ctx, P3T_EINVAL, "bad kinds-soft arguments");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    return launch_kinds_soft(ctx, n, pos, mass, p, kinds, acc, pot);
}

extern "C" int p3t_kinds_neighbors(p3t_ctx *ctx, int64_t n, const double *pos,
                                   const p3t_kinds *kinds, const int64_t *nn_off,
                                   const int32_t *nn_idx, int64_t *off, int32_t *idx, int64_t cap,
                                   int64_t *nnz) {
    if (!ctx) return P3T_EINVAL;
    if (n < 1 || n > INT32_MAX || !pos || !kinds || !kinds_ok(kinds, n) || !nn_off || !off ||
        !nnz || cap < 0 || (cap > 0 && !idx))
        return set_error(ctx, P3T_EINVAL, "bad kinds-neighbour arguments");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    // the normal particles' lists come from the caller: check them first
    const int64_t n_normal = n - kinds->n_special;
    if (n_normal > 0 && (rc = validate_csr(ctx, n_normal, nn_off, nn_idx))) return rc;
    return launch_kinds_neighbors(ctx, n, pos, kinds, nn_off, nn_idx, off, idx, cap, nnz);
}

// neighbour lists of the current build into buf_off/buf_idx, grown as needed
static int step_neighbors(p3t_ctx *ctx, int64_t n_rows, int64_t *nnz) {
    int rc;
    // the search reads the build's near lists: walk again if they were released
    if ((rc = ensure_lists(ctx))) return rc;
    if ((rc = ensure(ctx, ctx->step_off, (size_t)(n_rows + 1) * sizeof(int64_t)))) return rc;
    int64_t cap = (int64_t)(ctx->step_idx.bytes / sizeof(int32_t));
    if (cap < 1) {
        if ((rc = ensure(ctx, ctx->step_idx, (size_t)n_rows * sizeof(int32_t)))) return rc;
        cap = (int64_t)(ctx->step_idx.bytes / sizeof(int32_t));
    }
    rc = launch_neighbors(ctx, ptr<int64_t>(ctx->step_off), ptr<int32_t>(ctx->step_idx), cap, nnz,
                          nullptr, nullptr);
    if (rc == P3T_ECAPACITY) {
        if ((rc = ensure(ctx, ctx->step_idx, (size_t)*nnz * sizeof(int32_t)))) return rc;
        rc = launch_neighbors(ctx, ptr<int64_t>(ctx->step_off), ptr<int32_t>(ctx->step_idx), *nnz,
                              nnz, nullptr, nullptr);
    }
    return rc;
}

extern "C" int p3t_step(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass,
                        double *acc, double *pot, const p3t_params *p, const p3t_kinds *kinds,
                        const p3t_hermite_params *hp, p3t_hermite_stats *stats) {
    if (!ctx) return P3T_EINVAL;
    if (!pos || !vel || !mass || !acc || p3t_check_params(p) != P3T_OK || !hermite_params_ok(hp) ||
        n < 1 || !kinds_ok(kinds, n))
        return set_error(ctx, P3T_EINVAL, "bad step arguments");
    // Section 2.2: the neighbour radius is r_cut plus a buffer, so every pair
    // with a hard part (s < r_out) is on the lists the step integrates; a
    // smaller radius would drop the (1 - K) force of the pairs between h and r_out
    if (p->r_search < p->r_out ||
        (has_special(kinds) && (kinds->r_search_ns < kinds->r_out_ns ||
                                (kinds->split_ss && kinds->r_search_ss < kinds->r_out_ss))))
        return set_error(ctx, P3T_EINVAL, "p3t_step needs r_search >= r_out for every kind of pair");
    const int64_t n_sp = has_special(kinds) ? kinds->n_special : 0, n_tree = n - n_sp;
    if (!ctx->built || ctx->n != n_tree || n_tree < 1)
        return set_error(ctx, P3T_ESTATE, "p3t_step needs a build of the normal particles");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    const double half = 0.5 * hp->dt_soft;
    if ((rc = launch_kick_drift(ctx, n, pos, vel, acc, half, 0.0))) return rc;
    int64_t nnz = 0;
    if ((rc = step_neighbors(ctx, n_tree, &nnz))) return rc;
    ctx->nnz = nnz;
    const int64_t *hoff = ptr<int64_t>(ctx->step_off);
    const int32_t *hidx = ptr<int32_t>(ctx->step_idx);
    if (n_sp > 0) {
        // merge in the pairs with special particles
        if ((rc = ensure(ctx, ctx->step_off2, (size_t)(n + 1) * sizeof(int64_t)))) return rc;
        int64_t cap = (int64_t)(ctx->step_idx2.bytes / sizeof(int32_t));
        if (cap < nnz + 1) {
            if ((rc = ensure(ctx, ctx->step_idx2, (size_t)(nnz + 1) * sizeof(int32_t)))) return rc;
            cap = (int64_t)(ctx->step_idx2.bytes / sizeof(int32_t));
        }
        int64_t tot = 0;
        rc = launch_kinds_neighbors(ctx, n, pos, kinds, hoff, hidx, ptr<int64_t>(ctx->step_off2),
                                    ptr<int32_t>(ctx->step_idx2), cap, &tot);
        if (rc == P3T_ECAPACITY) {
            if ((rc = ensure(ctx, ctx->step_idx2, (size_t)tot * sizeof(int32_t)))) return rc;
            rc = launch_kinds_neighbors(ctx, n, pos, kinds, hoff, hidx,
                                        ptr<int64_t>(ctx->step_off2), ptr<int32_t>(ctx->step_idx2),
                                        tot, &tot);
        }
        if (rc) return rc;
        hoff = ptr<int64_t>(ctx->step_off2);
        hidx = ptr<int32_t>(ctx->step_idx2);
    }
    if ((rc = launch_hermite(ctx, n, pos, vel, mass, hoff, hidx, p, kinds, hp, nullptr, stats)))
        return rc;
    if ((rc = p3t_build_tree(ctx, n_tree, pos, mass, p))) return rc;
    if ((rc = p3t_long_force(ctx, acc, pot))) return rc;
    if (n_sp > 0 && (rc = launch_kinds_soft(ctx, n, pos, mass, p, kinds, acc, pot))) return rc;
    return launch_kick_drift(ctx, n, pos, vel, acc, half, 0.0);
}

extern "C" int p3t_direct(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                          const p3t_params *p, int mode, double *acc, double *pot) {
    if (!ctx) return P3T_EINVAL;
    if (n < 1 || !pos || !mass || !acc || p3t_check_params(p) != P3T_OK ||
        (mode != P3T_DIRECT_NEWTON && mode != P3T_DIRECT_SOFT && mode != P3T_DIRECT_HARD))
        return set_error(ctx, P3T_EINVAL, "bad direct-sum arguments");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    return launch_direct(ctx, n, pos, mass, p, mode, acc, pot);
}

extern "C" int p3t_get_stats(p3t_ctx *ctx, p3t_stats *out) {
    if (!ctx || !out) return P3T_EINVAL;
    if (ctx->ms_build < 0.0 && elapsed_ms(ctx, EV_BUILD, &ctx->ms_build)) ctx->ms_build = 0.0;
    if (ctx->ms_walk < 0.0 && elapsed_ms(ctx, EV_WALK, &ctx->ms_walk)) ctx->ms_walk = 0.0;
    if (ctx->ms_force < 0.0 && elapsed_ms(ctx, EV_FORCE, &ctx->ms_force)) ctx->ms_force = 0.0;
    if (ctx->ms_nbr < 0.0 && elapsed_ms(ctx, EV_NBR, &ctx->ms_nbr)) ctx->ms_nbr = 0.0;
    if (ctx->ms_vjp < 0.0 && elapsed_ms(ctx, EV_VJP, &ctx->ms_vjp)) ctx->ms_vjp = 0.0;
    memset(out, 0, sizeof(*out));
    out->n = ctx->n;
    out->n_nodes = ctx->n_nodes;
    out->n_leaves = ctx->n_leaves;
    out->n_groups = ctx->n_groups;
    out->depth = ctx->depth;
    out->n_cell_entries = ctx->list_total[0];
    out->n_part_entries = ctx->list_total[1];
    out->n_near_entries = ctx->list_total[2];
    out->cell_extent = ctx->list_extent[0];
    out->part_extent = ctx->list_extent[1];
    out->near_extent = ctx->list_extent[2];
    out->n_pp_near = ctx->n_pp_near;
    out->walk_fixed_stride = ctx->walk_fixed;
    out->n_pc = ctx->n_pc;
    out->n_pp = ctx->n_pp;
    out->nnz = ctx->nnz;
    out->walk_global_stack = ctx->walk_global;
    out->ms_build = ctx->ms_build;
    out->ms_walk = ctx->ms_walk;
    out->ms_force = ctx->ms_force;
    out->ms_neighbors = ctx->ms_nbr;
    out->ms_vjp = ctx->ms_vjp;
    return P3T_OK;
}

extern "C" int p3t_copy_array(p3t_ctx *ctx, int which, void *dst, int64_t bytes) {
    if (!ctx || !dst || bytes < 0) return P3T_EINVAL;
    if (!ctx->built) return set_error(ctx, P3T_ESTATE, "no tree");
    int rc = check_hip(ctx, hipSetDevice(ctx->device), "set device");
    if (rc) return rc;
    if ((rc = ensure_lists(ctx))) return rc;
    if ((rc = check_hip(ctx, hipStreamSynchronize(ctx->stream), "sync"))) return rc;
    const int64_t n = ctx->n, nn = ctx->n_nodes, G = ctx->n_groups, stride = nn + 1;
    const void *src = nullptr;
    int64_t size = 0, pitch = 0, spitch = 0, rows = 0;   // strided copies of node records
    switch (which) {
    case P3T_ARR_SORTED_KEYS: src = ctx->keys[0].p; size = n * 8; break;
    case P3T_ARR_PERM: src = ctx->vals[0].p; size = n * 4; break;
    case P3T_ARR_NODE_LEVEL: src = ctx->node_level.p; size = nn * 4; break;
    case P3T_ARR_NODE_FIRST: src = ctx->node_first.p; size = nn * 4; break;
    case P3T_ARR_NODE_COUNT: src = ctx->node_count.p; size = nn * 4; break;
    case P3T_ARR_NODE_CHILD: src = ctx->node_child.p; size = nn * 4; break;
    case P3T_ARR_NODE_NCHILD: src = ctx->node_nchild.p; size = nn * 4; break;
    case P3T_ARR_NODE_PARENT: src = ctx->node_parent.p; size = nn * 4; break;
    case P3T_ARR_NODE_PREFIX: src = ctx->node_prefix.p; size = nn * 8; break;
    case P3T_ARR_NODE_MASS:
        src = (const char *)ctx->node_mp.p + offsetof(NodeMP, M); pitch = 8; spitch = sizeof(NodeMP);
        rows = nn; break;
    case P3T_ARR_NODE_COM:
        src = ctx->node_mp.p; pitch = 24; spitch = sizeof(NodeMP); rows = nn; break;
    case P3T_ARR_NODE_QUAD:
        src = (const char *)ctx->node_mp.p + offsetof(NodeMP, q); pitch = 48; spitch = sizeof(NodeMP);
        rows = nn; break;
    case P3T_ARR_NODE_BOX:
        src = (const char *)ctx->node_walk.p + offsetof(NodeWalk, lo); pitch = 48;
        spitch = sizeof(NodeWalk); rows = nn; break;
    case P3T_ARR_GROUP_NODE:
        src = (const char *)ctx->grp.p + offsetof(GroupInfo, node); pitch = 4;
        spitch = sizeof(GroupInfo); rows = G; break;
    case P3T_ARR_CELL_BEG: src = ctx->off.p; size = G * 8; break;
    case P3T_ARR_CELL_END: src = ctx->seg_end.p; size = G * 8; break;
    case P3T_ARR_PART_END: src = (const int64_t *)ctx->seg_end.p + stride; size = G * 8; break;
    case P3T_ARR_NEAR_END: src = (const int64_t *)ctx->seg_end.p + 2 * stride; size = G * 8; break;
    case P3T_ARR_CELL_IDX: src = ctx->c_idx.p; size = ctx->list_extent[0] * 4; break;
    case P3T_ARR_PART_BEG: src = (const int64_t *)ctx->off.p + stride; size = G * 8; break;
    case P3T_ARR_PART_IDX: src = ctx->p_idx.p; size = ctx->list_extent[1] * 4; break;
    case P3T_ARR_ROOT: src = ctx->root.p; size = 32; break;
    case P3T_ARR_NEAR_BEG: src = (const int64_t *)ctx->off.p + 2 * stride; size = G * 8; break;
    case P3T_ARR_NEAR_IDX: src = ctx->n_idx.p; size = ctx->list_extent[2] * 4; break;
    default: return set_error(ctx, P3T_EINVAL, "unknown array id %d", which);
    }
    if (rows) size = rows * pitch;
    if (bytes != size)
        return set_error(ctx, P3T_EINVAL, "array %d holds %lld bytes, %lld requested", which,
                         (long long)size, (long long)bytes);
    if (size == 0) return P3T_OK;
    if (rows)
        return check_hip(ctx, hipMemcpy2D(dst, pitch, src, spitch, pitch, rows, hipMemcpyDeviceToHost),
                         "copy array");
    return check_hip(ctx, hipMemcpy(dst, src, size, hipMemcpyDeviceToHost), "copy array");
}
