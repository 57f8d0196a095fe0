// internal.h -- data layout and launch interfaces shared by the library's
// translation units (not part of the public ABI; see include/p3t.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "p3t.h"

namespace p3t {

constexpr int kMaxLevel = 21;        // 63-bit keys, 3 bits per level
constexpr int kLevels = kMaxLevel + 1;

// Root cube of the last build (device resident).
struct RootInfo {
    double lo[3];
    double L;          // power-of-two side
    double scale;      // 2^21 / L
    int32_t bad_input; // non-finite position or non-positive mass seen
    int32_t pad;
};

// Sorted particle record: position and mass in one aligned 32-byte line
// segment, so that a gathered list entry costs one read.
struct alignas(32) PosMass {
    double x, y, z, m;
};

// Per-node record read by the tree walk (96 bytes, one read per visit).
struct NodeWalk {
    double cx, cy, cz;      // centre of mass
    double l2;              // squared cell side (L 2^-level)^2
    double lo[3], hi[3];    // tight member box
    int32_t child_first, n_child, first, count;
};

// Per-node multipole read by the interaction kernels (80 bytes).
struct NodeMP {
    double cx, cy, cz, M;
    double q[6];            // traceless quadrupole xx yy zz xy xz yz about the com
};

// Per-group record, groups ordered by first particle.
struct GroupInfo {
    double lo[3], hi[3];    // member box
    double c[3];            // box centre, origin of the FP32 offsets
    int32_t first, count, node, pad;
};

// Changeover constants for a given gamma = r_in / r_out.
struct Changeover {
    double r_out, inv_rout, gamma, inv_1mg;   // 1 / (1 - gamma)
    double C;                                  // W/y below r_in
    // W(y)/y on [gamma, 1): w6 y^6 + w5 y^5 + ... + w1 y + w0 + wl ln(y) + wm / y
    double w[7];
    double wl, wm;
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// The walk's per-group lists: 0 = accepted cells (node ids), 1 = far particles,
// 2 = near particles (sorted particle indices); group g's entries of list k are
// idx[k][beg[k][g] .. end[k][g]).  Kernels with one block per group take group
// order[blockIdx.x]: groups sorted by decreasing estimated work, so that the
// longest blocks start first and the launch has no long tail.
struct ListsDev {
    const int64_t *beg[3];
    const int64_t *end[3];
    const int32_t *idx[3];
    const int32_t *order;
};

}  // namespace p3t

struct p3t_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    p3t_alloc_fn alloc = nullptr;
    p3t_free_fn free_ = nullptr;
    void *user = nullptr;
    char err[512] = {0};

    int built = 0;
    int lists_released = 0;   // 1: the list arrays were freed; the next call that needs them walks again
    int64_t n = 0;
    p3t_params prm{};
    p3t::Changeover chg{};

    int64_t n_nodes = 0, n_groups = 0, n_leaves = 0, depth = 0;
    int64_t list_total[3] = {0, 0, 0};    // entries of C, F, N over all groups
    int64_t list_extent[3] = {0, 0, 0};   // entries the list arrays span (segments may leave gaps)
    int64_t n_pc = 0, n_pp = 0, n_pp_near = 0, nnz = 0;
    int64_t level_start[p3t::kLevels + 2] = {0};
    int walk_global = 0, walk_fixed = 0;
    int32_t walk_lds_cap = 0;   // entries of the walk's LDS stack to use (0: all of it)
    bool groups_generic = false;  // groups compacted by a plain scan (as for the largest n)
    // sizes seen by the last two-pass or fixed-stride walk, used to reserve
    // fixed-stride list segments on the next build
    int64_t hint_groups = 0, hint_max[3] = {0, 0, 0};
    int32_t hint_n_crit = -1;
    int32_t nbr_cap = 0;   // neighbour row slot size for the next p3t_neighbors (0: default)
    unsigned long long nbr_tag = 0;   // number of neighbour searches so far (tags their readback words)
    double ms_build = 0, ms_walk = 0, ms_force = 0, ms_nbr = 0, ms_vjp = 0;
    hipEvent_t ev[12] = {nullptr};  // start/end pairs: build, force, neighbours, vjp, walk, hermite
    int64_t *hpin = nullptr;      // pinned host readback area (64 int64)
    void *scratch = nullptr;      // device address of the library's static workspace on this device

    p3t::DevBuf root, keys[2], vals[2], hist, histc, rs_tot, xm, xm_in;
    p3t::DevBuf lvlrange, tblk, tblk_off, gtile;
    p3t::DevBuf node_level, node_first, node_count, node_child, node_nchild, node_parent,
        node_prefix, node_S, node_walk, node_mp;
    p3t::DevBuf gflag, gscan, grp;
    p3t::DevBuf cnt, off, c_idx, p_idx, n_idx;
    p3t::DevBuf wstack, readback, scan_tmp, nbr_cnt, nbr_slots, nbr_scan;
    p3t::DevBuf vjp_gx, vjp_gm, vjp_cell, bbox;
    p3t::DevBuf seg_end, gorder, grank, ghist;
    p3t::DevBuf hard_ix, hard_state;   // hard part: components and integrator state
    p3t::DevBuf hard_giant;            // ... and the step bookkeeping of the largest components
    // the hard part's concurrent classes (aux_streams); the neighbour search
    // runs on aux[0] too, never at the same time (each host-synchronised)
    hipStream_t aux[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t aev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int aux_ready = 0;
    // The neighbour search runs on aux[0] from the point where the lists are
    // complete (ev_lists, recorded on `stream` by every walk), beside whatever
    // the context's stream does meanwhile; ev_sync orders the two.
    hipEvent_t ev_lists = nullptr, ev_sync[2] = {nullptr, nullptr};
    p3t::DevBuf step_off, step_idx;    // neighbour CSR of p3t_step
    p3t::DevBuf step_off2, step_idx2;  // ... merged with the special particles' pairs
    p3t::DevBuf kinds_cnt;
};

namespace p3t {

// Allocation helpers (context allocator or hipMalloc); return 0 or P3T_ENOMEM.
int ensure(p3t_ctx *ctx, DevBuf &b, size_t bytes);
// The device readback area (kReadbackWords int64 words), allocated and cleared
// on first use.
constexpr int kReadbackWords = 64;
int ensure_readback(p3t_ctx *ctx);
void release(p3t_ctx *ctx, DevBuf &b);
int set_error(p3t_ctx *ctx, int status, const char *fmt, ...);
int check_hip(p3t_ctx *ctx, hipError_t e, const char *what);

// Device-wide exclusive prefix sum (out may alias in).  `total` (device, may be
// null) receives the sum of all n inputs.
int scan_exclusive_i64(p3t_ctx *ctx, const int64_t *in, int64_t *out, int64_t n, int64_t *total);
int scan_exclusive_i32(p3t_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *total);
// The same on stream st with the workspace tmp (at least scan_tmp_bytes(n)
// bytes, so that the call allocates nothing).
size_t scan_tmp_bytes(int64_t n);
int scan_exclusive_i64_on(p3t_ctx *ctx, hipStream_t st, DevBuf &tmp, const int64_t *in,
                          int64_t *out, int64_t n, int64_t *total);
// Exclusive prefix sum of each row of a [rows][cols] array (one block per
// row, one launch); totals[r] receives the sum of row r.
int scan_rows_i32(p3t_ctx *ctx, const int32_t *in, int32_t *out, int32_t *totals, int rows,
                  int64_t cols);

// Readback slots (int64 words of ctx->readback / ctx->hpin) written during a
// build: the node count of each level (kLevels int32), then the input check.
constexpr int kRbTopoBad = kLevels + 1;
// The walk's statistics from this slot on (kRbWalkWords words, cleared by the
// group selection before every walk of a build).
constexpr int kRbWalk = 24;
constexpr int kRbWalkWords = 13;

// Tree build stages (tree.hip).
// root cube, Morton keys, stable sort (keys[0] / vals[0]) and the sorted
// particle records xm
int build_sorted(p3t_ctx *ctx, const double *pos, const double *mass, int64_t n);
int build_topology(p3t_ctx *ctx, int64_t n);    // sets ctx->n_nodes, level_start, depth
int build_moments(p3t_ctx *ctx);
int build_groups(p3t_ctx *ctx);                 // sets ctx->n_groups

// Walk (walk.hip): lists and their statistics; sets n_groups and list sizes.
// stats_cleared: the walk's statistics slots are already zero (a build clears
// them in the group selection); a walk after p3t_release_lists clears them.
int build_lists(p3t_ctx *ctx, bool stats_cleared);

// Interactions (force.hip).
int launch_force(p3t_ctx *ctx, double *acc, double *pot);

// The hard part's auxiliary streams and their events, made on first use
// (hard.hip); each takes a hardware queue of its own beside the context's
// stream, so the context makes no other streams.
int aux_streams(p3t_ctx *ctx);

// Neighbour lists (neighbors.hip).  The search and the row count run on
// ctx->aux[0], between the timing events t0 and t1 (either may be null); the
// caller's arrays are written on ctx->stream after them.
int launch_neighbors(p3t_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *nnz,
                     hipEvent_t t0, hipEvent_t t1);

// VJP (vjp.hip).  launch_vjp takes its workspaces from the context;
// launch_vjp_ws from the caller: gx [3 n], gm [n] and cadj [10 n_nodes] doubles
// (gx and gm are written before they are read, cadj is cleared first).
int launch_vjp(p3t_ctx *ctx, const double *w, const double *c, double *gpos, double *gmass);
int launch_vjp_ws(p3t_ctx *ctx, const double *w, const double *c, double *gpos, double *gmass,
                  double *gx, double *gm, double *cadj);

// Hard part (hard.hip): force and jerk over neighbour lists; Hermite block-step
// integration over one soft step.
int launch_hard_force(p3t_ctx *ctx, int64_t n, const double *pos, const double *vel,
                      const double *mass, const int64_t *off, const int32_t *idx,
                      const p3t_params *p, const p3t_kinds *kd, double *acc, double *jerk,
                      double *pot);
int launch_hermite(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass,
                   const int64_t *off, const int32_t *idx, const p3t_params *p,
                   const p3t_kinds *kd, const p3t_hermite_params *hp, int32_t *nsteps,
                   p3t_hermite_stats *stats);
// Checks a caller's symmetric neighbour CSR of n rows before any kernel walks it
// (offsets non-decreasing from >= 0, entries in [0, n), no self entry, every
// listed particle's own row non-empty); idx may be NULL only if every row is
// empty.  P3T_OK or P3T_EINVAL (synchronises the stream).
int validate_csr(p3t_ctx *ctx, int64_t n, const int64_t *off, const int32_t *idx);

// Particle kinds (kinds.hip): soft sums of the pairs with a special particle,
// and the neighbour lists of all particles with a radius per kind of pair.
int launch_kinds_soft(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                      const p3t_params *p, const p3t_kinds *kd, double *acc, double *pot);
int launch_kinds_neighbors(p3t_ctx *ctx, int64_t n, const double *pos, const p3t_kinds *kd,
                           const int64_t *nn_off, const int32_t *nn_idx, int64_t *off,
                           int32_t *idx, int64_t cap, int64_t *nnz);

// Constants of K and W for gamma = r_in / r_out (p3t_api.hip).
Changeover make_changeover(double r_in, double r_out);

// O(N^2) direct sums (direct.hip).
int launch_direct(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                  const p3t_params *p, int mode, double *acc, double *pot);

// Elementwise leapfrog helper (force.hip).
int launch_kick_drift(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *acc,
                      double dt_kick, double dt_drift);

template <class T>
inline T *ptr(const DevBuf &b) { return static_cast<T *>(b.p); }

// Device view of the lists of the last build.
ListsDev lists_dev(const p3t_ctx *ctx);

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace p3t
