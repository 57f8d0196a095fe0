/*
 * p3t.h -- C ABI of the MI355X (gfx950) long-range tree-force library.
 *
 * The library computes, for N particles, the long-range ("soft") part of the
 * gravitational force of the P3T scheme (Iwasawa, Portegies Zwart & Makino,
 * Section 2.1): the acceleration a_i = sum_j m_j K(s_ij) d_ij / s_ij^3 and the
 * potential phi_i = -sum_j m_j W(s_ij) / s_ij, with d_ij = x_j - x_i, Plummer
 * softened distance s_ij = sqrt(|d_ij|^2 + eps^2), and the changeover functions
 * K and W of Section 2.1 (inner cutoff r_in, outer cutoff r_out, gamma = r_in /
 * r_out).  The sum is evaluated with a Barnes-Hut octree with moments up to
 * the quadrupole (Section 2.2), walked once per group of at most n_crit
 * particles; the same walk yields, for every particle, the list of particles
 * within distance h (Section 2.2, "neighbour sphere" plus "buffer shell"),
 * which feeds the host-side Hermite integrator of the hard part.
 *
 * Conventions shared by every call:
 *   - all particle arrays are in the caller's ORIGINAL particle order;
 *   - pointers documented "device" are hipMalloc'd (or torch-allocated) memory
 *     on the context's device; "host" pointers are ordinary host memory;
 *   - positions/accelerations are row-major [n][3] float64, masses/potentials
 *     [n] float64, whatever the precision mode;
 *   - all work is enqueued on the context's stream, except the neighbour
 *     search of p3t_neighbors, which runs on a second stream of the context
 *     (see there); calls that must read a size back (p3t_build_tree,
 *     p3t_neighbors) synchronise;
 *   - a context is not thread-safe; use one per host thread;
 *   - every call returns P3T_OK (0) or a negative P3T_E* status; on error the
 *     caller's output buffers are left untouched and p3t_last_error() holds a
 *     message.  No C++ exception crosses this interface.
 */
#ifndef P3T_H
#define P3T_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define P3T_OK 0
#define P3T_EINVAL (-1)    /* invalid argument or parameter */
#define P3T_ENOMEM (-2)    /* device allocation failed */
#define P3T_ECAPACITY (-3) /* caller buffer too small; required size reported */
#define P3T_ESTATE (-4)    /* call out of order (e.g. force before build) */
#define P3T_EHIP (-5)      /* HIP runtime error */
#define P3T_ELIMIT (-6)    /* a bounded iteration reached its limit */

#define P3T_PREC_FP64 0    /* every interaction in FP64 */
#define P3T_PREC_MIXED 1   /* FP64 group-relative offsets, FP32 interactions, compensated sums */

/* Method parameters (Section 2.1, Table 1 symbols).
 *   eps        Plummer softening length (>= 0)
 *   r_in       inner cutoff of K and W (0 <= r_in < r_out); gamma = r_in / r_out
 *   r_out      outer cutoff r_cut (> 0)
 *   theta      opening angle (>= 0); a cell of side l with centre of mass at
 *              distance D from a group's box is used as a multipole iff
 *              theta * D > l and the cell's box is at least h away from it
 *   r_search   neighbour radius h (> 0), h = r_cut + buffer width
 *   n_crit     maximum group size (>= n_leaf)
 *   n_leaf     maximum leaf size (>= 1); leaves at depth 21 may hold more
 *   use_quadrupole  1: monopole + quadrupole, 0: monopole only
 *   precision  P3T_PREC_FP64 or P3T_PREC_MIXED */
typedef struct {
    double eps, r_in, r_out, theta, r_search;
    int32_t n_crit, n_leaf, use_quadrupole, precision;
} p3t_params;

/* Counters of the last calls. */
typedef struct {
    int64_t n, n_nodes, n_leaves, n_groups, depth;
    int64_t n_cell_entries;   /* sum over groups of |C_g| (accepted cells) */
    int64_t n_part_entries;   /* sum over groups of |F_g|: particles of opened leaves whose box
                                 is at least max(h, r_out) from the group box */
    int64_t n_near_entries;   /* sum over groups of |N_g|: particles of the other opened leaves;
                                 the walk's particle list is P_g = F_g + N_g */
    int64_t cell_extent, part_extent, near_extent; /* entries spanned by the CELL/PART/NEAR
                                 index arrays: segments may leave unused gaps between them */
    int64_t n_pc, n_pp;       /* interactions: sum_g n_g |C_g|, sum_g n_g |P_g| */
    int64_t n_pp_near;        /* the part of n_pp over near particles: sum_g n_g |N_g| */
    int64_t nnz;              /* neighbour pairs found by the last p3t_neighbors */
    int32_t walk_global_stack;/* 1 if some group's walk needed the global-memory stack */
    int32_t walk_fixed_stride;/* 1 if the lists were written in one walk into segments
                                 reserved from the previous build's sizes */
    double ms_build, ms_force, ms_neighbors, ms_vjp; /* GPU time of the last calls */
    double ms_walk;           /* the part of ms_build spent in the group walk (lists) */
} p3t_stats;

/* Optional device allocator (e.g. a framework's caching allocator). */
typedef void *(*p3t_alloc_fn)(size_t bytes, void *user);
typedef void (*p3t_free_fn)(void *ptr, void *user);

typedef struct p3t_ctx p3t_ctx;

/* Create a context on HIP device `device` whose work goes to `hip_stream`
 * (a hipStream_t; NULL = the default stream).  `alloc`/`free_` may both be NULL
 * (hipMalloc/hipFree are used) or both set; the context owns every internal
 * workspace.  *out receives the context.  Errors: EINVAL, EHIP.
 * The tree walk keeps each group's pending nodes on a stack in LDS and moves a
 * group whose stack outgrows it to a stack in global memory; the environment
 * variable P3T_WALK_LDS_STACK=k (64 <= k < 1536) at creation caps the LDS stack
 * at k entries (results are the same; it exercises the global-memory path). */
int p3t_create(p3t_ctx **out, int device, void *hip_stream, p3t_alloc_fn alloc,
               p3t_free_fn free_, void *alloc_user);

/* Release every workspace and the context (NULL is ignored). */
void p3t_destroy(p3t_ctx *ctx);

/* Host-only parameter check (no device access): P3T_OK or P3T_EINVAL. */
int p3t_check_params(const p3t_params *p);

/* Build the tree, groups and interaction lists (Section 2.2) for n particles.
 *   pos   device [n][3] float64, mass device [n] float64 (> 0, finite)
 * The positions and masses are copied (sorted) into the context, so the caller
 * may reuse its buffers afterwards.  Synchronises the stream to size the lists.
 * Errors: EINVAL (bad n, parameters, non-finite positions or non-positive
 * masses), ENOMEM, EHIP. */
int p3t_build_tree(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                   const p3t_params *p);

/* Long-range acceleration and potential (Section 2.1 soft force, Section 2.2
 * tree) of every particle of the last build.
 *   acc  device [n][3] float64 out;  pot  device [n] float64 out, or NULL
 * Errors: ESTATE (no tree), EINVAL, EHIP. */
int p3t_long_force(p3t_ctx *ctx, double *acc, double *pot);

/* For every particle i, the particles j != i with |x_j - x_i| < h (Section 2.2),
 * as CSR in original indices, ascending within each row; particle i is
 * isolated iff offsets[i+1] == offsets[i].
 *   offsets  device [n+1] int64 out;  idx  device [cap] int32 out
 *   nnz      host out: number of pairs (set also when ECAPACITY is returned)
 * The search runs on a second stream of the context, from the point where the
 * last build's lists were complete, beside whatever the context's stream is
 * still running (it reads only the tree and the lists, and writes workspaces
 * of its own); the call waits for the search alone, then writes offsets and
 * idx on the context's stream, which runs everything queued after the call
 * after the search.  Errors: ESTATE, EINVAL, ECAPACITY (cap < nnz: offsets and
 * idx untouched), EHIP. */
int p3t_neighbors(p3t_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *nnz);

/* Vector-Jacobian product of L = sum_i w_i . a_i + c_i phi_i with respect to
 * positions and masses, with the tree, groups and lists of the last build held
 * fixed (the derivative ignores changes of list membership).  The pair and
 * cell terms are evaluated in the last build's precision (P3T_PREC_MIXED:
 * FP32 on offsets from the group's centre taken in FP64, changeover factors
 * in FP64); all sums and the push-down through the tree are FP64.
 *   w  device [n][3] float64; c device [n] float64 or NULL (taken as 0)
 *   gpos device [n][3] float64 out; gmass device [n] float64 out
 * Errors: ESTATE, EINVAL, ENOMEM, EHIP. */
int p3t_long_force_vjp(p3t_ctx *ctx, const double *w, const double *c, double *gpos,
                       double *gmass);

/* p3t_long_force_vjp for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same result, from the same kernels, with every workspace
 * taken from a static 64 MiB array that the library holds on each device until
 * the process ends (its device address is resolved by p3t_create).  The call
 * itself allocates nothing and does not synchronise the stream.
 *   workspace: 4 n + 10 n_nodes doubles (n_nodes from p3t_get_stats), each of
 *   the two per-particle parts rounded up to 256 bytes; larger builds return
 *   ECAPACITY (about n = 2^20 with up to 4 * 10^5 nodes fits).
 * All calls on one device share that array and leave their intermediate
 * values in it: two calls that may run at the same time on one device (from
 * two contexts, or on different streams) race and give wrong results; calls
 * ordered on one stream are safe.  The build's lists must be present: after
 * p3t_release_lists the call returns ESTATE (walking again would allocate);
 * p3t_long_force or p3t_long_force_vjp restores them.
 * Arguments and outputs as p3t_long_force_vjp.
 * Errors: ESTATE, EINVAL, ECAPACITY, EHIP. */
int p3t_long_force_vjp_noalloc(p3t_ctx *ctx, const double *w, const double *c, double *gpos,
                               double *gmass);

/* Frees the interaction-list arrays of the last build (the largest part of a
 * build's memory) and keeps the tree, moments and groups.  The next call that
 * needs the lists (p3t_long_force, p3t_neighbors, p3t_long_force_vjp,
 * p3t_step, p3t_copy_array of a list) walks the tree again first; the walk is
 * deterministic, so the lists, forces and VJP are the same as without the
 * release.  For a backward pass under memory pressure: release after the
 * forward, recompute in the VJP.  Errors: ESTATE (no build), EHIP. */
int p3t_release_lists(p3t_ctx *ctx);

/* Leapfrog helpers of the shared-timestep soft step (Section 2.1, kick under
 * H_soft; drift): v += dt_kick * a, then x += dt_drift * v, elementwise over
 * [n][3] device arrays.  Errors: EINVAL, EHIP. */
int p3t_kick_drift(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *acc,
                   double dt_kick, double dt_drift);

/* Particle kinds (Section 3.2.2, the SMBH runs): the last n_special particles
 * of the arrays are special.  A normal-special pair takes its own cutoffs,
 * softening and neighbour radius; a special-special pair its own softening and,
 * with split_ss = 0, no soft part at all (K = W = 0: the pair is integrated
 * wholly by Hermite, and two special particles are always neighbours); special
 * particles take their own Hermite accuracy parameters.  The tree covers the
 * normal particles only; a NULL p3t_kinds or n_special = 0 means one kind.
 *   r_in_ns < r_out_ns, r_search_ns > 0, eps_ns >= 0
 *   split_ss 0 or 1; with 1: r_in_ss < r_out_ss, r_search_ss > 0; eps_ss >= 0
 *   eta_sp, eta_s_sp > 0 */
typedef struct {
    int64_t n_special;
    double r_in_ns, r_out_ns, r_search_ns, eps_ns;
    int32_t split_ss;
    double r_in_ss, r_out_ss, r_search_ss, eps_ss;
    double eta_sp, eta_s_sp;
} p3t_kinds;

/* Soft force and potential of every pair that involves a special particle
 * (each pair with its own parameters), O(n n_special): ADDED to the rows of the
 * normal particles (which hold the tree's sum over normal pairs) and WRITTEN
 * to the rows of the special particles.
 *   pos device [n][3]; mass device [n]; acc device [n][3] in/out; pot device
 *   [n] in/out or NULL.  Errors: EINVAL, EHIP. */
int p3t_kinds_soft(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
                   const p3t_params *p, const p3t_kinds *kinds, double *acc, double *pot);

/* Neighbour lists of all n particles with a radius per kind of pair: a normal
 * particle's row is its row of the normal lists (nn_off, nn_idx over the first
 * n - n_special particles, as p3t_neighbors writes them) followed by the
 * special particles within r_search_ns; a special particle's row lists the
 * normal particles within r_search_ns and the other special particles (all of
 * them when split_ss = 0, else those within r_search_ss); rows ascending.
 * The normal lists are checked like the hard part's (symmetric, in range, no
 * self entry; nn_idx may be NULL only if every row is empty), EINVAL otherwise.
 *   off device [n+1] int64 out; idx device [cap] int32 out; nnz host out (set
 *   also on ECAPACITY).  Synchronises.  Errors: EINVAL, ECAPACITY, ENOMEM, EHIP. */
int p3t_kinds_neighbors(p3t_ctx *ctx, int64_t n, const double *pos, const p3t_kinds *kinds,
                        const int64_t *nn_off, const int32_t *nn_idx, int64_t *off,
                        int32_t *idx, int64_t cap, int64_t *nnz);

/* ---- Hard part (Section 2.1: H_hard; Section 2.2: evaluated over the
 * neighbour lists).  Neighbour lists are CSR in original indices, as
 * p3t_neighbors writes them: offsets device [n+1] int64, idx device
 * [offsets[n]] int32; they must be symmetric (j on i's list iff i on j's),
 * free of self entries and in range, which is checked (EINVAL otherwise); idx
 * may be NULL only if every row is empty. */

/* Hard force, its jerk and the hard potential of every particle from its
 * list (Section 2.1, F_hard with the cutoff function K; potential of H_hard):
 *   a_i    = sum_j m_j (1 - K(s)) d / s^3,   d = x_j - x_i, v = v_j - v_i
 *   jerk_i = sum_j m_j [(1 - K)(v - 3 (d.v) d / s^2) / s^3 - K'(s) ((d.v)/s) d / s^3]
 *   phi_i  = -sum_j m_j (1 - W(s)) / s
 * in FP64, summed in list order.  Uses eps, r_in, r_out of *p for pairs of
 * normal particles and *kinds (or NULL) for pairs with a special particle.
 *   pos, vel device [n][3]; mass device [n]; acc, jerk device [n][3] out;
 *   pot device [n] out or NULL.  Isolated particles (empty rows) get zeros.
 * Synchronises the stream (list check).  Errors: EINVAL, ENOMEM, EHIP. */
int p3t_hard_force(p3t_ctx *ctx, int64_t n, const double *pos, const double *vel,
                   const double *mass, const int64_t *offsets, const int32_t *idx,
                   const p3t_params *p, const p3t_kinds *kinds, double *acc, double *jerk,
                   double *pot);

/* Parameters of the Hermite integration of H_hard (Section 2.1).
 *   dt_soft  the soft step, integrated over (> 0, a whole multiple of dt_max)
 *   dt_max   the largest Hermite step (0 < dt_max <= dt_soft)
 *   eta      accuracy parameter of the timestep criterion (> 0)
 *   eta_s    accuracy parameter of the first-step criterion (> 0; the paper
 *            uses eta / 10)
 *   a0       acceleration floor of the criteria, alpha m / r_cut^2 (>= 0)
 *   max_block_steps  bound on the block steps of one cluster (0: 2^22);
 *            reaching it ends the call with P3T_ELIMIT */
typedef struct {
    double dt_soft, dt_max, eta, eta_s, a0;
    int64_t max_block_steps;
} p3t_hermite_params;

typedef struct {
    int64_t n_hard;          /* particles with a non-empty list */
    int64_t n_clusters;      /* connected components of the neighbour graph among them */
    int64_t max_cluster;     /* members of the largest component */
    int64_t steps;           /* Hermite steps summed over particles */
    int64_t max_block_steps; /* block steps of the busiest component */
    double ms;               /* GPU time of the call */
} p3t_hermite_stats;

/* Advance H_hard over dt_soft (Section 2.1, step 3 of the scheme; Section 2.2,
 * steps 5-6 of the GPU procedure), in place on pos and vel: particles with an
 * empty row are isolated and drift, x += dt_soft v; the others are integrated
 * with the fourth-order Hermite scheme and block timesteps dt_max / 2^k
 * under the hard force of their list, the list held fixed.  Timestep: first
 * step eta_s sqrt((|a|^2 + a0^2) / |a'|^2); later
 * eta sqrt((sqrt(|a|^2 + a0^2) |a''| + |a'|^2) / (|a'| |a'''| + |a''|^2)), with
 * a'' and a''' from Hermite interpolation; a step doubles only where the
 * particle's time is a multiple of the doubled step.  Each connected
 * component of the neighbour graph is integrated on its own: by a group of
 * lanes of a wavefront (fewer than 64 members), a workgroup (fewer than 1024)
 * or grid-wide launches per block step.
 *   nsteps   device [n] int32 out (Hermite steps per particle) or NULL
 *   stats    host out or NULL
 * Synchronises the stream.  Errors: EINVAL, ENOMEM, ELIMIT, EHIP. */
int p3t_hermite_hard(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass,
                     const int64_t *offsets, const int32_t *idx, const p3t_params *p,
                     const p3t_kinds *kinds, const p3t_hermite_params *hp, int32_t *nsteps,
                     p3t_hermite_stats *stats);

/* One step of the P3T scheme (Section 2.2's GPU procedure), in place:
 * v += dt_soft/2 a_soft; neighbour lists of the current build; p3t_hermite_hard
 * over dt_soft; rebuild at the new positions; a_soft (and the soft potential
 * if pot is not NULL) at the new positions into acc; v += dt_soft/2 a_soft.
 * On entry the context must hold a build of the normal particles (all n, or
 * the first n - n_special with kinds) at the current positions and acc their
 * soft acceleration (p3t_build_tree + p3t_long_force, + p3t_kinds_soft with
 * kinds); on return both hold for the new positions, so steps chain.  With
 * kinds the neighbour lists are merged by p3t_kinds_neighbors and the hard
 * part and soft sums take each pair's own parameters.
 *   pos, vel device [n][3]; mass device [n]; acc device [n][3] in/out;
 *   pot device [n] out or NULL; stats: the hard part's, host out or NULL.
 * The neighbour radius must reach the outer cutoff (Section 2.2: h = r_cut plus
 * a buffer): r_search >= r_out, and with kinds r_search_ns >= r_out_ns (and
 * r_search_ss >= r_out_ss when split_ss = 1); otherwise the pairs between h and
 * r_out would lose their hard force, and the call returns EINVAL.
 * Errors: ESTATE, EINVAL, ENOMEM, ELIMIT, EHIP. */
int p3t_step(p3t_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass, double *acc,
             double *pot, const p3t_params *p, const p3t_kinds *kinds,
             const p3t_hermite_params *hp, p3t_hermite_stats *stats);

/* ---- Direct summation (the exact sums the tree approximates; for energies
 * and diagnostics).  For every particle i, over all j != i, in FP64:
 *   P3T_DIRECT_NEWTON  a_i = sum m_j d / s^3,          phi_i = -sum m_j / s
 *   P3T_DIRECT_SOFT    a_i = sum m_j K(s) d / s^3,     phi_i = -sum m_j W(s) / s
 *   P3T_DIRECT_HARD    a_i = sum m_j (1-K(s)) d / s^3, phi_i = -sum m_j (1-W(s)) / s
 * (Section 2.1: F_soft and F_hard, H_soft and H_hard; d = x_j - x_i, s the
 * softened distance).  O(n^2) work; uses eps, r_in, r_out of *p.
 *   pos device [n][3]; mass device [n]; acc device [n][3] out; pot device [n]
 *   out or NULL.  Errors: EINVAL, EHIP. */
#define P3T_DIRECT_NEWTON 0
#define P3T_DIRECT_SOFT 1
#define P3T_DIRECT_HARD 2
int p3t_direct(p3t_ctx *ctx, int64_t n, const double *pos, const double *mass,
               const p3t_params *p, int mode, double *acc, double *pot);

/* Statistics of the last calls.  Errors: EINVAL. */
int p3t_get_stats(p3t_ctx *ctx, p3t_stats *out);

/* Inspection of the last build, for tests and tools: copies an internal array
 * into HOST memory `dst` of `bytes` bytes (synchronous).  Array ids and element
 * types are listed below; the element count of each is given by p3t_get_stats
 * (n, n_nodes, n_groups, list sizes).  Errors: ESTATE, EINVAL (unknown id or
 * bytes not the array's size), EHIP. */
enum {
    P3T_ARR_SORTED_KEYS = 0,   /* uint64 [n]   Morton keys in sorted order */
    P3T_ARR_PERM = 1,          /* int32  [n]   sorted position -> original index */
    P3T_ARR_NODE_LEVEL = 2,    /* int32  [n_nodes] */
    P3T_ARR_NODE_FIRST = 3,    /* int32  [n_nodes] first sorted particle */
    P3T_ARR_NODE_COUNT = 4,    /* int32  [n_nodes] */
    P3T_ARR_NODE_CHILD = 5,    /* int32  [n_nodes] first child id */
    P3T_ARR_NODE_NCHILD = 6,   /* int32  [n_nodes] 0 for leaves */
    P3T_ARR_NODE_PARENT = 7,   /* int32  [n_nodes] -1 for the root */
    P3T_ARR_NODE_PREFIX = 8,   /* uint64 [n_nodes] key prefix at the node's level */
    P3T_ARR_NODE_MASS = 9,     /* double [n_nodes] */
    P3T_ARR_NODE_COM = 10,     /* double [n_nodes][3] */
    P3T_ARR_NODE_QUAD = 11,    /* double [n_nodes][6] xx yy zz xy xz yz */
    P3T_ARR_NODE_BOX = 12,     /* double [n_nodes][6] lo xyz, hi xyz */
    P3T_ARR_GROUP_NODE = 13,   /* int32  [n_groups] node id, ordered by first particle */
    /* Lists: group g's entries of a list are IDX[BEG[g] .. END[g]); the segments of
     * different groups may lie in any order, with unused gaps between them. */
    P3T_ARR_CELL_BEG = 14,     /* int64  [n_groups] */
    P3T_ARR_CELL_IDX = 15,     /* int32  [cell_extent] node ids of C_g */
    P3T_ARR_PART_BEG = 16,     /* int64  [n_groups] */
    P3T_ARR_PART_IDX = 17,     /* int32  [part_extent] sorted particle indices of F_g */
    P3T_ARR_ROOT = 18,         /* double [4] lo xyz, side L */
    P3T_ARR_NEAR_BEG = 19,     /* int64  [n_groups] */
    P3T_ARR_NEAR_IDX = 20,     /* int32  [near_extent] sorted particle indices of N_g */
    P3T_ARR_CELL_END = 21,     /* int64  [n_groups] */
    P3T_ARR_PART_END = 22,     /* int64  [n_groups] */
    P3T_ARR_NEAR_END = 23      /* int64  [n_groups] */
};
int p3t_copy_array(p3t_ctx *ctx, int which, void *dst, int64_t bytes);

/* Human-readable status, and the context's last error message. */
const char *p3t_status_string(int status);
const char *p3t_last_error(p3t_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* P3T_H */
