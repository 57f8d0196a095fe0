/*
 * p3t_oracle.c -- plain FP64 CPU oracle for the P3T long-range (soft) tree force.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no source with the GPU library.
 *
 * What it computes, step by step, in the order of the method:
 *   soft force (Section 2.1, equation for F_soft): a_i = sum_j m_j K(s_ij) d_ij / s_ij^3
 *     with d_ij = x_j - x_i, s_ij = sqrt(|d_ij|^2 + eps^2) (softened distance
 *     of the Hamiltonian, Section 2.1) and the cutoff function K (Section 2.1,
 *     polynomial K(x), x = (y - gamma)/(1 - gamma), y = s / r_cut);
 *   soft potential (Section 2.1, H_soft): phi_i = -sum_j m_j W(s_ij) / s_ij with the
 *     transition function W (Section 2.1, W(y; gamma) and G(y; gamma)), read with
 *     the denominator of G as (gamma - 1)^7 -- with the printed (1 - gamma)^7
 *     the identity K = W - s dW/ds fails and W jumps at y = gamma;
 *   Barnes-Hut tree with moments up to the quadrupole (Section 2.2) evaluated for
 *     groups of particles, and for each particle the list of particles within
 *     distance h (Section 2.2, neighbour sphere and buffer shell).
 *
 * Tree, group and list conventions (the paper leaves them open):
 *   root cube  lo_a = min x_a, L = 2^ceil(log2(max extent)) (L = 1 if extent 0);
 *   keys       q_a = min(floor((x_a - lo_a) * 2^21 / L), 2^21 - 1), 63-bit
 *              interleave, bit 3b+2 <- q_x bit b, 3b+1 <- q_y, 3b <- q_z;
 *   sort       by key, ties by original index;
 *   node       (level l, key prefix) = contiguous sorted range; split into its
 *              non-empty octants iff count > n_leaf and l < 21; ids in BFS order;
 *   moments    M and S = sum m x folded left in sorted order (leaves) or octant
 *              order (internal), com = S / M; traceless quadrupole about com;
 *              tight member AABB; cell side l = L 2^-level;
 *   groups     node g with (count <= n_crit or leaf) and no ancestor such;
 *              ordered by first particle;
 *   walk       cell c accepted for group g iff theta^2 D^2(com_c, box_g) > side_c^2
 *              and B^2(box_c, box_g) >= h^2; otherwise a leaf's particles join
 *              the particle list and an internal cell's children are visited;
 *   cell term  a += K(y_c) [-M r/s^3 + Q r/s^5 - 5/2 (r.Q.r) r/s^7],
 *              phi += W(y_c) [-M/s - (r.Q.r)/(2 s^5)], r = x_i - com_c;
 *   neighbours j in the particle list, j != i, dx*dx+dy*dy+dz*dz < h*h (FP64).
 *
 * Compiled with -ffp-contract=off and without fast-math: every decision-feeding
 * quantity (keys, com, distances) is a fixed IEEE operation sequence.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_LEVEL 21

typedef struct {
    double eps, r_in, r_out, theta, r_search;
    int32_t n_crit, n_leaf, use_quadrupole, precision;
} or_params;

typedef struct {
    int64_t n;
    or_params p;
    double lo[3], L;
    uint64_t *key;        /* [n] original order */
    int64_t *perm;        /* [n] sorted position -> original index */
    uint64_t *skey;       /* [n] sorted keys */
    double *x, *y, *z, *m;/* [n] sorted */
    /* nodes (BFS order) */
    int64_t n_nodes, cap_nodes;
    int32_t *level;
    int64_t *first, *count, *child_first, *parent;
    int32_t *n_child;
    uint64_t *prefix;
    double *M, *com, *Q, *blo, *bhi, *side; /* com/blo/bhi: [3*nodes]; Q: [6*nodes] xx yy zz xy xz yz */
    /* groups ordered by first particle */
    int64_t n_groups;
    int64_t *grp;         /* node id of each group */
    /* per-group lists (CSR) */
    int64_t *c_off, *c_idx;  /* accepted cells (node ids, ascending) */
    int64_t *p_off, *p_idx;  /* particles of opened leaves (sorted indices, ascending) */
    int64_t n_pp, n_pc;      /* interaction counts sum_g n_g |P_g|, sum_g n_g |C_g| */
} or_tree;

/* ------------------------------------------------------------------------ */
/* Changeover functions (Section 2.1).                                       */
/* ------------------------------------------------------------------------ */

/* K as a function of y = s / r_cut, gamma = r_in / r_cut. */
double or_K(double y, double gam)
{
    if (y < gam) return 0.0;
    if (y >= 1.0) return 1.0;
    double x = (y - gam) / (1.0 - gam);
    double x2 = x * x;
    return x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
}

/* dK/dy */
double or_dK(double y, double gam)
{
    if (y < gam || y >= 1.0) return 0.0;
    double x = (y - gam) / (1.0 - gam);
    double u = x * (1.0 - x);
    return 140.0 * u * u * u / (1.0 - gam);
}

/* The constant slope of W below the inner cutoff: W = C(gamma) y for y < gamma. */
double or_C(double g)
{
    double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g;
    double gm1 = g - 1.0;
    double gm7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
    return 7.0 * (g6 - 9.0 * g5 + 45.0 * g4 - 60.0 * g3 * log(g) - 45.0 * g2 + 9.0 * g - 1.0)
           / (3.0 * gm7);
}

/* G(y; gamma) of the paper with denominator (gamma - 1)^7. */
static double or_G(double y, double g)
{
    double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g, g7 = g6 * g;
    double y2 = y * y, y3 = y2 * y, y4 = y3 * y, y5 = y4 * y, y6 = y5 * y, y7 = y6 * y;
    double gm1 = g - 1.0;
    double gm7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
    double num = -(10.0 / 3.0) * y7
                 + 14.0 * (g + 1.0) * y6
                 - 21.0 * (g2 + 3.0 * g + 1.0) * y5
                 + (35.0 * (g3 + 9.0 * g2 + 9.0 * g + 1.0) / 3.0) * y4
                 - 70.0 * (g3 + 3.0 * g2 + g) * y3
                 + 210.0 * (g3 + g2) * y2
                 - 140.0 * g3 * y * log(y)
                 + (g7 - 7.0 * g6 + 21.0 * g5 - 35.0 * g4);
    return num / gm7;
}

/* W(y; gamma) */
double or_W(double y, double g)
{
    if (y < g) return or_C(g) * y;
    if (y >= 1.0) return 1.0;
    return or_G(y, g) + (1.0 - or_G(1.0, g)) * y;
}

/* W(y)/y, finite at y = 0. */
double or_W_over_y(double y, double g)
{
    if (y < g) return or_C(g);
    if (y >= 1.0) return 1.0 / y;
    return or_W(y, g) / y;
}

/* ------------------------------------------------------------------------ */
/* Root cube and Morton keys.                                                */
/* ------------------------------------------------------------------------ */

static double root_side(double ext)
{
    if (!(ext > 0.0)) return 1.0;
    int e;
    double f = frexp(ext, &e);         /* ext = f 2^e, f in [0.5, 1) */
    return (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

static uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < OR_MAX_LEVEL; b++)
        r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

uint64_t or_morton(double x, double y, double z, const double lo[3], double L)
{
    double scale = ldexp(1.0, OR_MAX_LEVEL) / L;
    double c[3] = {x, y, z};
    uint64_t q[3];
    for (int a = 0; a < 3; a++) {
        double t = floor((c[a] - lo[a]) * scale);
        uint64_t qi = (uint64_t)t;
        if (qi > (1ull << OR_MAX_LEVEL) - 1) qi = (1ull << OR_MAX_LEVEL) - 1;
        q[a] = qi;
    }
    return (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
}

/* ------------------------------------------------------------------------ */

static const uint64_t *g_sort_keys;
static int cmp_key_idx(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki < kj) return -1;
    if (ki > kj) return 1;
    return (i < j) ? -1 : (i > j);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x < y) ? -1 : (x > y);
}

static void grow_nodes(or_tree *t)
{
    int64_t c = t->cap_nodes ? 2 * t->cap_nodes : 1024;
    t->level = realloc(t->level, c * sizeof(int32_t));
    t->first = realloc(t->first, c * sizeof(int64_t));
    t->count = realloc(t->count, c * sizeof(int64_t));
    t->child_first = realloc(t->child_first, c * sizeof(int64_t));
    t->parent = realloc(t->parent, c * sizeof(int64_t));
    t->n_child = realloc(t->n_child, c * sizeof(int32_t));
    t->prefix = realloc(t->prefix, c * sizeof(uint64_t));
    t->cap_nodes = c;
}

static int64_t add_node(or_tree *t, int32_t lev, int64_t first, uint64_t pfx, int64_t par)
{
    if (t->n_nodes == t->cap_nodes) grow_nodes(t);
    int64_t id = t->n_nodes++;
    t->level[id] = lev;
    t->first[id] = first;
    t->count[id] = 0;
    t->child_first[id] = -1;
    t->n_child[id] = 0;
    t->prefix[id] = pfx;
    t->parent[id] = par;
    return id;
}

static int is_leaf(const or_tree *t, int64_t c) { return t->n_child[c] == 0; }

/* point-to-box squared distance, per-axis gap then ((tx^2 + ty^2) + tz^2) */
static double d2_point_box(const double p[3], const double lo[3], const double hi[3])
{
    double t[3];
    for (int a = 0; a < 3; a++) {
        double u = lo[a] - p[a];
        double v = p[a] - hi[a];
        double w = u > 0.0 ? u : 0.0;
        t[a] = v > w ? v : w;
    }
    return t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
}

/* box-to-box squared gap distance, same operation order */
static double d2_box_box(const double alo[3], const double ahi[3], const double blo[3],
                         const double bhi[3])
{
    double t[3];
    for (int a = 0; a < 3; a++) {
        double u = alo[a] - bhi[a];
        double v = blo[a] - ahi[a];
        double w = u > 0.0 ? u : 0.0;
        t[a] = v > w ? v : w;
    }
    return t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
}

/* Cell acceptance for group g (see header). */
static int accept_cell(const or_tree *t, int64_t c, int64_t g)
{
    const double *glo = t->blo + 3 * g, *ghi = t->bhi + 3 * g;
    double th2 = t->p.theta * t->p.theta;
    double h2 = t->p.r_search * t->p.r_search;
    double D2 = d2_point_box(t->com + 3 * c, glo, ghi);
    double B2 = d2_box_box(t->blo + 3 * c, t->bhi + 3 * c, glo, ghi);
    double l2 = t->side[c] * t->side[c];
    return (th2 * D2 > l2) && (B2 >= h2);
}

/* Moments, children before parents (reverse BFS order). */
static void compute_moments(or_tree *t)
{
    int64_t nn = t->n_nodes;
    if (!t->M) {
        t->M = calloc(nn, sizeof(double));
        t->com = calloc(3 * nn, sizeof(double));
        t->Q = calloc(6 * nn, sizeof(double));
        t->blo = calloc(3 * nn, sizeof(double));
        t->bhi = calloc(3 * nn, sizeof(double));
        t->side = calloc(nn, sizeof(double));
    }
    double *S = calloc(3 * nn, sizeof(double));
    for (int64_t id = nn - 1; id >= 0; id--) {
        double Mc = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
        if (is_leaf(t, id)) {
            for (int64_t k = t->first[id]; k < t->first[id] + t->count[id]; k++) {
                Mc = Mc + t->m[k];
                Sx = Sx + t->m[k] * t->x[k];
                Sy = Sy + t->m[k] * t->y[k];
                Sz = Sz + t->m[k] * t->z[k];
            }
        } else {
            for (int64_t c = t->child_first[id]; c < t->child_first[id] + t->n_child[id]; c++) {
                Mc = Mc + t->M[c];
                Sx = Sx + S[3 * c];
                Sy = Sy + S[3 * c + 1];
                Sz = Sz + S[3 * c + 2];
            }
        }
        t->M[id] = Mc;
        S[3 * id] = Sx; S[3 * id + 1] = Sy; S[3 * id + 2] = Sz;
        double cx = Sx / Mc, cy = Sy / Mc, cz = Sz / Mc;
        t->com[3 * id] = cx; t->com[3 * id + 1] = cy; t->com[3 * id + 2] = cz;
        double q[6] = {0, 0, 0, 0, 0, 0};
        double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t k = t->first[id]; k < t->first[id] + t->count[id]; k++) {
            double d[3] = {t->x[k] - cx, t->y[k] - cy, t->z[k] - cz};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double mk = t->m[k];
            q[0] += mk * (3.0 * d[0] * d[0] - r2);
            q[1] += mk * (3.0 * d[1] * d[1] - r2);
            q[2] += mk * (3.0 * d[2] * d[2] - r2);
            q[3] += mk * 3.0 * d[0] * d[1];
            q[4] += mk * 3.0 * d[0] * d[2];
            q[5] += mk * 3.0 * d[1] * d[2];
            double pk[3] = {t->x[k], t->y[k], t->z[k]};
            for (int a = 0; a < 3; a++) {
                if (pk[a] < lo3[a]) lo3[a] = pk[a];
                if (pk[a] > hi3[a]) hi3[a] = pk[a];
            }
        }
        for (int a = 0; a < 6; a++) t->Q[6 * id + a] = q[a];
        for (int a = 0; a < 3; a++) { t->blo[3 * id + a] = lo3[a]; t->bhi[3 * id + a] = hi3[a]; }
        t->side[id] = ldexp(t->L, -t->level[id]);
    }
    free(S);

}

/* ------------------------------------------------------------------------ */
/* Build: root, keys, sort, tree, moments, groups, walk.                      */
/* ------------------------------------------------------------------------ */

/* Build with the walk restricted to every walk_stride-th group (walk_stride = 1:
 * all groups); the lists of the other groups are left empty.  Used to sample
 * very large problems. */
int or_build_ex(int64_t n, const double *pos, const double *mass, const or_params *p,
                int64_t walk_stride, or_tree **out);

int or_build(int64_t n, const double *pos, const double *mass, const or_params *p, or_tree **out)
{
    return or_build_ex(n, pos, mass, p, 1, out);
}

int or_build_ex(int64_t n, const double *pos, const double *mass, const or_params *p,
                int64_t walk_stride, or_tree **out)
{
    if (walk_stride < 1) return -1;
    if (n < 1 || !pos || !mass || !p || !out) return -1;
    or_tree *t = calloc(1, sizeof(or_tree));
    t->n = n;
    t->p = *p;

    /* root cube */
    double hi[3];
    for (int a = 0; a < 3; a++) { t->lo[a] = pos[a]; hi[a] = pos[a]; }
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            double v = pos[3 * i + a];
            if (v < t->lo[a]) t->lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double ext = 0.0;
    for (int a = 0; a < 3; a++) {
        double e = hi[a] - t->lo[a];
        if (e > ext) ext = e;
    }
    t->L = root_side(ext);

    /* keys */
    t->key = malloc(n * sizeof(uint64_t));
    for (int64_t i = 0; i < n; i++)
        t->key[i] = or_morton(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], t->lo, t->L);

    /* stable sort */
    t->perm = malloc(n * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) t->perm[i] = i;
    g_sort_keys = t->key;
    qsort(t->perm, n, sizeof(int64_t), cmp_key_idx);
    t->skey = malloc(n * sizeof(uint64_t));
    t->x = malloc(n * sizeof(double));
    t->y = malloc(n * sizeof(double));
    t->z = malloc(n * sizeof(double));
    t->m = malloc(n * sizeof(double));
    for (int64_t s = 0; s < n; s++) {
        int64_t o = t->perm[s];
        t->skey[s] = t->key[o];
        t->x[s] = pos[3 * o];
        t->y[s] = pos[3 * o + 1];
        t->z[s] = pos[3 * o + 2];
        t->m[s] = mass[o];
    }

    /* octree, breadth first: children appended in octant order */
    int64_t root = add_node(t, 0, 0, 0, -1);
    t->count[root] = n;
    for (int64_t id = 0; id < t->n_nodes; id++) {
        int32_t lev = t->level[id];
        if (t->count[id] <= t->p.n_leaf || lev >= OR_MAX_LEVEL) continue;
        int shift = 3 * (OR_MAX_LEVEL - (lev + 1));
        int64_t f = t->first[id], e = f + t->count[id];
        int64_t cur = -1;
        uint64_t prev = 0;
        for (int64_t k = f; k < e; k++) {
            uint64_t pf = t->skey[k] >> shift;
            if (k == f || pf != prev) {
                int64_t c = add_node(t, lev + 1, k, pf, id);
                if (k == f) t->child_first[id] = c;
                t->n_child[id]++;
                if (cur >= 0) t->count[cur] = k - t->first[cur];
                cur = c;
                prev = pf;
            }
        }
        t->count[cur] = e - t->first[cur];
    }

    compute_moments(t);
    int64_t nn = t->n_nodes;

    /* groups */
    int64_t ng = 0;
    int64_t *tmp = malloc(nn * sizeof(int64_t));
    for (int64_t id = 0; id < nn; id++) {
        int cand = (t->count[id] <= t->p.n_crit) || is_leaf(t, id);
        int top = (t->parent[id] < 0) || (t->count[t->parent[id]] > t->p.n_crit);
        if (cand && top) tmp[ng++] = id;
    }
    /* order by first particle: group ranges are disjoint, so sort (first, id) */
    int64_t *order = malloc(ng * 2 * sizeof(int64_t));
    for (int64_t k = 0; k < ng; k++) { order[2 * k] = t->first[tmp[k]]; order[2 * k + 1] = tmp[k]; }
    qsort(order, ng, 2 * sizeof(int64_t), cmp_i64);
    t->n_groups = ng;
    t->grp = malloc((ng ? ng : 1) * sizeof(int64_t));
    for (int64_t k = 0; k < ng; k++) t->grp[k] = order[2 * k + 1];
    free(order);
    free(tmp);

    /* walk: per group, visit cells from the root */
    int64_t **cl = calloc(ng, sizeof(int64_t *)), **pl = calloc(ng, sizeof(int64_t *));
    int64_t *cn = calloc(ng, sizeof(int64_t)), *pn = calloc(ng, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t gi = 0; gi < ng; gi++) {
        if (gi % walk_stride != 0) {
            cl[gi] = malloc(sizeof(int64_t));
            pl[gi] = malloc(sizeof(int64_t));
            continue;
        }
        int64_t g = t->grp[gi];
        int64_t ccap = 64, pcap = 256, scap = 256, sp = 0;
        int64_t *cc = malloc(ccap * sizeof(int64_t)), *pp = malloc(pcap * sizeof(int64_t));
        int64_t *stk = malloc(scap * sizeof(int64_t));
        int64_t nc = 0, np = 0;
        stk[sp++] = 0;
        while (sp > 0) {
            int64_t c = stk[--sp];
            if (accept_cell(t, c, g)) {
                if (nc == ccap) { ccap *= 2; cc = realloc(cc, ccap * sizeof(int64_t)); }
                cc[nc++] = c;
            } else if (is_leaf(t, c)) {
                for (int64_t k = t->first[c]; k < t->first[c] + t->count[c]; k++) {
                    if (np == pcap) { pcap *= 2; pp = realloc(pp, pcap * sizeof(int64_t)); }
                    pp[np++] = k;
                }
            } else {
                for (int64_t ch = t->child_first[c]; ch < t->child_first[c] + t->n_child[c]; ch++) {
                    if (sp == scap) { scap *= 2; stk = realloc(stk, scap * sizeof(int64_t)); }
                    stk[sp++] = ch;
                }
            }
        }
        free(stk);
        qsort(cc, nc, sizeof(int64_t), cmp_i64);
        qsort(pp, np, sizeof(int64_t), cmp_i64);
        cl[gi] = cc; pl[gi] = pp; cn[gi] = nc; pn[gi] = np;
    }
    t->c_off = malloc((ng + 1) * sizeof(int64_t));
    t->p_off = malloc((ng + 1) * sizeof(int64_t));
    t->c_off[0] = 0; t->p_off[0] = 0;
    t->n_pp = 0; t->n_pc = 0;
    for (int64_t gi = 0; gi < ng; gi++) {
        t->c_off[gi + 1] = t->c_off[gi] + cn[gi];
        t->p_off[gi + 1] = t->p_off[gi] + pn[gi];
        int64_t n_g = t->count[t->grp[gi]];
        t->n_pp += n_g * pn[gi];
        t->n_pc += n_g * cn[gi];
    }
    t->c_idx = malloc((t->c_off[ng] ? t->c_off[ng] : 1) * sizeof(int64_t));
    t->p_idx = malloc((t->p_off[ng] ? t->p_off[ng] : 1) * sizeof(int64_t));
    for (int64_t gi = 0; gi < ng; gi++) {
        memcpy(t->c_idx + t->c_off[gi], cl[gi], cn[gi] * sizeof(int64_t));
        memcpy(t->p_idx + t->p_off[gi], pl[gi], pn[gi] * sizeof(int64_t));
        free(cl[gi]); free(pl[gi]);
    }
    free(cl); free(pl); free(cn); free(pn);
    *out = t;
    return 0;
}

void or_free(or_tree *t)
{
    if (!t) return;
    void *ptrs[] = {t->key, t->perm, t->skey, t->x, t->y, t->z, t->m, t->level, t->first,
                    t->count, t->child_first, t->parent, t->n_child, t->prefix, t->M, t->com,
                    t->Q, t->blo, t->bhi, t->side, t->grp, t->c_off, t->c_idx, t->p_off, t->p_idx};
    for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); k++) free(ptrs[k]);
    free(t);
}


/* Replace positions and masses, keeping keys, order, topology, groups and lists
 * frozen; moments are recomputed.  Used for finite differences with frozen lists. */
int or_refresh(or_tree *t, const double *pos, const double *mass)
{
    for (int64_t s = 0; s < t->n; s++) {
        int64_t o = t->perm[s];
        t->x[s] = pos[3 * o];
        t->y[s] = pos[3 * o + 1];
        t->z[s] = pos[3 * o + 2];
        t->m[s] = mass[o];
    }
    compute_moments(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Force and potential.                                                       */
/* ------------------------------------------------------------------------ */

/* Particle-particle term of particle i (sorted) from j (sorted). */
static void pp_term(const or_tree *t, int64_t i, int64_t j, double acc[3], double *phi)
{
    double gam = t->p.r_in / t->p.r_out;
    double d[3] = {t->x[j] - t->x[i], t->y[j] - t->y[i], t->z[j] - t->z[i]};
    double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + t->p.eps * t->p.eps;
    double s = sqrt(s2);
    double y = s / t->p.r_out;
    double K = or_K(y, gam);
    double f = t->m[j] * K / (s2 * s);
    for (int a = 0; a < 3; a++) acc[a] += f * d[a];
    *phi -= t->m[j] * or_W_over_y(y, gam) / t->p.r_out;
}

/* Particle-cell term of particle i (sorted) from cell c. */
static void pc_term(const or_tree *t, int64_t i, int64_t c, double acc[3], double *phi)
{
    double gam = t->p.r_in / t->p.r_out;
    const double *cm = t->com + 3 * c;
    double r[3] = {t->x[i] - cm[0], t->y[i] - cm[1], t->z[i] - cm[2]};
    double s2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + t->p.eps * t->p.eps;
    double s = sqrt(s2);
    double y = s / t->p.r_out;
    double K = or_K(y, gam);
    double Wy = or_W_over_y(y, gam);    /* W / y */
    double W = Wy * y;
    double M = t->M[c];
    double s3 = s2 * s;
    double a[3], ph;
    for (int k = 0; k < 3; k++) a[k] = -M * r[k] / s3;
    ph = -M / s;
    if (t->p.use_quadrupole) {
        const double *q = t->Q + 6 * c;
        double Qr[3] = {q[0] * r[0] + q[3] * r[1] + q[4] * r[2],
                        q[3] * r[0] + q[1] * r[1] + q[5] * r[2],
                        q[4] * r[0] + q[5] * r[1] + q[2] * r[2]};
        double rQr = r[0] * Qr[0] + r[1] * Qr[1] + r[2] * Qr[2];
        double s5 = s3 * s2, s7 = s5 * s2;
        for (int k = 0; k < 3; k++) a[k] += Qr[k] / s5 - 2.5 * rQr * r[k] / s7;
        ph += -0.5 * rQr / s5;
    }
    for (int k = 0; k < 3; k++) acc[k] += K * a[k];
    /* W multiplies the whole cell potential; below r_in it is C(gamma) y */
    *phi += W * ph;
}

/* acc [n][3], pot [n] in original particle order */
int or_force(const or_tree *t, double *acc, double *pot)
{
    int64_t ng = t->n_groups;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t gi = 0; gi < ng; gi++) {
        int64_t g = t->grp[gi];
        for (int64_t i = t->first[g]; i < t->first[g] + t->count[g]; i++) {
            double a[3] = {0, 0, 0}, ph = 0.0;
            for (int64_t k = t->p_off[gi]; k < t->p_off[gi + 1]; k++) {
                int64_t j = t->p_idx[k];
                if (j != i) pp_term(t, i, j, a, &ph);
            }
            for (int64_t k = t->c_off[gi]; k < t->c_off[gi + 1]; k++) pc_term(t, i, t->c_idx[k], a, &ph);
            int64_t o = t->perm[i];
            acc[3 * o] = a[0]; acc[3 * o + 1] = a[1]; acc[3 * o + 2] = a[2];
            if (pot) pot[o] = ph;
        }
    }
    return 0;
}

/* Forces of the members of the listed groups only (rows of other particles
 * are left untouched); used to sample large problems. */
int or_force_groups(const or_tree *t, const int64_t *gids, int64_t ng, double *acc, double *pot)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ng; k++) {
        int64_t gi = gids[k];
        int64_t g = t->grp[gi];
        for (int64_t i = t->first[g]; i < t->first[g] + t->count[g]; i++) {
            double a[3] = {0, 0, 0}, ph = 0.0;
            for (int64_t q = t->p_off[gi]; q < t->p_off[gi + 1]; q++) {
                int64_t j = t->p_idx[q];
                if (j != i) pp_term(t, i, j, a, &ph);
            }
            for (int64_t q = t->c_off[gi]; q < t->c_off[gi + 1]; q++) pc_term(t, i, t->c_idx[q], a, &ph);
            int64_t o = t->perm[i];
            acc[3 * o] = a[0]; acc[3 * o + 1] = a[1]; acc[3 * o + 2] = a[2];
            if (pot) pot[o] = ph;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists: CSR in original order, ascending original indices.        */
/* ------------------------------------------------------------------------ */

/* Pass 1 (idx == NULL): counts into offsets[1..n]; pass 2: fill. */
int or_neighbors(const or_tree *t, int64_t *offsets, int64_t *idx)
{
    int64_t n = t->n, ng = t->n_groups;
    double h2 = t->p.r_search * t->p.r_search;
    if (!idx) {
        memset(offsets, 0, (n + 1) * sizeof(int64_t));
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t gi = 0; gi < ng; gi++) {
        int64_t g = t->grp[gi];
        for (int64_t i = t->first[g]; i < t->first[g] + t->count[g]; i++) {
            int64_t o = t->perm[i], cnt = 0;
            int64_t base = idx ? offsets[o] : 0;
            for (int64_t k = t->p_off[gi]; k < t->p_off[gi + 1]; k++) {
                int64_t j = t->p_idx[k];
                if (j == i) continue;
                double dx = t->x[j] - t->x[i], dy = t->y[j] - t->y[i], dz = t->z[j] - t->z[i];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < h2) {
                    if (idx) idx[base + cnt] = t->perm[j];
                    cnt++;
                }
            }
            if (!idx) offsets[o + 1] = cnt;
            else qsort(idx + base, cnt, sizeof(int64_t), cmp_i64);
        }
    }
    if (!idx)
        for (int64_t i = 0; i < n; i++) offsets[i + 1] += offsets[i];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Vector-Jacobian product of L = sum_i w_i . a_i + c_i phi_i with respect to */
/* positions and masses, lists and tree frozen.                               */
/* ------------------------------------------------------------------------ */

int or_vjp(const or_tree *t, const double *w, const double *cw, double *gpos, double *gmass)
{
    int64_t n = t->n, nn = t->n_nodes, ng = t->n_groups;
    double gam = t->p.r_in / t->p.r_out, ro = t->p.r_out, e2 = t->p.eps * t->p.eps;
    double *gx = calloc(3 * n, sizeof(double)), *gm = calloc(n, sizeof(double)); /* sorted */
    double *gcom = calloc(3 * nn, sizeof(double)), *gM = calloc(nn, sizeof(double));
    double *gQ = calloc(9 * nn, sizeof(double));
    /* sequential: scatter to j and to cells would race */
    for (int64_t gi = 0; gi < ng; gi++) {
        int64_t g = t->grp[gi];
        for (int64_t i = t->first[g]; i < t->first[g] + t->count[g]; i++) {
            int64_t o = t->perm[i];
            double wi[3] = {w[3 * o], w[3 * o + 1], w[3 * o + 2]};
            double ci = cw ? cw[o] : 0.0;
            for (int64_t k = t->p_off[gi]; k < t->p_off[gi + 1]; k++) {
                int64_t j = t->p_idx[k];
                if (j == i) continue;
                double d[3] = {t->x[j] - t->x[i], t->y[j] - t->y[i], t->z[j] - t->z[i]};
                double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + e2;
                double s = sqrt(s2), s3 = s2 * s, s4 = s2 * s2;
                double y = s / ro;
                double K = or_K(y, gam), dK = or_dK(y, gam) / ro;
                double W = or_W_over_y(y, gam) * y;
                double gs = K / s3, dgs = dK / s3 - 3.0 * K / s4;
                double wd = wi[0] * d[0] + wi[1] * d[1] + wi[2] * d[2];
                double mj = t->m[j];
                for (int a = 0; a < 3; a++) {
                    double gd = mj * (gs * wi[a] + dgs * wd * d[a] / s + ci * K * d[a] / s3);
                    gx[3 * j + a] += gd;
                    gx[3 * i + a] -= gd;
                }
                gm[j] += gs * wd - ci * W / s;
            }
            for (int64_t k = t->c_off[gi]; k < t->c_off[gi + 1]; k++) {
                int64_t c = t->c_idx[k];
                const double *cm = t->com + 3 * c;
                double r[3] = {t->x[i] - cm[0], t->y[i] - cm[1], t->z[i] - cm[2]};
                double s2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + e2;
                double s = sqrt(s2), s3 = s2 * s, s5 = s3 * s2, s7 = s5 * s2, s9 = s7 * s2;
                double y = s / ro;
                double K = or_K(y, gam), dK = or_dK(y, gam);
                double W = or_W_over_y(y, gam) * y;
                double dW = (y > 0.0) ? (W - K) / y : 0.0;   /* K = W - y W' */
                double M = t->M[c];
                double Q[9] = {0};
                if (t->p.use_quadrupole) {
                    const double *q = t->Q + 6 * c;
                    Q[0] = q[0]; Q[4] = q[1]; Q[8] = q[2];
                    Q[1] = Q[3] = q[3]; Q[2] = Q[6] = q[4]; Q[5] = Q[7] = q[5];
                }
                double Qr[3], Qw[3];
                for (int a = 0; a < 3; a++) {
                    Qr[a] = Q[3 * a] * r[0] + Q[3 * a + 1] * r[1] + Q[3 * a + 2] * r[2];
                    Qw[a] = Q[3 * a] * wi[0] + Q[3 * a + 1] * wi[1] + Q[3 * a + 2] * wi[2];
                }
                double q = r[0] * Qr[0] + r[1] * Qr[1] + r[2] * Qr[2];
                double rw = r[0] * wi[0] + r[1] * wi[1] + r[2] * wi[2];
                double Qrw = Qr[0] * wi[0] + Qr[1] * wi[1] + Qr[2] * wi[2];
                double A[3], Hw[3];
                for (int a = 0; a < 3; a++) {
                    A[a] = -M * r[a] / s3 + Qr[a] / s5 - 2.5 * q * r[a] / s7;
                    /* Hessian of the cell potential applied to w */
                    double hq = 2.0 * Qw[a] / s5 - 10.0 * Qr[a] * rw / s7 - 10.0 * r[a] * Qrw / s7
                                - 5.0 * q * wi[a] / s7 + 35.0 * q * r[a] * rw / s9;
                    Hw[a] = M * wi[a] / s3 - 3.0 * M * r[a] * rw / s5 - 0.5 * hq;
                }
                double Phi = -M / s - 0.5 * q / s5;
                double wA = wi[0] * A[0] + wi[1] * A[1] + wi[2] * A[2];
                for (int a = 0; a < 3; a++) {
                    double gr = dK / ro * wA * r[a] / s + ci * dW / ro * Phi * r[a] / s
                                - K * Hw[a] - ci * W * A[a];
                    gx[3 * i + a] += gr;
                    gcom[3 * c + a] -= gr;
                }
                gM[c] += K * (-rw / s3) - ci * W / s;
                if (t->p.use_quadrupole)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            gQ[9 * c + 3 * a + b] += K * (wi[a] * r[b] / s5 - 2.5 * rw * r[a] * r[b] / s7)
                                                   - ci * W * 0.5 * r[a] * r[b] / s5;
            }
        }
    }
    /* push cell adjoints down to member particles */
    for (int64_t c = 0; c < nn; c++) {
        double M = t->M[c];
        const double *cm = t->com + 3 * c;
        const double *Qb = gQ + 9 * c;
        double tr = Qb[0] + Qb[4] + Qb[8];
        if (gM[c] == 0.0 && gcom[3 * c] == 0.0 && gcom[3 * c + 1] == 0.0 && gcom[3 * c + 2] == 0.0 &&
            tr == 0.0) {
            int nz = 0;
            for (int a = 0; a < 9; a++) nz |= (Qb[a] != 0.0);
            if (!nz) continue;
        }
        for (int64_t k = t->first[c]; k < t->first[c] + t->count[c]; k++) {
            double d[3] = {t->x[k] - cm[0], t->y[k] - cm[1], t->z[k] - cm[2]};
            double mk = t->m[k];
            double dQd = 0.0, d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            for (int a = 0; a < 3; a++) {
                double sym = 0.0;
                for (int b = 0; b < 3; b++) {
                    sym += (Qb[3 * a + b] + Qb[3 * b + a]) * d[b];
                    dQd += d[a] * Qb[3 * a + b] * d[b];
                }
                gx[3 * k + a] += mk / M * gcom[3 * c + a] + mk * (3.0 * sym - 2.0 * tr * d[a]);
            }
            gm[k] += gM[c] + (d[0] * gcom[3 * c] + d[1] * gcom[3 * c + 1] + d[2] * gcom[3 * c + 2]) / M
                     + 3.0 * dQd - d2 * tr;
        }
    }
    for (int64_t s = 0; s < n; s++) {
        int64_t o = t->perm[s];
        for (int a = 0; a < 3; a++) gpos[3 * o + a] = gx[3 * s + a];
        gmass[o] = gm[s];
    }
    free(gx); free(gm); free(gcom); free(gM); free(gQ);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Accessors for the ctypes wrapper.                                          */
/* ------------------------------------------------------------------------ */

int64_t or_n_nodes(const or_tree *t) { return t->n_nodes; }
int64_t or_n_groups(const or_tree *t) { return t->n_groups; }
void or_root(const or_tree *t, double lo_L[4])
{
    lo_L[0] = t->lo[0]; lo_L[1] = t->lo[1]; lo_L[2] = t->lo[2]; lo_L[3] = t->L;
}
void or_counts(const or_tree *t, int64_t out[4])
{
    out[0] = t->c_off[t->n_groups];
    out[1] = t->p_off[t->n_groups];
    out[2] = t->n_pc;
    out[3] = t->n_pp;
}

/* Copy out: keys/perm (n); node topology (n_nodes); node moments; groups; lists. */
void or_get_keys(const or_tree *t, uint64_t *key, int64_t *perm)
{
    memcpy(key, t->key, t->n * sizeof(uint64_t));
    memcpy(perm, t->perm, t->n * sizeof(int64_t));
}
void or_get_nodes(const or_tree *t, int32_t *level, int64_t *first, int64_t *count,
                  int64_t *child_first, int32_t *n_child, uint64_t *prefix, int64_t *parent)
{
    int64_t nn = t->n_nodes;
    memcpy(level, t->level, nn * sizeof(int32_t));
    memcpy(first, t->first, nn * sizeof(int64_t));
    memcpy(count, t->count, nn * sizeof(int64_t));
    memcpy(child_first, t->child_first, nn * sizeof(int64_t));
    memcpy(n_child, t->n_child, nn * sizeof(int32_t));
    memcpy(prefix, t->prefix, nn * sizeof(uint64_t));
    memcpy(parent, t->parent, nn * sizeof(int64_t));
}
void or_get_moments(const or_tree *t, double *M, double *com, double *Q, double *blo, double *bhi,
                    double *side)
{
    int64_t nn = t->n_nodes;
    memcpy(M, t->M, nn * sizeof(double));
    memcpy(com, t->com, 3 * nn * sizeof(double));
    memcpy(Q, t->Q, 6 * nn * sizeof(double));
    memcpy(blo, t->blo, 3 * nn * sizeof(double));
    memcpy(bhi, t->bhi, 3 * nn * sizeof(double));
    memcpy(side, t->side, nn * sizeof(double));
}
void or_get_groups(const or_tree *t, int64_t *grp) { memcpy(grp, t->grp, t->n_groups * sizeof(int64_t)); }
void or_get_lists(const or_tree *t, int64_t *c_off, int64_t *c_idx, int64_t *p_off, int64_t *p_idx)
{
    int64_t ng = t->n_groups;
    memcpy(c_off, t->c_off, (ng + 1) * sizeof(int64_t));
    memcpy(p_off, t->p_off, (ng + 1) * sizeof(int64_t));
    memcpy(c_idx, t->c_idx, t->c_off[ng] * sizeof(int64_t));
    memcpy(p_idx, t->p_idx, t->p_off[ng] * sizeof(int64_t));
}
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel regions (k < 1: leave as is). */
void or_set_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
