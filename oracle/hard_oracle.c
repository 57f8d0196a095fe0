/*
 * hard_oracle.c -- plain FP64 CPU oracle for the hard part of the P3T scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests and the benchmark's CPU baseline use it.  It
 * shares no source with the GPU library.
 *
 * What it computes, in the order of the method (Section 2.1):
 *
 *   hard force   F_hard,i / m_i = sum_j m_j (1 - K(s_ij)) d_ij / s_ij^3 over the
 *                particles j on i's neighbour list (Section 2.2: the hard force
 *                is evaluated over the list of particles within h), with
 *                d_ij = x_j - x_i and the softened distance s_ij;
 *   its jerk     the time derivative along the motion, v_ij = v_j - v_i,
 *                ds/dt = (d.v)/s:
 *                  j_i = sum_j m_j [ (1 - K) (v - 3 (d.v) d / s^2) / s^3
 *                                    - K'(s) ((d.v)/s) d / s^3 ];
 *   hard potential  phi_i = -sum_j m_j (1 - W(s_ij)) / s_ij (the pair term of
 *                H_hard);
 *   integration  of H_hard over one soft step with the fourth-order Hermite
 *                scheme and block timesteps (Section 2.1, step 3; timestep
 *                criteria of Section 2.1, the first-step form with eta_s):
 *                predictor x_p = x + v dt + a dt^2/2 + j dt^3/6,
 *                          v_p = v + a dt + j dt^2/2;
 *                force and jerk of the active particles from predicted states;
 *                second and third derivatives at the start of the step by
 *                interpolation of a and j at both ends,
 *                  a2 = (-6 (a0 - a1) - dt (4 j0 + 2 j1)) / dt^2,
 *                  a3 = (12 (a0 - a1) + 6 dt (j0 + j1)) / dt^3;
 *                corrector x = x_p + a2 dt^4/24 + a3 dt^5/120,
 *                          v = v_p + a2 dt^3/6 + a3 dt^4/24;
 *                derivatives carried to the end of the step: a2 + a3 dt, a3.
 *                Particles with an empty neighbour list are isolated and drift.
 *
 * Conventions (the paper leaves them open):
 *   timesteps   dt_soft is a whole multiple of dt_max (so every block step ends
 *               inside the soft step); dt_i = dt_max / 2^k, k <= OR_MAX_LEVEL; the first dt is the
 *               largest such value not above the first-step criterion; later
 *               the step doubles when 2 dt fits the criterion, 2 dt <= dt_max
 *               and t_i is a multiple of 2 dt, else it halves until it fits (or
 *               reaches dt_max / 2^OR_MAX_LEVEL); a criterion whose denominator
 *               is zero allows dt_max;
 *   block step  t_next = min_i (t_i + dt_i); every particle with
 *               t_i + dt_i == t_next is active; all non-isolated particles are
 *               predicted to t_next, then all active forces are evaluated, then
 *               all active particles are corrected;
 *   a0          the softening term of the criteria is passed in (alpha m / r_cut^2
 *               with m chosen by the caller);
 *   kinds       optionally the last n_special particles are special (the SMBHs of
 *               Section 3.2.2): a normal-special pair takes its own r_in, r_cut and
 *               softening, a special-special pair its own softening and, when it
 *               is not split, K = W = 0 (the pair is wholly hard: no soft force);
 *               special particles take their own eta and eta_s.
 *
 * Compiled with -ffp-contract=off and without fast-math, like the tree oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_LEVEL 40
#define OR_MAX_BLOCK_STEPS (1LL << 26)

double or_K(double y, double gam);
double or_dK(double y, double gam);
double or_W(double y, double g);

typedef struct {
    double dt_soft, dt_max, eta, eta_s, a0;
} or_hermite_params;

typedef struct {
    int64_t n_special;                 /* the last n_special particles are special */
    double r_in_ns, r_out_ns, eps_ns;  /* normal-special pairs */
    int32_t split_ss;                  /* special-special: 0 = wholly hard */
    double r_in_ss, r_out_ss, eps_ss;
    double eta_sp, eta_s_sp;           /* timestep accuracy of special particles */
} or_kinds;

typedef struct {
    double eps, r_in, r_out;
    int split;
} or_pair;

/* parameters of the pair (i, j) by the kinds of i and j */
static or_pair pair_of(int64_t n, const or_kinds *kd, int64_t i, int64_t j, double eps,
                       double r_in, double r_out)
{
    const int64_t first = kd ? n - kd->n_special : n;
    const int si = i >= first, sj = j >= first;
    or_pair q = {eps, r_in, r_out, 1};
    if (si && sj) {
        q.eps = kd->eps_ss;
        q.r_in = kd->r_in_ss;
        q.r_out = kd->r_out_ss;
        q.split = kd->split_ss;
    } else if (si || sj) {
        q.eps = kd->eps_ns;
        q.r_in = kd->r_in_ns;
        q.r_out = kd->r_out_ns;
    }
    return q;
}

/* Hard force, jerk and potential on particle i from its list, at the given
 * positions and velocities ([n][3] row-major). */
static void hard_one(int64_t n, const or_kinds *kd, int64_t i, const double *pos,
                     const double *vel, const double *mass, const int64_t *off,
                     const int32_t *idx, double eps0, double r_in0, double r_out0, double a[3],
                     double jk[3], double *phi)
{
    a[0] = a[1] = a[2] = 0.0;
    jk[0] = jk[1] = jk[2] = 0.0;
    double p = 0.0;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        const int64_t j = idx[e];
        const or_pair q = pair_of(n, kd, i, j, eps0, r_in0, r_out0);
        const double eps = q.eps, r_out = q.r_out, gam = q.r_in / q.r_out;
        const double dx = pos[3 * j] - pos[3 * i];
        const double dy = pos[3 * j + 1] - pos[3 * i + 1];
        const double dz = pos[3 * j + 2] - pos[3 * i + 2];
        const double vx = vel[3 * j] - vel[3 * i];
        const double vy = vel[3 * j + 1] - vel[3 * i + 1];
        const double vz = vel[3 * j + 2] - vel[3 * i + 2];
        const double s2 = dx * dx + dy * dy + dz * dz + eps * eps;
        const double s = sqrt(s2);
        const double y = s / r_out;
        /* a pair that is not split is wholly hard: K = W = 0 */
        const double K = q.split ? or_K(y, gam) : 0.0;
        const double Ks = q.split ? or_dK(y, gam) / r_out : 0.0;   /* dK/ds */
        const double W = q.split ? or_W(y, gam) : 0.0;
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
        p -= mj * (1.0 - W) / s;
    }
    if (phi) *phi = p;
}

int or_hard_force(int64_t n, const double *pos, const double *vel, const double *mass,
                  const int64_t *off, const int32_t *idx, double eps, double r_in, double r_out,
                  const or_kinds *kd, double *acc, double *jerk, double *pot)
{
    for (int64_t i = 0; i < n; ++i)
        hard_one(n, kd, i, pos, vel, mass, off, idx, eps, r_in, r_out, acc + 3 * i,
                 jerk + 3 * i, pot ? pot + i : NULL);
    return 0;
}

static double norm3(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* Timestep criterion of later steps (Section 2.1), with the first term of the
 * denominator read as |a^(1)| |a^(3)|: as printed, |a^(0)| |a^(3)| would not
 * have the units of the other terms (a^2 / time^4). */
static double crit_full(const double *a, const double *j, const double *a2, const double *a3,
                        const or_hermite_params *hp, double eta)
{
    const double na = norm3(a), nj = norm3(j), n2 = norm3(a2), n3 = norm3(a3);
    const double num = sqrt(na * na + hp->a0 * hp->a0) * n2 + nj * nj;
    const double den = nj * n3 + n2 * n2;
    if (den == 0.0) return hp->dt_max;
    return eta * sqrt(num / den);
}

/* First-step criterion (Section 2.1, with eta_s). */
static double crit_first(const double *a, const double *j, const or_hermite_params *hp,
                         double eta_s)
{
    const double na = norm3(a), nj = norm3(j);
    if (nj == 0.0) return hp->dt_max;
    return eta_s * sqrt((na * na + hp->a0 * hp->a0) / (nj * nj));
}

/*
 * Integrate H_hard over hp->dt_soft (in place on pos and vel).  nsteps[i]
 * receives the number of Hermite steps of particle i (0 for isolated ones).
 * Returns 0, -1 on invalid parameters, -2 when the block-step cap is reached.
 */
int or_hermite(int64_t n, double *pos, double *vel, const double *mass, const int64_t *off,
               const int32_t *idx, double eps, double r_in, double r_out,
               const or_hermite_params *hp, const or_kinds *kd, int32_t *nsteps,
               int64_t *n_block_steps)
{
    const int64_t first_sp = kd ? n - kd->n_special : n;
    if (!(hp->dt_soft > 0.0) || !(hp->dt_max > 0.0) || hp->dt_max > hp->dt_soft ||
        fmod(hp->dt_soft, hp->dt_max) != 0.0)
        return -1;
    const double t_end = hp->dt_soft;
    const double dt_min = ldexp(hp->dt_max, -OR_MAX_LEVEL);
    double *a = calloc(3 * n, sizeof(double)), *jk = calloc(3 * n, sizeof(double));
    double *a2 = calloc(3 * n, sizeof(double)), *a3 = calloc(3 * n, sizeof(double));
    double *xp = malloc(3 * n * sizeof(double)), *vp = malloc(3 * n * sizeof(double));
    double *a1 = calloc(3 * n, sizeof(double)), *j1 = calloc(3 * n, sizeof(double));
    double *t = calloc(n, sizeof(double)), *dt = calloc(n, sizeof(double));
    char *hard = calloc(n, 1);
    int rc = 0;
    for (int64_t i = 0; i < n; ++i) {
        hard[i] = off[i + 1] > off[i];
        nsteps[i] = 0;
    }
    /* the lists must be symmetric: every listed particle is itself non-isolated */
    for (int64_t i = 0; i < n && rc == 0; ++i)
        for (int64_t e = off[i]; e < off[i + 1]; ++e)
            if (idx[e] < 0 || idx[e] >= n || idx[e] == i || !hard[idx[e]]) rc = -1;
    if (rc) {
        free(a); free(jk); free(a2); free(a3); free(xp); free(vp); free(a1); free(j1);
        free(t); free(dt); free(hard);
        return rc;
    }
    /* isolated particles drift through the whole soft step */
    for (int64_t i = 0; i < n; ++i)
        if (!hard[i])
            for (int k = 0; k < 3; ++k) pos[3 * i + k] += t_end * vel[3 * i + k];
    /* initial force, jerk and timestep */
    for (int64_t i = 0; i < n; ++i) {
        if (!hard[i]) continue;
        hard_one(n, kd, i, pos, vel, mass, off, idx, eps, r_in, r_out, a + 3 * i, jk + 3 * i,
                 NULL);
        const double c = crit_first(a + 3 * i, jk + 3 * i, hp,
                                    i >= first_sp ? kd->eta_s_sp : hp->eta_s);
        double d = hp->dt_max;
        while (d > c && d > dt_min) d *= 0.5;
        dt[i] = d;
    }
    int64_t steps = 0;
    for (;;) {
        double t_next = INFINITY;
        for (int64_t i = 0; i < n; ++i)
            if (hard[i] && t[i] + dt[i] < t_next) t_next = t[i] + dt[i];
        if (!(t_next <= t_end)) break;           /* every particle is at t_end */
        if (++steps > OR_MAX_BLOCK_STEPS) { rc = -2; break; }
        /* predict every non-isolated particle to t_next */
        for (int64_t i = 0; i < n; ++i) {
            if (!hard[i]) continue;
            const double h = t_next - t[i];
            for (int k = 0; k < 3; ++k) {
                const int64_t q = 3 * i + k;
                xp[q] = pos[q] + vel[q] * h + a[q] * (h * h / 2.0) + jk[q] * (h * h * h / 6.0);
                vp[q] = vel[q] + a[q] * h + jk[q] * (h * h / 2.0);
            }
        }
        /* forces of the active particles from the predicted states */
        for (int64_t i = 0; i < n; ++i)
            if (hard[i] && t[i] + dt[i] == t_next)
                hard_one(n, kd, i, xp, vp, mass, off, idx, eps, r_in, r_out, a1 + 3 * i,
                         j1 + 3 * i, NULL);
        /* correct them and choose their next timesteps */
        for (int64_t i = 0; i < n; ++i) {
            if (!(hard[i] && t[i] + dt[i] == t_next)) continue;
            const double h = dt[i];
            for (int k = 0; k < 3; ++k) {
                const int64_t q = 3 * i + k;
                const double s2 = (-6.0 * (a[q] - a1[q]) - h * (4.0 * jk[q] + 2.0 * j1[q])) / (h * h);
                const double s3 = (12.0 * (a[q] - a1[q]) + 6.0 * h * (jk[q] + j1[q])) / (h * h * h);
                pos[q] = xp[q] + s2 * (h * h * h * h / 24.0) + s3 * (h * h * h * h * h / 120.0);
                vel[q] = vp[q] + s2 * (h * h * h / 6.0) + s3 * (h * h * h * h / 24.0);
                a[q] = a1[q];
                jk[q] = j1[q];
                a2[q] = s2 + s3 * h;
                a3[q] = s3;
            }
            t[i] = t_next;
            nsteps[i] += 1;
            const double c = crit_full(a + 3 * i, jk + 3 * i, a2 + 3 * i, a3 + 3 * i, hp,
                                       i >= first_sp ? kd->eta_sp : hp->eta);
            double d = h;
            if (2.0 * d <= c && 2.0 * d <= hp->dt_max && fmod(t[i], 2.0 * d) == 0.0)
                d = 2.0 * d;
            else
                while (d > c && d > dt_min) d *= 0.5;
            dt[i] = d;
        }
    }
    if (n_block_steps) *n_block_steps = steps;
    free(a); free(jk); free(a2); free(a3); free(xp); free(vp); free(a1); free(j1);
    free(t); free(dt); free(hard);
    return rc;
}
