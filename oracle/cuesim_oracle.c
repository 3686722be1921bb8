/*
 * cuesim_oracle.c -- FP64 CPU oracle of one time step of the cue-diffusion axon-guidance
 * simulation (Mihut, Morgan & Kaiser 2014, "GPU Simulation of Axon Growth and Guidance
 * through Cue Diffusion").
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference that the GPU library is checked
 * against.  Tests, the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never does.  It shares no code with the GPU library.
 *
 * A time step has two parts, in this order (Sec. 1: growth per neuron each time step as an
 * independent process; Sec. 3.5: the cue environment drives the steering):
 *   F1  explicit finite-difference diffusion of every cue species with first-order decay,
 *       zero-flux walls (a neighbour outside the grid is replaced by the cell itself);
 *   F2  point sources add their per-step amount q / dx^dim to their cell;
 *   C1  each active growth cone samples the cue gradient at its tip: central differences at
 *       cell centres, interpolated multilinearly to the tip, summed over species with sign;
 *   C2  deterministic turn toward the direction of (heading + gain * gradient) -- the
 *       vector-addition steering of Sec. 3.5, Eqs. 6-7, where the turn angle follows from
 *       the dot product (cosine) and cross product (sine) -- capped at pi/30 per step, the
 *       turn magnitude Sec. 3.5 fixes;
 *   C3  angular noise from a counter-based, stateless Philox stream keyed by
 *       (cone, step, tag, simulation), the per-thread generator style Sec. 5.1 recommends;
 *   C4  advance a fixed distance per step along the heading (Sec. 3.5 steering);
 *   C5  a cone that leaves the simulation bounds stops (Sec. 3.4);
 *   C6  contact: squared distance strictly below the squared radius (Sec. 3.3 sphere test),
 *       nearest target wins, lowest index on an exact tie; the cone stops there (Sec. 3.4).
 *
 * Readings where the paper is silent (grid centring, decay discretisation, source units,
 * gain, noise law, exit-before-contact, no contact test at t = 0) are the ones documented
 * with the design; every rule above is executed literally, in FP64, with no blocking or
 * reordering.
 */
#include "cuesim_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as      */
/* 1, 2, 3", SC'11).  Round: two 32x32->64 multiplies of counter words 0 and 2 by the    */
/* published multipliers; the high halves are xored with the other two words and the    */
/* key.  The key is bumped by the published Weyl constants between rounds.               */
/* ------------------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)mul0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)mul1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += weyl0;
        k1 += weyl1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1) from the top 23 bits, centred in its bin: (2m + 1) * 2^-24 with
 * m < 2^23 needs 24 significant bits, so it is exact in FP32 as well as FP64 and every
 * implementation sees the same uniform. */
static double uniform23(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

void oracle_normals4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                     double z[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    /* Box-Muller: radius from the first uniform of a pair, angle from the second. */
    for (int pair = 0; pair < 2; ++pair) {
        double u_r = uniform23(x[2 * pair]);
        double u_a = uniform23(x[2 * pair + 1]);
        double radius = sqrt(-2.0 * log(u_r));
        z[2 * pair] = radius * cos(2.0 * ORACLE_PI * u_a);
        z[2 * pair + 1] = radius * sin(2.0 * ORACLE_PI * u_a);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Grid helpers.                                                                          */
/* ------------------------------------------------------------------------------------ */
static int64_t n_cells(const oracle_params* p)
{
    return (int64_t)p->nx * p->ny * (p->dim == 3 ? p->nz : 1);
}

static int axis_size(const oracle_params* p, int a)
{
    return a == 0 ? p->nx : (a == 1 ? p->ny : p->nz);
}

static int64_t cell_index(const oracle_params* p, const int idx[3])
{
    int64_t l = p->dim == 3 ? idx[2] : 0;
    return (l * p->ny + idx[1]) * p->nx + idx[0];
}

/* Value of the neighbour of cell idx one step along axis a in direction d (+1/-1); a
 * neighbour outside the grid is the cell itself (zero-flux wall). */
static double neighbour(const oracle_params* p, const double* c, const int idx[3], int a, int d)
{
    int nb[3] = {idx[0], idx[1], idx[2]};
    nb[a] += d;
    if (nb[a] < 0 || nb[a] >= axis_size(p, a))
        return c[cell_index(p, idx)];
    return c[cell_index(p, nb)];
}

/* ------------------------------------------------------------------------------------ */
/* F1 + F2: field update.                                                                 */
/* ------------------------------------------------------------------------------------ */
void oracle_field_step(const oracle_params* p, const double* const in[2], double* const out[2])
{
    const int nz = p->dim == 3 ? p->nz : 1;
    const double cell_volume = pow(p->dx, p->dim);
    for (int s = 0; s < p->n_species; ++s) {
        const double r = p->D[s] * p->dt / (p->dx * p->dx);
        const double kdt = p->k[s] * p->dt;
        const double* c = in[s];
        double* c_new = out[s];
        /* F1: c' = c + r * sum_axes (c[+e] + c[-e] - 2c) - k dt c */
#pragma omp parallel for collapse(2) schedule(static)
        for (int l = 0; l < nz; ++l) {
            for (int j = 0; j < p->ny; ++j) {
                for (int i = 0; i < p->nx; ++i) {
                    int idx[3] = {i, j, l};
                    double centre = c[cell_index(p, idx)];
                    double laplacian_sum = 0.0;
                    for (int a = 0; a < p->dim; ++a)
                        laplacian_sum += neighbour(p, c, idx, a, +1) + neighbour(p, c, idx, a, -1)
                                         - 2.0 * centre;
                    c_new[cell_index(p, idx)] = centre + r * laplacian_sum - kdt * centre;
                }
            }
        }
        /* F2: each source adds its per-step amount, spread over its cell's volume. */
        for (int m = 0; m < p->n_sources[s]; ++m)
            c_new[p->source_cell[s][m]] += p->source_q[s][m] / cell_volume;
    }
}

double oracle_mass(const oracle_params* p, const double* field)
{
    double total = 0.0;
    int64_t n = n_cells(p);
    for (int64_t x = 0; x < n; ++x)
        total += field[x];
    return total * pow(p->dx, p->dim);
}

/* ------------------------------------------------------------------------------------ */
/* C1: gradient sampling.                                                                 */
/* ------------------------------------------------------------------------------------ */

/* Central-difference gradient component along axis a at the centre of cell idx. */
static double centre_gradient(const oracle_params* p, const double* c, const int idx[3], int a)
{
    return (neighbour(p, c, idx, a, +1) - neighbour(p, c, idx, a, -1)) / (2.0 * p->dx);
}

/* The 2^dim cell centres around point p: the lower corner `base` and the fractions along
 * each axis.  Cell centres sit at (i + 1/2) dx: u is the tip in units of cell-centre
 * spacing, clamped to the outermost centres. */
static void tip_corners(const oracle_params* p, const double* point, int base[3], double frac[3])
{
    for (int a = 0; a < 3; ++a) {
        base[a] = 0;
        frac[a] = 0.0;
    }
    for (int a = 0; a < p->dim; ++a) {
        int n = axis_size(p, a);
        double u = point[a] / p->dx - 0.5;
        if (u < 0.0) u = 0.0;
        if (u > (double)(n - 1)) u = (double)(n - 1);
        int i0 = (int)floor(u);
        if (i0 > n - 2) i0 = n - 2;
        base[a] = i0;
        frac[a] = u - (double)i0;
    }
}

/* Cell and multilinear weight of one corner (bit a of `corner` = upper along axis a). */
static double corner_cell(const oracle_params* p, const int base[3], const double frac[3],
                          int corner, int idx[3])
{
    double weight = 1.0;
    idx[0] = idx[1] = idx[2] = 0;
    for (int a = 0; a < p->dim; ++a) {
        int upper = (corner >> a) & 1;
        idx[a] = base[a] + upper;
        weight *= upper ? frac[a] : (1.0 - frac[a]);
    }
    return weight;
}

void oracle_sample_gradient(const oracle_params* p, const double* field, const double* point,
                            double g[3])
{
    int base[3];
    double frac[3];
    tip_corners(p, point, base, frac);
    g[0] = g[1] = g[2] = 0.0;
    for (int corner = 0; corner < (1 << p->dim); ++corner) {
        int idx[3];
        double weight = corner_cell(p, base, frac, corner, idx);
        for (int a = 0; a < p->dim; ++a)
            g[a] += weight * centre_gradient(p, field, idx, a);
    }
}

/* ------------------------------------------------------------------------------------ */
/* C2-C6: one cone step.                                                                  */
/* ------------------------------------------------------------------------------------ */
static double domain_length(const oracle_params* p, int a)
{
    return (double)axis_size(p, a) * p->dx;
}

/* Distance of an uncapped turn angle from the cap, kept as a running minimum (recorded
   only; it does not change the trajectory).  A turn this close to the cap can take the
   other side of it under rounding, which switches the turn's derivative. */
static void note_cap_margin(const oracle_params* p, double angle, double* cap_margin)
{
    if (cap_margin) {
        double m = fabs(fabs(angle) - p->max_turn);
        if (m < *cap_margin) *cap_margin = m;
    }
}

/* C2 (2D): rotate heading angle theta toward theta + angle(h + gain*g), capped. */
static double turn_2d(const oracle_params* p, double theta, const double g[3], int* ambiguous,
                      double* cap_margin)
{
    double hx = cos(theta), hy = sin(theta);
    double cross = hx * g[1] - hy * g[0];      /* sine part (Sec. 3.5, Eq. 7 discussion) */
    double dot = hx * g[0] + hy * g[1];        /* cosine part */
    double y = p->turn_gain * cross;
    double x = 1.0 + p->turn_gain * dot;
    if (y == 0.0) y = 0.0;                     /* -0 -> +0: anti-parallel turns by +cap */
    if (x < 0.0 && fabs(y) <= 1e-5 * fabs(x)) *ambiguous = 1;
    double delta = atan2(y, x);
    note_cap_margin(p, delta, cap_margin);
    if (delta > p->max_turn) delta = p->max_turn;
    if (delta < -p->max_turn) delta = -p->max_turn;
    return theta + delta;
}

/* C2 (3D): rotate h toward h + gain*g in the plane they span, by at most max_turn. */
static void turn_3d(const oracle_params* p, double h[3], const double g[3], int* ambiguous,
                    double* cap_margin)
{
    double along = g[0] * h[0] + g[1] * h[1] + g[2] * h[2];
    double perp[3] = {g[0] - along * h[0], g[1] - along * h[1], g[2] - along * h[2]};
    double perp_norm = sqrt(perp[0] * perp[0] + perp[1] * perp[1] + perp[2] * perp[2]);
    double x = 1.0 + p->turn_gain * along;
    if (x < 0.0 && p->turn_gain * perp_norm <= 1e-5 * fabs(x)) *ambiguous = 1;
    if (perp_norm == 0.0)
        return;
    double phi = atan2(p->turn_gain * perp_norm, x);
    note_cap_margin(p, phi, cap_margin);
    if (phi > p->max_turn) phi = p->max_turn;
    double c = cos(phi), s = sin(phi);
    for (int a = 0; a < 3; ++a)
        h[a] = c * h[a] + s * perp[a] / perp_norm;
}

/* Interpolated concentration of one field at point p: the multilinear interpolation of
 * cell-centre values with the same corners and weights as the gradient sample. */
static double sample_value(const oracle_params* p, const double* field, const double* point)
{
    int base[3];
    double frac[3];
    tip_corners(p, point, base, frac);
    double v = 0.0;
    for (int corner = 0; corner < (1 << p->dim); ++corner) {
        int idx[3];
        double weight = corner_cell(p, base, frac, corner, idx);
        v += weight * field[cell_index(p, idx)];
    }
    return v;
}

/* C2 under the SNR law (Sec. 3.5, Eq. 5; 2D): the growth cone compares the cue across its
 * width and turns by the fixed angle to the right (clockwise) when a normal deviate with
 * mean SNR and unit variance is positive, else to the left.  Outside the detection window
 * [c_min, c_max], or with no gradient, it does not turn.  sin(theta - theta_g) |g| equals
 * sin(theta) g_x - cos(theta) g_y, so theta_g itself is never formed. */
static double turn_snr_2d(const oracle_params* p, double theta, const double g[3], double c,
                          double z0, int* ambiguous)
{
    const double tol = 1e-4;
    if (fabs(c - p->c_min) <= tol * p->c_min || fabs(c - p->c_max) <= tol * p->c_max)
        *ambiguous = 1;
    if (c < p->c_min || c > p->c_max || (g[0] == 0.0 && g[1] == 0.0))
        return theta;
    double gamma = c / p->kd;
    double side = sin(theta) * g[0] - cos(theta) * g[1];      /* |g| sin(theta - theta_g) */
    double snr = p->snr_scale * (p->cone_width / c) * sqrt(gamma / pow(1.0 + gamma, 3.0)) * side;
    double x = snr + z0;
    if (fabs(x) <= tol)
        *ambiguous = 1;
    return x > 0.0 ? theta - p->max_turn : theta + p->max_turn;
}

/* C3 (3D): tangent-plane Gaussian rotation of h, then renormalisation. */
static void noise_3d(const oracle_params* p, double h[3], const double z[4])
{
    double along = z[0] * h[0] + z[1] * h[1] + z[2] * h[2];
    double w[3];
    for (int a = 0; a < 3; ++a)
        w[a] = p->noise_sigma * (z[a] - along * h[a]);
    double angle = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (angle > 0.0) {
        double c = cos(angle), s = sin(angle);
        for (int a = 0; a < 3; ++a)
            h[a] = c * h[a] + s * w[a] / angle;
    }
    double norm = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    for (int a = 0; a < 3; ++a)
        h[a] /= norm;
}

static void step_one_cone(const oracle_params* p, oracle_state* s, int i,
                          const double* const fields[2])
{
    const int dim = p->dim;
    const int64_t n = s->step;        /* the step being taken is n -> n+1 */
    double* pos = s->pos + (int64_t)i * dim;
    int ambiguous = 0;

    /* C1: signed sum of the species' interpolated gradients. */
    double g[3] = {0.0, 0.0, 0.0};
    for (int sp = 0; sp < p->n_species; ++sp) {
        double gs[3];
        oracle_sample_gradient(p, fields[sp], pos, gs);
        for (int a = 0; a < dim; ++a)
            g[a] += p->sign[sp] * gs[a];
    }

    /* C2 + C3: turn, then noise.  3D draws a block keyed by (cone, step, tag 0, simulation)
     * and uses three of its deviates.  2D needs at most two per step, so one block keyed by
     * (cone, step / 2, tag 0, simulation) serves two steps: its first Box-Muller pair for
     * the even step, its second for the odd one (z[0], z[1] below). */
    double z[4];
    if (dim == 2) {
        double zz[4];
        oracle_normals4(p->seed, (uint32_t)i, (uint32_t)(n >> 1), 0u, p->sim_index, zz);
        z[0] = zz[2 * (n & 1)];
        z[1] = zz[2 * (n & 1) + 1];
        z[2] = z[3] = 0.0;
    } else {
        oracle_normals4(p->seed, (uint32_t)i, (uint32_t)n, 0u, p->sim_index, z);
    }
    for (int q = 0; q < 4; ++q)
        z[q] *= p->noise_sign;
    double h[3];
    if (dim == 2) {
        double theta;
        if (p->turn_law == 1) {
            double c = sample_value(p, fields[0], pos);
            theta = turn_snr_2d(p, s->dir[i], g, c, z[0], &ambiguous);
            theta += p->noise_sigma * z[1];
        } else {
            theta = turn_2d(p, s->dir[i], g, &ambiguous,
                            s->cap_margin ? s->cap_margin + i : NULL);
            theta += p->noise_sigma * z[0];
        }
        theta -= 2.0 * ORACLE_PI * floor((theta + ORACLE_PI) / (2.0 * ORACLE_PI));
        s->dir[i] = theta;
        h[0] = cos(theta);
        h[1] = sin(theta);
        h[2] = 0.0;
    } else {
        double* hd = s->dir + (int64_t)i * 3;
        turn_3d(p, hd, g, &ambiguous, s->cap_margin ? s->cap_margin + i : NULL);
        noise_3d(p, hd, z);
        h[0] = hd[0]; h[1] = hd[1]; h[2] = hd[2];
    }

    /* C4: advance a fixed distance. */
    for (int a = 0; a < dim; ++a)
        pos[a] += p->step_len * h[a];

    /* Near-tie margins (recorded only; they do not change the trajectory). */
    for (int a = 0; a < dim; ++a) {
        double L = domain_length(p, a);
        if (fabs(pos[a]) <= p->flag_tol || fabs(L - pos[a]) <= p->flag_tol)
            ambiguous = 1;
    }

    /* C5: leaving the simulation bounds stops the cone (checked before contact). */
    int outside = 0;
    for (int a = 0; a < dim; ++a)
        if (pos[a] < 0.0 || pos[a] >= domain_length(p, a))
            outside = 1;
    if (outside) {
        s->status[i] = ORACLE_EXITED;
        s->event_step[i] = (int32_t)(n + 1);
    } else {
        /* C6: strict squared-distance test against every target (brute force). */
        const double R = p->contact_radius;
        double best_d2 = INFINITY, second_d = INFINITY, best_d = INFINITY;
        int best = -1;
        for (int t = 0; t < p->n_targets; ++t) {
            const double* tp = p->target_pos + (int64_t)t * dim;
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a)
                d2 += (pos[a] - tp[a]) * (pos[a] - tp[a]);
            double d = sqrt(d2);
            if (fabs(d - R) <= p->flag_tol)
                ambiguous = 1;
            if (d < R + p->flag_tol) {
                if (d < best_d) { second_d = best_d; best_d = d; }
                else if (d < second_d) second_d = d;
            }
            if (d2 < best_d2) {        /* strict: the lowest index wins an exact tie */
                best_d2 = d2;
                best = t;
            }
        }
        if (second_d - best_d <= p->flag_tol)
            ambiguous = 1;
        if (best >= 0 && best_d2 < R * R) {
            s->status[i] = ORACLE_CONTACT;
            s->target[i] = best;
            s->event_step[i] = (int32_t)(n + 1);
        }
    }
    if (ambiguous && s->flag_step[i] < 0)
        s->flag_step[i] = (int32_t)(n + 1);
}

void oracle_cone_step(const oracle_params* p, oracle_state* s)
{
    const double* fields[2] = {s->field[0], s->field[1]};
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < s->n_cones; ++i)
        if (s->status[i] == ORACLE_ACTIVE)
            step_one_cone(p, s, i, fields);
}

int oracle_run(const oracle_params* p, oracle_state* s, int64_t n_steps)
{
    const int64_t cells = n_cells(p);
    double* scratch[2] = {NULL, NULL};
    for (int sp = 0; sp < p->n_species; ++sp) {
        scratch[sp] = (double*)malloc((size_t)cells * sizeof(double));
        if (!scratch[sp]) {
            free(scratch[0]);
            return -1;
        }
    }
    for (int64_t it = 0; it < n_steps; ++it) {
        const double* in[2] = {s->field[0], s->field[1]};
        double* out[2] = {scratch[0], scratch[1]};
        oracle_field_step(p, in, out);
        for (int sp = 0; sp < p->n_species; ++sp)
            memcpy(s->field[sp], scratch[sp], (size_t)cells * sizeof(double));
        oracle_cone_step(p, s);
        s->step += 1;
    }
    free(scratch[0]);
    free(scratch[1]);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Reverse-mode gradient of a trajectory loss (2D).                                       */
/*                                                                                        */
/* L = sum_i w_i |p_i^N - t_{a(i)}|^2 over the cones' tips after N steps (a frozen cone   */
/* keeps the tip it stopped at), differentiated with respect to every source amount q,    */
/* and D and k of every species, along the forward run's branch: the exit and contact    */
/* decisions and the turn cap's active side are held as the forward run took them.       */
/*                                                                                        */
/* The forward run is recorded in full (c^n for n = 0..N and the cone states at the      */
/* start of every step), then the steps are reversed from N-1 down to 0:                  */
/*   cones of step n:  adjoints of (p, theta) through advance, turn and gradient sample;   */
/*                     the sample's adjoint is scattered into a^{n+1}, the field adjoint  */
/*   field of step n:  c^{n+1} = c^n + r Lap c^n - k dt c^n + S q, so                     */
/*                     dL/dq_m += a^{n+1}[cell_m] / dx^dim,                               */
/*                     dL/dD   += sum a^{n+1} (dt / dx^2) Lap c^n,                        */
/*                     dL/dk   += sum a^{n+1} (-dt c^n),                                  */
/*                     a^n = a^{n+1} + r Lap a^{n+1} - k dt a^{n+1}                       */
/*                     (the zero-flux Laplacian is symmetric, so its transpose is itself). */
/* ------------------------------------------------------------------------------------ */

/* Lap(c) at every cell of one 2D field (zero-flux walls): the sum over in-grid neighbours
 * of (neighbour - cell). */
static void laplacian_2d(const oracle_params* p, const double* c, double* out)
{
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            int idx[3] = {i, j, 0};
            double here = c[cell_index(p, idx)];
            double sum = 0.0;
            for (int a = 0; a < 2; ++a)
                sum += (neighbour(p, c, idx, a, +1) - here) + (neighbour(p, c, idx, a, -1) - here);
            out[cell_index(p, idx)] = sum;
        }
}

/* Linear index of the neighbour of cell idx along axis a, direction d (the cell itself
 * outside the grid). */
static int64_t neighbour_index(const oracle_params* p, const int idx[3], int a, int d)
{
    int nb[3] = {idx[0], idx[1], idx[2]};
    nb[a] += d;
    if (nb[a] < 0 || nb[a] >= axis_size(p, a))
        return cell_index(p, idx);
    return cell_index(p, nb);
}

/* Reverse of one 2D cone step.  In: the state at the start of the step (pos, theta), the
 * updated fields, the deviate z0 and the adjoints (ap[2], ath) of the state after the
 * step.  Out: ap, ath become the adjoints of the state before the step, and the gradient
 * sample's adjoint is added into afield[s]. */
static void cone_reverse_2d(const oracle_params* p, const double* const fields[2],
                            double* const afield[2], const double pos[2], double theta,
                            double z0, double ap[2], double* ath)
{
    /* recompute the forward quantities of the step */
    int base[2];
    double frac[2];
    int inside[2];
    for (int a = 0; a < 2; ++a) {
        int n = axis_size(p, a);
        double u = pos[a] / p->dx - 0.5;
        inside[a] = u > 0.0 && u < (double)(n - 1);
        if (u < 0.0) u = 0.0;
        if (u > (double)(n - 1)) u = (double)(n - 1);
        int i0 = (int)floor(u);
        if (i0 > n - 2) i0 = n - 2;
        base[a] = i0;
        frac[a] = u - (double)i0;
    }
    double g[2] = {0.0, 0.0};
    for (int sp = 0; sp < p->n_species; ++sp) {
        double gs[3];
        oracle_sample_gradient(p, fields[sp], pos, gs);
        g[0] += p->sign[sp] * gs[0];
        g[1] += p->sign[sp] * gs[1];
    }
    const double lam = p->turn_gain;
    double hx = cos(theta), hy = sin(theta);
    double y = lam * (hx * g[1] - hy * g[0]);
    double x = 1.0 + lam * (hx * g[0] + hy * g[1]);
    double delta = atan2(y, x);
    int capped = delta > p->max_turn || delta < -p->max_turn;
    delta = fmin(fmax(delta, -p->max_turn), p->max_turn);
    double theta_new = theta + delta + p->noise_sigma * z0;   /* the wrap is a constant shift */

    /* advance: p' = p + s (cos theta', sin theta') */
    double a_thn = *ath + p->step_len * (-sin(theta_new) * ap[0] + cos(theta_new) * ap[1]);
    /* theta' = theta + delta(theta, g) + noise */
    double a_theta = a_thn;
    double a_g[2] = {0.0, 0.0};
    if (!capped) {
        double den = x * x + y * y;
        double a_y = a_thn * x / den, a_x = -a_thn * y / den;
        a_theta += a_y * (-lam * (hx * g[0] + hy * g[1])) + a_x * y;
        a_g[0] = a_y * (-lam * hy) + a_x * (lam * hx);
        a_g[1] = a_y * (lam * hx) + a_x * (lam * hy);
    }
    /* gradient sample: g_a = sum_s sign_s sum_corners w(u) G_{s,a}[corner] */
    for (int sp = 0; sp < p->n_species; ++sp) {
        const double* c = fields[sp];
        double* ac = afield[sp];
        for (int corner = 0; corner < 4; ++corner) {
            int idx[3] = {0, 0, 0};
            int up[2];
            double w = 1.0;
            for (int a = 0; a < 2; ++a) {
                up[a] = (corner >> a) & 1;
                idx[a] = base[a] + up[a];
                w *= up[a] ? frac[a] : (1.0 - frac[a]);
            }
            /* the corner's central-difference gradient and its dependence on the tip */
            double G[2];
            for (int a = 0; a < 2; ++a)
                G[a] = (neighbour(p, c, idx, a, +1) - neighbour(p, c, idx, a, -1)) / (2.0 * p->dx);
            double sum = a_g[0] * G[0] + a_g[1] * G[1];
            for (int b = 0; b < 2; ++b) {
                if (!inside[b])
                    continue;
                double dw = up[b] ? 1.0 : -1.0;   /* d w / d frac_b */
                for (int a = 0; a < 2; ++a)
                    if (a != b)
                        dw *= up[a] ? frac[a] : (1.0 - frac[a]);
                ap[b] += p->sign[sp] * dw / p->dx * sum;
            }
            /* scatter into the field adjoint */
            for (int a = 0; a < 2; ++a) {
                double v = p->sign[sp] * w * a_g[a] / (2.0 * p->dx);
                ac[neighbour_index(p, idx, a, +1)] += v;
                ac[neighbour_index(p, idx, a, -1)] -= v;
            }
        }
    }
    *ath = a_theta;
}

int oracle_adjoint(const oracle_params* p, oracle_state* s, int64_t n_steps,
                   const int32_t* assign, const double* weight, double* loss,
                   double* dL_dq, double* dL_dD, double* dL_dk, double* magnitude,
                   double* cone_adjoint)
{
    if (p->dim != 2)
        return -2;
    const int64_t cells = n_cells(p);
    const int ns = p->n_species;
    const int M = s->n_cones;
    const int64_t N = n_steps;
    const int64_t n0 = s->step;
    /* tape: fields c^n (n = 0..N) per species, cone (x, y, theta) at the start of each step */
    double* tape_c = (double*)malloc((size_t)(N + 1) * ns * cells * sizeof(double));
    double* tape_cone = (double*)malloc((size_t)(N > 0 ? N : 1) * M * 3 * sizeof(double) + 8);
    double* afield = (double*)calloc((size_t)ns * cells, sizeof(double));
    double* lap = (double*)malloc((size_t)cells * sizeof(double));
    double* aprev = (double*)malloc((size_t)cells * sizeof(double));
    double* acone = (double*)calloc((size_t)M * 3 + 1, sizeof(double));
    if (!tape_c || !tape_cone || !afield || !lap || !aprev || !acone) {
        free(tape_c); free(tape_cone); free(afield); free(lap); free(aprev); free(acone);
        return -1;
    }
    for (int sp = 0; sp < ns; ++sp)
        memcpy(tape_c + (size_t)sp * cells, s->field[sp], (size_t)cells * sizeof(double));
    for (int64_t n = 0; n < N; ++n) {
        for (int i = 0; i < M; ++i) {
            tape_cone[((size_t)n * M + i) * 3 + 0] = s->pos[2 * i];
            tape_cone[((size_t)n * M + i) * 3 + 1] = s->pos[2 * i + 1];
            tape_cone[((size_t)n * M + i) * 3 + 2] = s->dir[i];
        }
        if (oracle_run(p, s, 1) != 0) {
            free(tape_c); free(tape_cone); free(afield); free(lap); free(aprev); free(acone);
            return -1;
        }
        for (int sp = 0; sp < ns; ++sp)
            memcpy(tape_c + ((size_t)(n + 1) * ns + sp) * cells, s->field[sp],
                   (size_t)cells * sizeof(double));
    }
    /* loss and its adjoint at the final tips */
    double L = 0.0;
    for (int i = 0; i < M; ++i) {
        const double* t = p->target_pos + (int64_t)assign[i] * 2;
        double dx0 = s->pos[2 * i] - t[0], dx1 = s->pos[2 * i + 1] - t[1];
        L += weight[i] * (dx0 * dx0 + dx1 * dx1);
        acone[3 * i + 0] = 2.0 * weight[i] * dx0;
        acone[3 * i + 1] = 2.0 * weight[i] * dx1;
        acone[3 * i + 2] = 0.0;
    }
    *loss = L;
    int q_off[2] = {0, p->n_sources[0]};
    const int nq = p->n_sources[0] + (ns > 1 ? p->n_sources[1] : 0);
    for (int sp = 0; sp < ns; ++sp) {
        for (int m = 0; m < p->n_sources[sp]; ++m)
            dL_dq[q_off[sp] + m] = 0.0;
        dL_dD[sp] = 0.0;
        dL_dk[sp] = 0.0;
    }
    /* magnitude (optional): the same sums taken over absolute values of their terms,
       [dL/dq ..., dL/dD per species, dL/dk per species]; the scale of rounding error that a
       sum of these terms can carry (its cancellation) */
    if (magnitude)
        for (int m = 0; m < nq + 2 * ns; ++m)
            magnitude[m] = 0.0;
    const double vol = p->dx * p->dx;
    for (int64_t n = N - 1; n >= 0; --n) {
        const double* fnext[2] = {tape_c + ((size_t)(n + 1) * ns) * cells,
                                  tape_c + ((size_t)(n + 1) * ns + (ns > 1 ? 1 : 0)) * cells};
        double* af[2] = {afield, afield + (size_t)(ns > 1 ? 1 : 0) * cells};
        /* cones active at the start of step n0 + n */
        for (int i = 0; i < M; ++i) {
            int32_t e = s->event_step[i];
            if (s->status[i] != ORACLE_ACTIVE && e <= n0 + n)
                continue;
            double z[4];
            const int64_t m = n0 + n;
            oracle_normals4(p->seed, (uint32_t)i, (uint32_t)(m >> 1), 0u, p->sim_index, z);
            const double* st = tape_cone + ((size_t)n * M + i) * 3;
            double pos[2] = {st[0], st[1]};
            cone_reverse_2d(p, fnext, af, pos, st[2], z[2 * (m & 1)] * p->noise_sign,
                            acone + 3 * i, acone + 3 * i + 2);
        }
        /* field of step n: parameters, then a^n = A a^{n+1} */
        for (int sp = 0; sp < ns; ++sp) {
            const double* c = tape_c + ((size_t)n * ns + sp) * cells;
            double* a = afield + (size_t)sp * cells;
            for (int m = 0; m < p->n_sources[sp]; ++m) {
                dL_dq[q_off[sp] + m] += a[p->source_cell[sp][m]] / vol;
                if (magnitude)
                    magnitude[q_off[sp] + m] += fabs(a[p->source_cell[sp][m]]) / vol;
            }
            laplacian_2d(p, c, lap);
            double sD = 0.0, sk = 0.0, mD = 0.0, mk = 0.0;
            for (int64_t x = 0; x < cells; ++x) {
                sD += a[x] * lap[x];
                sk += a[x] * c[x];
                mD += fabs(a[x] * lap[x]);
                mk += fabs(a[x] * c[x]);
            }
            dL_dD[sp] += sD * p->dt / (p->dx * p->dx);
            dL_dk[sp] += -p->dt * sk;
            if (magnitude) {
                magnitude[nq + sp] += mD * p->dt / (p->dx * p->dx);
                magnitude[nq + ns + sp] += p->dt * mk;
            }
            const double r = p->D[sp] * p->dt / (p->dx * p->dx);
            const double kdt = p->k[sp] * p->dt;
            laplacian_2d(p, a, lap);
            for (int64_t x = 0; x < cells; ++x)
                aprev[x] = a[x] + r * lap[x] - kdt * a[x];
            memcpy(a, aprev, (size_t)cells * sizeof(double));
        }
    }
    if (cone_adjoint)
        memcpy(cone_adjoint, acone, (size_t)M * 3 * sizeof(double));
    free(tape_c); free(tape_cone); free(afield); free(lap); free(aprev); free(acone);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Connectivity (Sec. 3.4, Figs. 4-5).                                                    */
/* ------------------------------------------------------------------------------------ */
int64_t oracle_connectivity(int32_t n_neurons, int32_t n_cones, const int32_t* status,
                            const int32_t* target, const int32_t* cone_owner,
                            const int32_t* target_owner, int32_t* row_start, int32_t* edges)
{
    /* degree of every neuron, then the start of its list (V_a) */
    for (int v = 0; v <= n_neurons; ++v)
        row_start[v] = 0;
    for (int i = 0; i < n_cones; ++i)
        if (status[i] == ORACLE_CONTACT)
            row_start[cone_owner[i] + 1] += 1;
    for (int v = 0; v < n_neurons; ++v)
        row_start[v + 1] += row_start[v];
    /* the lists (E_a): cones visited in increasing index, appended to their owner's list */
    int32_t* fill = (int32_t*)malloc(((size_t)n_neurons + 1) * sizeof(int32_t));
    if (!fill)
        return -1;
    memcpy(fill, row_start, (size_t)n_neurons * sizeof(int32_t));
    for (int i = 0; i < n_cones; ++i)
        if (status[i] == ORACLE_CONTACT)
            edges[fill[cone_owner[i]]++] = target_owner[target[i]];
    free(fill);
    return row_start[n_neurons];
}

int oracle_bfs_levels(int32_t n_neurons, const int32_t* row_start, const int32_t* edges,
                      int32_t root, int32_t* level)
{
    /* textbook queue-based breadth-first search */
    int32_t* queue = (int32_t*)malloc(((size_t)n_neurons + 1) * sizeof(int32_t));
    if (!queue)
        return -1;
    for (int v = 0; v < n_neurons; ++v)
        level[v] = -1;
    int head = 0, tail = 0;
    level[root] = 0;
    queue[tail++] = root;
    while (head < tail) {
        int v = queue[head++];
        for (int e = row_start[v]; e < row_start[v + 1]; ++e) {
            int u = edges[e];
            if (level[u] < 0) {
                level[u] = level[v] + 1;
                queue[tail++] = u;
            }
        }
    }
    free(queue);
    return 0;
}
