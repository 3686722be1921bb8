/* oracle_driver.c -- runs every entry point of the FP64 oracle on small seeded scenarios
 * (2D and 3D, one and two species, both turn laws, the reverse sweep with and without its
 * optional outputs, connectivity and breadth-first levels, the smallest grid) so that a
 * build under the address and undefined-behaviour sanitizers exercises all of its code.
 * Exit status 0 when every call succeeded and every value is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cuesim_oracle.h"

static uint64_t rng_state = 88172645463325252ull;
static double uniform(void) {   /* xorshift64: inputs only */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * 0x1p-53;
}

static int failures = 0;
#define CHECK(cond)                                                    \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                \
        }                                                              \
    } while (0)

typedef struct {
    oracle_params p;
    oracle_state s;
    int32_t* cells[2];
    double* q[2];
    double* targets;
} scenario;

static void make(scenario* sc, int dim, int nx, int ny, int nz, int ns, int n_src, int M,
                 int T, int turn_law) {
    memset(sc, 0, sizeof *sc);
    oracle_params* p = &sc->p;
    p->dim = dim;
    p->nx = nx;
    p->ny = ny;
    p->nz = dim == 3 ? nz : 1;
    p->dx = 1.0;
    p->dt = dim == 3 ? 0.15 : 0.2;
    p->n_species = ns;
    const int64_t cells = (int64_t)nx * ny * p->nz;
    for (int s = 0; s < ns; ++s) {
        p->D[s] = s ? 0.5 : 1.0;
        p->k[s] = s ? 0.02 : 0.01;
        p->sign[s] = s ? -1.0 : 1.0;
        p->n_sources[s] = n_src;
        sc->cells[s] = malloc(sizeof(int32_t) * (n_src ? n_src : 1));
        sc->q[s] = malloc(sizeof(double) * (n_src ? n_src : 1));
        for (int m = 0; m < n_src; ++m) {
            /* corners, a repeated cell, then random cells */
            sc->cells[s][m] = m == 0 ? 0 : m == 1 ? (int32_t)(cells - 1) : m == 2 ? 0
                                                 : (int32_t)(uniform() * cells);
            sc->q[s][m] = 0.5 + 1.5 * uniform();
        }
        p->source_cell[s] = sc->cells[s];
        p->source_q[s] = sc->q[s];
    }
    p->n_targets = T;
    sc->targets = malloc(sizeof(double) * dim * (T ? T : 1));
    const double L[3] = {nx, ny, p->nz};
    for (int t = 0; t < T; ++t)
        for (int a = 0; a < dim; ++a) sc->targets[t * dim + a] = uniform() * L[a];
    p->target_pos = sc->targets;
    p->contact_radius = 1.0;
    p->step_len = 0.5;
    p->turn_gain = 10.0;
    p->max_turn = 3.14159265358979 / 30.0;
    p->noise_sigma = 0.1;
    p->seed = 0x1234567890abcdefull;
    p->sim_index = 7;
    p->noise_sign = 1.0;
    p->flag_tol = 1e-4 * nx;
    p->turn_law = turn_law;
    p->snr_scale = 50.0;
    p->cone_width = 1.0;
    p->kd = 0.5;
    p->c_min = 1e-3;
    p->c_max = 1e3;
    oracle_state* s = &sc->s;
    s->n_cones = M;
    for (int sp = 0; sp < ns; ++sp) s->field[sp] = calloc((size_t)cells, sizeof(double));
    s->pos = malloc(sizeof(double) * dim * (M ? M : 1));
    s->dir = malloc(sizeof(double) * (dim == 2 ? 1 : 3) * (M ? M : 1));
    s->status = calloc(M ? M : 1, sizeof(int32_t));
    s->target = malloc(sizeof(int32_t) * (M ? M : 1));
    s->event_step = malloc(sizeof(int32_t) * (M ? M : 1));
    s->flag_step = malloc(sizeof(int32_t) * (M ? M : 1));
    s->cap_margin = malloc(sizeof(double) * (M ? M : 1));
    for (int i = 0; i < M; ++i) {
        for (int a = 0; a < dim; ++a) {
            /* the first cones sit right at the walls */
            double v = i < 2 * dim ? (i % 2 ? L[a] - 1e-3 : 1e-3) : uniform() * L[a];
            s->pos[i * dim + a] = v;
        }
        if (dim == 2) {
            s->dir[i] = 6.283185307179586 * uniform() - 3.141592653589793;
        } else {
            double h[3] = {uniform() - 0.5, uniform() - 0.5, uniform() - 0.5};
            double n = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
            for (int a = 0; a < 3; ++a) s->dir[i * 3 + a] = h[a] / n;
        }
        s->target[i] = -1;
        s->event_step[i] = -1;
        s->flag_step[i] = -1;
        s->cap_margin[i] = INFINITY;
    }
}

static void release(scenario* sc) {
    for (int s = 0; s < 2; ++s) {
        free(sc->cells[s]);
        free(sc->q[s]);
        free(sc->s.field[s]);
    }
    free(sc->targets);
    free(sc->s.pos);
    free(sc->s.dir);
    free(sc->s.status);
    free(sc->s.target);
    free(sc->s.event_step);
    free(sc->s.flag_step);
    free(sc->s.cap_margin);
}

static int all_finite(const double* v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static void run_forward(int dim, int nx, int ny, int nz, int ns, int M, int T, int law,
                        int steps) {
    scenario sc;
    make(&sc, dim, nx, ny, nz, ns, 5, M, T, law);
    CHECK(oracle_run(&sc.p, &sc.s, steps) == 0);
    const int64_t cells = (int64_t)nx * ny * (dim == 3 ? nz : 1);
    for (int s = 0; s < ns; ++s) {
        CHECK(all_finite(sc.s.field[s], cells));
        CHECK(isfinite(oracle_mass(&sc.p, sc.s.field[s])));
    }
    CHECK(all_finite(sc.s.pos, (int64_t)M * dim));
    double pt[3] = {0.0, 0.0, 0.0}, g[3];
    oracle_sample_gradient(&sc.p, sc.s.field[0], pt, g);
    CHECK(isfinite(g[0]) && isfinite(g[1]));
    pt[0] = nx - 1e-9;
    pt[1] = ny - 1e-9;
    pt[2] = dim == 3 ? nz - 1e-9 : 0.0;
    oracle_sample_gradient(&sc.p, sc.s.field[0], pt, g);
    CHECK(isfinite(g[0]) && isfinite(g[1]));
    /* connectivity of the run: neuron = cone % 7, target -> (3 t) % 7 */
    int32_t* owner = malloc(sizeof(int32_t) * (M ? M : 1));
    int32_t* towner = malloc(sizeof(int32_t) * (T ? T : 1));
    for (int i = 0; i < M; ++i) owner[i] = i % 7;
    for (int t = 0; t < T; ++t) towner[t] = (3 * t) % 7;
    int32_t row[8], level[7];
    int32_t* edges = malloc(sizeof(int32_t) * (M ? M : 1));
    const int64_t E = oracle_connectivity(7, M, sc.s.status, sc.s.target, owner, towner, row,
                                          edges);
    CHECK(E >= 0 && row[7] == E);
    CHECK(oracle_bfs_levels(7, row, edges, 0, level) == 0 && level[0] == 0);
    free(owner);
    free(towner);
    free(edges);
    release(&sc);
}

static void run_adjoint(int ns, int M, int steps, int with_outputs) {
    scenario sc;
    make(&sc, 2, 24, 19, 1, ns, 4, M, 6, 0);
    int32_t* assign = malloc(sizeof(int32_t) * (M ? M : 1));
    double* w = malloc(sizeof(double) * (M ? M : 1));
    for (int i = 0; i < M; ++i) {
        assign[i] = i % 6;
        w[i] = 0.5 + (double)i / (M ? M : 1);
    }
    double loss, dq[8], dD[2], dk[2], mag[12];
    double* acone = malloc(sizeof(double) * 3 * (M ? M : 1));
    CHECK(oracle_adjoint(&sc.p, &sc.s, steps, assign, w, &loss, dq, dD, dk,
                         with_outputs ? mag : NULL, with_outputs ? acone : NULL) == 0);
    CHECK(isfinite(loss) && all_finite(dq, 4 * ns) && all_finite(dD, ns) && all_finite(dk, ns));
    if (with_outputs) CHECK(all_finite(mag, 4 * ns + 2 * ns) && all_finite(acone, 3 * M));
    free(assign);
    free(w);
    free(acone);
    release(&sc);
}

int main(void) {
    run_forward(2, 33, 29, 1, 1, 40, 12, 0, 60);
    run_forward(2, 33, 29, 1, 2, 40, 12, 0, 60);
    run_forward(2, 33, 29, 1, 1, 40, 12, 1, 40);   /* SNR turn law */
    run_forward(3, 9, 7, 6, 2, 30, 8, 0, 40);
    run_forward(2, 2, 2, 1, 1, 6, 1, 0, 10);       /* smallest grid */
    run_forward(2, 16, 5, 1, 1, 0, 0, 0, 5);       /* no cones, no targets */
    run_adjoint(1, 12, 30, 1);
    run_adjoint(2, 12, 30, 0);
    run_adjoint(1, 0, 5, 1);
    double z[4];
    oracle_normals4(1, 2, 3, 4, 5, z);
    CHECK(all_finite(z, 4));
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle driver: ok (%d threads)\n", oracle_num_threads());
    return 0;
}
