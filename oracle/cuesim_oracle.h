/*
 * cuesim_oracle.h -- FP64 CPU oracle of the cue-diffusion / growth-cone time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct simulator that
 * the GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Every array is owned by the caller.  Fields are row-major with x fastest:
 *   index(i, j, l) = (l * ny + j) * nx + i        (l = 0, nz = 1 in 2D).
 * Cone headings: 2D -> one angle in radians per cone, wrapped to [-pi, pi);
 *                3D -> one unit vector (hx, hy, hz) per cone.
 */
#ifndef CUESIM_ORACLE_H
#define CUESIM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_ACTIVE = 0, ORACLE_CONTACT = 1, ORACLE_EXITED = 2 };

typedef struct oracle_params {
    int32_t dim;                 /* 2 or 3 */
    int32_t nx, ny, nz;          /* cells per axis (nz = 1 in 2D) */
    double dx, dt;
    int32_t n_species;           /* 1 or 2 */
    double D[2], k[2], sign[2];  /* diffusion, first-order decay, +1 attract / -1 repel */
    int32_t n_sources[2];
    const int32_t* source_cell[2];  /* linear cell index per source */
    const double* source_q[2];      /* amount emitted per step */
    int32_t n_targets;
    const double* target_pos;    /* [T][dim] */
    double contact_radius;
    double step_len, turn_gain, max_turn, noise_sigma;
    uint64_t seed;
    uint32_t sim_index;
    double noise_sign;           /* +1 normally; -1 negates every normal deviate (mirror test) */
    double flag_tol;             /* near-tie margin tau for the flag record */
    /* Turn law: 0 = vector addition (the default), 1 = the SNR decision of Sec. 3.5, Eq. 5
     * (2D): inside the detection window c_min <= c <= c_max (c: species 0 at the tip), turn
     * by max_turn to the right when SNR + Z0 > 0, else to the left, where
     * SNR = snr_scale * mu * sqrt(gamma / (1 + gamma)^3) * sin(theta - theta_g),
     * gamma = c / kd, mu = cone_width * |g| / c, theta_g the direction of g; the angular
     * noise is then noise_sigma * Z1. */
    int32_t turn_law;
    double snr_scale, cone_width, kd, c_min, c_max;
} oracle_params;

typedef struct oracle_state {
    int64_t step;                /* completed steps n */
    double* field[2];            /* n_cells doubles per species */
    int32_t n_cones;
    double* pos;                 /* [M][dim] */
    double* dir;                 /* 2D: [M] angle; 3D: [M][3] unit vector */
    int32_t* status;             /* ORACLE_ACTIVE / CONTACT / EXITED */
    int32_t* target;             /* contacted target, -1 if none */
    int32_t* event_step;         /* step at which status changed, -1 if none */
    int32_t* flag_step;          /* first step with a near-tie margin <= flag_tol, -1 if none */
    double* cap_margin;          /* may be NULL: per cone, the smallest distance (rad) of an
                                    uncapped vector-law turn angle from max_turn so far */
} oracle_state;

/* Philox4x32-10 bijection (Salmon et al., SC'11). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Four standard normal deviates from one Philox block by Box-Muller on 23-bit uniforms. */
void oracle_normals4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                     double z[4]);

/* Interpolated cue gradient of one field at point p (the gradient-sampling rule). */
void oracle_sample_gradient(const oracle_params* p, const double* field, const double* point,
                            double g[3]);

/* One field update of every species (stencil + decay, then sources): in -> out. */
void oracle_field_step(const oracle_params* p, const double* const in[2], double* const out[2]);

/* One step of every active cone against the already-updated fields (state->step = n
 * before the call; the cone part of step n -> n+1).  Does not advance state->step. */
void oracle_cone_step(const oracle_params* p, oracle_state* s);

/* n_steps full steps: field update, then cones.  Returns 0, or -1 on allocation failure. */
int oracle_run(const oracle_params* p, oracle_state* s, int64_t n_steps);

/* Trajectory loss L = sum_i weight[i] * |p_i^N - target[assign[i]]|^2 after n_steps steps
 * from state s (which is advanced by them), and its gradient along the forward run's
 * branch (exit/contact decisions and the active side of the turn cap held fixed) with
 * respect to every source amount (dL_dq: species 0's sources, then species 1's), and D
 * and k of every species (dL_dD, dL_dk: [n_species]).  2D only.  Returns 0, -1 on
 * allocation failure, -2 for 3D.  Records the whole forward run (n_steps + 1 fields).
 * magnitude (may be NULL; [n_q + 2 n_species], ordered like dL_dq, dL_dD, dL_dk) receives
 * the same sums taken over the absolute values of their terms: the size of the terms each
 * gradient component cancels, which bounds the rounding error a lower-precision
 * evaluation of that component can carry.  cone_adjoint (may be NULL; [M][3]) receives
 * the derivative of L with respect to every cone's state (x, y, theta) at the start of the
 * run: set against the loss's own derivative at the tips, it measures how strongly the run
 * amplifies a perturbation of that cone. */
int oracle_adjoint(const oracle_params* p, oracle_state* s, int64_t n_steps,
                   const int32_t* assign, const double* weight, double* loss,
                   double* dL_dq, double* dL_dD, double* dL_dk, double* magnitude,
                   double* cone_adjoint);

/* Adjacency list of the connections (a cone with status CONTACT links its owner neuron to
 * the owner of its target): row_start[n_neurons + 1] (V_a) and edges (E_a, capacity
 * n_cones; each neuron's list in increasing cone index).  Returns the edge count, -1 on
 * allocation failure. */
int64_t oracle_connectivity(int32_t n_neurons, int32_t n_cones, const int32_t* status,
                            const int32_t* target, const int32_t* cone_owner,
                            const int32_t* target_owner, int32_t* row_start, int32_t* edges);

/* Breadth-first levels from root (-1 where unreachable).  Returns 0, -1 on allocation
 * failure. */
int oracle_bfs_levels(int32_t n_neurons, const int32_t* row_start, const int32_t* edges,
                      int32_t root, int32_t* level);

/* Total cue amount sum(c) * dx^dim of one species. */
double oracle_mass(const oracle_params* p, const double* field);

/* Number of OpenMP threads the oracle's loops use (1 when built without OpenMP). */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
