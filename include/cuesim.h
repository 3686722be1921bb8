/*
 * cuesim.h -- C ABI of the MI355X (gfx950) cue-diffusion / growth-cone simulator.
 *
 * The library advances the data-parallel hot path of the axon-guidance simulation of
 * Mihut, Morgan & Kaiser (2014): every time step first updates the guidance-cue
 * environment, then moves every growth cone one independent step (Sec. 1: growth per
 * neuron each time step as a parallel, independent process; Sec. 3.5: cue-diffusion
 * guidance).  Concretely, one step n -> n+1 is:
 *
 *   1. each cue species s: c' = c + r * sum_axes(c[+e] + c[-e] - 2c) - k dt c,
 *      r = D dt / dx^2 (5-point stencil in 2D, 7-point in 3D), with zero-flux walls: a
 *      neighbour outside the grid is replaced by the cell itself;
 *   2. each point source adds q / dx^dim to its cell;
 *   3. each ACTIVE cone samples g = sum_s sign_s * grad c_s at its tip (central differences
 *      at cell centres, bilinear / trilinear interpolation to the tip; cell (i,j[,l]) has
 *      its centre at ((i+1/2)dx, (j+1/2)dx[, (l+1/2)dx]));
 *   4. turns its heading toward the direction of h + turn_gain * g (the vector-addition
 *      steering of Sec. 3.5, Eqs. 6-7: angle from the dot and cross products), by at most
 *      max_turn (pi/30 in Sec. 3.5);
 *   5. adds angular noise from Philox4x32-10 with key = (seed lo, seed hi) (the stateless
 *      per-thread generator style of Sec. 5.1).  Each 128-bit block (x0, x1, x2, x3) gives
 *      two Box-Muller pairs on uniforms u = ((x >> 9) + 0.5) * 2^-23: (Z0, Z1) from
 *      (u0, u1) and (Z2, Z3) from (u2, u3), Z0 = sqrt(-2 ln u0) cos(2 pi u1),
 *      Z1 = sqrt(-2 ln u0) sin(2 pi u1).
 *      2D: one block serves two steps: counter = (original cone index, floor(n / 2), 0,
 *      sim_index); step n takes the pair (Z0, Z1) when n is even and (Z2, Z3) when n is odd,
 *      and theta += noise_sigma * (the pair's first deviate), wrapped to [-pi, pi).
 *      3D: one block per step: counter = (original cone index, n, 0, sim_index); h is
 *      rotated by |w| toward w = noise_sigma * (z - (z.h) h), z = (Z0, Z1, Z2), then
 *      renormalised;
 *   6. advances step_len along the heading (a fixed distance per step, Sec. 3.5);
 *   7. stops as EXITED (event step n+1) if it left [0, n_a dx) on any axis (Sec. 3.4);
 *   8. otherwise stops as CONTACT (event step n+1) if its squared distance to some target
 *      is strictly below contact_radius^2 (the sphere test of Sec. 3.3); the nearest target
 *      is recorded, the lowest index on an exact tie.
 *
 * Arithmetic is FP32 on the device: sine and cosine from the library's own reduction and
 * polynomials (within 1.4 * 2^-24 of the exact values), the Box-Muller logarithm and square
 * root and the turn's reciprocal from the hardware (about one ulp), every fused multiply-add
 * explicit; the per-step, tiled and batched paths give bitwise identical states for any
 * blocking depth or tile shape.  All entry points return a sim_status and never abort
 * or throw across the ABI.  Handles are not thread-safe: calls on one handle must not
 * overlap; different handles are independent.
 */
#ifndef CUESIM_H
#define CUESIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sim_status {
    SIM_OK = 0,
    SIM_EINVAL = -1,   /* bad argument: NULL pointer, size, non-finite value, bad item */
    SIM_ECFL = -2,     /* unstable or non-positive scheme: D dt/dx^2 > 1/(2 dim) or
                          2 dim D dt/dx^2 + k dt > 1 for some species */
    SIM_ENOMEM = -3,   /* device or host allocation failed */
    SIM_EDEVICE = -4,  /* a HIP call failed; see sim_last_error */
    SIM_ERANGE = -5,   /* destination buffer too small (bytes_written = size needed) */
    SIM_ESTATE = -6,   /* the handle hit a sticky device error earlier: only
                          sim_last_error and sim_destroy remain usable */
    SIM_ENONFINITE = -7 /* a mass check (a SIM_MASS read, or the periodic check of
                          sim_set_mass_check) found a non-finite total: the fields hold NaN
                          or Inf.  Sticky: sim_step and sim_adjoint_run refuse with this
                          status (and sim_synchronize reports it) until the state has been
                          replaced through sim_write_state and a SIM_MASS read finds every
                          total finite again.  Reads and writes stay usable. */
} sim_status;

/* Cone status codes (CONE_STATUS items and the kind column of EVENTS). */
enum { SIM_CONE_ACTIVE = 0, SIM_CONE_CONTACT = 1, SIM_CONE_EXITED = 2 };

typedef enum sim_item {
    SIM_FIELD = 0,           /* float[cells] of species `index`, x fastest        (r/w) */
    SIM_CONE_POS = 1,        /* float[M][dim]                                      (r/w) */
    SIM_CONE_DIR = 2,        /* 2D: float[M] angle in [-pi, pi); 3D: float[M][3]  (r/w) */
    SIM_CONE_STATUS = 3,     /* int32[M] SIM_CONE_*                                (r/w) */
    SIM_CONE_TARGET = 4,     /* int32[M] contacted target index, -1 if none        (r/w) */
    SIM_CONE_EVENT_STEP = 5, /* int32[M] step at which the cone stopped, -1        (r/w) */
    SIM_EVENTS = 6,          /* int32[E][4] (cone, target, step, kind) sorted by
                                (step, cone); one row per stopped cone             (r)   */
    SIM_MASS = 7,            /* double[n_species]: sum(c) dx^dim, FP64 accumulation (r)  */
    SIM_STEP = 8,            /* int64[1] completed steps                           (r/w) */
    SIM_COUNTS = 9,          /* int32[3]: active, contact, exited                  (r)   */
    SIM_KERNEL_TIME = 10,    /* double[2]: summed device milliseconds and number of
                                launches of the step kernel since timing was last
                                enabled (see sim_set_timing)                       (r)   */
    SIM_TILING = 11          /* int32[8]: steps per launch B, halo H, core width TX,
                                core height TY, number of tiles, columns per lane,
                                loaded height, LDS bytes per tile (B = 1: no tiling) (r) */
} sim_item;

#define SIM_MAX_SPECIES 2

/*
 * Simulation parameters.  Every array is read during sim_create and copied; the caller
 * keeps ownership and may free it when sim_create returns.  Arrays are host pointers.
 */
typedef struct sim_params {
    uint32_t struct_size;              /* = sizeof(sim_params) */
    int32_t dim;                       /* 2 or 3 */
    int32_t nx, ny, nz;                /* cells per axis, each >= 2 (nz ignored in 2D) */
    double dx, dt;                     /* cell side and time step, > 0 */
    int32_t n_species;                 /* 1 or 2 */
    double D[SIM_MAX_SPECIES];         /* diffusion coefficient >= 0 */
    double k[SIM_MAX_SPECIES];         /* first-order decay rate >= 0 */
    double sign[SIM_MAX_SPECIES];      /* weight of the species in g: +1 attract, -1 repel */
    int32_t n_sources[SIM_MAX_SPECIES];
    const int32_t* source_cell[SIM_MAX_SPECIES];  /* linear cell index (x fastest) */
    const float* source_q[SIM_MAX_SPECIES];       /* amount added per step */
    const float* init_field[SIM_MAX_SPECIES];     /* NULL = zero field */
    int32_t n_cones;                   /* M >= 0 */
    const float* cone_pos;             /* [M][dim], inside [0, n_a dx) */
    const float* cone_dir;             /* 2D: [M] angle; 3D: [M][3] unit vectors */
    int32_t n_targets;                 /* T >= 0 */
    const float* target_pos;           /* [T][dim] */
    double contact_radius;             /* >= 0 */
    double step_len;                   /* >= 0 */
    double turn_gain;                  /* finite */
    double max_turn;                   /* in [0, pi] */
    double noise_sigma;                /* >= 0, radians */
    uint64_t seed;
    uint32_t sim_index;                /* fourth Philox counter word */
    int32_t block_steps;               /* steps fused into one launch of the tiled kernel;
                                          0 = library default, 1 = one kernel sequence per
                                          step (no temporal blocking), max 32 */
    int32_t tile_cols_per_lane;        /* tiled kernel row width 64 * this (2 or 4);
                                          0 = chosen by the library's planner */
    int32_t tile_height;               /* loaded tile height in rows; 0 = planner's choice.
                                          A hint that does not fit is ignored */
    /* Turn law (2D): SIM_TURN_VECTOR (0) is step 4 above.  SIM_TURN_SNR (1) is the
     * decision of Sec. 3.5, Eq. 5: with c the concentration of species 0 at the tip
     * (interpolated from the cell centres like the gradient) inside the detection window
     * [c_min, c_max] and g != 0, the heading turns by max_turn to the right (clockwise)
     * when SNR + z0 > 0 and to the left otherwise, where (z0, z1) is the step's normal
     * pair of step 5 (2D layout: (Z0, Z1) on even steps, (Z2, Z3) on odd ones) and
     *   SNR = snr_scale * mu * sqrt(gamma / (1 + gamma)^3) * sin(theta - theta_g),
     *   gamma = c / kd, mu = cone_width * |g| / c, theta_g = the direction of g;
     * outside the window it does not turn.  The angular noise is then noise_sigma * z1
     * (z0 decided the turn).  turn_gain is unused.  Requires dim = 2, kd > 0,
     * 0 < c_min <= c_max, cone_width >= 0, all finite.  The trajectory-loss gradient
     * (sim_adjoint_run) is defined for SIM_TURN_VECTOR only. */
    int32_t turn_law;
    double snr_scale, cone_width, kd, c_min, c_max;
} sim_params;

enum { SIM_TURN_VECTOR = 0, SIM_TURN_SNR = 1 };

typedef struct sim_handle sim_handle;

/* Validate *p, allocate device state on the current HIP device and upload it.  hip_stream
 * is the hipStream_t every later operation is enqueued on (NULL: a stream the library
 * creates and owns).  On success *out owns the simulation until sim_destroy; on failure
 * *out = NULL and sim_last_error(NULL) describes the problem. */
sim_status sim_create(const sim_params* p, void* hip_stream, sim_handle** out);

/* Enqueue n_steps >= 0 time steps on the handle's stream and return without waiting.
 * SIM_ENONFINITE (nothing enqueued) once a mass check has found a non-finite total. */
sim_status sim_step(sim_handle* h, int64_t n_steps);

/* Mass check every `every` steps (0 = off, the default): whenever the step count reaches a
 * multiple of `every`, sim_step enqueues the FP64 mass of every species (the same reduction
 * as a SIM_MASS read, no host synchronisation); a non-finite total makes the handle
 * SIM_ENONFINITE, reported by the first sim_step or sim_synchronize that finds the check
 * completed.  SIM_EINVAL if every < 0. */
sim_status sim_set_mass_check(sim_handle* h, int64_t every);

/* Wait for the stream, then copy `what` (species `index` for FIELD, else 0) into the
 * caller's host buffer dst of dst_bytes.  Cones come back in the caller's original order.
 * *bytes_written (may be NULL) receives the size of the item; SIM_ERANGE if dst_bytes is
 * smaller (nothing is copied).  SIM_MASS is a mass check: its totals are written in any
 * case, and it returns SIM_ENONFINITE (sticky, see above) if one is not finite, SIM_OK
 * (clearing that state) if all are. */
sim_status sim_read_state(sim_handle* h, sim_item what, int32_t index, void* dst,
                          size_t dst_bytes, size_t* bytes_written);

/* Wait for the stream, then replace `what` from the caller's host buffer src (bytes must
 * equal the item size).  Used to restart from a saved or externally computed state. */
sim_status sim_write_state(sim_handle* h, sim_item what, int32_t index, const void* src,
                           size_t bytes);

/* Non-owning device pointer to the current FIELD of species `index` (float[cells]),
 * valid until the next sim_step / sim_write_state / sim_destroy on the handle. */
sim_status sim_device_ptr(sim_handle* h, sim_item what, int32_t index, void** dev_ptr,
                          size_t* bytes);

/* Enable (1) or disable (0) HIP-event timing of every launch of the step kernel (the
 * tiled kernel; with block_steps = 1 and in 3D, the field kernel, whose one launch covers
 * the stencil and sources of every species); enabling resets the totals read back through
 * SIM_KERNEL_TIME. */
sim_status sim_set_timing(sim_handle* h, int32_t enable);

/* Block until all work enqueued on the handle's stream has finished.  SIM_ENONFINITE if a
 * mass check has found a non-finite total. */
sim_status sim_synchronize(sim_handle* h);

/* Release all resources; NULL is a no-op.  Returns SIM_EDEVICE if a HIP call failed
 * (resources are released regardless). */
sim_status sim_destroy(sim_handle* h);

/* Message for the last failed call on h, or for the calling thread's last failed
 * sim_create when h is NULL.  Library-owned, valid until the next call on h. */
const char* sim_last_error(const sim_handle* h);

/* ----------------------------------------------------------------------------------------
 * Gradient of a trajectory loss (2D simulations).
 *
 * L = sum_i weight[i] * |p_i^N - t_assign[i]|^2 over the cones' tips after a run (a stopped
 * cone keeps the tip it stopped at), differentiated by reverse-mode (adjoint) sweeps of the
 * step above with respect to every source amount q, and D and k of every species.  The
 * derivative is taken along the run's branch: the exit and contact decisions and the active
 * side of the turn cap are held as the run took them (the cone rules of Sec. 3.4-3.5 are
 * not differentiable at those switches).  Memory: checkpoints of the fields and cone state
 * every checkpoint_every steps.  When every field state of the run fits within the tape
 * limit (sim_adjoint_set_tape_limit), the run records them all as it goes and the reverse
 * sweep re-runs only the cone steps; otherwise the sweep re-runs each segment of
 * checkpoint_every + 1 fields per species from its checkpoint just before reversing it.
 * Both ways give the same gradient, bit for bit.
 * ---------------------------------------------------------------------------------------- */

/* Advance n_steps >= 0 steps (as sim_step does), checkpointing every checkpoint_every >= 1
 * steps, and return the loss in *loss (synchronises the stream).  assign[M] (target index
 * per cone, 0 <= assign[i] < n_targets) and weight[M] are host arrays copied during the
 * call.  Replaces any earlier record on the handle.  SIM_EINVAL for a 3D handle, bad
 * counts or indices, non-finite weights; SIM_ENOMEM if the checkpoints do not fit. */
sim_status sim_adjoint_run(sim_handle* h, int64_t n_steps, int32_t checkpoint_every,
                           const int32_t* assign, const float* weight, double* loss);

/* Reverse sweep of the last sim_adjoint_run (the handle must not have been stepped since;
 * SIM_ESTATE otherwise).  Writes host arrays dL_dq[sum of n_sources] (species 0's sources
 * in the caller's order, then species 1's), dL_dD[n_species] and dL_dk[n_species].  May be
 * called again for the same record: its device workspace is allocated by the first call and
 * kept, with the record, until the next sim_adjoint_run or sim_destroy.  Synchronises the
 * stream. */
sim_status sim_adjoint_backward(sim_handle* h, double* dL_dq, double* dL_dD, double* dL_dk);

/* Device memory (bytes) that the gradient may spend on recorded states: every field state
 * of the run (recorded by sim_adjoint_run as it steps, freed with the record) and every
 * cone state (re-run once by sim_adjoint_backward), instead of re-running each checkpoint
 * segment from its checkpoint just before reversing it.  0 (the default) means half the
 * device memory free when sim_adjoint_run starts.  Set it before sim_adjoint_run.  When
 * the whole run's states do not fit within the limit, each segment is re-run from its
 * checkpoint; both ways give the same gradient.  SIM_EINVAL if max_bytes < 0. */
sim_status sim_adjoint_set_tape_limit(sim_handle* h, int64_t max_bytes);

/* ----------------------------------------------------------------------------------------
 * Connectivity (Sec. 3.4, Figs. 4-5): a cone that stopped on a target is a connection from
 * the neuron owning the cone to the neuron owning the target.
 * ---------------------------------------------------------------------------------------- */

/* Build the adjacency list of the connections made so far (on the device) and copy it to
 * the caller's host arrays: row_start[n_neurons + 1] (V_a: neuron v's neighbours are
 * edges[row_start[v] .. row_start[v+1]-1]) and edges (E_a, one entry per contacting cone,
 * within a neuron in increasing cone index; a neighbour appears once per connection).
 * cone_owner[M] and target_owner[T] (values in [0, n_neurons)) are host arrays.  *n_edges
 * receives the edge count; SIM_ERANGE if edge_capacity is smaller (row_start is still
 * written, edges is not).  The graph is kept on the handle for sim_bfs_levels. */
sim_status sim_connectivity(sim_handle* h, int32_t n_neurons, const int32_t* cone_owner,
                            const int32_t* target_owner, int32_t* row_start, int32_t* edges,
                            int64_t edge_capacity, int64_t* n_edges);

/* sim_connectivity for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments,
 * result and errors, but every device buffer comes from one fixed array in the library
 * (about 10.6 MB per GPU, held until the process ends) and the call allocates nothing.
 * Limits: at most 262144 cones, 262144 targets and 262144 neurons, else SIM_EINVAL before
 * any device work.  The graph is not kept for sim_bfs_levels.  All calls on one GPU share
 * the array: calls that overlap on one GPU (from several threads or handles) race. */
sim_status sim_connectivity_noalloc(sim_handle* h, int32_t n_neurons,
                                    const int32_t* cone_owner, const int32_t* target_owner,
                                    int32_t* row_start, int32_t* edges, int64_t edge_capacity,
                                    int64_t* n_edges);

/* Level-synchronous breadth-first traversal of the last sim_connectivity graph from root
 * (one device launch per level, one thread per vertex): level[n_neurons] (host) receives
 * the number of edges on a shortest path from root, -1 where unreachable.  SIM_ESTATE if no
 * graph was built. */
sim_status sim_bfs_levels(sim_handle* h, int32_t root, int32_t* level);

/* ----------------------------------------------------------------------------------------
 * Batches: many independent 2D simulations (same n_species and block_steps, any grid size,
 * cone and target counts) advanced together.  Each block of steps is ONE persistent
 * launch in which a fixed grid of workgroups pulls (simulation, tile) work items from an
 * atomic queue, so uneven simulations share the GPU; every simulation computes exactly what
 * it would compute alone (its own Philox key and sim_index).
 * ---------------------------------------------------------------------------------------- */
typedef struct sim_batch sim_batch;

/* Create n simulations from params[0..n-1] (each validated as by sim_create; arrays
 * copied).  All share block_steps and tile_cols_per_lane (0 = 2 for a batch); each keeps
 * its own tile_height hint.  graph_launches > 0 captures that many full-depth launches in a hipGraph that
 * sim_batch_step replays; 0 launches directly.  Errors as sim_create; *out = NULL on error
 * and sim_batch_last_error(NULL) describes it. */
sim_status sim_batch_create(const sim_params* const* params, int32_t n, void* hip_stream,
                            int32_t graph_launches, sim_batch** out);

/* Enqueue n_steps >= 0 steps of every simulation of the batch. */
sim_status sim_batch_step(sim_batch* b, int64_t n_steps);

/* sim_read_state of simulation `sim` (0 <= sim < n). */
sim_status sim_batch_read_state(sim_batch* b, int32_t sim, sim_item what, int32_t index,
                                void* dst, size_t dst_bytes, size_t* bytes_written);

/* Block until the batch's stream is idle. */
sim_status sim_batch_synchronize(sim_batch* b);

/* Release everything; NULL is a no-op. */
sim_status sim_batch_destroy(sim_batch* b);

/* Message for the last failed call on b (or the thread's last failed batch create). */
const char* sim_batch_last_error(const sim_batch* b);

#ifdef __cplusplus
}
#endif
#endif
