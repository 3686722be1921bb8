// sim.hip -- host side of the C ABI (include/cuesim.h): parameter validation, device
// allocation and upload, the step loop, state read-back and write, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "cuesim.h"
#include "internal.hpp"
#include "validate.hpp"
#include "tiled.hpp"

using namespace cuesim;

namespace {

thread_local std::string g_create_error;

// Steps between refreshes of the spatial order of 3D cones (a cone moves step_len per step;
// 8, 16, 32 and 64 were measured at 256^3, 32 was fastest).
constexpr int kOrderRefresh = 32;
// Gradient sweep: the samples' fixed-point sums are added kSumGroup steps at a time (an even
// number, so that the two-step reverse launches stay within a group) into a ring of
// kSumRing = 2 kSumGroup per-step buffers per species; each two-step launch clears the
// buffers of the group before its own, which the group after it reuses.  At 1024^2 (one
// species, 100-step segments) groups of 8 steps measured best: 24.1 ms per sweep against
// 24.9 with 4, 27.0 with 2 and 24.6 with one buffer per step of the segment (800 MiB, cleared
// per segment); the ring takes 128 MiB.
constexpr int kSumGroup = 8;
constexpr int kSumRing = 2 * kSumGroup;
static_assert(kSumGroup >= 2 && kSumGroup % 2 == 0, "groups of whole step pairs");

}  // namespace

// Record of the last sim_adjoint_run: checkpoints every `every` steps of the forward run
// (fields and caller-order cone state), the loss's per-cone target tips and weights.
struct AdjointRun {
    int64_t n0 = 0, n_steps = 0;
    int every = 1, n_ckpt = 0;
    float* ckpt_field = nullptr;        // [n_ckpt][n_species][n_cells]
    float* ckpt_pos = nullptr;          // [n_ckpt][M][2]
    float* ckpt_dir = nullptr;          // [n_ckpt][M]
    int32_t* ckpt_int = nullptr;        // [n_ckpt][3][M]: status, target, event_step
    float* tip_target = nullptr;        // [M][2]: t_a(i)
    float* weight = nullptr;            // [M]
    float* acone = nullptr;             // [M][3]
    double* loss_partial = nullptr;     // [cone workgroups]
    float* tape = nullptr;              // [n_steps + 1][n_species][n_cells]: every field state
                                        // of the run, recorded as it ran (null: not recorded)
    // The reverse sweep's workspace, allocated by its first call and kept for further calls
    // on the same record (freed with the record).
    struct Work {
        bool ready = false;
        bool whole = false;             // the window is the whole run (else one segment)
        float* tape_own = nullptr;      // the window's field states when the run did not record
        float4* tape_cones = nullptr;   // the cone state at every step of the window
        long long* scatter = nullptr;   // fixed-point sample adjoints, a ring of steps:
                                        // [kSumRing][species][cells]
        int32_t* rec_at = nullptr;      // one segment's sample records [K][M][species][12]
        float* rec_v = nullptr;
        uint32_t* step_max = nullptr;   // [K]
        float* afield = nullptr;        // the field adjoint, ping-pong per species
        double* acc = nullptr;          // FP64 accumulators
        int32_t* q_cell = nullptr;      // source cells, and the sources listed per box
        int32_t* q_start = nullptr;
        int32_t* q_index = nullptr;
    } work;
};


struct sim_handle {
    // geometry and coefficients
    int dim = 2, nx = 0, ny = 0, nz = 1;
    int64_t n_cells = 0;
    double dx = 1.0, dt = 1.0;
    int n_species = 1;
    StencilCoef coef[SIM_MAX_SPECIES] = {};
    int n_cones = 0, n_targets = 0;
    ConeRules rules = {};

    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;

    // device state
    float* field[SIM_MAX_SPECIES][2] = {};
    int cur[SIM_MAX_SPECIES] = {0, 0};
    Field2DStep field2d = {};   // 2D un-blocked field step with its per-box source lists
    ConeArrays cones = {};
    float4* target_pts = nullptr;
    int32_t* target_cells = nullptr;
    double* mass_partial = nullptr;
    double* mass_out = nullptr;
    // periodic mass check: every mass_every steps (0: off) sim_step enqueues the FP64 mass of
    // every species; a non-finite total raises the device flag mass_flag, copied to the
    // pinned host word mass_flag_host behind the event mass_event.  `nonfinite` is sticky:
    // set by a check that saw a non-finite total, cleared by a SIM_MASS read whose totals
    // are all finite.
    int64_t mass_every = 0;
    int32_t* mass_flag = nullptr;
    int32_t* mass_flag_host = nullptr;
    hipEvent_t mass_event = nullptr;
    bool mass_pending = false;
    bool nonfinite = false;

    // temporal blocking
    int block_steps = 1;
    TiledPlan plan = {};
    TiledState tiled = {};
    bool cones_bucketed = false;   // active cones live in the tile buckets

    // 3D: field step with its per-box source lists; active cones in spatial order,
    // refreshed every kOrderRefresh steps
    Field3D field3d = {};
    ConeOrder3D order3d = {};
    bool cones_ordered = false;    // tips and headings of active cones live in order3d
    int since_refresh = 0;

    int64_t step = 0;
    bool poisoned = false;
    std::string err;

    // caller-order inputs the adjoint needs
    std::vector<float> target_host;                          // [T][dim]
    std::vector<int32_t> src_caller_cell[SIM_MAX_SPECIES];   // per source, caller order
    std::vector<int32_t> src_merged_cell[SIM_MAX_SPECIES];   // merged, sorted by cell
    std::vector<float> src_merged_q[SIM_MAX_SPECIES];        // their amounts / dx^dim
    AdjointRun* adj = nullptr;
    int64_t adj_tape_limit = 0;   // bytes the gradient may record (0: half the free memory)
    float* record = nullptr;      // recording a run (per-step path): tape of its field states
    int64_t record_n0 = 0;        // step of the tape's first state
    GraphBuffers graph = {};                                 // last sim_connectivity
    int graph_cones = 0;

    // timing of the step kernel
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

namespace {

sim_status fail(sim_handle* h, sim_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return st;
}

bool sticky(hipError_t e) {
    return e == hipErrorIllegalAddress || e == hipErrorLaunchFailure ||
           e == hipErrorAssert || e == hipErrorECCNotCorrectable;
}

sim_status device_fail(sim_handle* h, hipError_t e, const char* what) {
    if (h && sticky(e)) h->poisoned = true;
    return fail(h, e == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EDEVICE, "%s: %s (%d)", what,
                hipGetErrorString(e), (int)e);
}

#define HIP_TRY(h, expr)                                       \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return device_fail(h, e_, #expr); \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc((void**)p, count * sizeof(T));
}

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_events(sim_handle* h) {
    for (auto& ev : h->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    h->events.clear();
}

static void adjoint_work_release(AdjointRun::Work& w) {
    dfree(w.tape_own);
    dfree(w.tape_cones);
    dfree(w.scatter);
    dfree(w.rec_at);
    dfree(w.rec_v);
    dfree(w.step_max);
    dfree(w.afield);
    dfree(w.acc);
    dfree(w.q_cell);
    dfree(w.q_start);
    dfree(w.q_index);
    w = AdjointRun::Work();
}

void adjoint_release(sim_handle* h) {
    AdjointRun* a = h->adj;
    if (!a) return;
    dfree(a->ckpt_field);
    dfree(a->ckpt_pos);
    dfree(a->ckpt_dir);
    dfree(a->ckpt_int);
    dfree(a->tip_target);
    dfree(a->weight);
    dfree(a->acone);
    dfree(a->loss_partial);
    dfree(a->tape);
    adjoint_work_release(a->work);
    delete a;
    h->adj = nullptr;
}

void graph_release(sim_handle* h) {
    GraphBuffers& g = h->graph;
    dfree(g.owner);
    dfree(g.target_owner);
    dfree(g.key);
    dfree(g.cone);
    dfree(g.key_sorted);
    dfree(g.cone_sorted);
    dfree(g.degree);
    dfree(g.row_start);
    dfree(g.edges);
    dfree(g.level);
    dfree(g.grew);
    if (g.scratch) (void)hipFree(g.scratch);
    g = GraphBuffers{};
}

void release(sim_handle* h) {
    adjoint_release(h);
    graph_release(h);
    for (int s = 0; s < SIM_MAX_SPECIES; ++s) {
        for (int b = 0; b < 2; ++b) dfree(h->field[s][b]);
    }
    dfree(h->cones.pos);
    dfree(h->cones.dir);
    dfree(h->cones.status);
    dfree(h->cones.target);
    dfree(h->cones.event_step);
    dfree(h->target_pts);
    dfree(h->target_cells);
    dfree(h->mass_partial);
    dfree(h->mass_out);
    dfree(h->mass_flag);
    if (h->mass_flag_host) (void)hipHostFree(h->mass_flag_host);
    h->mass_flag_host = nullptr;
    if (h->mass_event) (void)hipEventDestroy(h->mass_event);
    h->mass_event = nullptr;
    tiled_release(h->tiled);
    order3d_release(h->order3d);
    field3d_release(h->field3d);
    field2d_release(h->field2d);
    drop_events(h);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    h->stream = nullptr;
}

// Fold a finished periodic mass check into the sticky flag (never waits).
void poll_mass_check(sim_handle* h) {
    if (!h->mass_pending || hipEventQuery(h->mass_event) != hipSuccess) return;
    h->mass_pending = false;
    if (*(volatile int32_t*)h->mass_flag_host) h->nonfinite = true;
}

sim_status nonfinite_fail(sim_handle* h) {
    return fail(h, SIM_ENONFINITE,
                "a mass check found a non-finite total: replace the state (sim_write_state) "
                "and read SIM_MASS to clear");
}

int dir_width(int dim) { return dim == 2 ? 1 : 3; }

// Validate the parameter struct (validate.cpp).  Returns SIM_OK or an error with
// g_create_error set.
sim_status validate(const sim_params* p) {
    char msg[512];
    const sim_status st = validate_params(p, msg, sizeof msg);
    if (st != SIM_OK) return fail(nullptr, st, "%s", msg);
    return SIM_OK;
}

// Bucket targets into cubic cells of side >= contact radius (host counting sort, once).
sim_status build_targets(sim_handle* h, const sim_params* p) {
    const int dim = p->dim;
    const double L[3] = {h->nx * h->dx, h->ny * h->dx, h->nz * h->dx};
    const double longest = std::max(L[0], std::max(L[1], dim == 3 ? L[2] : 0.0));
    const int max_per_axis = dim == 2 ? 512 : 128;
    double cell = std::max(p->contact_radius, longest / max_per_axis);
    if (!(cell > 0)) cell = longest;
    int g[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) g[a] = std::max(1, (int)std::ceil(L[a] / cell));
    const int64_t n_cells = (int64_t)g[0] * g[1] * g[2];
    std::vector<int32_t> start(n_cells + 1, 0);
    std::vector<int64_t> key(p->n_targets);
    for (int t = 0; t < p->n_targets; ++t) {
        int c[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            const double v = std::floor((double)p->target_pos[(int64_t)t * dim + a] / cell);
            c[a] = (int)std::min<double>(std::max<double>(v, 0.0), g[a] - 1);
        }
        key[t] = ((int64_t)c[2] * g[1] + c[1]) * g[0] + c[0];
        start[key[t] + 1] += 1;
    }
    for (int64_t c = 0; c < n_cells; ++c) start[c + 1] += start[c];
    std::vector<float4> pts(std::max(1, p->n_targets));
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int t = 0; t < p->n_targets; ++t) {
        const float* tp = p->target_pos + (int64_t)t * dim;
        float4 v;
        v.x = tp[0];
        v.y = tp[1];
        v.z = dim == 3 ? tp[2] : 0.0f;
        int32_t idx = t;
        std::memcpy(&v.w, &idx, sizeof idx);
        pts[fill[key[t]]++] = v;
    }
    HIP_TRY(h, dalloc(&h->target_pts, pts.size()));
    HIP_TRY(h, dalloc(&h->target_cells, start.size()));
    HIP_TRY(h, hipMemcpy(h->target_pts, pts.data(), pts.size() * sizeof(float4),
                         hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->target_cells, start.data(), start.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    TargetGrid& tg = h->rules.targets;
    tg.pts = h->target_pts;
    tg.cell_start = h->target_cells;
    tg.gx = g[0];
    tg.gy = g[1];
    tg.gz = g[2];
    tg.inv_cell = (float)(1.0 / cell);
    tg.r = (float)p->contact_radius;
    tg.r2 = (float)(p->contact_radius * p->contact_radius);
    return SIM_OK;
}

// Merge sources sharing a cell (amounts summed in double) and scale by 1/dx^dim; the field
// kernels take them from these host lists.
void merge_sources(sim_handle* h, const sim_params* p, int s) {
    std::map<int32_t, double> merged;
    const double vol = std::pow(p->dx, p->dim);
    for (int m = 0; m < p->n_sources[s]; ++m)
        merged[p->source_cell[s][m]] += (double)p->source_q[s][m] / vol;
    h->src_merged_cell[s].clear();
    h->src_merged_q[s].clear();
    for (auto& kv : merged) {
        h->src_merged_cell[s].push_back(kv.first);
        h->src_merged_q[s].push_back((float)kv.second);
    }
}

sim_status item_size(sim_handle* h, sim_item what, int32_t index, size_t* bytes) {
    const size_t M = (size_t)h->n_cones;
    switch (what) {
        case SIM_FIELD:
            if (index < 0 || index >= h->n_species)
                return fail(h, SIM_EINVAL, "species index %d out of range", index);
            *bytes = (size_t)h->n_cells * sizeof(float);
            return SIM_OK;
        case SIM_CONE_POS: *bytes = M * h->dim * sizeof(float); break;
        case SIM_CONE_DIR: *bytes = M * dir_width(h->dim) * sizeof(float); break;
        case SIM_CONE_STATUS:
        case SIM_CONE_TARGET:
        case SIM_CONE_EVENT_STEP: *bytes = M * sizeof(int32_t); break;
        case SIM_MASS: *bytes = (size_t)h->n_species * sizeof(double); break;
        case SIM_STEP: *bytes = sizeof(int64_t); break;
        case SIM_COUNTS: *bytes = 3 * sizeof(int32_t); break;
        case SIM_KERNEL_TIME: *bytes = 2 * sizeof(double); break;
        case SIM_TILING: *bytes = 8 * sizeof(int32_t); break;
        case SIM_EVENTS: *bytes = 0; break;  // computed by the caller of item_size
        default: return fail(h, SIM_EINVAL, "unknown item %d", (int)what);
    }
    if (index != 0) return fail(h, SIM_EINVAL, "index must be 0 for item %d", (int)what);
    return SIM_OK;
}

// Bring active cones from the tile buckets back into the caller-order arrays.
sim_status unbucket(sim_handle* h) {
    if (h->cones_ordered) {
        HIP_TRY(h, order3d_end(h->order3d, h->cones, h->stream));
        h->cones_ordered = false;
    }
    if (!h->cones_bucketed) return SIM_OK;
    HIP_TRY(h, tiled_unbucket(h->plan, h->tiled, h->cones, h->stream));
    h->cones_bucketed = false;
    return SIM_OK;
}

// A start/stop event pair for the next timed launch (both null when timing is off).  The
// launch records them itself (hipExtLaunchKernel: the dispatch packet carries the
// timestamps), so timing adds no commands between launches.
sim_status timing_events(sim_handle* h, hipEvent_t* start, hipEvent_t* stop) {
    *start = *stop = nullptr;
    if (!h->timing) return SIM_OK;
    HIP_TRY(h, hipEventCreate(start));
    HIP_TRY(h, hipEventCreate(stop));
    h->events.emplace_back(*start, *stop);
    return SIM_OK;
}

sim_status collect_timing(sim_handle* h) {
    for (auto& ev : h->events) {
        float ms = 0.0f;
        HIP_TRY(h, hipEventSynchronize(ev.second));
        HIP_TRY(h, hipEventElapsedTime(&ms, ev.first, ev.second));
        h->timed_ms += ms;
        h->timed_launches += 1;
    }
    drop_events(h);
    return SIM_OK;
}

// One un-blocked step: one launch for the stencil and sources of every species, then the
// cones (2D: in caller order; 3D: in spatial order).
sim_status plain_step(sim_handle* h) {
    hipEvent_t t0, t1;
    sim_status st = timing_events(h, &t0, &t1);
    if (st != SIM_OK) return st;
    const float* in[SIM_MAX_SPECIES] = {};
    float* out[SIM_MAX_SPECIES] = {};
    for (int s = 0; s < h->n_species; ++s) {
        in[s] = h->field[s][h->cur[s]];
        out[s] = h->field[s][h->cur[s] ^ 1];
    }
    if (h->dim == 3)
        HIP_TRY(h, launch_field3d(h->field3d, in, out, h->coef, h->stream, t0, t1));
    else
        HIP_TRY(h, launch_field2d_rows(h->field2d, in, out, h->coef, h->stream, t0, t1));
    for (int s = 0; s < h->n_species; ++s) h->cur[s] ^= 1;
    if (h->record)   // recording a run: the new state goes to the tape
        for (int s = 0; s < h->n_species; ++s)
            HIP_TRY(h, hipMemcpyAsync(h->record + ((size_t)(h->step + 1 - h->record_n0) *
                                                       h->n_species + s) * h->n_cells,
                                      h->field[s][h->cur[s]], (size_t)h->n_cells * 4,
                                      hipMemcpyDeviceToDevice, h->stream));
    const float* f0 = h->field[0][h->cur[0]];
    const float* f1 = h->n_species > 1 ? h->field[1][h->cur[1]] : f0;
    if (h->dim == 2) {
        HIP_TRY(h, launch_cones2d(h->rules, f0, f1, h->cones, (uint32_t)h->step, h->stream));
    } else if (h->order3d.n > 0) {
        if (!h->cones_ordered) {
            HIP_TRY(h, order3d_begin(h->order3d, h->rules, h->cones, h->stream));
            h->cones_ordered = true;
            h->since_refresh = 0;
        } else if (h->since_refresh >= kOrderRefresh) {
            HIP_TRY(h, order3d_refresh(h->order3d, h->rules, h->stream));
            h->since_refresh = 0;
        }
        HIP_TRY(h, launch_cones3d_ordered(h->rules, f0, f1, h->order3d, h->cones,
                                          (uint32_t)h->step, h->stream));
        h->since_refresh += 1;
    }
    h->step += 1;
    return SIM_OK;
}

sim_status tiled_steps(sim_handle* h, int64_t n) {
    if (!h->cones_bucketed) {
        HIP_TRY(h, tiled_bucket(h->plan, h->tiled, h->cones, h->stream));
        h->cones_bucketed = true;
    }
    while (n > 0) {
        const int b = (int)std::min<int64_t>(n, h->plan.block_steps);
        hipEvent_t t0, t1;
        sim_status st = timing_events(h, &t0, &t1);
        if (st != SIM_OK) return st;
        HIP_TRY(h, tiled_launch(h->plan, h->tiled, b, h->stream, t0, t1));
        for (int s = 0; s < h->n_species; ++s) h->cur[s] ^= 1;
        h->step += b;
        n -= b;
    }
    return SIM_OK;
}

// sim_create with an optional forced tile row width (batches need one kernel variant).
sim_status create_impl(const sim_params* p, void* hip_stream, int force_cpl, sim_handle** out) {
    if (!out) return fail(nullptr, SIM_EINVAL, "out is NULL");
    *out = nullptr;
    sim_status st = validate(p);
    if (st != SIM_OK) return st;
    sim_handle* h = new (std::nothrow) sim_handle();
    if (!h) return fail(nullptr, SIM_ENOMEM, "host allocation failed");
    auto bail = [&](sim_status s) {
        g_create_error = h->err;
        release(h);
        delete h;
        return s;
    };
    h->dim = p->dim;
    h->nx = p->nx;
    h->ny = p->ny;
    h->nz = p->dim == 3 ? p->nz : 1;
    h->n_cells = (int64_t)h->nx * h->ny * h->nz;
    h->dx = p->dx;
    h->dt = p->dt;
    h->n_species = p->n_species;
    h->n_cones = p->n_cones;
    h->n_targets = p->n_targets;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(device_fail(h, e, "hipGetDevice"));
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(device_fail(h, e, "hipStreamCreate"));
        h->own_stream = true;
    }
    for (int s = 0; s < p->n_species; ++s) {
        const double r = p->D[s] * p->dt / (p->dx * p->dx);
        h->coef[s].r = (float)r;
        h->coef[s].kdt = (float)(p->k[s] * p->dt);
    }
    ConeRules& R = h->rules;
    R.nx = h->nx;
    R.ny = h->ny;
    R.nz = h->nz;
    R.inv_dx = (float)(1.0 / p->dx);
    R.half_inv_dx = (float)(0.5 / p->dx);
    R.Lx = (float)(h->nx * p->dx);
    R.Ly = (float)(h->ny * p->dx);
    R.Lz = (float)(h->nz * p->dx);
    R.step_len = (float)p->step_len;
    R.gain = (float)p->turn_gain;
    R.max_turn = (float)p->max_turn;
    R.turn_law = p->turn_law;
    R.snr_coef = (float)(p->snr_scale * p->cone_width);
    R.inv_kd = p->turn_law == SIM_TURN_SNR ? (float)(1.0 / p->kd) : 0.0f;
    R.c_min = (float)p->c_min;
    R.c_max = (float)p->c_max;
    R.tan_max = p->max_turn <= kSmallCap ? (float)std::tan(p->max_turn) : 0.0f;
    R.sigma = (float)p->noise_sigma;
    R.sign0 = (float)p->sign[0];
    R.sign1 = p->n_species > 1 ? (float)p->sign[1] : 0.0f;
    R.n_species = p->n_species;
    R.key.k0 = (uint32_t)(p->seed & 0xffffffffu);
    R.key.k1 = (uint32_t)(p->seed >> 32);
    R.key.sim_index = p->sim_index;

    // fields
    for (int s = 0; s < p->n_species; ++s) {
        for (int b = 0; b < 2; ++b) {
            e = dalloc(&h->field[s][b], (size_t)h->n_cells);
            if (e != hipSuccess) return bail(device_fail(h, e, "field allocation"));
        }
        if (p->init_field[s])
            e = hipMemcpy(h->field[s][0], p->init_field[s], h->n_cells * sizeof(float),
                          hipMemcpyHostToDevice);
        else
            e = hipMemset(h->field[s][0], 0, h->n_cells * sizeof(float));
        if (e != hipSuccess) return bail(device_fail(h, e, "field upload"));
        merge_sources(h, p, s);
        h->src_caller_cell[s].assign(p->source_cell[s], p->source_cell[s] + p->n_sources[s]);
    }
    // cones (caller order)
    const size_t M = (size_t)p->n_cones;
    h->cones.n = p->n_cones;
    if ((e = dalloc(&h->cones.pos, M * p->dim)) != hipSuccess ||
        (e = dalloc(&h->cones.dir, M * dir_width(p->dim))) != hipSuccess ||
        (e = dalloc(&h->cones.status, M)) != hipSuccess ||
        (e = dalloc(&h->cones.target, M)) != hipSuccess ||
        (e = dalloc(&h->cones.event_step, M)) != hipSuccess)
        return bail(device_fail(h, e, "cone allocation"));
    if (M > 0) {
        std::vector<int32_t> minus1(M, -1);
        if ((e = hipMemcpy(h->cones.pos, p->cone_pos, M * p->dim * 4, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(h->cones.dir, p->cone_dir, M * dir_width(p->dim) * 4,
                           hipMemcpyHostToDevice)) ||
            (e = hipMemset(h->cones.status, 0, M * 4)) ||
            (e = hipMemcpy(h->cones.target, minus1.data(), M * 4, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(h->cones.event_step, minus1.data(), M * 4, hipMemcpyHostToDevice)))
            return bail(device_fail(h, e, "cone upload"));
    }
    if (p->dim == 3)
        e = field3d_prepare(h->field3d, h->nx, h->ny, h->nz, h->n_species, h->src_merged_cell,
                            h->src_merged_q);
    else
        e = field2d_prepare(h->field2d, h->nx, h->ny, h->n_species, h->src_merged_cell,
                            h->src_merged_q);
    if (e != hipSuccess) return bail(device_fail(h, e, "field step set-up"));
    if (p->dim == 3 && M > 0) {
        e = order3d_allocate(h->order3d, p->n_cones, h->nx, h->ny, h->nz);
        if (e != hipSuccess) return bail(device_fail(h, e, "cone order allocation"));
    }
    st = build_targets(h, p);
    if (st != SIM_OK) return bail(st);
    h->target_host.assign(p->target_pos, p->target_pos + (size_t)p->n_targets * p->dim);
    if ((e = dalloc(&h->mass_partial, kMassPartials)) != hipSuccess ||
        (e = dalloc(&h->mass_out, SIM_MAX_SPECIES)) != hipSuccess ||
        (e = dalloc(&h->mass_flag, 1)) != hipSuccess ||
        (e = hipMemset(h->mass_flag, 0, sizeof(int32_t))) != hipSuccess ||
        (e = hipHostMalloc((void**)&h->mass_flag_host, sizeof(int32_t))) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->mass_event, hipEventDisableTiming)) != hipSuccess)
        return bail(device_fail(h, e, "mass buffers"));
    *h->mass_flag_host = 0;

    // temporal blocking plan
    h->block_steps = p->block_steps == 0 ? kDefaultBlockSteps : p->block_steps;
    if (h->block_steps > 1) {
        h->plan = tiled_plan(h->dim, h->nx, h->ny, h->nz, h->n_species, p->step_len / p->dx,
                             h->block_steps, h->n_cones,
                             force_cpl ? force_cpl : p->tile_cols_per_lane, p->tile_height);
        h->plan.inv_dx = h->rules.inv_dx;
        for (int s = 0; s < h->n_species; ++s) h->plan.coef[s] = h->coef[s];
        if (h->plan.block_steps <= 1) {
            h->block_steps = 1;   // no tile shape fits: fall back to one step per launch
        } else {
            e = tiled_allocate(h->plan, h->tiled, h->n_cones, h->rules, p, h->field, h->cones,
                               h->stream);
            if (e != hipSuccess) return bail(device_fail(h, e, "tiled state allocation"));
        }
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return bail(device_fail(h, e, "create synchronisation"));
    *out = h;
    return SIM_OK;
}

}  // namespace

struct sim_batch {
    std::vector<sim_handle*> sims;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* table = nullptr;            // concatenated device argument tables
    int2* base = nullptr;             // every (simulation, tile), largest simulations first
    int n_base = 0;
    int4* items = nullptr;            // (simulation, tile, part) work items of the next launch
    int item_cap = 0;
    LaunchState* launch = nullptr;
    int n_species = 1, cpl = 2, block_steps = 1;
    size_t lds_bytes = 0;
    int64_t step = 0;
    int graph_launches = 0;           // launches captured in `graph` (0: no graph)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::string err;
};

namespace {

sim_status batch_fail(sim_batch* b, sim_status st, const char* msg) {
    if (b)
        b->err = msg;
    else
        g_create_error = msg;
    return st;
}

#define BATCH_TRY(b, expr)                                                        \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            char m_[256];                                                         \
            snprintf(m_, sizeof m_, "%s: %s (%d)", #expr, hipGetErrorString(e_), (int)e_); \
            return batch_fail(b, e_ == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EDEVICE, m_); \
        }                                                                         \
    } while (0)

void batch_release(sim_batch* b) {
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
    for (sim_handle* h : b->sims) {
        if (!h) continue;
        release(h);
        delete h;
    }
    b->sims.clear();
    if (b->table) (void)hipFree(b->table);
    if (b->items) (void)hipFree(b->items);
    if (b->base) (void)hipFree(b->base);
    if (b->launch) (void)hipFree(b->launch);
    b->table = nullptr;
    b->items = nullptr;
    b->base = nullptr;
    b->launch = nullptr;
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    b->stream = nullptr;
}

// One launch of `steps` steps for every simulation of the batch.
sim_status batch_launch(sim_batch* b, int steps) {
    BATCH_TRY(b, tiled_launch_batch((const TiledArgs2D*)b->table, b->items, b->base,
                                    b->n_base, b->item_cap, b->n_species, b->cpl,
                                    b->lds_bytes, steps, b->launch, b->stream));
    return SIM_OK;
}

// Mirror a completed launch of `steps` steps in every simulation's host-side state.
void batch_advance(sim_batch* b, int steps, int launches) {
    for (sim_handle* h : b->sims) {
        for (int l = 0; l < launches; ++l) {
            for (int s = 0; s < h->n_species; ++s) h->cur[s] ^= 1;
            h->tiled.cur ^= 1;
        }
        h->step += (int64_t)steps * launches;
    }
    b->step += (int64_t)steps * launches;
}

}  // namespace

namespace cuesim {

sim_status handle_fail(sim_handle* h, sim_status st, const char* msg) {
    return fail(h, st, "%s", msg);
}

int handle_cones(const sim_handle* h) { return h->n_cones; }

int handle_targets(const sim_handle* h) { return h->n_targets; }

int handle_device(const sim_handle* h) { return h->device; }

sim_status connectivity_validate(sim_handle* h, int32_t n_neurons, const int32_t* cone_owner,
                                 const int32_t* target_owner, const int32_t* row_start,
                                 const int32_t* edges, int64_t edge_capacity,
                                 const int64_t* n_edges) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    const int M = h->n_cones, T = h->n_targets;
    if (n_neurons < 1) return fail(h, SIM_EINVAL, "n_neurons < 1");
    if (!row_start || !n_edges || edge_capacity < 0 || (edge_capacity > 0 && !edges) ||
        (M > 0 && !cone_owner) || (T > 0 && !target_owner))
        return fail(h, SIM_EINVAL, "NULL pointer or negative capacity");
    for (int i = 0; i < M; ++i)
        if (cone_owner[i] < 0 || cone_owner[i] >= n_neurons)
            return fail(h, SIM_EINVAL, "cone_owner[%d] = %d out of range", i, cone_owner[i]);
    for (int t = 0; t < T; ++t)
        if (target_owner[t] < 0 || target_owner[t] >= n_neurons)
            return fail(h, SIM_EINVAL, "target_owner[%d] = %d out of range", t, target_owner[t]);
    return SIM_OK;
}

sim_status connectivity_build(sim_handle* h, const GraphBuffers& g, const int32_t* cone_owner,
                              const int32_t* target_owner, int32_t* row_start, int32_t* edges,
                              int64_t edge_capacity, int64_t* n_edges) {
    const int M = h->n_cones, T = h->n_targets;
    const size_t N = (size_t)g.n_neurons;
    if (M > 0)
        HIP_TRY(h, hipMemcpyAsync(g.owner, cone_owner, (size_t)M * 4, hipMemcpyHostToDevice,
                                  h->stream));
    if (T > 0)
        HIP_TRY(h, hipMemcpyAsync(g.target_owner, target_owner, (size_t)T * 4,
                                  hipMemcpyHostToDevice, h->stream));
    // stopped cones keep their final status and target in the caller-order arrays
    HIP_TRY(h, launch_adjacency(g, h->cones.status, h->cones.target, M, g.n_neurons,
                                h->stream));
    HIP_TRY(h, hipMemcpyAsync(row_start, g.row_start, (N + 1) * 4, hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const int64_t E = row_start[g.n_neurons];
    *n_edges = E;
    if (E > edge_capacity)
        return fail(h, SIM_ERANGE, "edge buffer holds %lld edges, %lld needed",
                    (long long)edge_capacity, (long long)E);
    if (E > 0) {
        HIP_TRY(h, hipMemcpyAsync(edges, g.edges, (size_t)E * 4, hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return SIM_OK;
}

}  // namespace cuesim

extern "C" {


sim_status sim_create(const sim_params* p, void* hip_stream, sim_handle** out) {
    return create_impl(p, hip_stream, 0, out);
}

sim_status sim_step(sim_handle* h, int64_t n_steps) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    if (n_steps < 0) return fail(h, SIM_EINVAL, "n_steps < 0");
    if (h->step + n_steps > 2147483647LL)
        return fail(h, SIM_EINVAL, "step count would exceed 2^31-1");
    poll_mass_check(h);
    if (h->nonfinite) return nonfinite_fail(h);
    if (n_steps == 0) return SIM_OK;
    while (n_steps > 0) {
        // with the periodic mass check on, stop at the next multiple of mass_every
        int64_t n = n_steps;
        if (h->mass_every > 0) n = std::min(n, h->mass_every - h->step % h->mass_every);
        sim_status st = SIM_OK;
        if (h->block_steps > 1) {
            st = tiled_steps(h, n);
        } else {
            for (int64_t i = 0; i < n && st == SIM_OK; ++i) st = plain_step(h);
        }
        if (st != SIM_OK) return st;
        n_steps -= n;
        if (h->mass_every > 0 && h->step % h->mass_every == 0) {
            for (int s = 0; s < h->n_species; ++s)
                HIP_TRY(h, launch_mass(h->field[s][h->cur[s]], h->n_cells, h->mass_partial,
                                       kMassPartials, h->mass_out + s, h->stream,
                                       h->mass_flag));
            HIP_TRY(h, hipMemcpyAsync(h->mass_flag_host, h->mass_flag, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(h, hipEventRecord(h->mass_event, h->stream));
            h->mass_pending = true;
        }
    }
    return SIM_OK;
}

sim_status sim_set_mass_check(sim_handle* h, int64_t every) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    if (every < 0) return fail(h, SIM_EINVAL, "every < 0");
    h->mass_every = every;
    return SIM_OK;
}

sim_status sim_read_state(sim_handle* h, sim_item what, int32_t index, void* dst,
                          size_t dst_bytes, size_t* bytes_written) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    size_t need = 0;
    sim_status st = item_size(h, what, index, &need);
    if (st != SIM_OK) return st;
    const size_t M = (size_t)h->n_cones;
    if (what == SIM_EVENTS || what == SIM_COUNTS) {
        st = unbucket(h);
        if (st != SIM_OK) return st;
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        std::vector<int32_t> status(M), target(M), ev(M);
        if (M) {
            HIP_TRY(h, hipMemcpy(status.data(), h->cones.status, M * 4, hipMemcpyDeviceToHost));
            HIP_TRY(h, hipMemcpy(target.data(), h->cones.target, M * 4, hipMemcpyDeviceToHost));
            HIP_TRY(h, hipMemcpy(ev.data(), h->cones.event_step, M * 4, hipMemcpyDeviceToHost));
        }
        if (what == SIM_COUNTS) {
            int32_t counts[3] = {0, 0, 0};
            for (size_t i = 0; i < M; ++i)
                if (status[i] >= 0 && status[i] <= 2) counts[status[i]] += 1;
            if (bytes_written) *bytes_written = sizeof counts;
            if (dst_bytes < sizeof counts) return fail(h, SIM_ERANGE, "buffer too small");
            if (!dst) return fail(h, SIM_EINVAL, "dst is NULL");
            std::memcpy(dst, counts, sizeof counts);
            return SIM_OK;
        }
        std::vector<int32_t> rows;
        std::vector<size_t> order;
        for (size_t i = 0; i < M; ++i)
            if (status[i] != kActive) order.push_back(i);
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return ev[a] < ev[b]; });
        for (size_t i : order) {
            rows.push_back((int32_t)i);
            rows.push_back(target[i]);
            rows.push_back(ev[i]);
            rows.push_back(status[i]);
        }
        need = rows.size() * sizeof(int32_t);
        if (bytes_written) *bytes_written = need;
        if (dst_bytes < need) return fail(h, SIM_ERANGE, "buffer too small: need %zu", need);
        if (need && !dst) return fail(h, SIM_EINVAL, "dst is NULL");
        if (need) std::memcpy(dst, rows.data(), need);
        return SIM_OK;
    }
    if (bytes_written) *bytes_written = need;
    if (dst_bytes < need) return fail(h, SIM_ERANGE, "buffer too small: need %zu", need);
    if (need && !dst) return fail(h, SIM_EINVAL, "dst is NULL");
    switch (what) {
        case SIM_FIELD:
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            HIP_TRY(h, hipMemcpy(dst, h->field[index][h->cur[index]], need, hipMemcpyDeviceToHost));
            return SIM_OK;
        case SIM_CONE_POS:
        case SIM_CONE_DIR:
        case SIM_CONE_STATUS:
        case SIM_CONE_TARGET:
        case SIM_CONE_EVENT_STEP: {
            st = unbucket(h);
            if (st != SIM_OK) return st;
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            const void* src = what == SIM_CONE_POS      ? (const void*)h->cones.pos
                              : what == SIM_CONE_DIR    ? (const void*)h->cones.dir
                              : what == SIM_CONE_STATUS ? (const void*)h->cones.status
                              : what == SIM_CONE_TARGET ? (const void*)h->cones.target
                                                        : (const void*)h->cones.event_step;
            if (need) HIP_TRY(h, hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
            return SIM_OK;
        }
        case SIM_MASS: {
            for (int s = 0; s < h->n_species; ++s)
                HIP_TRY(h, launch_mass(h->field[s][h->cur[s]], h->n_cells, h->mass_partial,
                                       kMassPartials, h->mass_out + s, h->stream));
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            double m[SIM_MAX_SPECIES];
            HIP_TRY(h, hipMemcpy(m, h->mass_out, h->n_species * sizeof(double),
                                 hipMemcpyDeviceToHost));
            const double vol = std::pow(h->dx, h->dim);
            bool finite = true;
            for (int s = 0; s < h->n_species; ++s) {
                m[s] *= vol;
                finite = finite && std::isfinite(m[s]);
            }
            std::memcpy(dst, m, need);
            // this check supersedes any earlier one: the flag follows what it found
            HIP_TRY(h, hipMemsetAsync(h->mass_flag, 0, sizeof(int32_t), h->stream));
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            *h->mass_flag_host = 0;
            h->mass_pending = false;
            h->nonfinite = !finite;
            if (!finite) return nonfinite_fail(h);
            return SIM_OK;
        }
        case SIM_STEP:
            std::memcpy(dst, &h->step, sizeof(int64_t));
            return SIM_OK;
        case SIM_TILING: {
            const TiledPlan& t = h->plan;
            const bool tiled = h->block_steps > 1;
            int32_t v[8] = {tiled ? t.block_steps : 1, tiled ? t.halo : 0, tiled ? t.core_x : 0,
                            tiled ? t.core_y : 0, tiled ? t.n_tiles : 0, tiled ? t.cpl : 0,
                            tiled ? t.height : 0, tiled ? (int32_t)t.lds_bytes : 0};
            std::memcpy(dst, v, sizeof v);
            return SIM_OK;
        }
        case SIM_KERNEL_TIME: {
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            st = collect_timing(h);
            if (st != SIM_OK) return st;
            double v[2] = {h->timed_ms, (double)h->timed_launches};
            std::memcpy(dst, v, sizeof v);
            return SIM_OK;
        }
        default:
            return fail(h, SIM_EINVAL, "item %d is not readable", (int)what);
    }
}

sim_status sim_write_state(sim_handle* h, sim_item what, int32_t index, const void* src,
                           size_t bytes) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    size_t need = 0;
    sim_status st = item_size(h, what, index, &need);
    if (st != SIM_OK) return st;
    if (bytes != need) return fail(h, SIM_EINVAL, "size %zu != item size %zu", bytes, need);
    if (need && !src) return fail(h, SIM_EINVAL, "src is NULL");
    switch (what) {
        case SIM_FIELD:
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            HIP_TRY(h, hipMemcpy(h->field[index][h->cur[index]], src, need, hipMemcpyHostToDevice));
            return SIM_OK;
        case SIM_CONE_POS:
        case SIM_CONE_DIR:
        case SIM_CONE_STATUS:
        case SIM_CONE_TARGET:
        case SIM_CONE_EVENT_STEP: {
            st = unbucket(h);
            if (st != SIM_OK) return st;
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            void* d = what == SIM_CONE_POS      ? (void*)h->cones.pos
                      : what == SIM_CONE_DIR    ? (void*)h->cones.dir
                      : what == SIM_CONE_STATUS ? (void*)h->cones.status
                      : what == SIM_CONE_TARGET ? (void*)h->cones.target
                                                : (void*)h->cones.event_step;
            if (need) HIP_TRY(h, hipMemcpy(d, src, need, hipMemcpyHostToDevice));
            return SIM_OK;
        }
        case SIM_STEP: {
            int64_t v;
            std::memcpy(&v, src, sizeof v);
            if (v < 0 || v > 2147483647LL) return fail(h, SIM_EINVAL, "step out of range");
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            h->step = v;
            if (h->block_steps > 1)
                HIP_TRY(h, tiled_set_launch_state(h->tiled, (uint32_t)v, h->cur[0], h->stream));
            return SIM_OK;
        }
        default:
            return fail(h, SIM_EINVAL, "item %d is not writable", (int)what);
    }
}

sim_status sim_device_ptr(sim_handle* h, sim_item what, int32_t index, void** dev_ptr,
                          size_t* bytes) {
    if (!h || !dev_ptr) return fail(h, SIM_EINVAL, "NULL argument");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    if (what != SIM_FIELD) return fail(h, SIM_EINVAL, "only SIM_FIELD has a device view");
    size_t need = 0;
    sim_status st = item_size(h, what, index, &need);
    if (st != SIM_OK) return st;
    *dev_ptr = h->field[index][h->cur[index]];
    if (bytes) *bytes = need;
    return SIM_OK;
}

sim_status sim_set_timing(sim_handle* h, int32_t enable) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    drop_events(h);
    h->timing = enable != 0;
    h->timed_ms = 0.0;
    h->timed_launches = 0;
    return SIM_OK;
}

sim_status sim_synchronize(sim_handle* h) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    poll_mass_check(h);
    if (h->nonfinite) return nonfinite_fail(h);
    return SIM_OK;
}

sim_status sim_destroy(sim_handle* h) {
    if (!h) return SIM_OK;
    hipError_t e = hipSuccess;
    if (h->stream) e = hipStreamSynchronize(h->stream);
    release(h);
    const bool bad = e != hipSuccess || h->poisoned;
    delete h;
    if (bad) return fail(nullptr, SIM_EDEVICE, "device error pending at destroy");
    return SIM_OK;
}

const char* sim_last_error(const sim_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

// ------------------------------------------------------------------------------------
// Trajectory-loss gradient (2D)
// ------------------------------------------------------------------------------------
namespace {

static int64_t cone_blocks(const sim_handle* h) { return adjoint_cone_blocks(std::max(h->n_cones, 1)); }

// Loss seed from the current (final) cone state: a_p = 2 w (p - t), a_theta = 0; the
// per-workgroup loss partials are left in adj->loss_partial.
static sim_status adjoint_seed(sim_handle* h) {
    sim_status st = unbucket(h);
    if (st != SIM_OK) return st;
    AdjointRun* a = h->adj;
    HIP_TRY(h, launch_adjoint_seed2d(h->cones.pos, a->tip_target, a->weight, a->acone,
                                     a->loss_partial, h->n_cones, h->stream));
    return SIM_OK;
}

// Bytes of every field state of a run of n_steps, of its cone states and of the ring of
// sample sums: what the gradient needs to re-run the cones of the whole run once.
static size_t adjoint_whole_bytes(const sim_handle* h, int64_t n_steps, int64_t every) {
    (void)every;
    const size_t ns = (size_t)h->n_species, cells = (size_t)h->n_cells;
    return (size_t)(n_steps + 1) * ns * cells * 4 + (size_t)kSumRing * ns * cells * 8 +
           (size_t)n_steps * std::max<size_t>((size_t)h->n_cones, 1) * 16;
}

// The handle's tape limit (sim_adjoint_set_tape_limit), or half the free device memory.
static size_t adjoint_tape_limit(const sim_handle* h) {
    if (h->adj_tape_limit > 0) return (size_t)h->adj_tape_limit;
    size_t free_bytes = 0, total_bytes = 0;
    if (hipMemGetInfo(&free_bytes, &total_bytes) != hipSuccess) free_bytes = 0;
    return free_bytes / 2;
}

// Ends the recording of a run's field states (both paths) when it goes out of scope.
struct RecordGuard {
    sim_handle* h = nullptr;
    ~RecordGuard() {
        if (!h) return;
        h->record = nullptr;
        if (h->block_steps > 1) (void)tiled_set_record(h->tiled, nullptr, 0, h->stream);
    }
};

}  // namespace

sim_status sim_adjoint_run(sim_handle* h, int64_t n_steps, int32_t checkpoint_every,
                           const int32_t* assign, const float* weight, double* loss) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    if (h->dim != 2) return fail(h, SIM_EINVAL, "the trajectory-loss gradient is 2D only");
    if (h->rules.turn_law != SIM_TURN_VECTOR)
        return fail(h, SIM_EINVAL, "the trajectory-loss gradient needs the vector turn law");
    if (n_steps < 0 || checkpoint_every < 1)
        return fail(h, SIM_EINVAL, "n_steps < 0 or checkpoint_every < 1");
    if (h->step + n_steps > 2147483647LL)
        return fail(h, SIM_EINVAL, "step count would exceed 2^31-1");
    if (!loss) return fail(h, SIM_EINVAL, "loss is NULL");
    const int M = h->n_cones;
    const int T = h->n_targets;
    if (M > 0 && (!assign || !weight)) return fail(h, SIM_EINVAL, "assign or weight is NULL");
    std::vector<float> tips((size_t)2 * M);
    for (int i = 0; i < M; ++i) {
        if (assign[i] < 0 || assign[i] >= T)
            return fail(h, SIM_EINVAL, "assign[%d] = %d is not a target index", i, assign[i]);
        if (!std::isfinite(weight[i])) return fail(h, SIM_EINVAL, "weight[%d] not finite", i);
        tips[2 * i] = h->target_host[(size_t)assign[i] * 2];
        tips[2 * i + 1] = h->target_host[(size_t)assign[i] * 2 + 1];
    }
    adjoint_release(h);
    AdjointRun* a = new (std::nothrow) AdjointRun();
    if (!a) return fail(h, SIM_ENOMEM, "adjoint record");
    h->adj = a;
    a->n0 = h->step;
    a->n_steps = n_steps;
    a->every = checkpoint_every;
    a->n_ckpt = (int)((n_steps + checkpoint_every - 1) / checkpoint_every);
    const size_t ns = (size_t)h->n_species, cells = (size_t)h->n_cells, Ms = (size_t)M;
    const size_t nck = (size_t)a->n_ckpt;
    hipError_t e;
    if ((e = dalloc(&a->ckpt_field, nck * ns * cells)) != hipSuccess ||
        (e = dalloc(&a->ckpt_pos, nck * Ms * 2)) != hipSuccess ||
        (e = dalloc(&a->ckpt_dir, nck * Ms)) != hipSuccess ||
        (e = dalloc(&a->ckpt_int, nck * 3 * Ms)) != hipSuccess ||
        (e = dalloc(&a->tip_target, Ms * 2)) != hipSuccess ||
        (e = dalloc(&a->weight, Ms)) != hipSuccess ||
        (e = dalloc(&a->acone, Ms * 3)) != hipSuccess ||
        (e = dalloc(&a->loss_partial, (size_t)cone_blocks(h))) != hipSuccess) {
        adjoint_release(h);
        if (e == hipErrorOutOfMemory)
            return fail(h, SIM_ENOMEM, "adjoint checkpoints: out of device memory");
        return device_fail(h, e, "adjoint allocation");
    }
    if (M > 0) {
        HIP_TRY(h, hipMemcpyAsync(a->tip_target, tips.data(), Ms * 2 * 4, hipMemcpyHostToDevice,
                                  h->stream));
        HIP_TRY(h, hipMemcpyAsync(a->weight, weight, Ms * 4, hipMemcpyHostToDevice, h->stream));
    }
    // When the whole run's states fit the tape limit, record every field state as the run
    // goes (the reverse sweep then re-runs only the cone steps); if the tape cannot be had,
    // the sweep re-runs the fields from the checkpoints instead.
    RecordGuard recording;
    if (a->n_ckpt > 1 && adjoint_whole_bytes(h, n_steps, checkpoint_every) < adjoint_tape_limit(h)) {
        if (dalloc(&a->tape, (size_t)(n_steps + 1) * ns * cells) != hipSuccess) {
            (void)hipGetLastError();
            a->tape = nullptr;
        } else {
            for (size_t s = 0; s < ns; ++s)
                HIP_TRY(h, hipMemcpyAsync(a->tape + s * cells, h->field[s][h->cur[s]], cells * 4,
                                          hipMemcpyDeviceToDevice, h->stream));
            recording.h = h;
            h->record = a->tape;
            h->record_n0 = h->step;
            if (h->block_steps > 1)
                HIP_TRY(h, tiled_set_record(h->tiled, a->tape, (uint32_t)h->step, h->stream));
        }
    }
    for (int j = 0; j < a->n_ckpt; ++j) {
        // the cones' state into the caller-order arrays; tile buckets stay valid, so the run
        // goes on without bucketing the cones again
        if (h->cones_bucketed && !h->cones_ordered) {
            HIP_TRY(h, tiled_sync_cones(h->plan, h->tiled, h->cones, h->stream));
        } else {
            sim_status st = unbucket(h);
            if (st != SIM_OK) return st;
        }
        // the checkpoint: fields and cone arrays in one copy launch
        CopySpans cp = {};
        size_t words = 0;
        auto span = [&](const void* src, void* dst, size_t bytes) {
            cp.src[cp.n] = src;
            cp.dst[cp.n] = dst;
            words += bytes / 4;
            cp.word_end[cp.n++] = words;
        };
        for (size_t s = 0; s < ns; ++s)
            span(h->field[s][h->cur[s]], a->ckpt_field + ((size_t)j * ns + s) * cells, cells * 4);
        if (M > 0) {
            int32_t* ci = a->ckpt_int + (size_t)j * 3 * Ms;
            span(h->cones.pos, a->ckpt_pos + (size_t)j * Ms * 2, Ms * 8);
            span(h->cones.dir, a->ckpt_dir + (size_t)j * Ms, Ms * 4);
            span(h->cones.status, ci, Ms * 4);
            span(h->cones.target, ci + Ms, Ms * 4);
            span(h->cones.event_step, ci + 2 * Ms, Ms * 4);
        }
        HIP_TRY(h, launch_copy_spans(cp, h->stream));
        const int64_t len = std::min<int64_t>(checkpoint_every, n_steps - (int64_t)j * checkpoint_every);
        const sim_status st = sim_step(h, len);
        if (st != SIM_OK) return st;
    }
    sim_status st = adjoint_seed(h);
    if (st != SIM_OK) return st;
    std::vector<double> part((size_t)cone_blocks(h), 0.0);
    if (M > 0)
        HIP_TRY(h, hipMemcpyAsync(part.data(), a->loss_partial, part.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    double L = 0.0;
    for (double v : part) L += v;
    *loss = M > 0 ? L : 0.0;
    return SIM_OK;
}

sim_status sim_adjoint_backward(sim_handle* h, double* dL_dq, double* dL_dD, double* dL_dk) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    AdjointRun* a = h->adj;
    if (!a) return fail(h, SIM_ESTATE, "no sim_adjoint_run to differentiate");
    if (h->step != a->n0 + a->n_steps)
        return fail(h, SIM_ESTATE, "the simulation was stepped after sim_adjoint_run");
    if (!dL_dq || !dL_dD || !dL_dk) return fail(h, SIM_EINVAL, "output pointer is NULL");
    const int ns = h->n_species, M = h->n_cones, nx = h->nx, ny = h->ny;
    const size_t cells = (size_t)h->n_cells, Ms = (size_t)M;
    const int K = (int)std::min<int64_t>(a->every, std::max<int64_t>(a->n_steps, 1));
    // accumulator slots: enough for the boxes of the single- and the two-step reverse field
    // kernels (both are used; the host sums every slot)
    const int fb = std::max(adjoint_field_blocks(nx, ny), adjoint_pair_blocks(nx, ny));
    int n_q[SIM_MAX_SPECIES] = {0, 0}, q_off[SIM_MAX_SPECIES] = {0, 0};
    for (int s = 0; s < ns; ++s) n_q[s] = (int)h->src_caller_cell[s].size();
    q_off[1] = n_q[0];
    const int nq_all = n_q[0] + (ns > 1 ? n_q[1] : 0);

    // Workspace.  The field states of the reverse sweep (a window of steps), the cone state at
    // every step of the window, one segment's per-step sample adjoints, the re-run's cones,
    // the field adjoint (ping-pong per species) and FP64 accumulators.  When the whole run's
    // fields fit comfortably (under half the free device memory), the window is the whole
    // run: the fields are re-run once and the cone steps of every segment are re-run at once,
    // one thread per (segment, cone), instead of segment after segment.
    const int n_seg = a->n_ckpt;
    const int64_t n_run = a->n_steps;
    // the run recorded its field states (sim_adjoint_run): only the cone steps are re-run
    const bool recorded = a->tape != nullptr;
    AdjointRun::Work& w = a->work;
    const bool fresh = !w.ready;   // first sweep of this record: allocate the workspace
    if (fresh)
        w.whole = recorded || (n_seg > 1 &&
                               adjoint_whole_bytes(h, n_run, a->every) < adjoint_tape_limit(h));
    const bool whole = w.whole;
    const int64_t window = whole ? n_run : K;
    float*& tape_own = w.tape_own;
    float4*& tape_cones = w.tape_cones;
    long long*& scatter = w.scatter;
    int32_t*& rec_at = w.rec_at;
    float*& rec_v = w.rec_v;
    uint32_t*& step_max = w.step_max;
    float*& afield = w.afield;
    double*& acc = w.acc;
    int32_t*& q_cell = w.q_cell;
    int32_t*& q_start = w.q_start;
    int32_t*& q_index = w.q_index;
    // on a device error the workspace is dropped (the next call allocates it again)
    auto free_all = [&]() { adjoint_work_release(w); };
    // each species' sources listed by the box of the two-step kernel that holds their cell:
    // q_start[s * (nbp + 1) + box] indexes q_index (source numbers within the species)
    const int nbp = adjoint_pair_blocks(nx, ny);
    std::vector<int32_t> q_start_h((size_t)ns * (nbp + 1)), q_index_h;
    for (int s = 0; s < ns; ++s) {
        std::vector<int32_t> st, ix;
        adjoint_pair_sources(nx, ny, h->src_caller_cell[s], st, ix);
        for (int b = 0; b <= nbp; ++b)
            q_start_h[(size_t)s * (nbp + 1) + b] = st[b] + (int32_t)q_index_h.size();
        q_index_h.insert(q_index_h.end(), ix.begin(), ix.end());
    }
    hipError_t e = hipSuccess;
    const size_t acc_n = (size_t)2 * ns * fb + (size_t)std::max(nq_all, 1);
    if (fresh &&
        ((!recorded && (e = dalloc(&tape_own, (size_t)(window + 1) * ns * cells)) != hipSuccess) ||
        (e = dalloc(&tape_cones, (size_t)window * std::max<size_t>(Ms, 1))) != hipSuccess ||
        (e = dalloc(&scatter, (size_t)kSumRing * ns * cells)) != hipSuccess ||
        (e = dalloc(&rec_at, (size_t)K * std::max<size_t>(Ms, 1) * ns * 12)) != hipSuccess ||
        (e = dalloc(&rec_v, (size_t)K * std::max<size_t>(Ms, 1) * ns * 12)) != hipSuccess ||
        (e = dalloc(&step_max, (size_t)K)) != hipSuccess ||
        (e = dalloc(&afield, (size_t)2 * ns * cells)) != hipSuccess ||
        (e = dalloc(&acc, acc_n)) != hipSuccess ||
        (e = dalloc(&q_cell, (size_t)std::max(nq_all, 1))) != hipSuccess ||
        (e = dalloc(&q_start, q_start_h.size())) != hipSuccess ||
        (e = dalloc(&q_index, std::max<size_t>(q_index_h.size(), 1))) != hipSuccess)) {
        free_all();
        if (e == hipErrorOutOfMemory)
            return fail(h, SIM_ENOMEM, "adjoint workspace: out of device memory");
        return device_fail(h, e, "adjoint workspace");
    }
#define ADJ_TRY(expr)                                                       \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            free_all();                                                     \
            return device_fail(h, e_, #expr);                               \
        }                                                                   \
    } while (0)
    if (fresh) {
        for (int s = 0; s < ns; ++s)
            if (n_q[s] > 0)
                ADJ_TRY(hipMemcpyAsync(q_cell + q_off[s], h->src_caller_cell[s].data(),
                                       n_q[s] * 4, hipMemcpyHostToDevice, h->stream));
        ADJ_TRY(hipMemcpyAsync(q_start, q_start_h.data(), q_start_h.size() * 4,
                               hipMemcpyHostToDevice, h->stream));
        if (!q_index_h.empty())
            ADJ_TRY(hipMemcpyAsync(q_index, q_index_h.data(), q_index_h.size() * 4,
                                   hipMemcpyHostToDevice, h->stream));
        w.ready = true;
    }
    ADJ_TRY(hipMemsetAsync(afield, 0, (size_t)2 * ns * cells * sizeof(float), h->stream));
    ADJ_TRY(hipMemsetAsync(acc, 0, acc_n * sizeof(double), h->stream));
    double* acc_D = acc;
    double* acc_k = acc + (size_t)ns * fb;
    double* acc_q = acc + (size_t)2 * ns * fb;
    sim_status st = adjoint_seed(h);   // final statuses now in h->cones (caller order)
    if (st != SIM_OK) {
        free_all();
        return st;
    }
    int64_t t_base = 0;   // run step whose field state is at the start of the window
    float* const tape = recorded ? a->tape : tape_own;
    auto field_at = [&](int64_t t, int s) {
        return tape + ((size_t)(t - t_base) * ns + s) * cells;
    };
    auto scatter_at = [&](int t, int s) {
        return scatter + ((size_t)(t % kSumRing) * ns + s) * cells;
    };
    int cur = 0;
    auto afield_at = [&](int s, int half) { return afield + ((size_t)s * 2 + half) * cells; };
    // re-run the fields of run steps [t0, t0 + len) from the checkpoint of segment j, and
    // the cone steps of segments j .. j + n - 1
    // (the fields only when the run did not record them)
    auto rerun = [&](int j, int64_t t0, int64_t len, int n) -> hipError_t {
        if (recorded)
            return launch_cones_segments2d(h->rules, tape, cells, ns, (int)t_base, j, n,
                                           a->every, (int)n_run, (uint32_t)a->n0, a->ckpt_pos,
                                           a->ckpt_dir, a->ckpt_int, M, tape_cones, h->stream);
        hipError_t r = hipMemcpyAsync(field_at(t0, 0), a->ckpt_field + (size_t)j * ns * cells,
                                      (size_t)ns * cells * 4, hipMemcpyDeviceToDevice,
                                      h->stream);
        // two steps per launch (every state is kept), the last one alone if odd
        int64_t t = t0;
        for (; t + 2 <= t0 + len && r == hipSuccess; t += 2) {
            const float* in[SIM_MAX_SPECIES] = {field_at(t, 0), field_at(t, ns - 1)};
            float* out1[SIM_MAX_SPECIES] = {field_at(t + 1, 0), field_at(t + 1, ns - 1)};
            float* out2[SIM_MAX_SPECIES] = {field_at(t + 2, 0), field_at(t + 2, ns - 1)};
            r = launch_field2d_pair(h->field2d, in, out1, out2, h->coef, h->stream);
        }
        if (t < t0 + len && r == hipSuccess) {
            const float* in[SIM_MAX_SPECIES] = {field_at(t, 0), field_at(t, ns - 1)};
            float* out[SIM_MAX_SPECIES] = {field_at(t + 1, 0), field_at(t + 1, ns - 1)};
            r = launch_field2d_rows(h->field2d, in, out, h->coef, h->stream);
        }
        if (r == hipSuccess)
            r = launch_cones_segments2d(h->rules, tape, cells, ns, (int)t_base, j, n, a->every,
                                        (int)n_run, (uint32_t)a->n0, a->ckpt_pos, a->ckpt_dir,
                                        a->ckpt_int, M, tape_cones, h->stream);
        return r;
    };
    if (whole) ADJ_TRY(rerun(0, 0, n_run, n_seg));
    for (int j = n_seg - 1; j >= 0; --j) {
        const int64_t t0 = (int64_t)j * a->every;
        const int len = (int)std::min<int64_t>(a->every, n_run - t0);
        if (!whole) {
            t_base = t0;
            ADJ_TRY(rerun(j, t0, len, 1));
        }
        // the segment's cone adjoints (their samples' adjoints recorded per step)
        ADJ_TRY(launch_cone_adjoint_segment2d(h->rules, field_at(t0, 0), cells, ns,
                                              (uint32_t)(a->n0 + t0), len, rec_at, rec_v,
                                              step_max,
                                              tape_cones + (size_t)(t0 - t_base) * Ms,
                                              h->cones.status, h->cones.event_step, a->acone,
                                              M, h->stream));
        ADJ_TRY(hipMemsetAsync(scatter, 0, (size_t)kSumRing * ns * cells * sizeof(long long),
                               h->stream));
        // reverse the segment's field steps, two per launch while two remain, in groups of
        // kSumGroup steps from the last one down: the group's sample sums first
        int t = len - 1;
        while (t >= 0) {
            const int g_lo = std::max(t - kSumGroup + 1, 0);
            ADJ_TRY(launch_sample_add2d(cells, ns, (uint32_t)(a->n0 + t0), len, g_lo,
                                        t - g_lo + 1, kSumRing, rec_at, rec_v, step_max,
                                        scatter, h->cones.status, h->cones.event_step, M,
                                        h->stream));
            for (; t >= g_lo + 1; t -= 2) {
                // the sums of steps t + kSumGroup and t + kSumGroup - 1 (the group before,
                // already reversed) are cleared for the group after this one
                for (int s = 0; s < ns; ++s)
                    ADJ_TRY(launch_field_adjoint2d_pair(
                        nx, ny, afield_at(s, cur), scatter_at(t, s), scatter_at(t - 1, s),
                        step_max, t, t - 1, field_at(t0 + t, s), field_at(t0 + t - 1, s),
                        afield_at(s, cur ^ 1), h->coef[s], acc_D + (size_t)s * fb,
                        acc_k + (size_t)s * fb, q_start + (size_t)s * (nbp + 1), q_index,
                        q_cell + q_off[s], acc_q + q_off[s], scatter_at(t + kSumGroup, s),
                        scatter_at(t + kSumGroup - 1, s), h->stream));
                cur ^= 1;
            }
            if (t == g_lo) {   // the segment's first step, when its length is odd
                for (int s = 0; s < ns; ++s)
                    ADJ_TRY(launch_field_adjoint2d(nx, ny, afield_at(s, cur), scatter_at(t, s),
                                                   step_max, t, field_at(t0 + t, s),
                                                   afield_at(s, cur ^ 1), h->coef[s],
                                                   acc_D + (size_t)s * fb,
                                                   acc_k + (size_t)s * fb, q_cell + q_off[s],
                                                   n_q[s], acc_q + q_off[s], h->stream));
                cur ^= 1;
                --t;
            }
        }
    }
    std::vector<double> host(acc_n);
    ADJ_TRY(hipMemcpyAsync(host.data(), acc, acc_n * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    ADJ_TRY(hipStreamSynchronize(h->stream));
#undef ADJ_TRY
    const double dx2 = h->dx * h->dx;
    for (int s = 0; s < ns; ++s) {
        double sD = 0.0, sk = 0.0;
        for (int b = 0; b < fb; ++b) {
            sD += host[(size_t)s * fb + b];
            sk += host[(size_t)(ns + s) * fb + b];
        }
        dL_dD[s] = sD * h->dt / dx2;
        dL_dk[s] = -h->dt * sk;
    }
    for (int m = 0; m < nq_all; ++m) dL_dq[m] = host[(size_t)2 * ns * fb + m] / dx2;
    return SIM_OK;
}

sim_status sim_adjoint_set_tape_limit(sim_handle* h, int64_t max_bytes) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (max_bytes < 0) return fail(h, SIM_EINVAL, "max_bytes < 0");
    h->adj_tape_limit = max_bytes;
    return SIM_OK;
}

// ------------------------------------------------------------------------------------
// Connectivity: adjacency list of the contacts and breadth-first levels
// ------------------------------------------------------------------------------------
sim_status sim_connectivity(sim_handle* h, int32_t n_neurons, const int32_t* cone_owner,
                            const int32_t* target_owner, int32_t* row_start, int32_t* edges,
                            int64_t edge_capacity, int64_t* n_edges) {
    sim_status st = connectivity_validate(h, n_neurons, cone_owner, target_owner, row_start,
                                          edges, edge_capacity, n_edges);
    if (st != SIM_OK) return st;
    const int M = h->n_cones, T = h->n_targets;
    graph_release(h);
    GraphBuffers& g = h->graph;
    const size_t Ms = (size_t)std::max(M, 1), N = (size_t)n_neurons;
    g.n_neurons = n_neurons;
    hipError_t e;
    if ((e = dalloc(&g.owner, Ms)) != hipSuccess ||
        (e = dalloc(&g.target_owner, (size_t)std::max(T, 1))) != hipSuccess ||
        (e = dalloc(&g.key, Ms)) != hipSuccess || (e = dalloc(&g.cone, Ms)) != hipSuccess ||
        (e = dalloc(&g.key_sorted, Ms)) != hipSuccess ||
        (e = dalloc(&g.cone_sorted, Ms)) != hipSuccess ||
        (e = dalloc(&g.degree, N)) != hipSuccess || (e = dalloc(&g.row_start, N + 1)) != hipSuccess ||
        (e = dalloc(&g.edges, Ms)) != hipSuccess || (e = dalloc(&g.level, N)) != hipSuccess ||
        (e = dalloc(&g.grew, 1)) != hipSuccess ||
        (e = hipMalloc((void**)&g.scratch, sort_pairs_scratch_bytes(M))) != hipSuccess) {
        graph_release(h);
        if (e == hipErrorOutOfMemory) return fail(h, SIM_ENOMEM, "connectivity buffers");
        return device_fail(h, e, "connectivity allocation");
    }
    h->graph_cones = M;
    return connectivity_build(h, g, cone_owner, target_owner, row_start, edges, edge_capacity,
                              n_edges);
}

sim_status sim_bfs_levels(sim_handle* h, int32_t root, int32_t* level) {
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(h, SIM_ESTATE, "handle poisoned by an earlier device error");
    GraphBuffers& g = h->graph;
    if (!g.row_start) return fail(h, SIM_ESTATE, "no sim_connectivity graph to traverse");
    if (!level) return fail(h, SIM_EINVAL, "level is NULL");
    const int N = g.n_neurons;
    if (root < 0 || root >= N) return fail(h, SIM_EINVAL, "root %d out of range", root);
    HIP_TRY(h, launch_bfs_init(g.level, N, root, h->stream));
    for (int depth = 0; depth < N; ++depth) {
        int32_t grew = 0;
        HIP_TRY(h, hipMemsetAsync(g.grew, 0, sizeof(int32_t), h->stream));
        HIP_TRY(h, launch_bfs_level(g.row_start, g.edges, N, depth, g.level, g.grew, h->stream));
        HIP_TRY(h, hipMemcpyAsync(&grew, g.grew, sizeof grew, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (!grew) break;
    }
    HIP_TRY(h, hipMemcpyAsync(level, g.level, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return SIM_OK;
}

sim_status sim_batch_create(const sim_params* const* params, int32_t n, void* hip_stream,
                            int32_t graph_launches, sim_batch** out) {
    if (!out) return batch_fail(nullptr, SIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || n < 1) return batch_fail(nullptr, SIM_EINVAL, "need at least one simulation");
    if (graph_launches < 0 || graph_launches > 1024)
        return batch_fail(nullptr, SIM_EINVAL, "graph_launches must be in [0, 1024]");
    for (int i = 0; i < n; ++i) {
        if (!params[i]) return batch_fail(nullptr, SIM_EINVAL, "params[i] is NULL");
        if (params[i]->dim != 2) return batch_fail(nullptr, SIM_EINVAL, "batches are 2D only");
        if (params[i]->n_species != params[0]->n_species)
            return batch_fail(nullptr, SIM_EINVAL, "all simulations need the same n_species");
        if (params[i]->block_steps != params[0]->block_steps)
            return batch_fail(nullptr, SIM_EINVAL, "all simulations need the same block_steps");
        if (params[i]->tile_cols_per_lane != params[0]->tile_cols_per_lane)
            return batch_fail(nullptr, SIM_EINVAL,
                              "all simulations need the same tile_cols_per_lane");
    }
    if (params[0]->tile_cols_per_lane != 0 && params[0]->tile_cols_per_lane != 2 &&
        params[0]->tile_cols_per_lane != 4)
        return batch_fail(nullptr, SIM_EINVAL, "tile_cols_per_lane must be 0, 2 or 4");
    sim_batch* b = new (std::nothrow) sim_batch();
    if (!b) return batch_fail(nullptr, SIM_ENOMEM, "host allocation failed");
    auto bail = [&](sim_status st) {
        const std::string msg = b->err.empty() ? g_create_error : b->err;
        batch_release(b);
        delete b;
        g_create_error = msg;
        return st;
    };
    hipError_t e;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(batch_fail(b, SIM_EDEVICE, "hipStreamCreate failed"));
        b->own_stream = true;
    }
    b->n_species = params[0]->n_species;
    b->cpl = params[0]->tile_cols_per_lane ? params[0]->tile_cols_per_lane : 2;
    int64_t total_cones = 0;
    for (int i = 0; i < n; ++i) {
        sim_params q = *params[i];
        if (q.block_steps == 0) q.block_steps = kDefaultBlockSteps;
        sim_handle* h = nullptr;
        sim_status st = create_impl(&q, b->stream, b->cpl, &h);
        if (st != SIM_OK) return bail(st);
        b->sims.push_back(h);
        if (h->block_steps <= 1 || h->plan.block_steps != b->sims[0]->plan.block_steps) {
            char m[160];
            snprintf(m, sizeof m, "simulation %d: no tiling with %d steps per launch fits", i,
                     q.block_steps);
            return bail(batch_fail(b, SIM_EINVAL, m));
        }
        b->lds_bytes = std::max(b->lds_bytes, h->plan.lds_bytes);
        b->n_base += h->plan.n_tiles;
        total_cones += h->n_cones;
    }
    b->block_steps = b->sims[0]->plan.block_steps;
    if (total_cones > INT32_MAX / 2)
        return bail(batch_fail(b, SIM_EINVAL, "too many cones in the batch"));
    b->item_cap = tiled_item_capacity(b->n_base, (int)total_cones);
    // concatenated argument tables, work items, shared launch state
    const size_t entry = tiled_table_entry_bytes();
    std::vector<int2> items;
    items.reserve(b->n_base);
    for (int i = 0; i < n; ++i)
        for (int t = 0; t < b->sims[i]->plan.n_tiles; ++t) items.push_back(make_int2(i, t));
    // largest simulations first, so the persistent grid finishes with small work items
    std::stable_sort(items.begin(), items.end(), [&](const int2& x, const int2& y) {
        return b->sims[x.x]->plan.height * b->sims[x.x]->n_cones >
               b->sims[y.x]->plan.height * b->sims[y.x]->n_cones;
    });
    if ((e = hipMalloc(&b->table, entry * n)) != hipSuccess ||
        (e = hipMalloc(&b->base, sizeof(int2) * items.size())) != hipSuccess ||
        (e = hipMalloc(&b->items, sizeof(int4) * b->item_cap)) != hipSuccess ||
        (e = hipMalloc(&b->launch, sizeof(LaunchState))) != hipSuccess)
        return bail(batch_fail(b, SIM_ENOMEM, "batch allocation failed"));
    for (int i = 0; i < n; ++i)
        if ((e = hipMemcpy((char*)b->table + entry * i, b->sims[i]->tiled.table, entry,
                           hipMemcpyDeviceToDevice)) != hipSuccess)
            return bail(batch_fail(b, SIM_EDEVICE, "table copy failed"));
    if ((e = hipMemcpy(b->base, items.data(), sizeof(int2) * items.size(),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return bail(batch_fail(b, SIM_EDEVICE, "item upload failed"));
    const LaunchState ls = tiled_launch_state(0);   // a persistent launch lists no slots
    if ((e = hipMemcpy(b->launch, &ls, sizeof ls, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(batch_fail(b, SIM_EDEVICE, "launch state upload failed"));
    if ((e = tiled_prepare_batch(b->n_species, b->cpl, b->lds_bytes)) != hipSuccess)
        return bail(batch_fail(b, SIM_EDEVICE, "kernel attribute failed"));
    // initial bucketing of every simulation's cones
    for (sim_handle* h : b->sims) {
        if ((e = tiled_bucket(h->plan, h->tiled, h->cones, b->stream)) != hipSuccess)
            return bail(batch_fail(b, SIM_EDEVICE, "bucketing failed"));
        h->cones_bucketed = true;
    }
    if ((e = tiled_build_items((const TiledArgs2D*)b->table, b->items, b->base, b->n_base,
                               b->item_cap, b->launch, b->stream, false)) != hipSuccess)
        return bail(batch_fail(b, SIM_EDEVICE, "work item listing failed"));
    // optional graph of `graph_launches` full-depth launches, replayed by sim_batch_step
    if (graph_launches > 0) {
        if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return bail(batch_fail(b, SIM_EDEVICE, "graph capture failed to start"));
        for (int l = 0; l < graph_launches; ++l) {
            e = tiled_launch_batch((const TiledArgs2D*)b->table, b->items, b->base,
                                   b->n_base, b->item_cap, b->n_species, b->cpl,
                                   b->lds_bytes, b->block_steps, b->launch, b->stream);
            if (e != hipSuccess) break;
        }
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess)
            return bail(batch_fail(b, SIM_EDEVICE, "graph capture failed"));
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess)
            return bail(batch_fail(b, SIM_EDEVICE, "graph instantiation failed"));
        b->graph_launches = graph_launches;
    }
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess)
        return bail(batch_fail(b, SIM_EDEVICE, "create synchronisation failed"));
    *out = b;
    return SIM_OK;
}

sim_status sim_batch_step(sim_batch* b, int64_t n_steps) {
    if (!b) return batch_fail(nullptr, SIM_EINVAL, "batch is NULL");
    if (n_steps < 0) return batch_fail(b, SIM_EINVAL, "n_steps < 0");
    if (b->step + n_steps > 2147483647LL)
        return batch_fail(b, SIM_EINVAL, "step count would exceed 2^31-1");
    bool rebucketed = false;
    for (sim_handle* h : b->sims) {
        if (h->poisoned) return batch_fail(b, SIM_ESTATE, "a simulation hit a device error");
        if (!h->cones_bucketed) {   // after a read of cones: put them back in the buckets
            BATCH_TRY(b, tiled_bucket(h->plan, h->tiled, h->cones, b->stream));
            h->cones_bucketed = true;
            rebucketed = true;
        }
    }
    if (rebucketed)
        BATCH_TRY(b, tiled_build_items((const TiledArgs2D*)b->table, b->items, b->base,
                                       b->n_base, b->item_cap, b->launch, b->stream, false));
    const int64_t per_graph = (int64_t)b->graph_launches * b->block_steps;
    while (per_graph > 0 && n_steps >= per_graph) {
        BATCH_TRY(b, hipGraphLaunch(b->graph_exec, b->stream));
        batch_advance(b, b->block_steps, b->graph_launches);
        n_steps -= per_graph;
    }
    while (n_steps > 0) {
        const int steps = (int)std::min<int64_t>(n_steps, b->block_steps);
        sim_status st = batch_launch(b, steps);
        if (st != SIM_OK) return st;
        batch_advance(b, steps, 1);
        n_steps -= steps;
    }
    return SIM_OK;
}

sim_status sim_batch_read_state(sim_batch* b, int32_t sim, sim_item what, int32_t index,
                                void* dst, size_t dst_bytes, size_t* bytes_written) {
    if (!b) return batch_fail(nullptr, SIM_EINVAL, "batch is NULL");
    if (sim < 0 || sim >= (int32_t)b->sims.size())
        return batch_fail(b, SIM_EINVAL, "simulation index out of range");
    sim_handle* h = b->sims[sim];
    const sim_status st = sim_read_state(h, what, index, dst, dst_bytes, bytes_written);
    if (st != SIM_OK) b->err = h->err;
    return st;
}

sim_status sim_batch_synchronize(sim_batch* b) {
    if (!b) return batch_fail(nullptr, SIM_EINVAL, "batch is NULL");
    BATCH_TRY(b, hipStreamSynchronize(b->stream));
    return SIM_OK;
}

sim_status sim_batch_destroy(sim_batch* b) {
    if (!b) return SIM_OK;
    hipError_t e = hipSuccess;
    if (b->stream) e = hipStreamSynchronize(b->stream);
    batch_release(b);
    delete b;
    if (e != hipSuccess) return batch_fail(nullptr, SIM_EDEVICE, "device error pending at destroy");
    return SIM_OK;
}

const char* sim_batch_last_error(const sim_batch* b) {
    return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
