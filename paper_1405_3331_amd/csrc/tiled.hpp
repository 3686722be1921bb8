// tiled.hpp -- temporally blocked, LDS-tiled step kernel: interface used by the host side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cuesim.h"
#include "internal.hpp"

namespace cuesim {

constexpr int kDefaultBlockSteps = 8;

// Tile geometry chosen once per simulation.
struct TiledPlan {
    int dim = 2;
    int block_steps = 1;     // B: steps advanced per launch (1 = tiling unavailable)
    int halo = 0;            // H: cells loaded around each tile core
    int core_x = 0, core_y = 0, core_z = 1;
    int tiles_x = 0, tiles_y = 0, tiles_z = 1;
    int n_tiles = 0;
    int height = 0;          // loaded tile height (rows), core_y + 2 * halo
    int move = 0;            // cells a tip can travel in one launch, ceil(B * s / dx)
    int cpl = 2;             // columns per lane: loaded tile width is 64 * cpl
    int cone_rows = 15;      // strip rows traded per occupied cone slot (load balance)
    int n_species = 1;
    int nx = 0, ny = 0, nz = 1;
    float inv_dx = 1.0f;
    StencilCoef coef[SIM_MAX_SPECIES] = {};
    size_t lds_bytes = 0;
};

// Launch-to-launch state of the tiled kernel, in device memory: completed steps, which half
// of every ping-pong pair is the input, and the work-queue counters (reset by the last
// workgroup of each launch).
struct LaunchState {
    uint32_t step;
    int32_t parity;
    int32_t next;
    int32_t exited;
    int32_t n_items;   // work items of the next launch (listed by the last workgroup)
    int32_t slots;     // work items a list laid out by die may hold (set by the host)
};

// Initial launch state; `slots` bounds the work items of a list laid out by die (the
// workgroups resident at once, and no more than its item capacity allows).
LaunchState tiled_launch_state(int slots);

struct TiledArgs2D;

// Device buffers owned by the tiled path.
struct TiledState {
    float4* bucket[2] = {nullptr, nullptr};    // per tile: cone slots (x, y, theta, id)
    int32_t* count[2] = {nullptr, nullptr};    // cones per tile
    int cur = 0;                               // bucket buffer holding the live cones
    int capacity = 0;                          // slots per tile
    int32_t* src_start = nullptr;              // per tile: range into src_entry
    int2* src_entry = nullptr;                 // (tile-local cell index, species)
    float* src_amount = nullptr;
    int32_t* tgt_start = nullptr;              // per tile: range into tgt_pts
    float4* tgt_pts = nullptr;                 // targets a tile's cones can reach
    TiledArgs2D* table = nullptr;              // device copy of this simulation's arguments
    LaunchState* launch = nullptr;             // device launch state
    int2* base = nullptr;                      // (simulation, tile) per tile
    int4* items = nullptr;                     // (simulation, tile, part) of the next launch
    int item_cap = 0;
    bool recording = false;                    // launches also write every sub-step's state
                                               // to the run tape (tiled_set_record)
};

// Choose B and the tile shape; block_steps = 1 in the result means no tiling fits.
// force_cpl != 0 restricts the row width to 64 * force_cpl columns, force_height != 0 the
// loaded tile height; a forced shape that does not fit falls back to the planner's choice.
TiledPlan tiled_plan(int dim, int nx, int ny, int nz, int n_species, double step_cells,
                     int block_steps, int n_cones, int force_cpl = 0, int force_height = 0);
// Allocate buckets and per-tile tables and upload the argument table; fields[s][b] are the
// simulation's ping-pong field buffers, cones its caller-order arrays.
hipError_t tiled_allocate(const TiledPlan& plan, TiledState& st, int n_cones,
                          const ConeRules& rules, const sim_params* p, float* const fields[][2],
                          ConeArrays cones, hipStream_t stream);
// Set the device launch state (step counter; parity = input half of the ping-pong pairs).
hipError_t tiled_set_launch_state(TiledState& st, uint32_t step, int parity, hipStream_t stream);
// Record mode: while tape is non-null every launch also writes the state after each of its
// sub-steps to tape + ((step - n0) * n_species + s) * cells (null: off).
hipError_t tiled_set_record(TiledState& st, float* tape, uint32_t n0, hipStream_t stream);
void tiled_release(TiledState& st);
// Move active cones from the caller-order arrays into the tile buckets.
hipError_t tiled_bucket(const TiledPlan& plan, TiledState& st, ConeArrays cones,
                        hipStream_t stream);
// Move active cones from the tile buckets back into the caller-order arrays.
hipError_t tiled_unbucket(const TiledPlan& plan, TiledState& st, ConeArrays cones,
                          hipStream_t stream);
// The same copy of the active cones into the caller-order arrays, leaving the buckets and
// counts in place, so that stepping continues without bucketing again.
hipError_t tiled_sync_cones(const TiledPlan& plan, const TiledState& st, ConeArrays cones,
                            hipStream_t stream);
// Advance `steps` (<= plan.block_steps) steps in one launch; flips st.cur like the device
// parity.
// start/stop (may be null): events the launch records around the kernel (timing).
hipError_t tiled_launch(const TiledPlan& plan, TiledState& st, int steps, hipStream_t stream,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

// Size in bytes of one argument-table entry (for batching several simulations).
size_t tiled_table_entry_bytes();
// One persistent launch over the work items of a batch whose argument tables are
// concatenated in `table`; all simulations share n_species, cpl and `launch`.  base lists
// every (simulation, tile); items receives the expanded (simulation, tile, part) list.
hipError_t tiled_launch_batch(const TiledArgs2D* table, int4* items, const int2* base,
                              int n_base, int item_cap, int n_species, int cpl,
                              size_t lds_bytes, int steps, LaunchState* launch,
                              hipStream_t stream);
// Upper bound on the work items of n_tiles tiles holding n_cones cones in total.
int tiled_item_capacity(int n_tiles, int n_cones);
// List the work items for the current cone counts (after cones were bucketed); by_die lays
// the list out for a launch of one workgroup per slot (a contiguous run of tiles per die),
// else in tile order for the persistent batch launch.
hipError_t tiled_build_items(const TiledArgs2D* table, int4* items, const int2* base,
                             int n_base, int item_cap, LaunchState* launch, hipStream_t stream,
                             bool by_die);
// Number of workgroups of the persistent batch launch for a given dynamic LDS size.
int tiled_persistent_grid(size_t lds_bytes);
// Allow the batch kernel variant lds_bytes of dynamic LDS (call before launching or
// capturing it).
hipError_t tiled_prepare_batch(int n_species, int cpl, size_t lds_bytes);

}  // namespace cuesim
