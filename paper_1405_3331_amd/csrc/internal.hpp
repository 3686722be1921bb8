// internal.hpp -- launchers shared between the host side of the library and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "cuesim.h"
#include "device.hpp"

namespace cuesim {

// Stencil coefficients of one species: c' = (c - kdt*c) + r*(sum(neighbours) - 2 dim c).
// Keeping decay and diffusion as separate terms (rather than folding them into one centre
// weight 1 - 2 dim r - k dt, whose FP32 rounding shifts the effective decay rate and is
// amplified ~1/(k dt) in the steady state) leaves only unbiased rounding.
struct StencilCoef {
    float r, kdt;
};

// Per-species source entries (unique cells, amounts already divided by dx^dim).

// Cone state in the caller's order (structure of arrays).
struct ConeArrays {
    float* pos;          // [M][dim]
    float* dir;          // 2D [M]; 3D [M][3]
    int32_t* status;
    int32_t* target;
    int32_t* event_step;
    int n;
};

// One 2D step's cones in the caller's order (kernels_plain.hip).
hipError_t launch_cones2d(const ConeRules& rules, const float* f0, const float* f1,
                          ConeArrays cones, uint32_t step, hipStream_t stream);

// 2D field step of every species in one launch, sources included (kernels_field2d.hip).
// Field2DStep holds the per-box source lists (row, column in the box, amount) built once by
// field2d_prepare from the merged, pre-scaled sources of each species.
struct Field2DStep {
    int nx = 0, ny = 0, n_species = 0, n_boxes = 0;
    int32_t* src_start = nullptr;   // [n_boxes + 1]
    int32_t* src_row = nullptr;     // per entry: row j
    int32_t* src_col = nullptr;     // per entry: thread of the box owning the cell
    float* src_q = nullptr;         // per entry: amount / dx^2
    // two steps per launch (launch_field2d_pair): per box of 256 x 4 cells, the sources on
    // the box and its one-cell ring, as (tile position, amount / dx^2)
    int n_pair_boxes = 0;
    int32_t* pair_start = nullptr;  // [n_pair_boxes + 1]
    int32_t* pair_pos = nullptr;    // per entry: row * 258 + column within the ringed box
    float* pair_q = nullptr;
};
struct Field2DStepArgs {
    const float* in[2];
    float* out[2];
    StencilCoef coef[2];
    int nx, ny, n_species;
    int tx, ty, per_xcd;
    const int32_t* src_start;
    const int32_t* src_row;
    const int32_t* src_col;
    const float* src_q;
};
hipError_t field2d_prepare(Field2DStep& f, int nx, int ny, int n_species,
                           const std::vector<int32_t>* cells, const std::vector<float>* q);
void field2d_release(Field2DStep& f);
// Two steps: out1 = the state after one step, out2 after two (every species).
hipError_t launch_field2d_pair(const Field2DStep& f, const float* const* in, float* const* out1,
                               float* const* out2, const StencilCoef* coef, hipStream_t stream);
// start/stop (may be null): events the launch itself records.
hipError_t launch_field2d_rows(const Field2DStep& f, const float* const* in, float* const* out,
                               const StencilCoef* coef, hipStream_t stream,
                               hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

// 3D field step of every species in one launch, sources included (kernels_field3d.hip).
// Field3D holds the per-box source lists (plane, thread, amount) built once by
// field3d_prepare from the merged, pre-scaled sources of each species.
struct Field3D {
    int nx = 0, ny = 0, nz = 0, n_species = 0, n_boxes = 0;
    int32_t* src_start = nullptr;    // [n_boxes + 1]
    int32_t* src_plane = nullptr;    // per entry: plane index l
    int32_t* src_thread = nullptr;   // per entry: thread of the box owning the cell
    float* src_q = nullptr;          // per entry: amount / dx^3
};
struct Field3DArgs {
    const float* in[2];
    float* out[2];
    StencilCoef coef[2];
    int nx, ny, nz, n_species;
    int tx, ty, tz, per_xcd;
    const int32_t* src_start;
    const int32_t* src_plane;
    const int32_t* src_thread;
    const float* src_q;
};
hipError_t field3d_prepare(Field3D& f, int nx, int ny, int nz, int n_species,
                           const std::vector<int32_t>* cells, const std::vector<float>* q);
void field3d_release(Field3D& f);
// start/stop (may be null): events the launch itself records.
hipError_t launch_field3d(const Field3D& f, const float* const* in, float* const* out,
                          const StencilCoef* coef, hipStream_t stream,
                          hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

// Active 3D cones in spatial order (kernels_cones3d.hip): per cone the tip (x, y, z, id)
// and heading (hx, hy, hz, 0), ping-pong halves, with the radix-sort keys, slots and scratch.
// Keys are Morton codes of the tip cell coarsened by `shift` bits per axis; stopped cones
// carry id -1 and the key `inactive`, past every active one.
struct ConeOrder3D {
    float4* tip[2] = {};
    float4* dir[2] = {};
    uint32_t* key[2] = {};
    int32_t* slot[2] = {};
    int32_t* scratch = nullptr;   // counting-sort histograms (sort_pairs)
    int cur = 0;
    int n = 0;
    int shift = 3;   // 8-cell Morton cells: 118.2 us per 256^3 step, against 119.1 with 4-cell
                     // and 118.3 / 119.5 with 16- / 32-cell ones (fewer sort passes, same order
                     // at the scale of a workgroup's block)
    uint32_t inactive = 0;
    int end_bit = 1;
};
hipError_t order3d_allocate(ConeOrder3D& o, int n, int nx, int ny, int nz);
void order3d_release(ConeOrder3D& o);
// Caller-order arrays -> ordered state (pack, sort, gather).
hipError_t order3d_begin(ConeOrder3D& o, const ConeRules& r, ConeArrays cones,
                         hipStream_t stream);
// Re-sort the ordered state by the current tips.
hipError_t order3d_refresh(ConeOrder3D& o, const ConeRules& r, hipStream_t stream);
// One step of the ordered cones; stopping cones are written to `cones` at once.
hipError_t launch_cones3d_ordered(const ConeRules& r, const float* f0, const float* f1,
                                  ConeOrder3D& o, ConeArrays cones, uint32_t step,
                                  hipStream_t stream);
// Tips and headings of the still-active ordered cones back into the caller-order arrays.
hipError_t order3d_end(const ConeOrder3D& o, ConeArrays cones, hipStream_t stream);

// Sample adjoints of one reverse step held as 64-bit fixed-point sums, so that the sum in a
// cell does not depend on the order in which the cones' contributions arrive (integer
// addition is associative): value = q * 2^(e - kFixedBits), where 2^e bounds the step's
// largest |contribution| (step_max[t] holds its FP32 bits, 0 for a step without any).
// Every contribution is at most 2^kFixedBits in magnitude after scaling, so up to
// 2^(62 - kFixedBits) of them can meet in one cell without overflow.
constexpr int kFixedBits = 40;

__device__ __forceinline__ int fixed_exponent(uint32_t max_bits) {
    if (max_bits == 0u) return 0;
    int e;
    (void)frexpf(__uint_as_float(max_bits), &e);   // max = f 2^e, 0.5 <= f < 1
    return e;
}

struct FixedStep {
    const long long* q;   // one species' sums of the step, one per cell
    double inv;           // 2^(e - kFixedBits)
    __device__ __forceinline__ float operator[](size_t x) const {
        return (float)((double)q[x] * inv);
    }
};

__device__ __forceinline__ FixedStep fixed_step(const long long* q, const uint32_t* step_max,
                                                int t) {
    return FixedStep{q, ldexp(1.0, fixed_exponent(step_max[t]) - kFixedBits)};
}

// Reverse pass of the 2D step (kernels_adjoint.hip).  Field adjoint grids have
// adjoint_field_blocks(nx, ny) workgroups, each owning one slot of acc_D / acc_k.
// A segment's fields are `fields + (t * n_species + s) * cells` for t = 0..len.
int adjoint_field_blocks(int nx, int ny);
int adjoint_cone_blocks(int n);
// Forward re-run of segments seg_first .. seg_first + n_seg - 1 of a run checkpointed every
// `every` of its n_steps steps from step n0; run step t's fields are at
// fields + ((t - t_base) * n_species + s) * cells and its cone states go to
// tape[(t - t_base) * M + i].
hipError_t launch_cones_segments2d(const ConeRules& rules, const float* fields, size_t cells,
                                   int n_species, int t_base, int seg_first, int n_seg,
                                   int every, int n_steps, uint32_t n0, const float* ckpt_pos,
                                   const float* ckpt_dir, const int32_t* ckpt_int, int M,
                                   float4* tape, hipStream_t stream);
// Reverse of a segment's cone steps: each cone's gradient samples' adjoints (12 cells per
// species and step) are written to the segment's records, rec_at / rec_v
// [len][n][n_species][12]; then the largest |contribution| of every step goes to
// step_max[len] (cleared by the call).
hipError_t launch_cone_adjoint_segment2d(const ConeRules& rules, const float* fields,
                                         size_t cells, int n_species, uint32_t seg0, int len,
                                         int32_t* rec_at, float* rec_v, uint32_t* step_max,
                                         const float4* tape, const int32_t* status,
                                         const int32_t* event_step, float* acone, int n,
                                         hipStream_t stream);
// The records of segment steps t_lo .. t_lo + n_steps - 1 added into their fixed-point sums
// with each step's scale: step t's sums of species s are e + ((t % ring) * n_species + s) *
// cells, a ring of `ring` steps whose slots for these steps must hold zeros.
hipError_t launch_sample_add2d(size_t cells, int n_species, uint32_t seg0, int len, int t_lo,
                               int n_steps, int ring, const int32_t* rec_at, const float* rec_v,
                               const uint32_t* step_max, long long* e, const int32_t* status,
                               const int32_t* event_step, int n, hipStream_t stream);
// One reverse field step with the sample adjoints of step t: e + (t * n_species) * cells
// holds the species' fixed-point sums (e points at this species' first step).
hipError_t launch_field_adjoint2d(int nx, int ny, const float* a_in, const long long* e_in,
                                  const uint32_t* step_max, int t, const float* c,
                                  float* a_out, StencilCoef coef, double* acc_D, double* acc_k,
                                  const int32_t* q_cell, int n_q, double* acc_q,
                                  hipStream_t stream);
// Two reverse steps per launch (n, then n - 1): a_in = a^{n+1}, e1/e0 = e^{n+1}/e^n (the
// fixed-point sums of segment steps t1 / t0),
// c1/c0 = c^n/c^{n-1}, a_out = a^{n-1}; adjoint_pair_blocks(nx, ny) boxes own acc_D/acc_k
// slots, and the sources are listed per box (adjoint_pair_sources: q_start[box] ..
// q_start[box + 1] - 1 index q_index, the source numbers m of q_cell / acc_q).  z1 and z0
// (may be null) are sums of other steps, which the launch sets to zero (each box its own
// cells); neither may be e1 or e0.
int adjoint_pair_blocks(int nx, int ny);
void adjoint_pair_sources(int nx, int ny, const std::vector<int32_t>& cells,
                          std::vector<int32_t>& start, std::vector<int32_t>& index);
hipError_t launch_field_adjoint2d_pair(int nx, int ny, const float* a_in, const long long* e1,
                                       const long long* e0, const uint32_t* step_max, int t1,
                                       int t0, const float* c1, const float* c0, float* a_out,
                                       StencilCoef coef, double* acc_D, double* acc_k,
                                       const int32_t* q_start, const int32_t* q_index,
                                       const int32_t* q_cell, double* acc_q,
                                       long long* z1, long long* z0, hipStream_t stream);
hipError_t launch_adjoint_seed2d(const float* pos, const float* tip_target, const float* weight,
                                 float* acone, double* partial, int n, hipStream_t stream);

// Adjacency list of the connections and its breadth-first levels (kernels_graph.hip).
struct GraphBuffers {
    int32_t* owner = nullptr;          // [M] neuron owning each cone
    int32_t* target_owner = nullptr;   // [T] neuron owning each target
    int32_t* key = nullptr;            // [M] sort keys / values and their sorted copies
    int32_t* cone = nullptr;
    int32_t* key_sorted = nullptr;
    int32_t* cone_sorted = nullptr;
    int32_t* degree = nullptr;         // [N]
    int32_t* row_start = nullptr;      // [N + 1]  (V_a)
    int32_t* edges = nullptr;          // [M]      (E_a; the first row_start[N] are used)
    int32_t* level = nullptr;          // [N]
    int32_t* grew = nullptr;           // [1]
    int32_t* scratch = nullptr;        // counting-sort histograms (sort_pairs)
    int n_neurons = 0;
};
hipError_t launch_adjacency(const GraphBuffers& g, const int32_t* status, const int32_t* target,
                            int n_cones, int n_neurons, hipStream_t stream);

// Host side of the connectivity build (sim.hip), shared by the entry points that build it:
// the argument checks, and the build itself into caller-provided device buffers g (owners
// uploaded, adjacency built on the handle's stream, copied into the caller's arrays).
sim_status connectivity_validate(sim_handle* h, int32_t n_neurons, const int32_t* cone_owner,
                                 const int32_t* target_owner, const int32_t* row_start,
                                 const int32_t* edges, int64_t edge_capacity,
                                 const int64_t* n_edges);
sim_status connectivity_build(sim_handle* h, const GraphBuffers& g, const int32_t* cone_owner,
                              const int32_t* target_owner, int32_t* row_start, int32_t* edges,
                              int64_t edge_capacity, int64_t* n_edges);
sim_status handle_fail(sim_handle* h, sim_status st, const char* msg);
int handle_cones(const sim_handle* h);
int handle_targets(const sim_handle* h);
int handle_device(const sim_handle* h);   // the device the handle was created on
hipError_t launch_bfs_init(int32_t* level, int n, int root, hipStream_t stream);
hipError_t launch_bfs_level(const int32_t* row_start, const int32_t* edges, int n, int depth,
                            int32_t* level, int32_t* grew, hipStream_t stream);

// Stable sort of n (key, value) pairs by the low key_bits bits of the keys (every key must
// be below 2^key_bits) with the project's counting passes (kernels_sort.hip).  keys/vals
// hold the input; keys_alt/vals_alt (same sizes) are the other half of each pass's
// ping-pong; *in_alt tells which pair holds the result.  scratch holds
// sort_pairs_scratch_bytes(n) bytes.
size_t sort_pairs_scratch_bytes(int n);
hipError_t sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                      int n, int key_bits, int32_t* scratch, hipStream_t stream, bool* in_alt);

// Sum of a field in FP64 (deterministic two-pass reduction) into *out (device); when
// nonfinite is given, a non-finite sum sets *nonfinite = 1 (device).
// Up to kMaxSpans device-to-device copies of whole 4-byte words in one launch: span k copies
// word_end[k] - word_end[k - 1] words from src[k] to dst[k] (word_end is cumulative).
constexpr int kMaxSpans = 8;
struct CopySpans {
    const void* src[kMaxSpans];
    void* dst[kMaxSpans];
    size_t word_end[kMaxSpans];
    int n;
};
hipError_t launch_copy_spans(const CopySpans& c, hipStream_t stream);

hipError_t launch_mass(const float* field, int64_t n, double* partial, int n_partial,
                       double* out, hipStream_t stream, int32_t* nonfinite = nullptr);
constexpr int kMassPartials = 1024;

}  // namespace cuesim
