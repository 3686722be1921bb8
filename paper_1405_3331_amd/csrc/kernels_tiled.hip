// kernels_tiled.hip -- temporally blocked, LDS-tiled step kernel for 2D grids.
//
// One launch advances B steps.  Each workgroup owns one tile: a core of TX x TY cells plus
// a halo of H cells on every side, loaded once from HBM into LDS.  Each sub-step updates
// the whole tile in LDS (the valid region shrinks by one cell per sub-step), adds the
// sources that fall in the tile, and then steps the growth cones bucketed to the tile
// against the just-updated LDS field -- the field update precedes the cone step within a
// step, as in the paper's time step.  After B sub-steps the core is written back and every
// surviving cone is appended to the bucket of the tile that now holds its tip.
//
// Halo: a cone bucketed to the core at block start is at most ceil((B-1) s / dx) cells away
// from the core before its last sub-step and samples cells up to 2 away from its own cell,
// while the valid region after sub-step b is the core grown by H - b; so
// H = B + ceil((B-1) s / dx) + 2 keeps every sample inside valid cells.  H is rounded up to
// a multiple of the per-lane segment width so that segments stay aligned to the grid.
//
// Layout of a tile row in LDS: one wavefront spans the loaded width W = 64 * CPL, lane l
// owning columns CPL*l .. CPL*l + CPL-1.  The eight wavefronts of a workgroup own
// consecutive strips of rows and update them in place (see strip_update).
//
// HBM traffic per launch: the tile with its halo is read once and the core written once,
// instead of B reads and B writes of every cell.
#include <hip/hip_ext.h>

#include "tiled.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <map>
#include <vector>

namespace cuesim {

namespace {

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxTileTargets = 256;        // targets staged in LDS per tile
constexpr size_t kLdsBudget = 154 * 1024;   // dynamic LDS; the rest is static (targets,
                                            // re-bucketing counters)
constexpr int kLoadBatch = 10;              // tile rows a wavefront has in flight at load
constexpr int kConeSlots = 1;               // cones per thread held in registers
constexpr int kPartCones = kConeSlots * kThreads;   // cones one work item steps
constexpr size_t kStaticLds = kMaxTileTargets * 16 + 3 * 9 * 4 + 16;   // static LDS per tile
constexpr int kGuardRows = 4;               // one above and three below each species plane
constexpr int kXcds = 8;                    // dies (XCDs); workgroup b of a launch runs on die
                                            // b % kXcds

}  // namespace

// Static description of one simulation for the tiled kernel (device-resident table entry).
// Everything that changes from launch to launch lives in LaunchState.
struct TiledArgs2D {
    float* field[SIM_MAX_SPECIES][2];   // [species][ping-pong buffer]
    StencilCoef coef[SIM_MAX_SPECIES];
    int nx, ny;
    int tiles_x, n_tiles;
    int tx_core, ty_core, halo, height;   // TX, TY, H, loaded height HL
    const int32_t* src_start;
    const int2* src_entry;     // (LDS index within the species plane, species)
    const float* src_amount;
    const int32_t* tgt_start;  // per tile: targets within reach of its cones this launch
    const float4* tgt_pts;
    float4* bucket[2];         // per tile: cone slots (x, y, theta, id bits); the input
                               // bucket's slots of a tile are owned by its workgroup and
                               // updated in place
    int32_t* count[2];         // the input counts are zeroed by each workgroup for reuse as
                               // the next launch's output
    int capacity;
    int cone_rows;             // stencil rows a wavefront gives up per cone slot it steps
    ConeArrays cones;
    ConeRules rules;
    float* record;             // non-null: every sub-step's field also goes to
                               // record + ((step - record_n0) * NS + s) * cells (a tape of
                               // every state of a run, for the trajectory-loss gradient)
    uint32_t record_n0;
};

namespace {

template <int CPL>
struct Row;
template <>
struct Row<2> {
    using T = float2;
};
template <>
struct Row<4> {
    using T = float4;
};

__device__ __forceinline__ float comp(const float2& v, int k) { return k == 0 ? v.x : v.y; }
__device__ __forceinline__ float comp(const float4& v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}
__device__ __forceinline__ void set_comp(float2& v, int k, float x) {
    if (k == 0) v.x = x; else v.y = x;
}
__device__ __forceinline__ void set_comp(float4& v, int k, float x) {
    if (k == 0) v.x = x; else if (k == 1) v.y = x; else if (k == 2) v.z = x; else v.w = x;
}

// Global-address-space view of a pointer held in a table: loads and stores through it are
// global (vector-memory only) rather than flat accesses, which would also count against
// the LDS wait counter.
template <class T>
using GlobalPtr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ GlobalPtr<T> gbl(T* p) {
    return (GlobalPtr<T>)p;
}
// HIP's vector structs do not bind to address-space-qualified references: move them as
// clang vectors.
using f4v = float __attribute__((ext_vector_type(4)));
using i2v = int __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 gload(GlobalPtr<const float4> p) {
    const f4v v = *(GlobalPtr<const f4v>)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int2 gload(GlobalPtr<const int2> p) {
    const i2v v = *(GlobalPtr<const i2v>)p;
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ void gstore(GlobalPtr<float4> p, float4 v) {
    *(GlobalPtr<f4v>)p = f4v{v.x, v.y, v.z, v.w};
}

// One tile row segment of CPL floats per lane: row gy, columns gx0 .. gx0 + CPL - 1 of the
// field, read at indices clamped into the grid, so every lane loads and nothing branches
// between the loads of a batch; cells outside the grid are zeroed when the segment is
// stored (store_row).  With ALIGNED (the segment starts at a multiple of CPL and the row
// length is one) the segment lies wholly inside or wholly outside the grid's columns and is
// one naturally aligned vector load.
template <int CPL>
using RowVec = float __attribute__((ext_vector_type(CPL)));

template <int CPL, bool ALIGNED>
__device__ __forceinline__ RowVec<CPL> load_row(GlobalPtr<const float> f, int nx, int ny,
                                                int gy, int gx0) {
    const size_t at = (size_t)min(max(gy, 0), ny - 1) * nx;
    if (ALIGNED) return *(GlobalPtr<const RowVec<CPL>>)(f + at + min(max(gx0, 0), nx - CPL));
    RowVec<CPL> v;
#pragma unroll
    for (int k = 0; k < CPL; ++k) v[k] = f[at + min(max(gx0 + k, 0), nx - 1)];
    return v;
}

// Load a tile plane (HL rows from grid row y0) into LDS rows 0 .. HL-1 at `dst`, the rows
// strided over the wavefronts, kLoadBatch rows in flight per wavefront: the batch's loads
// are all issued before the first is used.  A batch running past the tile re-reads its last
// row and parks the copy in guard row HL, which is never meaningful.  Cells outside the grid
// read as zero; cells inside never use them (they take their own value for out-of-grid
// neighbours).
template <int CPL, bool ALIGNED>
__device__ __forceinline__ void load_tile(float* dst, GlobalPtr<const float> f, int nx, int ny,
                                          int y0, int HL, int gx0, int cx, int wave,
                                          const bool (&col_in)[CPL]) {
    using V = typename Row<CPL>::T;
    constexpr int W = 64 * CPL;
    for (int ly0 = wave; ly0 < HL; ly0 += kLoadBatch * kWaves) {
        RowVec<CPL> v[kLoadBatch];
#pragma unroll
        for (int r = 0; r < kLoadBatch; ++r)
            v[r] = load_row<CPL, ALIGNED>(f, nx, ny, y0 + min(ly0 + r * kWaves, HL - 1), gx0);
#pragma unroll
        for (int r = 0; r < kLoadBatch; ++r) {
            const int ly = min(ly0 + r * kWaves, HL);
            const bool row_in = (unsigned)(y0 + ly) < (unsigned)ny;
            V out;
#pragma unroll
            for (int k = 0; k < CPL; ++k) set_comp(out, k, row_in && col_in[k] ? v[r][k] : 0.0f);
            *(V*)&dst[ly * W + cx] = out;
        }
    }
}

// LDS view of one species with tile-origin offset; indices are clamped to the tile so a
// sample can never leave the LDS allocation.
struct LdsField2D {
    const float* L;
    int x0, y0, width, height;
    __device__ float operator()(int i, int j) const {
        const int lx = min(max(i - x0, 0), width - 1);
        const int ly = min(max(j - y0, 0), height - 1);
        return L[ly * width + lx];
    }
};

// Value held by the lane below (lane_from_left) or above (lane_from_right) in the
// wavefront: a whole-wave DPP shift by one lane, which moves data between lanes inside the
// VALU instead of through the LDS crossbar.  Lane 0 (resp. 63) receives 0; it holds the
// tile's outermost column, which is never valid after the first sub-step.
__device__ __forceinline__ float lane_from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138 /* wave_shr:1 */,
                                                      0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130 /* wave_shl:1 */,
                                                      0xF, 0xF, false));
}

// How a tile meets the grid's first and last column (the zero-flux rule: a missing
// neighbour is the cell itself).  kWallAligned: every lane's segment starts at a multiple of
// CPL and so does nx, so column 0 can only be a segment's first cell and column nx - 1 a
// segment's last, and only the neighbours taken from the adjacent lanes need the rule.
enum ColumnWalls { kNoWall = 0, kWallAligned = 1, kWallAny = 2 };

// New value of the CPL cells of one row from the old rows above (s), at (c) and below (n).
// Horizontal neighbours across lanes come from the adjacent lanes' registers.  COLS applies
// the zero-flux rule at the grid's first and last column; at the first and last row the
// caller passes the row itself as the missing neighbour.
template <int CPL, int COLS>
__device__ __forceinline__ typename Row<CPL>::T row_update(const typename Row<CPL>::T& s,
                                                           const typename Row<CPL>::T& c,
                                                           const typename Row<CPL>::T& n,
                                                           int gx0, int nx, StencilCoef cf) {
    using V = typename Row<CPL>::T;
    float left = lane_from_left(comp(c, CPL - 1));   // column cx - 1
    float right = lane_from_right(comp(c, 0));       // column cx + CPL
    if (COLS == kWallAligned) {
        if (gx0 == 0) left = comp(c, 0);
        if (gx0 + CPL == nx) right = comp(c, CPL - 1);
    }
    V nv;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const float ck = comp(c, k);
        float w = k == 0 ? left : comp(c, k - 1);
        float e = k == CPL - 1 ? right : comp(c, k + 1);
        if (COLS == kWallAny) {
            if (gx0 + k == 0) w = ck;
            if (gx0 + k == nx - 1) e = ck;
        }
        const float lap = fmaf(-4.0f, ck, (w + e) + (comp(s, k) + comp(n, k)));
        set_comp(nv, k, fmaf(cf.r, lap, fmaf(-cf.kdt, ck, ck)));
    }
    return nv;
}

// One stencil + decay sub-step of one species over a wavefront's strip of rows
// [ybeg, yend), in place.  L points at tile row 0; rows -1 and HL .. HL+2 are guard rows
// (never meaningful) so reads, which reach at most two rows past the strip, need no
// clamping.  Within a wavefront every LDS read of a row is issued before that row's write,
// so interior rows are overwritten as soon as they are computed; the strip's first and
// last rows are read by the neighbouring wavefronts and are returned for writing after a
// barrier.  Four row registers cycle through their roles (above / at / below /
// prefetched), so rows are prefetched two ahead with no register moves: a prefetched row
// is either this strip's, still unmodified, or a neighbour's first row, written only after
// the barrier (or is never used).  The first and last rows are peeled off, so the loop body
// has no branches and the LDS wait counter can let prefetches stay in flight.  A strip
// never reaches outside the grid's rows; `top` (`bottom`) says that its first (last) row is
// the grid's first (last), whose missing neighbour is the row itself.
template <int CPL>
struct StripEdges {
    typename Row<CPL>::T first, last;
};

template <int CPL, int COLS>
__device__ __forceinline__ StripEdges<CPL> strip_update(float* L, int ybeg, int yend, int cx,
                                                        int gx0, int nx, bool top, bool bottom,
                                                        StencilCoef cf) {
    using V = typename Row<CPL>::T;
    constexpr int W = 64 * CPL;
    const float* rd = L + cx;
    float* wr = L + cx;
    auto load = [&](int yy) { return *(const V*)&rd[yy * W]; };
    auto store = [&](int yy, const V& v) { *(V*)&wr[yy * W] = v; };
    auto upd = [&](const V& s, const V& c, const V& n, int) {
        return row_update<CPL, COLS>(s, c, n, gx0, nx, cf);
    };
    StripEdges<CPL> out;
    V A = load(ybeg - 1), Bv = load(ybeg), C = load(ybeg + 1), D = load(ybeg + 2);
    // the strip's first row (returned, written after the barrier)
    if (yend - ybeg == 1) {
        out.first = upd(top ? Bv : A, Bv, bottom ? Bv : C, ybeg);
        out.last = out.first;
        return out;
    }
    out.first = upd(top ? Bv : A, Bv, C, ybeg);
    A = load(ybeg + 3);
    // interior rows [ybeg + 1, yend - 1), written in place: a branch-free body of four rows,
    // the registers (Bv, C, D, A) holding rows y - 1 .. y + 2 at its top
    int y = ybeg + 1;
    const int yin = yend - 1;
    for (; y + 4 <= yin; y += 4) {
        V nv = upd(Bv, C, D, y);
        Bv = load(y + 3);
        store(y, nv);
        nv = upd(C, D, A, y + 1);
        C = load(y + 4);
        store(y + 1, nv);
        nv = upd(D, A, Bv, y + 2);
        D = load(y + 5);
        store(y + 2, nv);
        nv = upd(A, Bv, C, y + 3);
        A = load(y + 6);
        store(y + 3, nv);
    }
    // 0..3 remaining interior rows, then the last row (returned)
    const int r = yin - y;
    if (r == 0) {
        out.last = upd(Bv, C, bottom ? C : D, y);
    } else if (r == 1) {
        store(y, upd(Bv, C, D, y));
        out.last = upd(C, D, bottom ? D : A, y + 1);
    } else if (r == 2) {
        const V v0 = upd(Bv, C, D, y);
        Bv = load(y + 3);
        store(y, v0);
        store(y + 1, upd(C, D, A, y + 1));
        out.last = upd(D, A, bottom ? A : Bv, y + 2);
    } else {
        const V v0 = upd(Bv, C, D, y);
        Bv = load(y + 3);
        store(y, v0);
        const V v1 = upd(C, D, A, y + 1);
        C = load(y + 4);
        store(y + 1, v1);
        store(y + 2, upd(D, A, Bv, y + 2));
        out.last = upd(A, Bv, bottom ? Bv : C, y + 3);
    }
    return out;
}

// Contact test against the targets staged for this tile (a superset of every target within
// the contact radius of any tip the tile's cones can reach in this launch), or against the
// whole grid when the tile's list did not fit in LDS.
struct TileContact {
    const float4* pts;
    int n;
    bool staged;
    const TargetGrid* grid;
    template <int dim>
    __device__ int find(float x, float y, float z) const {
        return staged ? contact_in_list<dim>(pts, n, grid->r2, x, y, z)
                      : contact_target<dim>(*grid, x, y, z);
    }
};

// The gradient footprint of a tip read from the LDS tile.  Its 12 cells lie between one
// cell before and two after the corner cell (i0, j0) along each axis, so one base address
// and constant offsets reach them all; at a grid wall the outer cell is the wall cell itself
// (the zero-flux ghost), substituted afterwards.  The base is clamped so that every read
// stays inside the tile: a tip bucketed to the tile never needs the clamp (the halo covers
// its footprint), and with it no tip can read outside the tile.  The values are those the
// per-cell accessor (LdsField2D) returns.
__device__ __forceinline__ Footprint2D footprint_lds(const LdsField2D& f, const ConeRules& r,
                                                    float x, float y) {
    Footprint2D p;
    corner(x, r.inv_dx, r.nx, p.i0, p.fx);
    corner(y, r.inv_dx, r.ny, p.j0, p.fy);
    p.im = max(p.i0 - 1, 0);
    p.ip = min(p.i0 + 2, r.nx - 1);
    p.jm = max(p.j0 - 1, 0);
    p.jp = min(p.j0 + 2, r.ny - 1);
    const int W = f.width;
    const int lx = min(max(p.i0 - f.x0, 1), W - 3);
    const int ly = min(max(p.j0 - f.y0, 1), f.height - 3);
    const float* b = f.L + ly * W + lx;
    p.a0 = b[-1];
    p.a1 = b[0];
    p.a2 = b[1];
    p.a3 = b[2];
    p.b0 = b[W - 1];
    p.b1 = b[W];
    p.b2 = b[W + 1];
    p.b3 = b[W + 2];
    p.c0 = b[-W];
    p.c1 = b[1 - W];
    p.d0 = b[2 * W];
    p.d1 = b[2 * W + 1];
    if (p.im == p.i0) {   // left wall
        p.a0 = p.a1;
        p.b0 = p.b1;
    }
    if (p.ip == p.i0 + 1) {   // right wall
        p.a3 = p.a2;
        p.b3 = p.b2;
    }
    if (p.jm == p.j0) {   // bottom wall
        p.c0 = p.a1;
        p.c1 = p.a2;
    }
    if (p.jp == p.j0 + 1) {   // top wall
        p.d0 = p.b1;
        p.d1 = p.b2;
    }
    return p;
}

// The cone step in two parts.  The first samples the signed gradient g at the tip from the
// LDS field (the only part that reads the field); the second turns, adds noise, advances
// and tests exit and contact using g and registers only, so it may run while the next
// sub-step already overwrites the field.
// The sample is (g_x, g_y, concentration of species 0; the last only under the SNR law).
template <int NS>
__device__ __forceinline__ float3 tile_cone_gradient(const float4& st, const LdsField2D& f0,
                                                     const LdsField2D& f1,
                                                     const ConeRules& rules) {
    float gxv = 0.0f, gyv = 0.0f, conc = 0.0f;
    if (__float_as_int(st.w) < 0) return make_float3(gxv, gyv, conc);
    const Footprint2D p0 = footprint_lds(f0, rules, st.x, st.y);
    gradient_from_2d(p0, corner_gradients_2d(p0, rules), gxv, gyv,
                     rules.turn_law == 1 ? &conc : nullptr);
    gxv *= rules.sign0;
    gyv *= rules.sign0;
    if (NS > 1) {
        float hx, hy;
        const Footprint2D p1 = footprint_lds(f1, rules, st.x, st.y);
        gradient_from_2d(p1, corner_gradients_2d(p1, rules), hx, hy, nullptr);
        gxv = fmaf(rules.sign1, hx, gxv);
        gyv = fmaf(rules.sign1, hy, gyv);
    }
    return make_float3(gxv, gyv, conc);
}

// Second part; a stopped cone has its final state written to the caller-order arrays and
// the sign bit of its id set.  One Philox block serves an even step and the next odd one:
// the odd step's two words wait in `spare` (`fresh`: no even step of this launch has
// filled them yet).
__device__ __forceinline__ void tile_cone_advance(float4& st, float2& sc, uint2& spare,
                                                  float3 g, const ConeRules& rules,
                                                  uint32_t step, bool fresh,
                                                  const TileContact& contact,
                                                  const ConeArrays& cones) {
    int id = __float_as_int(st.w);
    if (id < 0) return;
    float z[2];
    if ((step & 1u) == 0u || fresh) {
        const uint4 blk = noise_block_2d(rules.key, (uint32_t)id, step);
        if (step & 1u) {
            normal_pair(blk.z, blk.w, z);
        } else {
            normal_pair(blk.x, blk.y, z);
            spare = make_uint2(blk.z, blk.w);
        }
    } else {
        normal_pair(spare.x, spare.y, z);
    }
    float x = st.x, y = st.y, th = st.z;
    const ConeEvent ev =
        cone_step_2d(rules, g.x, g.y, g.z, z, x, y, th, sc.x, sc.y, contact);
    if (ev.status != kActive) {
        cones.pos[2 * id] = x;
        cones.pos[2 * id + 1] = y;
        cones.dir[id] = th;
        cones.status[id] = ev.status;
        cones.target[id] = ev.target;
        cones.event_step[id] = (int32_t)(step + 1);
        id = (int)((unsigned)id | 0x80000000u);
    }
    st = make_float4(x, y, th, __int_as_float(id));
}

// Cell of a coordinate, clamped to the grid (as a float first: a NaN tip maps to cell 0).
__device__ __forceinline__ int cell_of(float p, float inv_dx, int n) {
    return (int)fminf(fmaxf(floorf(p * inv_dx), 0.0f), (float)(n - 1));
}

// Destination tile of a cone's tip after a launch, restricted to the 3x3 neighbourhood of
// the tile it was stepped in (the halo guarantees it never moves further).
__device__ __forceinline__ int2 next_tile(const float4& st, int tx, int ty, int tiles_x,
                                          int tiles_y, float inv_dx, int nx, int ny,
                                          int tx_core, int ty_core) {
    int ntx = cell_of(st.x, inv_dx, nx) / tx_core;
    int nty = cell_of(st.y, inv_dx, ny) / ty_core;
    ntx = min(max(ntx, max(tx - 1, 0)), min(tx + 1, tiles_x - 1));
    nty = min(max(nty, max(ty - 1, 0)), min(ty + 1, tiles_y - 1));
    return make_int2(ntx, nty);
}

// The core of a tile from LDS to the fields dst[s] (row-major, the grid's row length),
// through global-address-space stores.  The tile's rows are strided over the wavefronts.
// STREAM: non-temporal stores, for the run tape, which is read only by a later reverse sweep
// (the recording forward run of a 1024^2 gradient: 8.1 against 8.4 ms).
template <int NS, int CPL, bool STREAM = false>
__device__ __forceinline__ void store_core(float* const dst[], const TiledArgs2D& a, int tx,
                                           int ty, int plane, int cx, int wave, bool aligned) {
    using V = typename Row<CPL>::T;
    constexpr int W = 64 * CPL;
    extern __shared__ __align__(16) float lds[];
    const int H = a.halo;
    const int cx0 = tx * a.tx_core, cy0 = ty * a.ty_core;
    for (int ly = wave; ly < a.ty_core; ly += kWaves) {
        const int gy = cy0 + ly;
        if (gy >= a.ny) break;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const V v = *(const V*)&lds[s * plane + (ly + H + 1) * W + cx];
            const GlobalPtr<float> row = gbl(dst[s]) + (size_t)gy * a.nx + cx0;
            if (aligned) {
                const int lx = cx - H;   // the segment is wholly inside or outside the core
                if (lx >= 0 && lx < a.tx_core && cx0 + lx < a.nx) {
                    RowVec<CPL> x;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) x[k] = comp(v, k);
                    if (STREAM)
                        __builtin_nontemporal_store(x, (GlobalPtr<RowVec<CPL>>)(row + lx));
                    else
                        *(GlobalPtr<RowVec<CPL>>)(row + lx) = x;
                }
                continue;
            }
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                const int lx = cx + k - H;   // core column of this lane's k-th cell
                if (lx >= 0 && lx < a.tx_core && cx0 + lx < a.nx) {
                    if (STREAM)
                        __builtin_nontemporal_store(comp(v, k), row + lx);
                    else
                        row[lx] = comp(v, k);
                }
            }
        }
    }
}

// Parts of a tile holding c cones when a part takes at most p of them (at least one part
// per tile).  The tile's cones are shared evenly among its parts (build_items).
__device__ __forceinline__ int tile_parts(int c, int p) { return max(1, (c + p - 1) / p); }

// One work item: one part of one tile of one simulation for `steps` sub-steps.  Every part
// of a tile computes the tile's field; each part steps its share of the tile's cones,
// [first_cone, first_cone + n_cones) with n_cones <= kPartCones, and only the part holding
// the first cone writes the field back, so a tile crowded with cones is spread over several
// workgroups.  par selects the input half of
// every ping-pong pair (fields and cone buckets); the other half is written.
template <int NS, int CPL, bool RECORD>
__device__ __forceinline__ void tile_body(const TiledArgs2D& a, int tile, int first_cone,
                                          int n_cones, int steps, uint32_t first_step,
                                          int par) {
    using V = typename Row<CPL>::T;
    constexpr int W = 64 * CPL;
    extern __shared__ __align__(16) float lds[];
    __shared__ int dest_count[9];
    __shared__ int dest_base[9];
    __shared__ int dest_fill[9];
    __shared__ float4 tile_targets[kMaxTileTargets];
    const float* in[SIM_MAX_SPECIES] = {a.field[0][par], a.field[NS > 1 ? 1 : 0][par]};
    float* out[SIM_MAX_SPECIES] = {a.field[0][par ^ 1], a.field[NS > 1 ? 1 : 0][par ^ 1]};
    float4* const bucket_in = a.bucket[par];
    float4* const bucket_out = a.bucket[par ^ 1];
    int32_t* const count_out = a.count[par ^ 1];

    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int tiles_y = a.n_tiles / a.tiles_x;
    const int HL = a.height, H = a.halo;
    const int x0 = tx * a.tx_core - H, y0 = ty * a.ty_core - H;
    // species plane: guard row, HL tile rows, three guard rows; row 0 at offset W
    const int plane = W * (HL + kGuardRows);
    // the wavefront index is uniform across a wavefront: keep it (and the strip bounds
    // derived from it) in scalar registers so strip bookkeeping is scalar work
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cx = CPL * lane;
    const int gx0 = x0 + cx;

    // 0. this part's cones and the tile's targets, fetched first so that their latency
    //    overlaps the tile load.  Every cone of the part stays in registers for the whole
    //    launch: cone i sits in thread i % kThreads, slot i / kThreads (a part holds at
    //    most kPartCones = kConeSlots * kThreads cones).
    const bool first_part = first_cone == 0;
    const GlobalPtr<const float4> live = gbl(bucket_in) + (size_t)tile * a.capacity + first_cone;
    const int t_lo = gbl(a.tgt_start)[tile], n_tt = gbl(a.tgt_start)[tile + 1] - t_lo;
    const TileContact contact{tile_targets, n_tt, n_tt <= kMaxTileTargets, &a.rules.targets};
    if (contact.staged)
        for (int k = threadIdx.x; k < n_tt; k += kThreads)
            tile_targets[k] = gload(gbl(a.tgt_pts) + t_lo + k);
    float4 mine[kConeSlots];
#pragma unroll
    for (int k = 0; k < kConeSlots; ++k) {
        const int i = threadIdx.x + k * kThreads;
        mine[k] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
        if (i < n_cones) mine[k] = gload(live + i);
    }

    // 1. load the tile, kLoadBatch rows in flight per wavefront; cells outside the grid
    //    read as zero and are never used by cells inside it, which take their own value
    //    for out-of-grid neighbours
    bool col_in[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) col_in[k] = (unsigned)(gx0 + k) < (unsigned)a.nx;
    // whole-segment vector loads and stores when segments cannot straddle the grid edge
    const bool aligned = (x0 % CPL) == 0 && (a.nx % CPL) == 0 && (a.tx_core % CPL) == 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const GlobalPtr<const float> f = gbl((const float*)in[s]);
        float* const dst = lds + s * plane + W;
        if (aligned)
            load_tile<CPL, true>(dst, f, a.nx, a.ny, y0, HL, gx0, cx, wave, col_in);
        else
            load_tile<CPL, false>(dst, f, a.nx, a.ny, y0, HL, gx0, cx, wave, col_in);
    }
    // sin and cos of every heading, carried alongside the cone from sub-step to sub-step, and
    // the second half of the current Philox block
    float2 trig[kConeSlots];
    uint2 spare[kConeSlots];
#pragma unroll
    for (int k = 0; k < kConeSlots; ++k) {
        trig[k] = make_float2(0.0f, 1.0f);
        spare[k] = make_uint2(0u, 0u);
        if (threadIdx.x + k * kThreads < n_cones) sincos_angle(mine[k].z, trig[k].x, trig[k].y);
    }
    if (threadIdx.x < 9) {
        dest_count[threadIdx.x] = 0;
        dest_fill[threadIdx.x] = 0;
    }
    __syncthreads();

    // Strips of the tile's rows inside the grid, [r0, r1), per wavefront, balanced against
    // the cone work: a wavefront stepping cones in k register slots gives up
    // k * cone_rows rows to the others, so that every wavefront does about the same work
    // between two barriers.  Boundaries are computed for every wavefront in scalar registers
    // and kept monotone.  Rows outside the grid are never computed: no cell inside the grid
    // reads them (at the grid's first and last row the missing neighbour is the row itself).
    const int r0 = max(0, -y0), r1 = min(HL, a.ny - y0);
    int ybeg = 0, yend = 0;
    {
        int cw[kConeSlots];   // wavefronts holding a cone in slot k
        int slots = 0;
#pragma unroll
        for (int k = 0; k < kConeSlots; ++k) {
            cw[k] = min(kWaves, (max(n_cones - k * kThreads, 0) + 63) / 64);
            slots += cw[k];
        }
        const float per = (float)(r1 - r0 + a.cone_rows * slots) / kWaves;
        int prev = r0;
        for (int w = 1; w <= kWaves; ++w) {
            int used = 0;
#pragma unroll
            for (int k = 0; k < kConeSlots; ++k) used += a.cone_rows * min(w, cw[k]);
            const int b = w == kWaves ? r1 : min(max(r0 + (int)rintf(w * per) - used, prev), r1);
            if (w == wave) ybeg = b;       // wavefront w's strip is [b(w), b(w + 1))
            if (w == wave + 1) yend = b;
            prev = b;
        }
        if (wave == 0) ybeg = r0;
    }
    const int src_lo = gbl(a.src_start)[tile], src_hi = gbl(a.src_start)[tile + 1];
    // the tile's first 64 source entries, one per lane, kept in registers for every sub-step
    const int n_src = src_hi - src_lo;
    int src_cell = -1, src_plane = 0;
    float src_q = 0.0f;
    if (lane < n_src) {
        const int2 ent = gload(gbl(a.src_entry) + src_lo + lane);
        src_cell = ent.x;
        src_plane = ent.y * plane;
        src_q = gbl(a.src_amount)[src_lo + lane];
    }
    const ConeRules& rules = a.rules;
    const int cols = x0 > 0 && x0 + W < a.nx ? kNoWall : aligned ? kWallAligned : kWallAny;
    const LdsField2D f0{lds + W, x0, y0, W, HL};
    const LdsField2D f1{lds + (NS > 1 ? plane : 0) + W, x0, y0, W, HL};

    for (int b = 0; b < steps; ++b) {
        // 2. stencil + decay, in place, strip per wavefront.  After this sub-step only rows
        //    [b + 1, HL - b - 1) are still valid (each sub-step loses one row at either
        //    edge of the tile), so rows outside that band are not computed.
        const int lo = max(ybeg, b + 1), hi = min(yend, HL - b - 1);
        const bool top = lo == -y0, bottom = hi == a.ny - y0;
        StripEdges<CPL> edge[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (lo < hi) {
                float* const L = lds + s * plane + W;
                if (cols == kNoWall)
                    edge[s] = strip_update<CPL, kNoWall>(L, lo, hi, cx, gx0, a.nx, top, bottom,
                                                         a.coef[s]);
                else if (cols == kWallAligned)
                    edge[s] = strip_update<CPL, kWallAligned>(L, lo, hi, cx, gx0, a.nx, top,
                                                              bottom, a.coef[s]);
                else
                    edge[s] = strip_update<CPL, kWallAny>(L, lo, hi, cx, gx0, a.nx, top, bottom,
                                                          a.coef[s]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (lo < hi) *(V*)&lds[s * plane + (lo + 1) * W + cx] = edge[s].first;
            if (hi - 1 > lo) *(V*)&lds[s * plane + hi * W + cx] = edge[s].last;
        }
        // 3. sources in this wavefront's rows [lo, hi) (entries are unique cells per
        //    species; rows no wavefront computes are not valid after this sub-step), added
        //    after its own edge rows: a wavefront's LDS operations take effect in order, and
        //    the barrier below publishes them with the rest of the sub-step
        if (n_src > 0 && lo < hi) {
            if (src_cell >= 0 && src_cell / W >= lo && src_cell / W < hi)
                lds[src_plane + W + src_cell] += src_q;
            for (int e = src_lo + 64 + lane; e < src_hi; e += 64) {
                const int2 ent = gload(gbl(a.src_entry) + e);
                const int row = ent.x / W;
                if (row >= lo && row < hi) lds[ent.y * plane + W + ent.x] += gbl(a.src_amount)[e];
            }
        }
        __syncthreads();
        // recording a run: the state after this sub-step goes to the tape (read from LDS
        // before the next sub-step's in-place update, hence the barrier)
        if (RECORD && first_part) {
            const size_t cells = (size_t)a.nx * a.ny;
            const size_t at = (size_t)(first_step + (uint32_t)b + 1u - a.record_n0) * NS;
            float* tape[SIM_MAX_SPECIES] = {a.record + at * cells,
                                            a.record + (at + (NS - 1)) * cells};
            store_core<NS, CPL, true>(tape, a, tx, ty, plane, cx, wave, aligned);
            __syncthreads();
        }
        // 4. cones against the updated field.  Every read of the field (the gradients)
        //    happens before the barrier; the cones then finish their step after it,
        //    overlapping the next sub-step's in-place stencil, which they no longer read.
        const uint32_t step = first_step + (uint32_t)b;
        if (n_cones > 0) {
            float3 g[kConeSlots];
#pragma unroll
            for (int k = 0; k < kConeSlots; ++k) g[k] = tile_cone_gradient<NS>(mine[k], f0, f1, rules);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kConeSlots; ++k)
                tile_cone_advance(mine[k], trig[k], spare[k], g[k], rules, step, b == 0,
                                  contact, a.cones);
        }
    }

    // 5. write the core back (one part per tile does)
    if (first_part) store_core<NS, CPL>(out, a, tx, ty, plane, cx, wave, aligned);

    // 6. re-bucket surviving cones, straight from registers, into the tile that now holds
    //    their tip (one of the 3 x 3 tiles around this one)
    int dest[kConeSlots];
#pragma unroll
    for (int k = 0; k < kConeSlots; ++k) {
        dest[k] = -1;
        if (threadIdx.x + k * kThreads < n_cones && __float_as_int(mine[k].w) >= 0) {
            const int2 nt = next_tile(mine[k], tx, ty, a.tiles_x, tiles_y, rules.inv_dx, a.nx,
                                      a.ny, a.tx_core, a.ty_core);
            dest[k] = (nt.y - ty + 1) * 3 + (nt.x - tx + 1);
            atomicAdd(&dest_count[dest[k]], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < 9 && dest_count[threadIdx.x] > 0) {
        const int dtx = tx + threadIdx.x % 3 - 1, dty = ty + threadIdx.x / 3 - 1;
        dest_base[threadIdx.x] = atomicAdd(&count_out[dty * a.tiles_x + dtx],
                                           dest_count[threadIdx.x]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kConeSlots; ++k) {
        const int d = dest[k];
        if (d < 0) continue;
        const int ntx = tx + d % 3 - 1, nty = ty + d / 3 - 1;
        const int slot = dest_base[d] + atomicAdd(&dest_fill[d], 1);
        gstore(gbl(bucket_out) + (size_t)(nty * a.tiles_x + ntx) * a.capacity + slot, mine[k]);
    }
}

// Candidate part sizes of a list laid out by die, largest first.  Only tiles of more than
// the smallest candidate's cones can need more than one part under any of them.
constexpr int kCand = 5;
__device__ __forceinline__ int candidate_size(int j) {
    return j == 0 ? kPartCones : j == 1 ? 384 : j == 2 ? 320 : j == 3 ? 256 : 192;
}
static_assert(kPartCones == 512, "candidate part sizes assume 512-cone parts");

// Parts of a tile of c cones under candidate j (constant divisors: no integer division).
__device__ __forceinline__ int candidate_parts(int c, int j) {
    switch (j) {
        case 1: return tile_parts(c, 384);
        case 2: return tile_parts(c, 320);
        case 3: return tile_parts(c, 256);
        case 4: return tile_parts(c, 192);
        default: return tile_parts(c, kPartCones);
    }
}

// Expand the base items (simulation, tile) into work items (simulation, tile, first cone,
// cones), one per part of a tile, from the tile counts of input half par_in; optionally zero
// the counts of half par_zero for reuse as the next output.  Run by one whole workgroup.
//
// BY_DIE (a launch of one workgroup per item): the part size is the smallest candidate whose
// list still fits ls->slots (the workgroups resident at once), so that the spare slots carry
// the crowded tiles' cones in more, smaller parts and every item still starts at once.  The
// extra parts of each candidate are counted in `extra` (kCand ints of LDS that the caller
// has zeroed before a barrier) by the few threads whose tile is crowded.  The list is laid
// out so that each die gets a contiguous run of the n items, in tile order -- neighbouring
// tiles, whose overlapping halo rows and columns the die's L2 then fetches once: item q goes
// to slot (q % per) * kXcds + q / per with per = ceil(n / kXcds), so that workgroup b (on die
// b % kXcds) takes item (b % kXcds) * per + b / kXcds; slots without an item hold
// simulation -1, and ls->n_items is the number of slots, kXcds * per.  Such a list serves one
// simulation whose base items are (0, k), so the count arrays are read from table[0] once
// rather than through base[] and the table for every tile.  Otherwise (a persistent launch,
// whose queue balances itself) parts take up to kPartCones cones.
template <bool BY_DIE>
__device__ void build_items(const TiledArgs2D* __restrict__ table, const int2* __restrict__ base,
                            int n_base, int par_in, int par_zero, bool zero, int4* items,
                            int item_cap, LaunchState* ls, int* extra) {
    __shared__ int wave_total[kWaves];
    const int slots = BY_DIE ? ls->slots : 0;   // issued early, beside the count loads
    const int per = (n_base + kThreads - 1) / kThreads;
    const int lo = min((int)threadIdx.x * per, n_base), hi = min(lo + per, n_base);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t* const counts_in = BY_DIE ? table[0].count[par_in] : nullptr;
    int32_t* const counts_zero = BY_DIE ? table[0].count[par_zero] : nullptr;
    auto count_of = [&](int k) {
        int32_t* const c = BY_DIE ? counts_in + k : &table[base[k].x].count[par_in][base[k].y];
        return __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    const int c_lo = lo < hi ? count_of(lo) : 0;   // the first count is kept in a register
    auto count_at = [&](int k) { return k == lo ? c_lo : count_of(k); };

    int chosen = 0;   // candidate part size in use
    if (BY_DIE) {
        for (int k = lo; k < hi; ++k) {
            const int c = count_at(k);
            if (c > candidate_size(kCand - 1)) {
#pragma unroll
                for (int j = 1; j < kCand; ++j) {
                    const int e = candidate_parts(c, j) - 1;
                    if (e > 0) atomicAdd(&extra[j], e);
                }
            }
        }
        __syncthreads();
        const int room = slots - n_base;
#pragma unroll
        for (int j = 1; j < kCand; ++j)   // the counts grow with j: keep the last that fits
            if (extra[j] <= room) chosen = j;
    }
    int mine = 0;
    for (int k = lo; k < hi; ++k) mine += candidate_parts(count_at(k), chosen);
    // exclusive scan of `mine` over the workgroup: within each wavefront by lane shuffles,
    // then across the wavefronts' totals
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wave_total[wave] = incl;
    __syncthreads();
    int at = incl - mine, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = wave_total[w];
        at += w < wave ? t : 0;
        total += t;
    }
    // (item_cap includes kXcds slots that a list laid out by die may leave empty; a list of
    // parts of up to kPartCones cones always fits, and a smaller size is only chosen when its
    // list fits ls->slots, which the host keeps within the same bound)
    const int n = min(total, BY_DIE ? item_cap - kXcds : item_cap);
    const int per_die = (n + kXcds - 1) / kXcds;
    // item `at` goes to slot r * kXcds + d with (d, r) = (at / per_die, at % per_die) when laid
    // out by die, stepped along without dividing again
    int d = BY_DIE ? at / max(per_die, 1) : 0, r = BY_DIE ? at - d * per_die : 0;
    for (int k = lo; k < hi; ++k) {
        const int c = count_at(k);
        const int parts = candidate_parts(c, chosen);
        // the tile's cones shared evenly: the first c % parts parts take one more
        const int each = parts == 1 ? c : c / parts, more = c - each * parts;
        int first = 0;
        const int2 bk = BY_DIE ? make_int2(0, k) : base[k];
        for (int q = 0; q < parts; ++q, ++at) {
            const int m = each + (q < more ? 1 : 0);
            if (at < n) items[BY_DIE ? r * kXcds + d : at] = make_int4(bk.x, bk.y, first, m);
            first += m;
            if (BY_DIE && ++r == per_die) {
                r = 0;
                ++d;
            }
        }
        if (zero) {
            if (BY_DIE)
                counts_zero[k] = 0;
            else
                table[bk.x].count[par_zero][bk.y] = 0;
        }
    }
    if (BY_DIE)   // the slots that hold no item (at most kXcds - 1, below kXcds * per)
        for (int b = threadIdx.x; b < kXcds * per_die; b += kThreads)
            if ((b % kXcds) * per_die + b / kXcds >= n) items[b] = make_int4(-1, 0, 0, 0);
    if (threadIdx.x == 0) ls->n_items = BY_DIE ? kXcds * per_die : n;
}

// The step kernel.  Work items (simulation, tile, first cone, cones) come from the list the
// previous launch (or k_build_items) wrote: one workgroup per slot of a list laid out by
// die, or, in persistent mode, a fixed grid pulling items from an atomic queue until it
// runs dry.  The launch state (step counter, ping-pong parity) is read by
// every workgroup at its start and advanced by the last workgroup to finish, so launches
// need no host-side bookkeeping and can be captured in a graph and replayed.
template <int NS, int CPL, bool RECORD>
__global__ __launch_bounds__(kThreads) void k_tiled2d(const TiledArgs2D* __restrict__ table,
                                                      int4* items, const int2* __restrict__ base,
                                                      int n_base, int item_cap, int steps,
                                                      LaunchState* ls, int persistent) {
    __shared__ int item_idx;
    __shared__ int last_out;
    __shared__ int extra_parts[kCand];
    const uint32_t first_step = ls->step;
    const int par = ls->parity;
    const int n_items = ls->n_items;
    if (!persistent) {
        // the item list has one slot per workgroup of the grid, laid out by die
        // (build_items): fetch it alongside the launch state (a slot past n_items, or one
        // holding simulation -1, is not used)
        const int4 it = items[blockIdx.x];
        if ((int)blockIdx.x < n_items && it.x >= 0)
            tile_body<NS, CPL, RECORD>(table[it.x], it.y, it.z, it.w, steps, first_step, par);
    } else {
        // the next item is taken from the queue while the current one runs, so the queue's
        // round trip is hidden behind the item's work
        if (threadIdx.x == 0) item_idx = atomicAdd(&ls->next, 1);
        __syncthreads();
        int i = item_idx;
        while (i < n_items) {
            int next = 0;
            if (threadIdx.x == 0) next = atomicAdd(&ls->next, 1);
            const int4 it = items[i];
            tile_body<NS, CPL, RECORD>(table[it.x], it.y, it.z, it.w, steps, first_step, par);
            // every thread read item_idx before tile_body's first barrier
            if (threadIdx.x == 0) item_idx = next;
            __syncthreads();   // the item is done with LDS; item_idx holds the next index
            i = item_idx;
        }
    }
    // The last workgroup to finish lists the next launch's work items from the final tile
    // counts, zeroes this launch's input counts and advances the launch state.  The only
    // data it reads that other workgroups wrote during the launch are those counts, which
    // are changed by read-modify-write atomics only (performed at the device's coherence
    // point, all of a workgroup's complete before it counts itself out: their results were
    // used before the barrier) and read back with agent-scope atomic loads.  So no fence is
    // needed -- an agent-scope fence would write back and invalidate the whole L2 of the
    // chiplet once per workgroup.  Everything else it writes is read by the next launch,
    // after the kernel boundary.
    if (threadIdx.x < kCand) extra_parts[threadIdx.x] = 0;   // for build_items
    __syncthreads();
    if (threadIdx.x == 0)
        last_out = __hip_atomic_fetch_add(&ls->exited, 1, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) == (int)gridDim.x - 1;
    __syncthreads();
    if (last_out) {
        if (persistent)
            build_items<false>(table, base, n_base, par ^ 1, par, true, items, item_cap, ls,
                               extra_parts);
        else
            build_items<true>(table, base, n_base, par ^ 1, par, true, items, item_cap, ls,
                              extra_parts);
        if (threadIdx.x == 0) {
            ls->exited = 0;
            ls->next = 0;
            ls->step = first_step + (uint32_t)steps;
            ls->parity = par ^ 1;
        }
    }
}

// Work items for the current cone counts (after cones were put into the buckets).
__global__ __launch_bounds__(kThreads) void k_build_items(const TiledArgs2D* __restrict__ table,
                                                          int4* items,
                                                          const int2* __restrict__ base,
                                                          int n_base, int item_cap,
                                                          LaunchState* ls, int by_die) {
    __shared__ int extra_parts[kCand];
    if (threadIdx.x < kCand) extra_parts[threadIdx.x] = 0;
    __syncthreads();
    if (by_die)
        build_items<true>(table, base, n_base, ls->parity, 0, false, items, item_cap, ls,
                          extra_parts);
    else
        build_items<false>(table, base, n_base, ls->parity, 0, false, items, item_cap, ls,
                           extra_parts);
}

// Initial bucketing from the caller-order arrays (active cones only).
__global__ void k_bucket2d(ConeArrays c, int nx, int ny, int tx_core, int ty_core, int tiles_x,
                           float inv_dx, float4* bucket, int32_t* count, int capacity) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n || c.status[i] != kActive) return;
    const float x = c.pos[2 * i], y = c.pos[2 * i + 1];
    const int t = cell_of(y, inv_dx, ny) / ty_core * tiles_x + cell_of(x, inv_dx, nx) / tx_core;
    const int slot = atomicAdd(&count[t], 1);
    bucket[(size_t)t * capacity + slot] = make_float4(x, y, c.dir[i], __int_as_float(i));
}

// Active cones from the buckets back into the caller-order arrays.
__global__ void k_unbucket2d(ConeArrays c, const float4* bucket, const int32_t* count,
                             int capacity) {
    const int t = blockIdx.x;
    const int n = count[t];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const float4 st = bucket[(size_t)t * capacity + k];
        const int id = __float_as_int(st.w);
        if (id < 0) continue;
        c.pos[2 * id] = st.x;
        c.pos[2 * id + 1] = st.y;
        c.dir[id] = st.z;
    }
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// The kernel variant for a species count and row width; `record` selects the one that also
// writes every sub-step's state to the run tape (only a recording run launches it).
const void* kernel_for(int n_species, int cpl, bool record = false) {
    if (record) {
        if (n_species == 1)
            return cpl == 4 ? (const void*)k_tiled2d<1, 4, true> : (const void*)k_tiled2d<1, 2, true>;
        return cpl == 4 ? (const void*)k_tiled2d<2, 4, true> : (const void*)k_tiled2d<2, 2, true>;
    }
    if (n_species == 1)
        return cpl == 4 ? (const void*)k_tiled2d<1, 4, false> : (const void*)k_tiled2d<1, 2, false>;
    return cpl == 4 ? (const void*)k_tiled2d<2, 4, false> : (const void*)k_tiled2d<2, 2, false>;
}

}  // namespace

namespace {

// Best tile plan by the cost model, restricted to row width 64 * only_cpl and loaded height
// only_height when those are non-zero.
TiledPlan plan_search(int dim, int nx, int ny, int nz, int n_species, double step_cells,
                      int block_steps, int n_cones, int only_cpl, int only_height) {
    TiledPlan best;
    best.dim = dim;
    best.nx = nx;
    best.ny = ny;
    best.nz = nz;
    best.n_species = n_species;
    best.block_steps = 1;
    if (dim != 2 || block_steps < 2) return best;
    double best_cost = 1e300;
    for (int B = block_steps; B >= 2; --B) {
        // halo: B sub-steps of shrinkage + cone travel before the last sub-step + the
        // gradient footprint (two cells); the small epsilon covers FP32 rounding of travel
        const int travel = (int)std::ceil((B - 1) * step_cells + 1e-3);
        const int H_min = B + travel + 2;
        const int move = (int)std::ceil(B * step_cells + 1e-3);
        for (int cpl : {2, 4}) {
            if (only_cpl && cpl != only_cpl) continue;
            // a halo (and so a core) that is a multiple of the lane segment keeps every
            // segment aligned: whole-segment vector loads and stores
            const int H = (H_min + cpl - 1) / cpl * cpl;
            const int W = 64 * cpl;
            const int TX = W - 2 * H;
            if (TX < 16 || TX <= move) continue;
            const int max_height =
                (int)(kLdsBudget / ((size_t)n_species * W * sizeof(float))) - kGuardRows;
            for (int HL = 2 * H + 16; HL <= max_height; ++HL) {
                if (only_height && HL != only_height) continue;
                const int TY = HL - 2 * H;
                if (TY <= move) continue;
                const size_t lds = (size_t)n_species * W * (HL + kGuardRows) * sizeof(float);
                const int tiles = ceil_div(nx, TX) * ceil_div(ny, TY);
                const int per_cu = ceil_div(tiles, 256);
                const size_t per_cu_lds = 160 * 1024;
                const int resident = std::max(1, std::min(2, (int)(per_cu_lds / (lds + kStaticLds))));
                // per-step cost in cell-updates per compute unit: each tile's loaded area
                // per sub-step plus its load/store per launch; one resident tile per CU
                // hides latency poorly.  Cones gather (attracted to the sources), and a tile
                // holding more than kPartCones of them takes extra workgroups: keep room
                // for a quarter of the cones in full parts beside one workgroup per tile,
                // or the launch runs in two generations.
                const int spare = std::min(tiles, ceil_div(n_cones, 4 * kPartCones));
                double cost = (double)per_cu * W * HL * (1.0 + 2.0 / B) / B;
                if (resident < 2 || ceil_div(tiles + spare, 256) > resident) cost *= 1.25;
                if (cost < best_cost * 0.999) {
                    best_cost = cost;
                    best.block_steps = B;
                    best.move = move;
                    best.halo = H;
                    best.cpl = cpl;
                    best.core_x = TX;
                    best.core_y = TY;
                    best.tiles_x = ceil_div(nx, TX);
                    best.tiles_y = ceil_div(ny, TY);
                    best.n_tiles = best.tiles_x * best.tiles_y;
                    best.lds_bytes = lds;
                    best.height = HL;
                    // one cone step costs about as much as a stencil row of ~30 cells per
                    // lane-slot pair: 15 rows of two-cell segments for one species
                    best.cone_rows = std::max(1, 30 / (cpl * n_species));
                }
            }
        }
        if (best.block_steps > 1) break;   // prefer the deepest blocking that fits
    }
    return best;
}

}  // namespace

TiledPlan tiled_plan(int dim, int nx, int ny, int nz, int n_species, double step_cells,
                     int block_steps, int n_cones, int force_cpl, int force_height) {
    if (force_cpl != 0 || force_height != 0) {
        const TiledPlan forced = plan_search(dim, nx, ny, nz, n_species, step_cells,
                                             block_steps, n_cones, force_cpl, force_height);
        if (forced.block_steps > 1) return forced;
    }
    return plan_search(dim, nx, ny, nz, n_species, step_cells, block_steps, n_cones, 0, 0);
}

hipError_t tiled_allocate(const TiledPlan& plan, TiledState& st, int n_cones,
                          const ConeRules& rules, const sim_params* p, float* const fields[][2],
                          ConeArrays cones, hipStream_t stream) {
    hipError_t e;
    const int W = 64 * plan.cpl;
    st.capacity = std::max(1, n_cones);
    const size_t slots = (size_t)plan.n_tiles * st.capacity;
    for (int b = 0; b < 2; ++b) {
        if ((e = hipMalloc(&st.bucket[b], slots * sizeof(float4))) != hipSuccess) return e;
        if ((e = hipMalloc(&st.count[b], plan.n_tiles * sizeof(int32_t))) != hipSuccess) return e;
        if ((e = hipMemsetAsync(st.count[b], 0, plan.n_tiles * sizeof(int32_t), stream)) != hipSuccess)
            return e;
    }
    st.cur = 0;
    // per-tile source entries: every unique source cell inside a tile's loaded region
    std::vector<std::vector<std::pair<int2, float>>> per_tile(plan.n_tiles);
    const double vol = std::pow(p->dx, p->dim);
    for (int s = 0; s < p->n_species; ++s) {
        std::map<int32_t, double> merged;
        for (int m = 0; m < p->n_sources[s]; ++m)
            merged[p->source_cell[s][m]] += (double)p->source_q[s][m] / vol;
        for (auto& kv : merged) {
            const int gx = kv.first % plan.nx, gy = kv.first / plan.nx;
            for (int ty = 0; ty < plan.tiles_y; ++ty) {
                const int y0 = ty * plan.core_y - plan.halo;
                if (gy < y0 || gy >= y0 + plan.height) continue;
                for (int tx = 0; tx < plan.tiles_x; ++tx) {
                    const int x0 = tx * plan.core_x - plan.halo;
                    if (gx < x0 || gx >= x0 + W) continue;
                    const int local = (gy - y0) * W + (gx - x0);
                    per_tile[ty * plan.tiles_x + tx].push_back({make_int2(local, s), (float)kv.second});
                }
            }
        }
    }
    std::vector<int32_t> start(plan.n_tiles + 1, 0);
    std::vector<int2> entry;
    std::vector<float> amount;
    for (int t = 0; t < plan.n_tiles; ++t) {
        for (auto& en : per_tile[t]) {
            entry.push_back(en.first);
            amount.push_back(en.second);
        }
        start[t + 1] = (int32_t)entry.size();
    }
    if ((e = hipMalloc(&st.src_start, start.size() * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(&st.src_entry, std::max<size_t>(1, entry.size()) * sizeof(int2))) != hipSuccess)
        return e;
    if ((e = hipMalloc(&st.src_amount, std::max<size_t>(1, amount.size()) * sizeof(float))) != hipSuccess)
        return e;
    if ((e = hipMemcpy(st.src_start, start.data(), start.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (!entry.empty()) {
        if ((e = hipMemcpy(st.src_entry, entry.data(), entry.size() * sizeof(int2),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        if ((e = hipMemcpy(st.src_amount, amount.data(), amount.size() * sizeof(float),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return e;
    }
    // per-tile target lists: every target within reach of a tip that starts the launch in
    // the tile core (core grown by the launch's travel, plus the contact radius)
    {
        const double reach = (plan.move + 1) * p->dx + p->contact_radius;
        std::vector<std::vector<float4>> lists(plan.n_tiles);
        for (int t = 0; t < p->n_targets; ++t) {
            const float tx_ = p->target_pos[2 * t], ty_ = p->target_pos[2 * t + 1];
            for (int ty = 0; ty < plan.tiles_y; ++ty) {
                const double ylo = ty * plan.core_y * p->dx - reach;
                const double yhi = (ty + 1) * plan.core_y * p->dx + reach;
                if (ty_ < ylo || ty_ > yhi) continue;
                for (int tx = 0; tx < plan.tiles_x; ++tx) {
                    const double xlo = tx * plan.core_x * p->dx - reach;
                    const double xhi = (tx + 1) * plan.core_x * p->dx + reach;
                    if (tx_ < xlo || tx_ > xhi) continue;
                    float4 v = make_float4(tx_, ty_, 0.0f, 0.0f);
                    int32_t idx = t;
                    std::memcpy(&v.w, &idx, sizeof idx);
                    lists[ty * plan.tiles_x + tx].push_back(v);
                }
            }
        }
        std::vector<int32_t> tstart(plan.n_tiles + 1, 0);
        std::vector<float4> tpts;
        for (int t = 0; t < plan.n_tiles; ++t) {
            tpts.insert(tpts.end(), lists[t].begin(), lists[t].end());
            tstart[t + 1] = (int32_t)tpts.size();
        }
        if (tpts.empty()) tpts.push_back(make_float4(0.0f, 0.0f, 0.0f, 0.0f));
        if ((e = hipMalloc(&st.tgt_start, tstart.size() * sizeof(int32_t))) != hipSuccess) return e;
        if ((e = hipMalloc(&st.tgt_pts, tpts.size() * sizeof(float4))) != hipSuccess) return e;
        if ((e = hipMemcpy(st.tgt_start, tstart.data(), tstart.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        if ((e = hipMemcpy(st.tgt_pts, tpts.data(), tpts.size() * sizeof(float4),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return e;
    }
    // argument table and launch state
    TiledArgs2D a = {};
    for (int s = 0; s < plan.n_species; ++s) {
        a.field[s][0] = fields[s][0];
        a.field[s][1] = fields[s][1];
        a.coef[s] = plan.coef[s];
    }
    a.nx = plan.nx;
    a.ny = plan.ny;
    a.tiles_x = plan.tiles_x;
    a.n_tiles = plan.n_tiles;
    a.tx_core = plan.core_x;
    a.ty_core = plan.core_y;
    a.halo = plan.halo;
    a.height = plan.height;
    a.src_start = st.src_start;
    a.src_entry = st.src_entry;
    a.src_amount = st.src_amount;
    a.tgt_start = st.tgt_start;
    a.tgt_pts = st.tgt_pts;
    a.bucket[0] = st.bucket[0];
    a.bucket[1] = st.bucket[1];
    a.count[0] = st.count[0];
    a.count[1] = st.count[1];
    a.capacity = st.capacity;
    a.cone_rows = plan.cone_rows;
    a.cones = cones;
    a.rules = rules;
    if ((e = hipMalloc(&st.table, sizeof(TiledArgs2D))) != hipSuccess) return e;
    if ((e = hipMemcpy(st.table, &a, sizeof a, hipMemcpyHostToDevice)) != hipSuccess) return e;
    // work items: one per tile plus one per kPartCones further cones in a crowded tile (a
    // list of smaller parts is used only when it fits the resident workgroups)
    st.item_cap = tiled_item_capacity(plan.n_tiles, n_cones);
    std::vector<int2> base(plan.n_tiles);
    for (int t = 0; t < plan.n_tiles; ++t) base[t] = make_int2(0, t);
    if ((e = hipMalloc(&st.base, base.size() * sizeof(int2))) != hipSuccess) return e;
    if ((e = hipMemcpy(st.base, base.data(), base.size() * sizeof(int2),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if ((e = hipMalloc(&st.items, (size_t)st.item_cap * sizeof(int4))) != hipSuccess) return e;
    if ((e = hipMalloc(&st.launch, sizeof(LaunchState))) != hipSuccess) return e;
    const LaunchState ls0 = tiled_launch_state(
        std::min(tiled_persistent_grid(plan.lds_bytes), st.item_cap - kXcds));
    if ((e = hipMemcpy(st.launch, &ls0, sizeof ls0, hipMemcpyHostToDevice)) != hipSuccess) return e;
    st.cur = 0;
    for (bool record : {false, true})
        if ((e = hipFuncSetAttribute(kernel_for(plan.n_species, plan.cpl, record),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)plan.lds_bytes)) != hipSuccess)
            return e;
    return hipSuccess;
}

hipError_t tiled_set_record(TiledState& st, float* tape, uint32_t n0, hipStream_t stream) {
    struct {
        float* record;
        uint32_t record_n0;
    } rec = {tape, n0};
    st.recording = tape != nullptr;
    static_assert(offsetof(TiledArgs2D, record_n0) == offsetof(TiledArgs2D, record) + sizeof(float*),
                  "record and record_n0 are adjacent");
    hipError_t e = hipMemcpyAsync((char*)st.table + offsetof(TiledArgs2D, record), &rec,
                                  sizeof(float*) + sizeof(uint32_t), hipMemcpyHostToDevice,
                                  stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

hipError_t tiled_set_launch_state(TiledState& st, uint32_t step, int parity, hipStream_t stream) {
    const int32_t head[2] = {(int32_t)step, parity};   // step and parity; items untouched
    st.cur = parity;
    hipError_t e = hipMemcpyAsync(st.launch, head, sizeof head, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

LaunchState tiled_launch_state(int slots) {
    LaunchState ls = {};
    ls.slots = slots;
    return ls;
}

int tiled_item_capacity(int n_tiles, int n_cones) {
    // the items, plus the slots a list laid out by die may leave empty
    return n_tiles + (n_cones + kPartCones - 1) / kPartCones + 1 + kXcds;
}

hipError_t tiled_build_items(const TiledArgs2D* table, int4* items, const int2* base,
                             int n_base, int item_cap, LaunchState* launch, hipStream_t stream,
                             bool by_die) {
    hipLaunchKernelGGL(k_build_items, dim3(1), dim3(kThreads), 0, stream,
                       table, items, base, n_base, item_cap, launch, by_die ? 1 : 0);
    return hipGetLastError();
}

void tiled_release(TiledState& st) {
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(st.bucket[b]);
        (void)hipFree(st.count[b]);
        st.bucket[b] = nullptr;
        st.count[b] = nullptr;
    }
    (void)hipFree(st.src_start);
    (void)hipFree(st.src_entry);
    (void)hipFree(st.src_amount);
    (void)hipFree(st.tgt_start);
    (void)hipFree(st.tgt_pts);
    (void)hipFree(st.table);
    (void)hipFree(st.launch);
    (void)hipFree(st.items);
    (void)hipFree(st.base);
    st.table = nullptr;
    st.launch = nullptr;
    st.items = nullptr;
    st.base = nullptr;
    st.tgt_start = nullptr;
    st.tgt_pts = nullptr;
    st.src_start = nullptr;
    st.src_entry = nullptr;
    st.src_amount = nullptr;
}

hipError_t tiled_bucket(const TiledPlan& plan, TiledState& st, ConeArrays cones,
                        hipStream_t stream) {
    hipError_t e;
    for (int b = 0; b < 2; ++b)
        if ((e = hipMemsetAsync(st.count[b], 0, plan.n_tiles * sizeof(int32_t), stream)) != hipSuccess)
            return e;
    if (cones.n > 0) {
        hipLaunchKernelGGL(k_bucket2d, dim3(ceil_div(cones.n, 256)), dim3(256), 0, stream,
                           cones, plan.nx, plan.ny, plan.core_x, plan.core_y, plan.tiles_x,
                           plan.inv_dx, st.bucket[st.cur], st.count[st.cur], st.capacity);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return tiled_build_items(st.table, st.items, st.base, plan.n_tiles, st.item_cap, st.launch,
                             stream, true);
}

hipError_t tiled_unbucket(const TiledPlan& plan, TiledState& st, ConeArrays cones,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_unbucket2d, dim3(plan.n_tiles), dim3(256), 0, stream, cones,
                       st.bucket[st.cur], st.count[st.cur], st.capacity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int b = 0; b < 2; ++b)
        if ((e = hipMemsetAsync(st.count[b], 0, plan.n_tiles * sizeof(int32_t), stream)) != hipSuccess)
            return e;
    return hipSuccess;
}

hipError_t tiled_sync_cones(const TiledPlan& plan, const TiledState& st, ConeArrays cones,
                            hipStream_t stream) {
    hipLaunchKernelGGL(k_unbucket2d, dim3(plan.n_tiles), dim3(256), 0, stream, cones,
                       st.bucket[st.cur], st.count[st.cur], st.capacity);
    return hipGetLastError();
}

hipError_t tiled_launch(const TiledPlan& plan, TiledState& st, int steps, hipStream_t stream,
                        hipEvent_t start, hipEvent_t stop) {
    const TiledArgs2D* table = st.table;
    int4* items = st.items;
    const int2* base = st.base;
    int n_base = plan.n_tiles;
    int item_cap = st.item_cap;
    LaunchState* ls = st.launch;
    int persistent = 0;
    void* args[] = {&table, &items, &base, &n_base, &item_cap, &steps, &ls, &persistent};
    const hipError_t e = hipExtLaunchKernel(kernel_for(plan.n_species, plan.cpl, st.recording),
                                            dim3(item_cap), dim3(kThreads), args,
                                            plan.lds_bytes, stream, start, stop, 0);
    if (e == hipSuccess) st.cur ^= 1;
    return e;
}

size_t tiled_table_entry_bytes() { return sizeof(TiledArgs2D); }

int tiled_persistent_grid(size_t lds_bytes) {
    const size_t per_cu_lds = 160 * 1024;
    const int resident = std::max(1, std::min(2, (int)(per_cu_lds / (lds_bytes + kStaticLds))));
    return 256 * resident;
}

hipError_t tiled_launch_batch(const TiledArgs2D* table, int4* items, const int2* base,
                              int n_base, int item_cap, int n_species, int cpl,
                              size_t lds_bytes, int steps, LaunchState* launch,
                              hipStream_t stream) {
    int persistent = 1;
    void* args[] = {&table, &items, &base, &n_base, &item_cap, &steps, &launch, &persistent};
    return hipLaunchKernel(kernel_for(n_species, cpl), dim3(tiled_persistent_grid(lds_bytes)),
                           dim3(kThreads), args, lds_bytes, stream);
}

hipError_t tiled_prepare_batch(int n_species, int cpl, size_t lds_bytes) {
    return hipFuncSetAttribute(kernel_for(n_species, cpl),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

}  // namespace cuesim
