// kernels_cones3d.hip -- the 3D cone step over cones held in spatial order.
//
// A 3D cone samples 32 cells per species around its tip (Sec. 3.5 gradient steering; trilinear).  In
// the caller's order neighbouring threads sit anywhere in the volume, so a wavefront touches
// a separate set of cache lines per cone and uses a few bytes of each.  Here the active
// cones are kept sorted by the Morton code of their tip cell (coarsened by `shift` bits per
// axis): a workgroup then covers one compact region, its gathers share lines in L1/L2, and
// the cone state itself streams as two aligned float4 per cone (tip x, y, z, id; heading).
// Cones move at most step_len per step, so the order is refreshed every few steps (the
// project's stable counting sort of the keys, kernels_sort.hip, then a gather of the state),
// not every step.
//
// Stopped cones leave the order: the step writes their final tip, heading, status, target
// and event step straight into the caller-order arrays and marks the ordered copy id = -1;
// a refresh moves them behind the active ones.  The caller-order tips and headings of the
// active cones are brought up to date only when the state is read (order3d_end).
#include "internal.hpp"

namespace cuesim {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;   // workgroups are dealt to the accelerator dies round-robin
// workgroups per die of the cone step: two per CU (32 CUs per die), each walking several
// blocks of its die's stretch, so a die works on a region of the fields its L2 can hold
// (256^3 workload: 62 us and 247 MB fetched per step, against 70 us and 336 MB with every
// block resident at once; one per CU fetched least, 186 MB, but took 67 us)
constexpr int kConeWgsPerXcd = 32 * 2;

__device__ __forceinline__ uint32_t spread3(uint32_t v) {   // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Cell of a coordinate, clamped to the grid (as a float first: a NaN tip maps to cell 0).
__device__ __forceinline__ uint32_t cell_coord(float p, float inv_dx, int n) {
    return (uint32_t)fminf(fmaxf(floorf(p * inv_dx), 0.0f), (float)(n - 1));
}

__device__ __forceinline__ uint32_t order_key(const ConeRules& r, float x, float y, float z,
                                              int shift) {
    return spread3(cell_coord(x, r.inv_dx, r.nx) >> shift) |
           (spread3(cell_coord(y, r.inv_dx, r.ny) >> shift) << 1) |
           (spread3(cell_coord(z, r.inv_dx, r.nz) >> shift) << 2);
}

// Caller order -> (tip, heading) with keys; inactive cones get id -1 and the key past every
// active one.
__global__ __launch_bounds__(kThreads) void k_pack3d(ConeRules r, ConeArrays c, float4* tip,
                                                     float4* dir, uint32_t* key, int32_t* slot,
                                                     int shift, uint32_t inactive) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= c.n) return;
    const float x = c.pos[3 * i], y = c.pos[3 * i + 1], z = c.pos[3 * i + 2];
    const bool active = c.status[i] == kActive;
    tip[i] = make_float4(x, y, z, __int_as_float(active ? i : -1));
    dir[i] = make_float4(c.dir[3 * i], c.dir[3 * i + 1], c.dir[3 * i + 2], 0.0f);
    key[i] = active ? order_key(r, x, y, z, shift) : inactive;
    slot[i] = i;
}

__global__ __launch_bounds__(kThreads) void k_keys3d(ConeRules r, const float4* __restrict__ tip,
                                                     int n, uint32_t* key, int32_t* slot,
                                                     int shift, uint32_t inactive) {
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const float4 p = tip[t];
    key[t] = __float_as_int(p.w) >= 0 ? order_key(r, p.x, p.y, p.z, shift) : inactive;
    slot[t] = t;
}

__global__ __launch_bounds__(kThreads) void k_gather3d(const int32_t* __restrict__ slot, int n,
                                                       const float4* __restrict__ tip_in,
                                                       const float4* __restrict__ dir_in,
                                                       float4* __restrict__ tip_out,
                                                       float4* __restrict__ dir_out) {
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const int s = slot[t];
    tip_out[t] = tip_in[s];
    dir_out[t] = dir_in[s];
}

struct Global3D {
    const float* f;
    int nx, ny;
    __device__ float operator()(int i, int j, int l) const { return f[(l * ny + j) * nx + i]; }
};

// The 3D gradient footprint of one species read row by row: each of the four rows
// (j0 + b, l0 + c) with four cells (im, i0, i0 + 1, ip) is one 16-byte load of the cells
// [s, s + 4), s = clamp(i0 - 1, 0, nx - 4), from which the four values are picked (at a wall
// the clamped indices repeat a cell, exactly as the per-cell accessor reads it); the other
// eight rows hold two adjacent cells each.  Needs nx >= 4.
__device__ __forceinline__ Footprint3D load_footprint_3d_rows(const float* __restrict__ f,
                                                              const ConeRules& r,
                                                              const Corner3D& k) {
    Footprint3D p;
    const size_t nx = (size_t)r.nx, plane = nx * (size_t)r.ny;
    const int s = min(max(k.i0 - 1, 0), r.nx - 4);
    const int am = k.im - s, a0 = k.i0 - s, ap = k.ip - s;
    auto row4 = [&](int j, int l) {
        float4 v;
        __builtin_memcpy(&v, f + (size_t)l * plane + (size_t)j * nx + s, sizeof v);
        return v;
    };
    auto pick = [](const float4& v, int i) {
        return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
    };
    auto row2 = [&](int j, int l) {
        float2 v;
        __builtin_memcpy(&v, f + (size_t)l * plane + (size_t)j * nx + k.i0, sizeof v);
        return v;
    };
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float4 v = row4(k.j0 + b, k.l0 + c);
            p.xm[b][c] = pick(v, am);
            p.blk[0][b][c] = pick(v, a0);
            p.blk[1][b][c] = pick(v, a0 + 1);
            p.xp[b][c] = pick(v, ap);
        }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float2 ym = row2(k.jm, k.l0 + c), yp = row2(k.jp, k.l0 + c);
        p.ym[0][c] = ym.x;
        p.ym[1][c] = ym.y;
        p.yp[0][c] = yp.x;
        p.yp[1][c] = yp.y;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const float2 zm = row2(k.j0 + b, k.lm), zp = row2(k.j0 + b, k.lp);
        p.zm[0][b] = zm.x;
        p.zm[1][b] = zm.y;
        p.zp[0][b] = zp.x;
        p.zp[1][b] = zp.y;
    }
    return p;
}

// One step of ordered cone t against the updated fields.
template <int NS>
__device__ __forceinline__ void step_ordered_cone(const ConeRules& r, const float* f0,
                                                  const float* f1, float4* tip, float4* dir,
                                                  const ConeArrays& c, uint32_t step, int t) {
    const float4 p = tip[t];
    const int id = __float_as_int(p.w);
    if (id < 0) return;
    const float4 h = dir[t];
    float x = p.x, y = p.y, z = p.z, hx = h.x, hy = h.y, hz = h.z;
    const Corner3D k = corner_3d(r, x, y, z);
    float gx, gy, gz;
    if (r.nx >= 4)
        gradient_from_3d(r, k, load_footprint_3d_rows(f0, r, k), gx, gy, gz);
    else
        gradient_from_3d(r, k, load_footprint_3d(Global3D{f0, r.nx, r.ny}, k), gx, gy, gz);
    gx *= r.sign0;
    gy *= r.sign0;
    gz *= r.sign0;
    if (NS > 1) {
        float ax, ay, az;
        if (r.nx >= 4)
            gradient_from_3d(r, k, load_footprint_3d_rows(f1, r, k), ax, ay, az);
        else
            gradient_from_3d(r, k, load_footprint_3d(Global3D{f1, r.nx, r.ny}, k), ax, ay,
                             az);
        gx = fmaf(r.sign1, ax, gx);
        gy = fmaf(r.sign1, ay, gy);
        gz = fmaf(r.sign1, az, gz);
    }
    const ConeEvent ev = cone_step_3d(r, gx, gy, gz, (uint32_t)id, step, x, y, z, hx, hy, hz,
                                      GridContact{&r.targets});
    dir[t] = make_float4(hx, hy, hz, 0.0f);
    if (ev.status == kActive) {
        tip[t] = make_float4(x, y, z, p.w);
        return;
    }
    tip[t] = make_float4(x, y, z, __int_as_float(-1));
    c.pos[3 * id] = x;
    c.pos[3 * id + 1] = y;
    c.pos[3 * id + 2] = z;
    c.dir[3 * id] = hx;
    c.dir[3 * id + 1] = hy;
    c.dir[3 * id + 2] = hz;
    c.status[id] = ev.status;
    c.target[id] = ev.target;
    c.event_step[id] = (int32_t)(step + 1);
}

// One step of every ordered cone.  The blocks of kThreads cones are split into one
// contiguous stretch of the order per accelerator die (workgroups are dealt to the dies
// round-robin), so a die works on one compact region of the fields; when there are more
// blocks than workgroups, the workgroups of a die walk its stretch block after block.  (Loading
// both species' footprints before combining either was measured slower: the wider register
// live range costs more than the extra loads in flight gain.)
template <int NS>
__global__ __launch_bounds__(kThreads) void k_cones3d_ordered(ConeRules r,
                                                              const float* __restrict__ f0,
                                                              const float* __restrict__ f1,
                                                              float4* tip, float4* dir, int n,
                                                              int per_xcd, ConeArrays c,
                                                              uint32_t step) {
    const int xcd = blockIdx.x % kXcds;
    const int wgs_per_xcd = gridDim.x / kXcds;
    for (int b = blockIdx.x / kXcds; b < per_xcd; b += wgs_per_xcd) {
        const int t = (xcd * per_xcd + b) * kThreads + threadIdx.x;
        if (t < n) step_ordered_cone<NS>(r, f0, f1, tip, dir, c, step, t);
    }
}

__global__ __launch_bounds__(kThreads) void k_unpack3d(const float4* __restrict__ tip,
                                                       const float4* __restrict__ dir, int n,
                                                       ConeArrays c) {
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const float4 p = tip[t];
    const int id = __float_as_int(p.w);
    if (id < 0) return;
    const float4 h = dir[t];
    c.pos[3 * id] = p.x;
    c.pos[3 * id + 1] = p.y;
    c.pos[3 * id + 2] = p.z;
    c.dir[3 * id] = h.x;
    c.dir[3 * id + 1] = h.y;
    c.dir[3 * id + 2] = h.z;
}

int blocks_for(int n) { return (n + kThreads - 1) / kThreads; }

int axis_bits(int n, int shift) {
    int bits = 1;
    while (bits < 10 && ((n - 1) >> shift) >= (1 << bits)) ++bits;
    return bits;
}

// Stable counting sort of (key, slot) (buffers 0 and 1 ping-pong), then the state gather
// into the other half of the state's ping-pong.
hipError_t sort_and_gather(ConeOrder3D& o, hipStream_t stream) {
    bool in_alt = false;
    hipError_t e = sort_pairs(o.key[0], o.slot[0], o.key[1], o.slot[1], o.n, o.end_bit,
                              o.scratch, stream, &in_alt);
    if (e != hipSuccess) return e;
    const int nxt = o.cur ^ 1;
    hipLaunchKernelGGL(k_gather3d, dim3(blocks_for(o.n)), dim3(kThreads), 0, stream,
                       o.slot[in_alt ? 1 : 0], o.n, o.tip[o.cur], o.dir[o.cur], o.tip[nxt],
                       o.dir[nxt]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    o.cur = nxt;
    return hipSuccess;
}

}  // namespace

hipError_t order3d_allocate(ConeOrder3D& o, int n, int nx, int ny, int nz) {
    o = ConeOrder3D{};
    o.n = n;
    const int bits = std::max(axis_bits(nx, o.shift), std::max(axis_bits(ny, o.shift),
                                                               axis_bits(nz, o.shift)));
    o.inactive = 1u << (3 * bits);
    o.end_bit = 3 * bits + 1;
    if (n == 0) return hipSuccess;
    hipError_t e;
    for (int b = 0; b < 2; ++b) {
        if ((e = hipMalloc((void**)&o.tip[b], (size_t)n * sizeof(float4))) != hipSuccess ||
            (e = hipMalloc((void**)&o.dir[b], (size_t)n * sizeof(float4))) != hipSuccess ||
            (e = hipMalloc((void**)&o.key[b], (size_t)n * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc((void**)&o.slot[b], (size_t)n * sizeof(int32_t))) != hipSuccess)
            return e;
    }
    return hipMalloc((void**)&o.scratch, sort_pairs_scratch_bytes(n));
}

void order3d_release(ConeOrder3D& o) {
    for (int b = 0; b < 2; ++b) {
        if (o.tip[b]) (void)hipFree(o.tip[b]);
        if (o.dir[b]) (void)hipFree(o.dir[b]);
        if (o.key[b]) (void)hipFree(o.key[b]);
        if (o.slot[b]) (void)hipFree(o.slot[b]);
    }
    if (o.scratch) (void)hipFree(o.scratch);
    o = ConeOrder3D{};
}

hipError_t order3d_begin(ConeOrder3D& o, const ConeRules& r, ConeArrays cones,
                         hipStream_t stream) {
    if (o.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack3d, dim3(blocks_for(o.n)), dim3(kThreads), 0, stream, r, cones,
                       o.tip[o.cur], o.dir[o.cur], o.key[0], o.slot[0], o.shift, o.inactive);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sort_and_gather(o, stream);
}

hipError_t order3d_refresh(ConeOrder3D& o, const ConeRules& r, hipStream_t stream) {
    if (o.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys3d, dim3(blocks_for(o.n)), dim3(kThreads), 0, stream, r,
                       o.tip[o.cur], o.n, o.key[0], o.slot[0], o.shift, o.inactive);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sort_and_gather(o, stream);
}

hipError_t launch_cones3d_ordered(const ConeRules& r, const float* f0, const float* f1,
                                  ConeOrder3D& o, ConeArrays cones, uint32_t step,
                                  hipStream_t stream) {
    if (o.n == 0) return hipSuccess;
    const int blocks = blocks_for(o.n);
    const int per_xcd = (blocks + kXcds - 1) / kXcds;
    const int wgs_per_xcd = std::min(per_xcd, kConeWgsPerXcd);
    if (r.n_species > 1)
        hipLaunchKernelGGL(k_cones3d_ordered<2>, dim3(wgs_per_xcd * kXcds), dim3(kThreads), 0,
                           stream, r, f0, f1, o.tip[o.cur], o.dir[o.cur], o.n, per_xcd, cones,
                           step);
    else
        hipLaunchKernelGGL(k_cones3d_ordered<1>, dim3(wgs_per_xcd * kXcds), dim3(kThreads), 0,
                           stream, r, f0, f1, o.tip[o.cur], o.dir[o.cur], o.n, per_xcd, cones,
                           step);
    return hipGetLastError();
}

hipError_t order3d_end(const ConeOrder3D& o, ConeArrays cones, hipStream_t stream) {
    if (o.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack3d, dim3(blocks_for(o.n)), dim3(kThreads), 0, stream,
                       o.tip[o.cur], o.dir[o.cur], o.n, cones);
    return hipGetLastError();
}

}  // namespace cuesim
