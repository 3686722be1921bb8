// kernels_field3d.hip -- one explicit step of every species of a 3D field, sources included.
//
// 7-point stencil with first-order decay, zero-flux walls (a missing neighbour is the cell
// itself), then the point sources of the step (c' += q / dx^3).  One launch covers every
// species.  A workgroup owns a box of kTX x kTY columns and kTZ consecutive planes of one
// species (64 x 8 x 16, the fastest of the shapes measured) and marches up the planes; each
// thread keeps the planes below, at and above its cell in registers and reads the four
// in-plane neighbours from lines the workgroup has just brought into L1/L2, so a cell is
// fetched from HBM about once per step: 8 algorithmic bytes per species-cell-update.
// Planes are taken kUnroll at a time with every load of the group issued before the
// arithmetic, which keeps kUnroll times more reads in flight than a plane-by-plane march.
// Walls are handled by clamping the neighbour index, which reads the cell itself exactly
// where the ghost value is the cell's own.
//
// Boxes are dealt to the accelerator dies in contiguous stretches (workgroups are assigned
// to dies round-robin), so boxes that share halo rows usually share an L2.
//
// The sources of a box are a short list (plane, thread, amount) built once on the host and
// sorted by plane; every thread walks it with the march and adds the amounts of its own
// cells after the stencil, as a separate FP32 add (the same rounding as a source pass).
#include <hip/hip_ext.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace cuesim {

namespace {

constexpr int kTX = 64, kTY = 8, kTZ = 16, kUnroll = 4;
constexpr int kThreads = kTX * kTY;
constexpr int kXcds = 8;

struct Boxes {
    int tx, ty, tz;   // boxes per axis
    int per_species() const { return tx * ty * tz; }
};

Boxes boxes_for(int nx, int ny, int nz) {
    return Boxes{(nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY, (nz + kTZ - 1) / kTZ};
}

__device__ __forceinline__ float stencil(float c, float w, float e, float s, float n,
                                         float below, float above, const StencilCoef& k) {
    const float lap = fmaf(-6.0f, c, ((w + e) + (s + n)) + (below + above));
    return fmaf(k.r, lap, fmaf(-k.kdt, c, c));
}

__global__ __launch_bounds__(kThreads) void k_field3d(Field3DArgs a) {
    const int n_boxes = a.n_species * a.tx * a.ty * a.tz;
    const int box = (blockIdx.x % kXcds) * a.per_xcd + blockIdx.x / kXcds;
    if (box >= n_boxes) return;
    int rest = box;
    const int bx = rest % a.tx;
    rest /= a.tx;
    const int by = rest % a.ty;
    rest /= a.ty;
    const int bz = rest % a.tz;
    const int s = rest / a.tz;
    // this workgroup's slice of the source list
    int e = a.src_start[box];
    const int e_end = a.src_start[box + 1];

    const int tid = threadIdx.x;
    const int i = bx * kTX + tid % kTX;
    const int j = by * kTY + tid / kTX;
    if (i >= a.nx || j >= a.ny) {
        return;   // no barriers below: idle threads may leave
    }
    const StencilCoef k = a.coef[s];
    const size_t plane = (size_t)a.nx * a.ny;
    const float* col = a.in[s] + (size_t)j * a.nx + i;
    float* dst = a.out[s] + (size_t)j * a.nx + i;
    const int dw = i > 0 ? -1 : 0, de = i < a.nx - 1 ? 1 : 0;
    const int ds = j > 0 ? -a.nx : 0, dn = j < a.ny - 1 ? a.nx : 0;
    const int nz = a.nz;
    const int z0 = bz * kTZ, z1 = min(z0 + kTZ, nz);

    float c = col[(size_t)z0 * plane];
    float below = col[(size_t)max(z0 - 1, 0) * plane];
    int l = z0;
    for (; l + kUnroll <= z1; l += kUnroll) {
        float up[kUnroll], w[kUnroll], ea[kUnroll], so[kUnroll], no[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const float* p = col + (size_t)(l + u) * plane;
            up[u] = col[(size_t)min(l + u + 1, nz - 1) * plane];
            w[u] = p[dw];
            ea[u] = p[de];
            so[u] = p[ds];
            no[u] = p[dn];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            float v = stencil(c, w[u], ea[u], so[u], no[u], below, up[u], k);
            while (e < e_end && a.src_plane[e] == l + u) {
                if (a.src_thread[e] == tid) v += a.src_q[e];
                ++e;
            }
            dst[(size_t)(l + u) * plane] = v;
            below = c;
            c = up[u];
        }
    }
    for (; l < z1; ++l) {
        const float* p = col + (size_t)l * plane;
        const float above = col[(size_t)min(l + 1, nz - 1) * plane];
        float v = stencil(c, p[dw], p[de], p[ds], p[dn], below, above, k);
        while (e < e_end && a.src_plane[e] == l) {
            if (a.src_thread[e] == tid) v += a.src_q[e];
            ++e;
        }
        dst[(size_t)l * plane] = v;
        below = c;
        c = above;
    }
}

}  // namespace

hipError_t field3d_prepare(Field3D& f, int nx, int ny, int nz, int n_species,
                           const std::vector<int32_t>* cells, const std::vector<float>* q) {
    field3d_release(f);
    const Boxes b = boxes_for(nx, ny, nz);
    const int n_boxes = n_species * b.per_species();
    // source entries per box, in plane order (cells are unique per species)
    std::vector<std::vector<std::pair<int64_t, float>>> per_box(n_boxes);
    for (int s = 0; s < n_species; ++s)
        for (size_t m = 0; m < cells[s].size(); ++m) {
            const int64_t cell = cells[s][m];
            const int i = (int)(cell % nx), j = (int)((cell / nx) % ny),
                      l = (int)(cell / ((int64_t)nx * ny));
            const int box = ((s * b.tz + l / kTZ) * b.ty + j / kTY) * b.tx + i / kTX;
            const int tid = (j % kTY) * kTX + i % kTX;
            per_box[box].push_back({(int64_t)l * kThreads + tid, q[s][m]});
        }
    std::vector<int32_t> start(n_boxes + 1, 0), plane_of, thread_of;
    std::vector<float> amount;
    for (int box = 0; box < n_boxes; ++box) {
        auto& v = per_box[box];
        std::sort(v.begin(), v.end(),
                  [](const std::pair<int64_t, float>& x, const std::pair<int64_t, float>& y) {
                      return x.first < y.first;
                  });
        for (auto& en : v) {
            plane_of.push_back((int32_t)(en.first / kThreads));
            thread_of.push_back((int32_t)(en.first % kThreads));
            amount.push_back(en.second);
        }
        start[box + 1] = (int32_t)plane_of.size();
    }
    const size_t n_src = std::max<size_t>(plane_of.size(), 1);
    hipError_t e;
    if ((e = hipMalloc((void**)&f.src_start, start.size() * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.src_plane, n_src * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.src_thread, n_src * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.src_q, n_src * sizeof(float))) != hipSuccess)
        return e;
    if ((e = hipMemcpy(f.src_start, start.data(), start.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (!plane_of.empty() &&
        ((e = hipMemcpy(f.src_plane, plane_of.data(), plane_of.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = hipMemcpy(f.src_thread, thread_of.data(), thread_of.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = hipMemcpy(f.src_q, amount.data(), amount.size() * sizeof(float),
                        hipMemcpyHostToDevice)) != hipSuccess))
        return e;
    f.nx = nx;
    f.ny = ny;
    f.nz = nz;
    f.n_species = n_species;
    f.n_boxes = n_boxes;
    return hipSuccess;
}

void field3d_release(Field3D& f) {
    if (f.src_start) (void)hipFree(f.src_start);
    if (f.src_plane) (void)hipFree(f.src_plane);
    if (f.src_thread) (void)hipFree(f.src_thread);
    if (f.src_q) (void)hipFree(f.src_q);
    f = Field3D{};
}

hipError_t launch_field3d(const Field3D& f, const float* const* in, float* const* out,
                          const StencilCoef* coef, hipStream_t stream, hipEvent_t start,
                          hipEvent_t stop) {
    const Boxes b = boxes_for(f.nx, f.ny, f.nz);
    Field3DArgs a = {};
    for (int s = 0; s < f.n_species; ++s) {
        a.in[s] = in[s];
        a.out[s] = out[s];
        a.coef[s] = coef[s];
    }
    a.nx = f.nx;
    a.ny = f.ny;
    a.nz = f.nz;
    a.n_species = f.n_species;
    a.tx = b.tx;
    a.ty = b.ty;
    a.tz = b.tz;
    a.per_xcd = (f.n_boxes + kXcds - 1) / kXcds;
    a.src_start = f.src_start;
    a.src_plane = f.src_plane;
    a.src_thread = f.src_thread;
    a.src_q = f.src_q;
    void* args[] = {&a};
    return hipExtLaunchKernel((const void*)k_field3d, dim3(a.per_xcd * kXcds), dim3(kThreads),
                              args, 0, stream, start, stop, 0);
}

}  // namespace cuesim
