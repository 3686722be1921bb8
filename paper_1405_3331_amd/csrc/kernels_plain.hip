// kernels_plain.hip -- the parts of an un-blocked 2D step besides the field update: the
// cones, one thread each in the caller's order, against the just-updated fields; and the
// FP64 mass of a field.
#include <hip/hip_ext.h>

#include <algorithm>

#include "internal.hpp"

namespace cuesim {

namespace {

struct Global2D {
    const float* f;
    int nx;
    __device__ float operator()(int i, int j) const { return f[j * nx + i]; }
};

__global__ __launch_bounds__(256) void k_cones2d(ConeRules r, const float* __restrict__ f0,
                                                 const float* __restrict__ f1, ConeArrays c,
                                                 uint32_t step) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n || c.status[i] != kActive) return;
    float x = c.pos[2 * i], y = c.pos[2 * i + 1], th = c.dir[i];
    float gx, gy, conc = 0.0f;
    gradient_2d(Global2D{f0, r.nx}, r, x, y, gx, gy, r.turn_law == 1 ? &conc : nullptr);
    gx *= r.sign0;
    gy *= r.sign0;
    if (r.n_species > 1) {
        float hx, hy;
        gradient_2d(Global2D{f1, r.nx}, r, x, y, hx, hy);
        gx = fmaf(r.sign1, hx, gx);
        gy = fmaf(r.sign1, hy, gy);
    }
    float sn, cs;
    sincos_angle(th, sn, cs);
    float z[2];
    noise_2d(r.key, (uint32_t)i, step, z);
    const ConeEvent ev = cone_step_2d(r, gx, gy, conc, z, x, y, th, sn, cs,
                                      GridContact{&r.targets});
    c.pos[2 * i] = x;
    c.pos[2 * i + 1] = y;
    c.dir[i] = th;
    if (ev.status != kActive) {
        c.status[i] = ev.status;
        c.target[i] = ev.target;
        c.event_step[i] = (int32_t)(step + 1);
    }
}

// FP64 sum: each block reduces a grid-stride slice (wavefront shuffles, then LDS), the
// second pass adds the block partials in a fixed order, so the result is deterministic.
constexpr int kMassThreads = 256;

__device__ double block_sum(double v) {
    __shared__ double part[kMassThreads / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kMassThreads / 64; ++w) t += part[w];
    return t;
}

__global__ __launch_bounds__(kMassThreads) void k_mass_partial(const float* __restrict__ f,
                                                                int64_t n,
                                                                double* __restrict__ partial) {
    double acc = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * kMassThreads + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * kMassThreads)
        acc += (double)f[x];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// The total goes to *out; a non-finite total also raises *nonfinite (when given).
__global__ __launch_bounds__(kMassThreads) void k_mass_final(const double* __restrict__ partial,
                                                              int n, double* __restrict__ out,
                                                              int32_t* __restrict__ nonfinite) {
    double acc = 0.0;
    for (int x = threadIdx.x; x < n; x += kMassThreads) acc += partial[x];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) {
        *out = t;
        if (nonfinite && !isfinite(t)) *nonfinite = 1;
    }
}

// Several device-to-device copies in one launch (a checkpoint's field and cone arrays):
// word w of the concatenated spans, in 4-byte words, by a grid-stride loop.
__global__ __launch_bounds__(256) void k_copy_spans(CopySpans c) {
    const size_t total = c.word_end[c.n - 1];
    for (size_t w = (size_t)blockIdx.x * 256 + threadIdx.x; w < total;
         w += (size_t)gridDim.x * 256) {
        int k = 0;
        while (w >= c.word_end[k]) ++k;
        const size_t off = w - (k > 0 ? c.word_end[k - 1] : 0);
        ((uint32_t*)c.dst[k])[off] = ((const uint32_t*)c.src[k])[off];
    }
}

}  // namespace

hipError_t launch_copy_spans(const CopySpans& c, hipStream_t stream) {
    if (c.n <= 0 || c.word_end[c.n - 1] == 0) return hipSuccess;
    const size_t total = c.word_end[c.n - 1];
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(k_copy_spans, dim3(blocks), dim3(256), 0, stream, c);
    return hipGetLastError();
}

hipError_t launch_cones2d(const ConeRules& rules, const float* f0, const float* f1,
                          ConeArrays cones, uint32_t step, hipStream_t stream) {
    if (cones.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cones2d, dim3((cones.n + 255) / 256), dim3(256), 0, stream, rules, f0,
                       f1, cones, step);
    return hipGetLastError();
}

hipError_t launch_mass(const float* field, int64_t n, double* partial, int n_partial,
                       double* out, hipStream_t stream, int32_t* nonfinite) {
    int blocks = (int)((n + kMassThreads - 1) / kMassThreads);
    if (blocks > n_partial) blocks = n_partial;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mass_partial, dim3(blocks), dim3(kMassThreads), 0, stream, field, n,
                       partial);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(kMassThreads), 0, stream, partial, blocks,
                       out, nonfinite);
    return hipGetLastError();
}

}  // namespace cuesim
