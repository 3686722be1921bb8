// internal.hpp -- launchers shared between the host side of the library and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
struct SourceList {
    const int32_t* cell;
    const float* q;
    int n;
};

// Cone state in the caller's order (structure of arrays).
struct ConeArrays {
    float* pos;          // [M][dim]
    float* dir;          // 2D [M]; 3D [M][3]
    int32_t* status;
    int32_t* target;
    int32_t* event_step;
    int n;
};

// One step without temporal blocking: stencil of every species (HBM in -> HBM out), then
// sources, then one thread per cone.  `in`/`out` index species.
hipError_t launch_field_plain(int dim, int nx, int ny, int nz, const float* in, float* out,
                              StencilCoef coef, hipStream_t stream);
hipError_t launch_sources(float* field, SourceList src, hipStream_t stream);
hipError_t launch_cones_plain(int dim, const ConeRules& rules, const float* f0,
                              const float* f1, ConeArrays cones, uint32_t step,
                              hipStream_t stream);

// Sum of a field in FP64 (deterministic two-pass reduction) into *out (device).
hipError_t launch_mass(const float* field, int64_t n, double* partial, int n_partial,
                       double* out, hipStream_t stream);
constexpr int kMassPartials = 1024;

}  // namespace cuesim
