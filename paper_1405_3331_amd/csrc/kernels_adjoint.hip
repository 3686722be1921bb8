// kernels_adjoint.hip -- reverse pass of the 2D time step, for the gradient of a trajectory
// loss L = sum_i w_i |p_i^N - t_a(i)|^2 with respect to the source amounts, D and k.
//
// The derivative is taken along the forward run's branch: the exit and contact decisions
// and the active side of the turn cap are held as the forward run took them (the cone
// rules of Sec. 3.4-3.5 have no derivative at those switches).
//
// The fields never depend on the cones, so within a checkpoint segment the cones can be
// handled apart from the fields, each cone by one thread over all the segment's steps:
//   k_cones_segment2d         re-runs the segment's cone steps against the re-run fields and
//                             records (x, y, theta) of every cone at the start of each step;
//   k_cone_adjoint_segment2d  walks the steps backwards carrying each cone's adjoint of
//                             (p, theta) through advance, capped turn and interpolated
//                             gradient; the gradient samples' adjoints are scattered into
//                             e^{n+1}, one buffer per step (12 cells per species per cone);
//   k_field_adjoint2d_rows    (kernels_field2d.hip) one launch per step: with
//                             b = a^{n+1} + e^{n+1}, a^n = b + r Lap b - k dt b (the
//                             zero-flux Laplacian is symmetric, so the adjoint stencil is
//                             the stencil), and
//                             per-workgroup FP64 sums of b Lap c^n (for dL/dD) and b c^n (for
//                             dL/dk) plus b at every source cell (dL/dq).
// HBM bytes per cell of the reverse field step: a^{n+1}, e^{n+1} and c^n read, a^n written.
#include "internal.hpp"

namespace cuesim {

namespace {

constexpr int kAdjThreads = 256;
constexpr int kSegThreads = 64;   // segment kernels: one short wave per CU where possible

__device__ double adj_block_sum(double v) {
    __shared__ double part[kAdjThreads / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();   // part[] may still be read from a previous call
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kAdjThreads / 64; ++w) t += part[w];
    return t;
}

// Reverse of the interpolated central-difference gradient of one species at (x, y).
// (agx, agy) is the adjoint of the sampled gradient, already weighted by the species
// sign.  Adds the adjoint of the tip position into (apx, apy) -- the interpolation
// weights depend on the tip; along an axis where the tip is clamped to the outermost
// centres they do not -- and scatters the adjoint of the 12 loaded values into af.
__device__ __forceinline__ void gradient_2d_reverse(const float* __restrict__ f,
                                                    float* __restrict__ af,
                                                    const ConeRules& r, float x, float y,
                                                    float agx, float agy, float& apx,
                                                    float& apy) {
    int i0, j0;
    float fx, fy;
    corner(x, r.inv_dx, r.nx, i0, fx);
    corner(y, r.inv_dx, r.ny, j0, fy);
    const float ux = fmaf(x, r.inv_dx, -0.5f), uy = fmaf(y, r.inv_dx, -0.5f);
    const bool free_x = ux > 0.0f && ux < (float)(r.nx - 1);
    const bool free_y = uy > 0.0f && uy < (float)(r.ny - 1);
    const int im = max(i0 - 1, 0), ip = min(i0 + 2, r.nx - 1);
    const int jm = max(j0 - 1, 0), jp = min(j0 + 2, r.ny - 1);
    const int nx = r.nx;
    const int ia0 = j0 * nx + im, ia1 = j0 * nx + i0, ia2 = j0 * nx + i0 + 1, ia3 = j0 * nx + ip;
    const int r1 = (j0 + 1) * nx;
    const int ib0 = r1 + im, ib1 = r1 + i0, ib2 = r1 + i0 + 1, ib3 = r1 + ip;
    const int ic0 = jm * nx + i0, ic1 = jm * nx + i0 + 1;
    const int id0 = jp * nx + i0, id1 = jp * nx + i0 + 1;
    const float h = r.half_inv_dx;
    // corner gradients (forward values, for the position term)
    const float gx00 = (f[ia2] - f[ia0]) * h, gx10 = (f[ia3] - f[ia1]) * h;
    const float gx01 = (f[ib2] - f[ib0]) * h, gx11 = (f[ib3] - f[ib1]) * h;
    const float gy00 = (f[ib1] - f[ic0]) * h, gy10 = (f[ib2] - f[ic1]) * h;
    const float gy01 = (f[id0] - f[ia1]) * h, gy11 = (f[id1] - f[ia2]) * h;
    const float w00 = (1.0f - fx) * (1.0f - fy), w10 = fx * (1.0f - fy);
    const float w01 = (1.0f - fx) * fy, w11 = fx * fy;
    // position: d w / d f along each axis, times d f / d p = 1 / dx where not clamped
    const float aw00 = agx * gx00 + agy * gy00, aw10 = agx * gx10 + agy * gy10;
    const float aw01 = agx * gx01 + agy * gy01, aw11 = agx * gx11 + agy * gy11;
    if (free_x) apx += r.inv_dx * ((1.0f - fy) * (aw10 - aw00) + fy * (aw11 - aw01));
    if (free_y) apy += r.inv_dx * ((1.0f - fx) * (aw01 - aw00) + fx * (aw11 - aw10));
    // field: each loaded value's adjoint (cells repeat at walls; the adds then combine)
    const float hx = h * agx, hy = h * agy;
    atomicAdd(&af[ia0], -w00 * hx);
    atomicAdd(&af[ia1], -w10 * hx - w01 * hy);
    atomicAdd(&af[ia2], w00 * hx - w11 * hy);
    atomicAdd(&af[ia3], w10 * hx);
    atomicAdd(&af[ib0], -w01 * hx);
    atomicAdd(&af[ib1], -w11 * hx + w00 * hy);
    atomicAdd(&af[ib2], w01 * hx + w10 * hy);
    atomicAdd(&af[ib3], w11 * hx);
    atomicAdd(&af[ic0], -w00 * hy);
    atomicAdd(&af[ic1], -w10 * hy);
    atomicAdd(&af[id0], w01 * hy);
    atomicAdd(&af[id1], w11 * hy);
}

struct Field2D {
    const float* f;
    int nx;
    __device__ float operator()(int i, int j) const { return f[j * nx + i]; }
};

// Reverse of one cone step (step index `step`) of cone i from its state (x, y, theta) at
// the start of the step; f0/f1 are the fields after the step's field update and af0/af1
// receive the adjoints of their sampled values.  (apx, apy, ath) holds the adjoint of the
// state after the step on entry and of the state before it on exit.
template <int NS>
__device__ __forceinline__ void cone_adjoint_step(const ConeRules& r, const float* f0,
                                                  const float* f1, float* af0, float* af1,
                                                  float4 st, int i, uint32_t step, float& apx,
                                                  float& apy, float& ath) {
    const float x = st.x, y = st.y, th = st.z;
    // forward quantities, computed exactly as the forward step computes them
    float gx, gy;
    gradient_2d(Field2D{f0, r.nx}, r, x, y, gx, gy);
    gx *= r.sign0;
    gy *= r.sign0;
    if (NS > 1) {
        float hx, hy;
        gradient_2d(Field2D{f1, r.nx}, r, x, y, hx, hy);
        gx = fmaf(r.sign1, hx, gx);
        gy = fmaf(r.sign1, hy, gy);
    }
    float s, c;
    sincosf(th, &s, &c);
    float cross = r.gain * (c * gy - s * gx);
    const float along = 1.0f + r.gain * (c * gx + s * gy);
    if (cross == 0.0f) cross = 0.0f;
    bool capped;
    const float turn = capped_turn(r, cross, along, &capped);
    float z[2];
    noise_2d(r.key, (uint32_t)i, step, z);
    float thn = th + turn;
    thn = thn + r.sigma * z[0];
    const float two_pi = 6.28318530717958647692f;
    thn = thn - two_pi * floorf((thn + 3.14159265358979323846f) * (1.0f / two_pi));
    float sn, cn;
    sincosf(thn, &sn, &cn);

    // reverse: p' = p + s (cos theta', sin theta')
    const float athn = ath + r.step_len * (cn * apy - sn * apx);
    // theta' = theta + turn(theta, g) + noise
    ath = athn;
    float agx = 0.0f, agy = 0.0f;
    if (!capped) {
        const float den = along * along + cross * cross;
        const float a_cross = athn * along / den, a_along = -athn * cross / den;
        const float dot = c * gx + s * gy;
        ath += a_cross * (-r.gain * dot) + a_along * cross;
        agx = r.gain * (a_along * c - a_cross * s);
        agy = r.gain * (a_cross * c + a_along * s);
    }
    gradient_2d_reverse(f0, af0, r, x, y, r.sign0 * agx, r.sign0 * agy, apx, apy);
    if (NS > 1) gradient_2d_reverse(f1, af1, r, x, y, r.sign1 * agx, r.sign1 * agy, apx, apy);
}

// A checkpoint segment of `len` steps from step seg0: fields[t] (species-major, `cells`
// each) is the field state after t steps of the segment, t = 0..len.
struct Segment2D {
    const float* fields;
    size_t cells;
    int n_species;
    uint32_t seg0;
    int len;
    __device__ const float* field(int t, int s) const {
        return fields + ((size_t)t * n_species + s) * cells;
    }
};

// Forward re-run of one segment's cone steps, one thread per cone over all the steps; the
// state at the start of step t goes to tape[t][i] whether or not the cone is still active.
// Same arithmetic as the forward step (gradient, turn, noise, advance, exit, contact).
template <int NS>
__global__ __launch_bounds__(kSegThreads) void k_cones_segment2d(ConeRules r, Segment2D seg,
                                                                 ConeArrays c,
                                                                 float4* __restrict__ tape) {
    const int i = blockIdx.x * kSegThreads + threadIdx.x;
    if (i >= c.n) return;
    float x = c.pos[2 * i], y = c.pos[2 * i + 1], th = c.dir[i];
    int status = c.status[i];
    for (int t = 0; t < seg.len; ++t) {
        tape[(size_t)t * c.n + i] = make_float4(x, y, th, 0.0f);
        if (status != kActive) continue;
        const float* f0 = seg.field(t + 1, 0);
        float gx, gy;
        gradient_2d(Field2D{f0, r.nx}, r, x, y, gx, gy);
        gx *= r.sign0;
        gy *= r.sign0;
        if (NS > 1) {
            float hx, hy;
            gradient_2d(Field2D{seg.field(t + 1, NS - 1), r.nx}, r, x, y, hx, hy);
            gx = fmaf(r.sign1, hx, gx);
            gy = fmaf(r.sign1, hy, gy);
        }
        float sn, cs;
        sincosf(th, &sn, &cs);
        float z[2];
        noise_2d(r.key, (uint32_t)i, seg.seg0 + (uint32_t)t, z);
        const ConeEvent ev = cone_step_2d(r, gx, gy, 0.0f, z, x, y, th, sn, cs,
                                          GridContact{&r.targets});
        status = ev.status;
    }
}

// Reverse of one segment's cone steps, one thread per cone from the last step to the first.
// status/event_step are the final ones of the run: a cone stopped at step n takes part in
// steps < n only.  The adjoint of the sample of step t goes to e + t * n_species * cells.
template <int NS>
__global__ __launch_bounds__(kSegThreads) void k_cone_adjoint_segment2d(
    ConeRules r, Segment2D seg, float* __restrict__ e, const float4* __restrict__ tape,
    const int32_t* __restrict__ status, const int32_t* __restrict__ event_step,
    float* __restrict__ acone, int n) {
    const int i = blockIdx.x * kSegThreads + threadIdx.x;
    if (i >= n) return;
    // steps < last take part (all steps when the cone is still active)
    const int64_t last = status[i] == kActive ? INT64_MAX : (int64_t)event_step[i];
    float apx = acone[3 * i], apy = acone[3 * i + 1], ath = acone[3 * i + 2];
    for (int t = seg.len - 1; t >= 0; --t) {
        const uint32_t step = seg.seg0 + (uint32_t)t;
        if ((int64_t)step >= last) continue;
        float* et = e + (size_t)t * seg.n_species * seg.cells;
        cone_adjoint_step<NS>(r, seg.field(t + 1, 0), seg.field(t + 1, NS - 1), et,
                              et + (NS - 1) * seg.cells, tape[(size_t)t * n + i], i, step, apx,
                              apy, ath);
    }
    acone[3 * i] = apx;
    acone[3 * i + 1] = apy;
    acone[3 * i + 2] = ath;
}

// Loss at the final tips and the seed of the cone adjoints: a_p = 2 w (p - t), a_theta = 0.
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_seed2d(
    const float* __restrict__ pos, const float* __restrict__ tip_target,
    const float* __restrict__ weight, float* __restrict__ acone, double* __restrict__ partial,
    int n) {
    const int i = blockIdx.x * kAdjThreads + threadIdx.x;
    double l = 0.0;
    if (i < n) {
        const float dx = pos[2 * i] - tip_target[2 * i];
        const float dy = pos[2 * i + 1] - tip_target[2 * i + 1];
        const float w = weight[i];
        acone[3 * i] = 2.0f * w * dx;
        acone[3 * i + 1] = 2.0f * w * dy;
        acone[3 * i + 2] = 0.0f;
        l = (double)w * ((double)dx * dx + (double)dy * dy);
    }
    const double t = adj_block_sum(l);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}


}  // namespace

int adjoint_cone_blocks(int n) { return (n + kAdjThreads - 1) / kAdjThreads; }

hipError_t launch_cones_segment2d(const ConeRules& rules, const float* fields, size_t cells,
                                  int n_species, uint32_t seg0, int len, ConeArrays cones,
                                  float4* tape, hipStream_t stream) {
    if (cones.n == 0 || len == 0) return hipSuccess;
    const Segment2D seg{fields, cells, n_species, seg0, len};
    const dim3 grid((cones.n + kSegThreads - 1) / kSegThreads);
    if (n_species > 1)
        hipLaunchKernelGGL(k_cones_segment2d<2>, grid, dim3(kSegThreads), 0, stream, rules, seg,
                           cones, tape);
    else
        hipLaunchKernelGGL(k_cones_segment2d<1>, grid, dim3(kSegThreads), 0, stream, rules, seg,
                           cones, tape);
    return hipGetLastError();
}

hipError_t launch_cone_adjoint_segment2d(const ConeRules& rules, const float* fields,
                                         size_t cells, int n_species, uint32_t seg0, int len,
                                         float* e, const float4* tape, const int32_t* status,
                                         const int32_t* event_step, float* acone, int n,
                                         hipStream_t stream) {
    if (n == 0 || len == 0) return hipSuccess;
    const Segment2D seg{fields, cells, n_species, seg0, len};
    const dim3 grid((n + kSegThreads - 1) / kSegThreads);
    if (n_species > 1)
        hipLaunchKernelGGL(k_cone_adjoint_segment2d<2>, grid, dim3(kSegThreads), 0, stream,
                           rules, seg, e, tape, status, event_step, acone, n);
    else
        hipLaunchKernelGGL(k_cone_adjoint_segment2d<1>, grid, dim3(kSegThreads), 0, stream,
                           rules, seg, e, tape, status, event_step, acone, n);
    return hipGetLastError();
}

hipError_t launch_adjoint_seed2d(const float* pos, const float* tip_target, const float* weight,
                                 float* acone, double* partial, int n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_seed2d, dim3(adjoint_cone_blocks(n)), dim3(kAdjThreads), 0,
                       stream, pos, tip_target, weight, acone, partial, n);
    return hipGetLastError();
}


}  // namespace cuesim
