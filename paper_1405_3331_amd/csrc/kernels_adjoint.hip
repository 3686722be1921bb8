// kernels_adjoint.hip -- reverse pass of the 2D time step, for the gradient of a trajectory
// loss L = sum_i w_i |p_i^N - t_a(i)|^2 with respect to the source amounts, D and k.
//
// The derivative is taken along the forward run's branch: the exit and contact decisions
// and the active side of the turn cap are held as the forward run took them (the cone
// rules of Sec. 3.4-3.5 have no derivative at those switches).
//
// The fields never depend on the cones, so within a checkpoint segment the cones can be
// handled apart from the fields, each cone by one thread over all the segment's steps:
//   k_cones_segments2d        re-runs the segment's cone steps against the re-run fields and
//                             records (x, y, theta) of every cone at the start of each step
//                             (when the whole run's fields fit in memory, every segment at
//                             once, one thread per segment and cone);
//   k_cone_adjoint_segment2d  walks the steps backwards carrying each cone's adjoint of
//                             (p, theta) through advance, capped turn and interpolated
//                             gradient, and records its gradient samples' adjoints (12
//                             cells and values per species, cone and step);
//   k_sample_max, k_sample_add  add the records of every step into e^{n+1}, one buffer of
//                             64-bit fixed-point sums per step and species, scaled by the
//                             step's largest contribution: integer additions, so the sums
//                             (and the whole gradient) do not depend on the order in which
//                             the cones' contributions arrive.  The sums are added a few
//                             steps at a time, just before those steps are reversed, into a
//                             small ring of per-step buffers (the reverse field launches
//                             clear the buffers they are done with);
//   k_field_adjoint2d_pair    (kernels_field2d.hip) two reverse steps per launch, and
//   k_field_adjoint2d_rows    one for the first step of a segment of odd length: with
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
constexpr int kSegThreads = 64;   // segment kernels: one wavefront per workgroup.  With the
                                  // reverse walk loading footprints a step ahead, a gradient's
                                  // reverse sweep at 1024^2 (8192 cones) takes 21.4-21.6 ms,
                                  // against 21.7-21.8 with 32 threads and 23.0 with 16; half-wave
                                  // workgroups were ~1.5% faster before that prefetch

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

// The adjoints of one gradient sample's 12 loaded cells: adds to af[at[k]] of v[k].
struct Scatter2D {
    int at[12];
    float v[12];
};

// Record of one sample's adjoints: rec_at / rec_v + ((t * n + i) * n_species + s) * 12.
__device__ __forceinline__ void write_record(int32_t* __restrict__ at, float* __restrict__ v,
                                             const Scatter2D& s) {
#pragma unroll
    for (int k = 0; k < 12; k += 4) {
        *(int4*)(at + k) = make_int4(s.at[k], s.at[k + 1], s.at[k + 2], s.at[k + 3]);
        *(float4*)(v + k) = make_float4(s.v[k], s.v[k + 1], s.v[k + 2], s.v[k + 3]);
    }
}

// Reverse of the interpolated central-difference gradient of one species at (x, y), from
// the footprint and corner gradients the forward sample used.  (agx, agy) is the adjoint of
// the sampled gradient, already weighted by the species sign.  Adds the adjoint of the tip
// position into (apx, apy) -- the interpolation weights depend on the tip; along an axis
// where the tip is clamped to the outermost centres they do not -- and returns the adjoint
// of the 12 loaded values (cells repeat at walls; their adds then combine).
__device__ __forceinline__ Scatter2D gradient_2d_reverse(const Footprint2D& p,
                                                         const CornerGradients2D& g,
                                                         const ConeRules& r, float x, float y,
                                                         float agx, float agy, float& apx,
                                                         float& apy) {
    const float fx = p.fx, fy = p.fy;
    const float ux = fmaf(x, r.inv_dx, -0.5f), uy = fmaf(y, r.inv_dx, -0.5f);
    const bool free_x = ux > 0.0f && ux < (float)(r.nx - 1);
    const bool free_y = uy > 0.0f && uy < (float)(r.ny - 1);
    const int nx = r.nx, i0 = p.i0, j0 = p.j0;
    const float w00 = (1.0f - fx) * (1.0f - fy), w10 = fx * (1.0f - fy);
    const float w01 = (1.0f - fx) * fy, w11 = fx * fy;
    // position: d w / d f along each axis, times d f / d p = 1 / dx where not clamped
    const float aw00 = fmaf(agy, g.gy00, agx * g.gx00), aw10 = fmaf(agy, g.gy10, agx * g.gx10);
    const float aw01 = fmaf(agy, g.gy01, agx * g.gx01), aw11 = fmaf(agy, g.gy11, agx * g.gx11);
    if (free_x) apx = fmaf(r.inv_dx, fmaf(fy, aw11 - aw01, (1.0f - fy) * (aw10 - aw00)), apx);
    if (free_y) apy = fmaf(r.inv_dx, fmaf(fx, aw11 - aw10, (1.0f - fx) * (aw01 - aw00)), apy);
    // field: each loaded value's adjoint
    const float h = r.half_inv_dx;
    const float hx = h * agx, hy = h * agy;
    const int r0 = j0 * nx, r1 = r0 + nx;
    Scatter2D s;
    s.at[0] = r0 + p.im;      s.v[0] = -w00 * hx;
    s.at[1] = r0 + i0;        s.v[1] = fmaf(-w10, hx, -(w01 * hy));
    s.at[2] = r0 + i0 + 1;    s.v[2] = fmaf(w00, hx, -(w11 * hy));
    s.at[3] = r0 + p.ip;      s.v[3] = w10 * hx;
    s.at[4] = r1 + p.im;      s.v[4] = -w01 * hx;
    s.at[5] = r1 + i0;        s.v[5] = fmaf(-w11, hx, w00 * hy);
    s.at[6] = r1 + i0 + 1;    s.v[6] = fmaf(w01, hx, w10 * hy);
    s.at[7] = r1 + p.ip;      s.v[7] = w11 * hx;
    s.at[8] = p.jm * nx + i0; s.v[8] = -w00 * hy;
    s.at[9] = s.at[8] + 1;    s.v[9] = -w10 * hy;
    s.at[10] = p.jp * nx + i0; s.v[10] = w01 * hy;
    s.at[11] = s.at[10] + 1;  s.v[11] = w11 * hy;
    return s;
}

struct Field2D {
    const float* f;
    int nx;
    __device__ float operator()(int i, int j) const { return f[j * nx + i]; }
};

// Reverse of one cone step (step index `step`) of cone i from its state (x, y, theta) at
// the start of the step, the footprints p0/p1 of its gradient samples in the fields after
// the step's field update, their corner gradients and the weighted gradient (gx, gy).  (apx, apy, ath) holds the adjoint of the state after the
// step on entry and of the state before it on exit; out[s] receives the adjoints of species
// s's sampled cells.
template <int NS>
__device__ __forceinline__ void cone_adjoint_step(const ConeRules& r, const Footprint2D& p0,
                                                  const Footprint2D& p1,
                                                  const CornerGradients2D& g0,
                                                  const CornerGradients2D& g1, float gx,
                                                  float gy, float4 st, int i, uint32_t step,
                                                  float& apx, float& apy, float& ath,
                                                  Scatter2D* out) {
    const float x = st.x, y = st.y, th = st.z;
    float s, c;
    sincos_angle(th, s, c);
    float cross, along;
    turn_terms(r, s, c, gx, gy, cross, along);
    bool capped;
    const float turn = capped_turn(r, cross, along, &capped);
    float z[2];
    noise_2d(r.key, (uint32_t)i, step, z);
    const float thn = wrap_heading(fmaf(r.sigma, z[0], th + turn));
    float sn, cn;
    sincos_angle(thn, sn, cn);

    // reverse: p' = p + s (cos theta', sin theta')
    const float athn = fmaf(r.step_len, fmaf(cn, apy, -(sn * apx)), ath);
    // theta' = theta + turn(theta, g) + noise
    ath = athn;
    float agx = 0.0f, agy = 0.0f;
    if (!capped) {
        const float den = fmaf(along, along, cross * cross);
        const float a_cross = athn * along / den, a_along = -athn * cross / den;
        const float dot = fmaf(c, gx, s * gy);
        ath = fmaf(a_cross, -r.gain * dot, fmaf(a_along, cross, ath));
        agx = r.gain * fmaf(a_along, c, -(a_cross * s));
        agy = r.gain * fmaf(a_cross, c, a_along * s);
    }
    out[0] = gradient_2d_reverse(p0, g0, r, x, y, r.sign0 * agx, r.sign0 * agy, apx, apy);
    if (NS > 1)
        out[NS - 1] = gradient_2d_reverse(p1, g1, r, x, y, r.sign1 * agx, r.sign1 * agy, apx,
                                          apy);
}

// The forward gradient sample of a step from its footprints, computed exactly as the
// forward step computes it.
template <int NS>
__device__ __forceinline__ void sample_2d(const ConeRules& r, const Footprint2D& p0,
                                          const Footprint2D& p1, CornerGradients2D& g0,
                                          CornerGradients2D& g1, float& gx, float& gy) {
    g0 = corner_gradients_2d(p0, r);
    g1 = NS > 1 ? corner_gradients_2d(p1, r) : g0;
    gradient_from_2d(p0, g0, gx, gy, nullptr);
    gx *= r.sign0;
    gy *= r.sign0;
    if (NS > 1) {
        float hx, hy;
        gradient_from_2d(p1, g1, hx, hy, nullptr);
        gx = fmaf(r.sign1, hx, gx);
        gy = fmaf(r.sign1, hy, gy);
    }
}

// A checkpoint segment of `len` steps from step seg0: fields[t] (species-major, `cells`
// each) is the field state after t steps of the segment, t = 0..len.
// Segments of a checkpointed run of n_steps steps from step n0, every `every` steps: run
// step t's field state (after t steps) is fields + ((t - t_base) * n_species + s) * cells;
// the checkpoint arrays hold each segment's cone state at its first step.
struct SegmentSet2D {
    const float* fields;
    size_t cells;
    int n_species;
    int t_base;
    int seg_first, every, n_steps;
    uint32_t n0;
    const float* ckpt_pos;         // [segments][M][2]
    const float* ckpt_dir;         // [segments][M]
    const int32_t* ckpt_status;    // [segments][3][M]: status first
    int M;
    __device__ const float* field(int t, int s) const {
        return fields + ((size_t)(t - t_base) * n_species + s) * cells;
    }
};

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

// Forward re-run of the cone steps of segments seg_first .. seg_first + gridDim.y - 1, one
// thread per (segment, cone) over all the segment's steps, each starting from its
// checkpoint; the state at the start of run step t goes to tape[t - t_base][i] whether or
// not the cone is still active.  Same arithmetic as the forward step (gradient, turn,
// noise, advance, exit, contact).
template <int NS>
__global__ __launch_bounds__(kSegThreads) void k_cones_segments2d(ConeRules r, SegmentSet2D set,
                                                                  float4* __restrict__ tape) {
    const int i = blockIdx.x * kSegThreads + threadIdx.x;
    if (i >= set.M) return;
    const int seg = set.seg_first + (int)blockIdx.y;
    const int t0 = seg * set.every;
    const int t1 = min(t0 + set.every, set.n_steps);
    const size_t M = (size_t)set.M;
    float x = set.ckpt_pos[((size_t)seg * M + i) * 2];
    float y = set.ckpt_pos[((size_t)seg * M + i) * 2 + 1];
    float th = set.ckpt_dir[(size_t)seg * M + i];
    int status = set.ckpt_status[(size_t)seg * 3 * M + i];
    for (int t = t0; t < t1; ++t) {
        tape[(size_t)(t - set.t_base) * M + i] = make_float4(x, y, th, 0.0f);
        if (status != kActive) continue;
        const float* f0 = set.field(t + 1, 0);
        float gx, gy;
        gradient_2d(Field2D{f0, r.nx}, r, x, y, gx, gy);
        gx *= r.sign0;
        gy *= r.sign0;
        if (NS > 1) {
            float hx, hy;
            gradient_2d(Field2D{set.field(t + 1, NS - 1), r.nx}, r, x, y, hx, hy);
            gx = fmaf(r.sign1, hx, gx);
            gy = fmaf(r.sign1, hy, gy);
        }
        float sn, cs;
        sincos_angle(th, sn, cs);
        float z[2];
        noise_2d(r.key, (uint32_t)i, set.n0 + (uint32_t)t, z);
        const ConeEvent ev = cone_step_2d(r, gx, gy, 0.0f, z, x, y, th, sn, cs,
                                          GridContact{&r.targets});
        status = ev.status;
    }
}

// Last step of a segment (from step seg0, len steps) in which cone i takes part: status and
// event_step are the run's final ones, and a cone stopped at step n takes part in steps < n
// only (-1: none of the segment's).
__device__ __forceinline__ int last_step(const Segment2D& seg, const int32_t* status,
                                         const int32_t* event_step, int i) {
    const int64_t last = status[i] == kActive ? INT64_MAX : (int64_t)event_step[i];
    return (int)max<int64_t>(min<int64_t>(seg.len - 1, last - 1 - (int64_t)seg.seg0), -1);
}

// Reverse of one segment's cone steps, one thread per cone from the last step to the first;
// the adjoints of step t's gradient samples are recorded (write_record) for k_sample_add.
// The forward states come from the run's cone tape, so the gathers of the step before do
// not wait for this step's adjoint: its footprints are loaded one step ahead and its state
// two.
template <int NS>
__global__ __launch_bounds__(kSegThreads) void k_cone_adjoint_segment2d(
    ConeRules r, Segment2D seg, int32_t* __restrict__ rec_at, float* __restrict__ rec_v,
    const float4* __restrict__ tape, const int32_t* __restrict__ status,
    const int32_t* __restrict__ event_step, float* __restrict__ acone, int n) {
    const int i = blockIdx.x * kSegThreads + threadIdx.x;
    if (i >= n) return;
    float apx = acone[3 * i], apy = acone[3 * i + 1], ath = acone[3 * i + 2];
    const int t_hi = last_step(seg, status, event_step, i);
    if (t_hi >= 0) {
        float4 st = tape[(size_t)t_hi * n + i];
        float4 next = tape[(size_t)max(t_hi - 1, 0) * n + i];
        Footprint2D p0 = footprint_2d(Field2D{seg.field(t_hi + 1, 0), r.nx}, r, st.x, st.y);
        Footprint2D p1 =
            NS > 1 ? footprint_2d(Field2D{seg.field(t_hi + 1, NS - 1), r.nx}, r, st.x, st.y)
                   : p0;
        for (int t = t_hi; t >= 0; --t) {
            // the step before: its state two steps ahead and its footprints one step ahead,
            // requested before this step's arithmetic (the samples do not depend on it)
            const float4 next2 = tape[(size_t)max(t - 2, 0) * n + i];
            Footprint2D q0 = p0, q1 = p1;
            if (t > 0) {
                q0 = footprint_2d(Field2D{seg.field(t, 0), r.nx}, r, next.x, next.y);
                q1 = NS > 1 ? footprint_2d(Field2D{seg.field(t, NS - 1), r.nx}, r, next.x,
                                           next.y)
                            : q0;
            }
            CornerGradients2D g0, g1;
            float gx, gy;
            sample_2d<NS>(r, p0, p1, g0, g1, gx, gy);
            Scatter2D out[NS];
            cone_adjoint_step<NS>(r, p0, p1, g0, g1, gx, gy, st, i, seg.seg0 + (uint32_t)t,
                                  apx, apy, ath, out);
            const size_t rec = (((size_t)t * n + i) * NS) * 12;
#pragma unroll
            for (int s = 0; s < NS; ++s) write_record(rec_at + rec + s * 12, rec_v + rec + s * 12,
                                                      out[s]);
            st = next;
            next = next2;
            p0 = q0;
            p1 = q1;
        }
    }
    acone[3 * i] = apx;
    acone[3 * i + 1] = apy;
    acone[3 * i + 2] = ath;
}

constexpr int kRecThreads = 256;

// Largest |contribution| of every step of the segment: a workgroup takes kMaxCones cones of
// one step (kMaxCones / kRecThreads per thread), reduces their maximum through the wavefronts
// and LDS, and applies one atomic maximum on the step's FP32 bits (non-negative floats order
// like their bits).  Few atomics meet on each step's word: with one per wavefront (128 per
// step at 8192 cones) they queued on those words, and a gradient's reverse sweep at 1024^2
// took 23.5 instead of 22.5 ms.
constexpr int kMaxCones = 8 * kRecThreads;

template <int NS>
__global__ __launch_bounds__(kRecThreads) void k_sample_max(
    Segment2D seg, const float* __restrict__ rec_v, const int32_t* __restrict__ status,
    const int32_t* __restrict__ event_step, uint32_t* __restrict__ step_max, int n) {
    const int t = blockIdx.y;
    float m = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxCones / kRecThreads; ++k) {
        const int i = blockIdx.x * kMaxCones + k * kRecThreads + threadIdx.x;
        if (i < n && t <= last_step(seg, status, event_step, i)) {
            const float4* v = (const float4*)(rec_v + (((size_t)t * n + i) * NS) * 12);
#pragma unroll
            for (int q = 0; q < 3 * NS; ++q) {
                const float4 x = v[q];
                m = fmaxf(m, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    __shared__ float wave_max[kRecThreads / 64];
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRecThreads / 64; ++w) m = fmaxf(m, wave_max[w]);
        if (m > 0.0f) atomicMax(&step_max[t], __float_as_uint(m));
    }
}

// Every (cone, step) record of steps t_lo .. t_lo + gridDim.y - 1 added into the step's
// fixed-point sums (slot t % ring of e): q = rint(v 2^(40 - e)) (the product is an exact
// power-of-two scaling in FP64), |q| <= 2^40.
template <int NS>
__global__ __launch_bounds__(kRecThreads) void k_sample_add(
    Segment2D seg, int t_lo, int ring, const int32_t* __restrict__ rec_at,
    const float* __restrict__ rec_v, const int32_t* __restrict__ status,
    const int32_t* __restrict__ event_step, const uint32_t* __restrict__ step_max,
    unsigned long long* __restrict__ e, int n) {
    const int i = blockIdx.x * kRecThreads + threadIdx.x;
    const int t = t_lo + blockIdx.y;
    if (i >= n || t > last_step(seg, status, event_step, i)) return;
    const size_t rec = (((size_t)t * n + i) * NS) * 12;
    // the whole record first (16-byte loads, all in flight together), then the additions
    float4 v[3 * NS];
    int4 at[3 * NS];
#pragma unroll
    for (int k = 0; k < 3 * NS; ++k) {
        v[k] = ((const float4*)(rec_v + rec))[k];
        at[k] = ((const int4*)(rec_at + rec))[k];
    }
    const double scale = ldexp(1.0, kFixedBits - fixed_exponent(step_max[t]));
#pragma unroll
    for (int k = 0; k < 12 * NS; ++k) {
        unsigned long long* dst = e + ((size_t)(t % ring) * NS + k / 12) * seg.cells;
        const float4 vq = v[k / 4];
        const int4 aq = at[k / 4];
        const float val = k % 4 == 0 ? vq.x : k % 4 == 1 ? vq.y : k % 4 == 2 ? vq.z : vq.w;
        const int cell = k % 4 == 0 ? aq.x : k % 4 == 1 ? aq.y : k % 4 == 2 ? aq.z : aq.w;
        const double x = (double)val * scale;
        // (a non-finite contribution, possible only from non-finite fields, adds nothing
        // rather than an undefined conversion)
        const long long q = isfinite(x) ? (long long)rint(x) : 0;
        if (q != 0) atomicAdd(dst + cell, (unsigned long long)q);
    }
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

hipError_t launch_cones_segments2d(const ConeRules& rules, const float* fields, size_t cells,
                                   int n_species, int t_base, int seg_first, int n_seg,
                                   int every, int n_steps, uint32_t n0, const float* ckpt_pos,
                                   const float* ckpt_dir, const int32_t* ckpt_int, int M,
                                   float4* tape, hipStream_t stream) {
    if (M == 0 || n_seg == 0) return hipSuccess;
    const SegmentSet2D set{fields, cells, n_species, t_base, seg_first, every, n_steps, n0,
                           ckpt_pos, ckpt_dir, ckpt_int, M};
    const dim3 grid((M + kSegThreads - 1) / kSegThreads, n_seg);
    if (n_species > 1)
        hipLaunchKernelGGL(k_cones_segments2d<2>, grid, dim3(kSegThreads), 0, stream, rules,
                           set, tape);
    else
        hipLaunchKernelGGL(k_cones_segments2d<1>, grid, dim3(kSegThreads), 0, stream, rules,
                           set, tape);
    return hipGetLastError();
}

hipError_t launch_cone_adjoint_segment2d(const ConeRules& rules, const float* fields,
                                         size_t cells, int n_species, uint32_t seg0, int len,
                                         int32_t* rec_at, float* rec_v, uint32_t* step_max,
                                         const float4* tape, const int32_t* status,
                                         const int32_t* event_step, float* acone, int n,
                                         hipStream_t stream) {
    if (len == 0) return hipSuccess;
    hipError_t err = hipMemsetAsync(step_max, 0, sizeof(uint32_t) * (size_t)len, stream);
    if (err != hipSuccess || n == 0) return err;
    const Segment2D seg{fields, cells, n_species, seg0, len};
    const dim3 grid((n + kSegThreads - 1) / kSegThreads);
    const dim3 max_grid((n + kMaxCones - 1) / kMaxCones, len);
    if (n_species > 1) {
        hipLaunchKernelGGL(k_cone_adjoint_segment2d<2>, grid, dim3(kSegThreads), 0, stream,
                           rules, seg, rec_at, rec_v, tape, status, event_step, acone, n);
        hipLaunchKernelGGL(k_sample_max<2>, max_grid, dim3(kRecThreads), 0, stream, seg, rec_v,
                           status, event_step, step_max, n);
    } else {
        hipLaunchKernelGGL(k_cone_adjoint_segment2d<1>, grid, dim3(kSegThreads), 0, stream,
                           rules, seg, rec_at, rec_v, tape, status, event_step, acone, n);
        hipLaunchKernelGGL(k_sample_max<1>, max_grid, dim3(kRecThreads), 0, stream, seg, rec_v,
                           status, event_step, step_max, n);
    }
    return hipGetLastError();
}

hipError_t launch_sample_add2d(size_t cells, int n_species, uint32_t seg0, int len, int t_lo,
                               int n_steps, int ring, const int32_t* rec_at, const float* rec_v,
                               const uint32_t* step_max, long long* e, const int32_t* status,
                               const int32_t* event_step, int n, hipStream_t stream) {
    if (n == 0 || n_steps <= 0) return hipSuccess;
    const Segment2D seg{nullptr, cells, n_species, seg0, len};
    const dim3 rec_grid((n + kRecThreads - 1) / kRecThreads, n_steps);
    unsigned long long* eu = (unsigned long long*)e;
    if (n_species > 1)
        hipLaunchKernelGGL(k_sample_add<2>, rec_grid, dim3(kRecThreads), 0, stream, seg, t_lo,
                           ring, rec_at, rec_v, status, event_step, step_max, eu, n);
    else
        hipLaunchKernelGGL(k_sample_add<1>, rec_grid, dim3(kRecThreads), 0, stream, seg, t_lo,
                           ring, rec_at, rec_v, status, event_step, step_max, eu, n);
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
