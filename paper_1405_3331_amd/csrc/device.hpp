// device.hpp -- device-side pieces of one time step shared by every gfx950 kernel:
// counter-based noise, gradient sampling, the cone turn / advance / exit / contact rule.
// FP32 throughout.  Field access goes through an accessor so the same cone arithmetic
// runs on HBM-resident fields and on LDS tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cuesim {

constexpr int kActive = 0;
constexpr int kContact = 1;
constexpr int kExited = 2;

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the 4x32 S-box, the
// key advanced by the Weyl increments between rounds.  Counter-based and stateless, so
// every cone draws its own stream with no per-thread state in memory (Sec. 5.1).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per S-box multiply gives both halves at once
        const uint64_t pa = (uint64_t)0xD2511F53u * c.x;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb,
                       (uint32_t)(pa >> 32) ^ c.w ^ k1, (uint32_t)pa);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (2m + 1) * 2^-24 with m the top 23 bits: exact in FP32.
__device__ __forceinline__ float unit_open(uint32_t x) {
    return (float)(x >> 9) * 0x1p-23f + 0x1p-24f;
}

// ------------------------------------------------------------------------------------
// sin and cos on a reduced argument |a| <= pi/4 (with a little slack): the Taylor series to
// a^9 and a^10, whose truncation errors (below 1.8e-9 and 1.2e-10 at pi/4) lie far under
// FP32 rounding, in Horner form.  Only fma, mul and add, so every kernel (and a host build)
// gets the same bits.
// ------------------------------------------------------------------------------------
constexpr double kPiD = 3.14159265358979323846;

__host__ __device__ __forceinline__ void sincos_reduced(float a, float& s, float& c) {
    const float a2 = a * a;
    float p = fmaf(a2, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
    p = fmaf(a2, p, (float)(1.0 / 120.0));
    p = fmaf(a2, p, (float)(-1.0 / 6.0));
    s = fmaf(a * a2, p, a);
    float q = fmaf(a2, (float)(-1.0 / 3628800.0), (float)(1.0 / 40320.0));
    q = fmaf(a2, q, (float)(-1.0 / 720.0));
    q = fmaf(a2, q, (float)(1.0 / 24.0));
    q = fmaf(a2, q, -0.5f);
    c = fmaf(a2, q, 1.0f);
}

// Rotate (s, c) = (sin a, cos a) by j quarter turns: the sine and cosine of a + j pi / 2.
__host__ __device__ __forceinline__ void quarter_turns(float j, float& s, float& c) {
    const int q = (int)j & 3;
    const float s0 = (q & 1) ? c : s, c0 = (q & 1) ? s : c;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

// sin and cos of an angle in radians, |th| up to a few turns (headings are kept in
// [-pi, pi)): j = rint(2 th / pi) quarter turns are taken off with pi / 2 split in two FP32
// parts (Cody and Waite), leaving |a| <= pi / 4.
__host__ __device__ __forceinline__ void sincos_angle(float th, float& s, float& c) {
    constexpr float kHalfPiHi = (float)(kPiD / 2.0);
    constexpr float kHalfPiLo = (float)(kPiD / 2.0 - (double)(float)(kPiD / 2.0));
    const float j = rintf(th * (float)(2.0 / kPiD));
    float a = fmaf(-j, kHalfPiHi, th);
    a = fmaf(-j, kHalfPiLo, a);
    sincos_reduced(a, s, c);
    quarter_turns(j, s, c);
}

// sin and cos of 2 pi u for u in (0, 1]: 4u = j + 2 r with j = rint(4u) exactly, and
// r = 2u - j / 2 in [-1/4, 1/4] exact as well (j / 2 is a multiple of a coarser power of two
// than 2u), so the only rounding before the series is that of a = pi r.
__host__ __device__ __forceinline__ void sincos_turn(float u, float& s, float& c) {
    const float t = 2.0f * u;
    const float j = rintf(2.0f * t);
    const float r = fmaf(-0.5f, j, t);
    sincos_reduced((float)kPiD * r, s, c);
    quarter_turns(j, s, c);
}

// One Box-Muller pair from two Philox words: radius sqrt(-2 ln u0) from the first uniform,
// angle 2 pi u1 from the second.  u0 lies in [2^-24, 1), a normal number, and -2 ln u0 in
// (1e-7, 34), so the hardware base-2 logarithm and square root (about one ulp each) need no
// range scaling.
__device__ __forceinline__ void box_muller(uint32_t w0, uint32_t w1, float& z0, float& z1) {
    const float r = __builtin_amdgcn_sqrtf((float)(-2.0 * 0.69314718055994530942) *
                                           __builtin_amdgcn_logf(unit_open(w0)));
    float s, c;
    sincos_turn(unit_open(w1), s, c);
    z0 = r * c;
    z1 = r * s;
}

struct NoiseKey {
    uint32_t k0, k1;       // seed low / high word
    uint32_t sim_index;    // fourth counter word
};

__device__ __forceinline__ void normal_pair(uint32_t w0, uint32_t w1, float* z) {
    box_muller(w0, w1, z[0], z[1]);
}

// 2D draws at most two deviates per step, so one Philox block, counter
// (cone, step / 2, 0, sim_index), serves two steps: its words (x, y) for the even step and
// (z, w) for the odd one.
__device__ __forceinline__ uint4 noise_block_2d(const NoiseKey& key, uint32_t cone,
                                                uint32_t step) {
    return philox4x32_10(make_uint4(cone, step >> 1, 0u, key.sim_index), key.k0, key.k1);
}
__device__ __forceinline__ void noise_2d(const NoiseKey& key, uint32_t cone, uint32_t step,
                                         float* z) {
    const uint4 x = noise_block_2d(key, cone, step);
    if (step & 1u)
        normal_pair(x.z, x.w, z);
    else
        normal_pair(x.x, x.y, z);
}

// Box-Muller pairs (Z0, Z1) from (u0, u1) and (Z2, Z3) from (u2, u3) of the block with
// counter (cone, step, 0, sim_index).  count selects how many deviates are needed (3D: 3).
template <int count>
__device__ __forceinline__ void normals(const NoiseKey& key, uint32_t cone, uint32_t step,
                                        float* z) {
    const uint4 x = philox4x32_10(make_uint4(cone, step, 0u, key.sim_index), key.k0, key.k1);
    float z1, z3;
    box_muller(x.x, x.y, z[0], z1);
    if (count > 1) z[1] = z1;
    if (count > 2) {
        box_muller(x.z, x.w, z[2], z3);
        if (count > 3) z[3] = z3;
    }
}

// ------------------------------------------------------------------------------------
// Static target grid: targets bucketed into cubic cells of side >= contact radius, so a
// 3^dim-cell neighbourhood holds every target that can be within range (the uniform-grid
// broadphase of Secs. 3.3 and 3.5).  pts[k] = (x, y, z, original index as bits).
// ------------------------------------------------------------------------------------
struct TargetGrid {
    const float4* pts;
    const int32_t* cell_start;   // [gx*gy*gz + 1]
    int gx, gy, gz;
    float inv_cell;
    float r;                     // contact radius (FP32)
    float r2;                    // contact radius squared (FP32)
};

// Keep (d2, idx) if it beats the best so far: strictly closer, or equally close with a
// lower original index.  best starts at (r2, -1), so only d2 < r2 is ever accepted.
__device__ __forceinline__ void closer(float d2, int idx, float& best_d2, int& best) {
    if (d2 < best_d2 || (d2 == best_d2 && best >= 0 && idx < best)) {
        best_d2 = d2;
        best = idx;
    }
}

// Squared distance of an offset (dz unused in 2D).
template <int dim>
__device__ __forceinline__ float dist2(float dx, float dy, float dz) {
    const float d2 = fmaf(dy, dy, dx * dx);
    return dim == 3 ? fmaf(dz, dz, d2) : d2;
}

// Nearest target in a list (x, y, z, original index as bits), same rule as below.  The
// smallest squared distance is found first, four targets at a time (the common case: no
// target within reach, decided with one min per target); only a tip with a target in reach
// takes the exact pass with the tie rule.  The squared distances are the same expressions in
// both passes, so the result is that of the exact pass alone.
template <int dim>
__device__ __forceinline__ int contact_in_list(const float4* pts, int n, float r2, float x,
                                               float y, float z) {
    auto d2 = [&](const float4& t) { return dist2<dim>(x - t.x, y - t.y, z - t.z); };
    float m = r2;
    int k = 0;
    for (; k + 4 <= n; k += 4) {
        const float4 a = pts[k], b = pts[k + 1], c = pts[k + 2], e = pts[k + 3];
        m = fminf(m, fminf(fminf(d2(a), d2(b)), fminf(d2(c), d2(e))));
    }
    for (; k < n; ++k) m = fminf(m, d2(pts[k]));
    if (!(m < r2)) return -1;
    float best_d2 = r2;
    int best = -1;
    for (k = 0; k < n; ++k) {
        const float4 t = pts[k];
        closer(d2(t), __float_as_int(t.w), best_d2, best);
    }
    return best;
}

// Target cells along one axis that can hold a target within the contact radius of p: a
// target closer than R differs from p by less than R on every axis, so its cell lies between
// those of p - R and p + R.  The bounds are widened by kCellSlack cells to absorb the FP32
// rounding of (p +- R) / cell, so the search stays exact; usually one or two cells per axis.
constexpr float kCellSlack = 1e-3f;
// The bounds are clamped as floats before the conversion, so a NaN or infinite tip gives an
// empty range (lo > hi) instead of an undefined conversion.
__device__ __forceinline__ void target_cell_range(float p, const TargetGrid& tg, int n, int& lo,
                                                  int& hi) {
    lo = (int)fminf(fmaxf(floorf(fmaf(p - tg.r, tg.inv_cell, -kCellSlack)), 0.0f), (float)n);
    hi = (int)fminf(fmaxf(floorf(fmaf(p + tg.r, tg.inv_cell, kCellSlack)), -1.0f),
                    (float)(n - 1));
}

// Nearest target with squared distance strictly below r2; ties on the squared distance go
// to the lowest original index.  Returns -1 when none is in range.
template <int dim>
__device__ __forceinline__ int contact_target(const TargetGrid& tg, float x, float y, float z) {
    int x_lo, x_hi, y_lo, y_hi, z_lo = 0, z_hi = 0;
    target_cell_range(x, tg, tg.gx, x_lo, x_hi);
    target_cell_range(y, tg, tg.gy, y_lo, y_hi);
    if (dim == 3) target_cell_range(z, tg, tg.gz, z_lo, z_hi);
    float best_d2 = tg.r2;
    int best = -1;
    for (int zz = z_lo; zz <= z_hi; ++zz)
        for (int yy = y_lo; yy <= y_hi; ++yy) {
            const int row = (zz * tg.gy + yy) * tg.gx;
            const int lo = tg.cell_start[row + x_lo];
            const int hi = tg.cell_start[row + x_hi + 1];
            for (int k = lo; k < hi; ++k) {
                const float4 t = tg.pts[k];
                closer(dist2<dim>(x - t.x, y - t.y, z - t.z), __float_as_int(t.w), best_d2,
                       best);
            }
        }
    return best;
}

// ------------------------------------------------------------------------------------
// Rule constants of the cone step (one simulation).
// ------------------------------------------------------------------------------------
struct ConeRules {
    int nx, ny, nz;
    float inv_dx, half_inv_dx;
    float Lx, Ly, Lz;            // domain extent n_a * dx
    float step_len, gain, max_turn, sigma;
    float tan_max;               // tan(max_turn) when max_turn <= kSmallCap, else 0
    int turn_law;                // 0 vector addition, 1 SNR decision (2D)
    float snr_coef;              // SNR law: snr_scale * cone_width
    float inv_kd, c_min, c_max;  // SNR law: 1 / kd and the detection window
    float sign0, sign1;          // species weights in g
    int n_species;
    NoiseKey key;
    TargetGrid targets;
};

// Tip coordinate -> lower corner cell and fraction along one axis (cell centres at
// (i + 1/2) dx; clamped so the tip is interpolated between in-grid centres).
__device__ __forceinline__ void corner(float p, float inv_dx, int n, int& i0, float& f) {
    float u = fmaf(p, inv_dx, -0.5f);
    u = fminf(fmaxf(u, 0.0f), (float)(n - 1));
    i0 = min((int)floorf(u), n - 2);
    f = u - (float)i0;
}

// Accessor concept: F(i, j) / F(i, j, l) returns the cue value of in-grid cell (i, j[, l])
// of one species.

// The footprint of the interpolated 2D gradient at a tip: the lower corner (i0, j0) of the
// 2x2 cell-centre block, the fractions, the clamped indices one beyond each side (ghost =
// own value at a wall) and the 12 cells read: rows j0, j0+1 at columns im, i0, i0+1, ip
// (a, b) and columns i0, i0+1 at rows jm, jp (c, d).
struct Footprint2D {
    int i0, j0, im, ip, jm, jp;
    float fx, fy;
    float a0, a1, a2, a3, b0, b1, b2, b3, c0, c1, d0, d1;
};

template <class F>
__device__ __forceinline__ Footprint2D footprint_2d(const F& f, const ConeRules& r, float x,
                                                    float y) {
    Footprint2D p;
    corner(x, r.inv_dx, r.nx, p.i0, p.fx);
    corner(y, r.inv_dx, r.ny, p.j0, p.fy);
    p.im = max(p.i0 - 1, 0);
    p.ip = min(p.i0 + 2, r.nx - 1);
    p.jm = max(p.j0 - 1, 0);
    p.jp = min(p.j0 + 2, r.ny - 1);
    const int i0 = p.i0, j0 = p.j0;
    p.a0 = f(p.im, j0);
    p.a1 = f(i0, j0);
    p.a2 = f(i0 + 1, j0);
    p.a3 = f(p.ip, j0);
    p.b0 = f(p.im, j0 + 1);
    p.b1 = f(i0, j0 + 1);
    p.b2 = f(i0 + 1, j0 + 1);
    p.b3 = f(p.ip, j0 + 1);
    p.c0 = f(i0, p.jm);
    p.c1 = f(i0 + 1, p.jm);
    p.d0 = f(i0, p.jp);
    p.d1 = f(i0 + 1, p.jp);
    return p;
}

// Central differences at the four corner centres: g?ab at corner (i0 + a, j0 + b).
struct CornerGradients2D {
    float gx00, gx10, gx01, gx11, gy00, gy10, gy01, gy11;
};

__device__ __forceinline__ CornerGradients2D corner_gradients_2d(const Footprint2D& p,
                                                                 const ConeRules& r) {
    CornerGradients2D g;
    g.gx00 = (p.a2 - p.a0) * r.half_inv_dx;
    g.gx10 = (p.a3 - p.a1) * r.half_inv_dx;
    g.gx01 = (p.b2 - p.b0) * r.half_inv_dx;
    g.gx11 = (p.b3 - p.b1) * r.half_inv_dx;
    g.gy00 = (p.b1 - p.c0) * r.half_inv_dx;
    g.gy10 = (p.b2 - p.c1) * r.half_inv_dx;
    g.gy01 = (p.d0 - p.a1) * r.half_inv_dx;
    g.gy11 = (p.d1 - p.a2) * r.half_inv_dx;
    return g;
}

// Bilinear interpolation of the corner gradients (and, if asked, of the cell values).
__device__ __forceinline__ void gradient_from_2d(const Footprint2D& p,
                                                 const CornerGradients2D& g, float& gx,
                                                 float& gy, float* value) {
    const float fx = p.fx, fy = p.fy;
    const float w00 = (1.0f - fx) * (1.0f - fy), w10 = fx * (1.0f - fy);
    const float w01 = (1.0f - fx) * fy, w11 = fx * fy;
    gx = fmaf(w11, g.gx11, fmaf(w01, g.gx01, fmaf(w10, g.gx10, w00 * g.gx00)));
    gy = fmaf(w11, g.gy11, fmaf(w01, g.gy01, fmaf(w10, g.gy10, w00 * g.gy00)));
    // the interpolated concentration itself, from the same corners and weights
    if (value) *value = fmaf(w11, p.b2, fmaf(w01, p.b1, fmaf(w10, p.a2, w00 * p.a1)));
}

// Interpolated central-difference gradient of one species at (x, y).
template <class F>
__device__ __forceinline__ void gradient_2d(const F& f, const ConeRules& r, float x, float y,
                                            float& gx, float& gy, float* value = nullptr) {
    const Footprint2D p = footprint_2d(f, r, x, y);
    gradient_from_2d(p, corner_gradients_2d(p, r), gx, gy, value);
}

// The footprint of the interpolated 3D gradient: the lower corner (i0, j0, l0) of the 2x2x2
// cell-centre block around the tip, the fractions along each axis, and the clamped indices
// one beyond each face (ghost = own value at a wall).
struct Corner3D {
    int i0, j0, l0, im, ip, jm, jp, lm, lp;
    float fx, fy, fz;
};

// The 32 distinct cells of the footprint: the 2x2x2 corner block and, beyond each of its
// faces, the 2x2 cells one further out.
struct Footprint3D {
    float blk[2][2][2], xm[2][2], xp[2][2], ym[2][2], yp[2][2], zm[2][2], zp[2][2];
};

__device__ __forceinline__ Corner3D corner_3d(const ConeRules& r, float x, float y, float z) {
    Corner3D k;
    corner(x, r.inv_dx, r.nx, k.i0, k.fx);
    corner(y, r.inv_dx, r.ny, k.j0, k.fy);
    corner(z, r.inv_dx, r.nz, k.l0, k.fz);
    k.im = max(k.i0 - 1, 0);
    k.ip = min(k.i0 + 2, r.nx - 1);
    k.jm = max(k.j0 - 1, 0);
    k.jp = min(k.j0 + 2, r.ny - 1);
    k.lm = max(k.l0 - 1, 0);
    k.lp = min(k.l0 + 2, r.nz - 1);
    return k;
}

template <class F>
__device__ __forceinline__ Footprint3D load_footprint_3d(const F& f, const Corner3D& k) {
    Footprint3D p;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            p.blk[0][b][c] = f(k.i0, k.j0 + b, k.l0 + c);
            p.blk[1][b][c] = f(k.i0 + 1, k.j0 + b, k.l0 + c);
            p.xm[b][c] = f(k.im, k.j0 + b, k.l0 + c);
            p.xp[b][c] = f(k.ip, k.j0 + b, k.l0 + c);
            p.ym[b][c] = f(k.i0 + b, k.jm, k.l0 + c);      // [x offset][z offset]
            p.yp[b][c] = f(k.i0 + b, k.jp, k.l0 + c);
            p.zm[b][c] = f(k.i0 + b, k.j0 + c, k.lm);      // [x offset][y offset]
            p.zp[b][c] = f(k.i0 + b, k.j0 + c, k.lp);
        }
    return p;
}

// Trilinear interpolation of the central differences at the eight corners.
__device__ __forceinline__ void gradient_from_3d(const ConeRules& r, const Corner3D& k,
                                                 const Footprint3D& p, float& gx, float& gy,
                                                 float& gz) {
    const float fx = k.fx, fy = k.fy, fz = k.fz;
    gx = gy = gz = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float w = (a ? fx : 1.0f - fx) * (b ? fy : 1.0f - fy) * (c ? fz : 1.0f - fz);
                // central differences at corner (i0+a, j0+b, l0+c)
                const float ex = (a ? p.xp[b][c] : p.blk[1][b][c]) - (a ? p.blk[0][b][c] : p.xm[b][c]);
                const float ey = (b ? p.yp[a][c] : p.blk[a][1][c]) - (b ? p.blk[a][0][c] : p.ym[a][c]);
                const float ez = (c ? p.zp[a][b] : p.blk[a][b][1]) - (c ? p.blk[a][b][0] : p.zm[a][b]);
                gx = fmaf(w, ex, gx);
                gy = fmaf(w, ey, gy);
                gz = fmaf(w, ez, gz);
            }
    gx *= r.half_inv_dx;
    gy *= r.half_inv_dx;
    gz *= r.half_inv_dx;
}

template <class F>
__device__ __forceinline__ void gradient_3d(const F& f, const ConeRules& r, float x, float y,
                                            float z, float& gx, float& gy, float& gz) {
    const Corner3D k = corner_3d(r, x, y, z);
    gradient_from_3d(r, k, load_footprint_3d(f, k), gx, gy, gz);
}

struct ConeEvent {
    int status;   // kActive / kContact / kExited after the step
    int target;   // contacted target or -1
};

// Contact test against the simulation's whole target grid.
struct GridContact {
    const TargetGrid* tg;
    template <int dim>
    __device__ int find(float x, float y, float z) const { return contact_target<dim>(*tg, x, y, z); }
};

// Caps up to this angle take the small-angle path of capped_turn (tan(0.19) < 0.2).
constexpr float kSmallCap = 0.19f;

// The capped turn toward h + gain*g: atan2(cross, along) clamped to +-max_turn, with
// cross = gain (h x g) and along = 1 + gain (h . g) (cross = -0 already replaced by +0).
// For a small cap the clamp is decided first: the angle exceeds the cap exactly when
// along <= 0 or |cross| >= along tan(max_turn); otherwise t = cross / along is below
// tan(max_turn) < 0.2 and atan(t) is its Taylor series to t^11 (truncation below 2e-9 t,
// under FP32 rounding).  *capped tells whether the clamp was applied.
__device__ __forceinline__ float capped_turn(const ConeRules& r, float cross, float along,
                                             bool* capped) {
    if (r.tan_max > 0.0f) {
        if (along > 0.0f && fabsf(cross) < along * r.tan_max) {
            *capped = false;
            const float t = cross * __builtin_amdgcn_rcpf(along);   // reciprocal: ~1 ulp
            const float t2 = t * t;
            float p = fmaf(t2, -1.0f / 11.0f, 1.0f / 9.0f);
            p = fmaf(t2, p, -1.0f / 7.0f);
            p = fmaf(t2, p, 1.0f / 5.0f);
            p = fmaf(t2, p, -1.0f / 3.0f);
            return fmaf(t * t2, p, t);
        }
        *capped = true;
        return cross >= 0.0f ? r.max_turn : -r.max_turn;
    }
    const float turn = atan2f(cross, along);
    *capped = turn > r.max_turn || turn < -r.max_turn;
    return fminf(fmaxf(turn, -r.max_turn), r.max_turn);
}

// The SNR turn law (Sec. 3.5, Eq. 5): inside the detection window [c_min, c_max] of the
// concentration c at the tip, turn by max_turn to the right (clockwise) when SNR + z0 > 0,
// else to the left, with SNR = A w / c * sqrt(gamma / (1 + gamma)^3) * |g| sin(theta -
// theta_g), gamma = c / kd; |g| sin(theta - theta_g) = sin(theta) g_x - cos(theta) g_y.
// Outside the window, or with no gradient, no turn.
__device__ __forceinline__ float snr_turn(const ConeRules& r, float s, float c, float gx,
                                          float gy, float conc, float z0) {
    if (!(conc >= r.c_min && conc <= r.c_max) || (gx == 0.0f && gy == 0.0f)) return 0.0f;
    const float gamma = conc * r.inv_kd;
    const float one = 1.0f + gamma;
    const float snr =
        r.snr_coef / conc * sqrtf(gamma / (one * one * one)) * fmaf(s, gx, -(c * gy));
    return snr + z0 > 0.0f ? -r.max_turn : r.max_turn;
}

// The two terms of the vector-law turn toward h + gain*g, h = (c, s) the heading:
// cross = gain (h x g) and along = 1 + gain (h . g), with cross = -0 replaced by +0 (an
// anti-parallel pull turns by +cap).  Shared by the forward step and its reverse, which must
// see the same branch.
__device__ __forceinline__ void turn_terms(const ConeRules& r, float s, float c, float gx,
                                           float gy, float& cross, float& along) {
    cross = r.gain * fmaf(c, gy, -(s * gx));
    along = fmaf(r.gain, fmaf(c, gx, s * gy), 1.0f);
    if (cross == 0.0f) cross = 0.0f;
}

// A heading wrapped back into [-pi, pi).
__device__ __forceinline__ float wrap_heading(float th) {
    const float two_pi = 6.28318530717958647692f;
    return fmaf(-two_pi, floorf((th + 3.14159265358979323846f) * (1.0f / two_pi)), th);
}

// One step of an active 2D cone: turn toward h + gain*g (capped) -- or by the SNR law's
// decision, which also needs the concentration `conc` of species 0 at the tip -- noise,
// advance, exit, contact.  z is the step's normal pair (noise_2d).  `contact` finds the
// nearest target in range (GridContact, or a list staged in LDS).  (s, c) carry
// sincos_angle(theta) in and that of the new heading out, so a caller stepping a cone
// repeatedly evaluates it once per step.
template <class Contact>
__device__ __forceinline__ ConeEvent cone_step_2d(const ConeRules& r, float gx, float gy,
                                                  float conc, const float* z, float& x,
                                                  float& y, float& theta, float& s, float& c,
                                                  const Contact& contact) {
    float th;
    if (r.turn_law == 1) {
        th = theta + snr_turn(r, s, c, gx, gy, conc, z[0]);
        th = fmaf(r.sigma, z[1], th);
    } else {
        float cross, along;
        turn_terms(r, s, c, gx, gy, cross, along);
        bool capped;
        const float turn = capped_turn(r, cross, along, &capped);
        th = theta + turn;
        th = fmaf(r.sigma, z[0], th);
    }
    th = wrap_heading(th);
    theta = th;
    sincos_angle(th, s, c);
    x = fmaf(r.step_len, c, x);
    y = fmaf(r.step_len, s, y);
    ConeEvent ev{kActive, -1};
    if (x < 0.0f || x >= r.Lx || y < 0.0f || y >= r.Ly) {
        ev.status = kExited;
        return ev;
    }
    const int t = contact.template find<2>(x, y, 0.0f);
    if (t >= 0) {
        ev.status = kContact;
        ev.target = t;
    }
    return ev;
}

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by,
                                      float bz) {
    return fmaf(az, bz, fmaf(ay, by, ax * bx));
}

// One step of an active 3D cone with unit heading (hx, hy, hz).
template <class Contact>
__device__ __forceinline__ ConeEvent cone_step_3d(const ConeRules& r, float gx, float gy,
                                                  float gz, uint32_t id, uint32_t step,
                                                  float& x, float& y, float& z, float& hx,
                                                  float& hy, float& hz,
                                                  const Contact& contact) {
    // turn in the plane of h and g, toward h + gain*g, by at most max_turn
    const float gh = dot3(gx, gy, gz, hx, hy, hz);
    const float px = fmaf(-gh, hx, gx), py = fmaf(-gh, hy, gy), pz = fmaf(-gh, hz, gz);
    const float pn = sqrtf(dot3(px, py, pz, px, py, pz));
    if (pn > 0.0f) {
        float phi = atan2f(r.gain * pn, fmaf(r.gain, gh, 1.0f));
        phi = fminf(phi, r.max_turn);
        float s, c;
        sincos_angle(phi, s, c);
        const float k = s / pn;
        hx = fmaf(c, hx, k * px);
        hy = fmaf(c, hy, k * py);
        hz = fmaf(c, hz, k * pz);
    }
    // tangent-plane Gaussian rotation
    float zn[3];
    normals<3>(r.key, id, step, zn);
    const float zh = dot3(zn[0], zn[1], zn[2], hx, hy, hz);
    const float wx = r.sigma * fmaf(-zh, hx, zn[0]);
    const float wy = r.sigma * fmaf(-zh, hy, zn[1]);
    const float wz = r.sigma * fmaf(-zh, hz, zn[2]);
    const float wn = sqrtf(dot3(wx, wy, wz, wx, wy, wz));
    if (wn > 0.0f) {
        float s, c;
        sincos_angle(wn, s, c);
        const float k = s / wn;
        hx = fmaf(c, hx, k * wx);
        hy = fmaf(c, hy, k * wy);
        hz = fmaf(c, hz, k * wz);
    }
    const float inv = 1.0f / sqrtf(dot3(hx, hy, hz, hx, hy, hz));
    hx *= inv;
    hy *= inv;
    hz *= inv;
    x = fmaf(r.step_len, hx, x);
    y = fmaf(r.step_len, hy, y);
    z = fmaf(r.step_len, hz, z);
    ConeEvent ev{kActive, -1};
    if (x < 0.0f || x >= r.Lx || y < 0.0f || y >= r.Ly || z < 0.0f || z >= r.Lz) {
        ev.status = kExited;
        return ev;
    }
    const int t = contact.template find<3>(x, y, z);
    if (t >= 0) {
        ev.status = kContact;
        ev.target = t;
    }
    return ev;
}

}  // namespace cuesim
