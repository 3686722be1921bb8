// kernels_field2d.hip -- one explicit 2D field step per launch (every species, sources
// included) and its reverse for the gradient sweep, both marching up the rows.
//
// A workgroup owns kRX columns x kRY rows (kAY for the reverse) of one species; each thread
// keeps the rows below, at and above its cell in registers and reads its two row neighbours
// from lines the workgroup has just brought into L1, so a cell is fetched from HBM about
// once.  Rows are taken in groups with every load of a group issued before the arithmetic.  A
// missing neighbour at a wall is the cell itself (clamped index).  The stencil expression
// is term for term the one of the temporally blocked kernel, so both paths give the same
// bits.  Boxes are dealt to the accelerator dies in contiguous stretches.
//
// Step (Sec. 3.4 cue field: diffusion with first-order decay and point sources):
//   c' = c + r ((w + e) + (s + n) - 4c) - k dt c, then c' += q / dx^2 at each source cell
//   (a separate FP32 add, the rounding of a source pass), from a per-box list built once.
//   Where every state is kept (the gradient sweep's re-run), k_field2d_pair takes two steps
//   per launch: a box of 256 x 4 cells holds c^n on the box and a two-cell ring in LDS,
//   steps the box and a one-cell ring (with the sources there), writes c^{n+1}, steps the
//   box again and writes c^{n+2}: 12 instead of 16 B per cell and two steps, same bits.
// Reverse, with b = a^{n+1} + e^{n+1} (e: the cone samples' adjoints of the step):
//   a^n = b + r Lap b - k dt b, and per-workgroup FP64 sums of b Lap c^n and b c^n.  Two
//   reverse steps are taken per launch where the segment allows (k_field_adjoint2d_pair):
//   a box of 256 x 4 cells holds b^{n+1} on the box and a two-cell ring in LDS, takes the
//   first step on the box and a one-cell ring, adds e^n and takes the second on the box;
//   per cell and two steps a^{n+1}, e^{n+1}, e^n, c^n, c^{n-1} are read and a^{n-1}
//   written (12 instead of 16 B per cell and step, and half the launches).  The launch also
//   clears, on its box, two buffers of sums of steps already reversed, for their reuse.
#include <hip/hip_ext.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace cuesim {

namespace {

// step: 256 columns x 8 rows, all 8 rows' loads at once; reverse: 256 x 4 (measured best)
constexpr int kRX = 256, kRY = 8, kRUnroll = 8;
constexpr int kAY = 4, kAUnroll = 4;
// two steps per launch (forward and reverse): boxes of 256 x kPY cells held with a two-cell
// ring (kPW x kPH) for the first step and a one-cell ring (kQW x kQH) for the second; 4 rows
// measured best (2, 6 and 8 rows slower)
constexpr int kPY = 4;
constexpr int kPW = kRX + 4, kPH = kPY + 4;
constexpr int kQW = kRX + 2, kQH = kPY + 2;
constexpr int kXcds = 8;

struct Tiles2D {
    int tx, ty;
};

Tiles2D tiles_for(int nx, int ny, int rows = kRY) {
    return Tiles2D{(nx + kRX - 1) / kRX, (ny + rows - 1) / rows};
}

__device__ __forceinline__ float stencil2d(float c, float w, float e, float s, float n,
                                           const StencilCoef& k) {
    const float lap = fmaf(-4.0f, c, (w + e) + (s + n));
    return fmaf(k.r, lap, fmaf(-k.kdt, c, c));
}

// Logical box of this workgroup (die-contiguous stretches of the box order).
__device__ __forceinline__ int box_of(int per_xcd) {
    return (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
}

__global__ __launch_bounds__(kRX) void k_field2d_rows(Field2DStepArgs a) {
    const int box = box_of(a.per_xcd);
    if (box >= a.n_species * a.tx * a.ty) return;
    const int bx = box % a.tx, by = (box / a.tx) % a.ty, s = box / (a.tx * a.ty);
    int e = a.src_start[box];
    const int e_end = a.src_start[box + 1];
    const int tid = threadIdx.x;
    const int i = bx * kRX + tid;
    if (i >= a.nx) return;   // no barriers below
    const StencilCoef k = a.coef[s];
    const int nx = a.nx, ny = a.ny;
    const float* col = a.in[s] + i;
    float* dst = a.out[s] + i;
    const int dw = i > 0 ? -1 : 0, de = i < nx - 1 ? 1 : 0;
    const int j0 = by * kRY, j1 = min(j0 + kRY, ny);
    float c = col[(size_t)j0 * nx];
    float below = col[(size_t)max(j0 - 1, 0) * nx];
    int j = j0;
    auto finish = [&](float v, int row) {
        while (e < e_end && a.src_row[e] == row) {
            if (a.src_col[e] == tid) v += a.src_q[e];
            ++e;
        }
        dst[(size_t)row * nx] = v;
    };
    for (; j + kRUnroll <= j1; j += kRUnroll) {
        float up[kRUnroll], w[kRUnroll], ea[kRUnroll];
#pragma unroll
        for (int u = 0; u < kRUnroll; ++u) {
            const float* p = col + (size_t)(j + u) * nx;
            up[u] = col[(size_t)min(j + u + 1, ny - 1) * nx];
            w[u] = p[dw];
            ea[u] = p[de];
        }
#pragma unroll
        for (int u = 0; u < kRUnroll; ++u) {
            finish(stencil2d(c, w[u], ea[u], below, up[u], k), j + u);
            below = c;
            c = up[u];
        }
    }
    for (; j < j1; ++j) {
        const float* p = col + (size_t)j * nx;
        const float above = col[(size_t)min(j + 1, ny - 1) * nx];
        finish(stencil2d(c, p[dw], p[de], below, above, k), j);
        below = c;
        c = above;
    }
}

__device__ double block_sum_fp64(double v) {
    __shared__ double part[kRX / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();   // part[] may still be read from a previous call
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRX / 64; ++w) t += part[w];
    return t;
}

// Reverse step of one species; box b of the launch owns acc_D[b] and acc_k[b].  Box 0 also
// adds b at every source cell into acc_q.
__global__ __launch_bounds__(kRX) void k_field_adjoint2d_rows(
    const float* __restrict__ a_in, const long long* __restrict__ e_q,
    const uint32_t* __restrict__ step_max, int t, const float* __restrict__ c,
    float* __restrict__ a_out, int nx, int ny, int tx, int ty, int per_xcd, StencilCoef k,
    double* __restrict__ acc_D, double* __restrict__ acc_k, const int32_t* __restrict__ q_cell,
    int n_q, double* __restrict__ acc_q) {
    const int box = box_of(per_xcd);
    if (box >= tx * ty) return;   // whole workgroup: the barriers below stay uniform
    const int bx = box % tx, by = box / tx;
    const int i = bx * kRX + threadIdx.x;
    const FixedStep e_in = fixed_step(e_q, step_max, t);
    double pD = 0.0, pk = 0.0;
    if (i < nx) {
        const float* ca = a_in + i;
        const FixedStep ce{e_in.q + i, e_in.inv};
        const float* cc = c + i;
        float* dst = a_out + i;
        const int dw = i > 0 ? -1 : 0, de = i < nx - 1 ? 1 : 0;
        const int j0 = by * kAY, j1 = min(j0 + kAY, ny);
        auto total = [&](size_t at, int off) { return ca[at + off] + ce[at + off]; };
        const size_t r0 = (size_t)j0 * nx, rm = (size_t)max(j0 - 1, 0) * nx;
        float b = total(r0, 0), b_below = total(rm, 0);
        float v = cc[r0], v_below = cc[rm];
        int j = j0;
        for (; j + kAUnroll <= j1; j += kAUnroll) {
            float bu[kAUnroll], bw[kAUnroll], be[kAUnroll], vu[kAUnroll], vw[kAUnroll],
                ve[kAUnroll];
#pragma unroll
            for (int u = 0; u < kAUnroll; ++u) {
                const size_t at = (size_t)(j + u) * nx;
                const size_t up = (size_t)min(j + u + 1, ny - 1) * nx;
                bu[u] = total(up, 0);
                bw[u] = total(at, dw);
                be[u] = total(at, de);
                vu[u] = cc[up];
                vw[u] = cc[at + dw];
                ve[u] = cc[at + de];
            }
#pragma unroll
            for (int u = 0; u < kAUnroll; ++u) {
                dst[(size_t)(j + u) * nx] = stencil2d(b, bw[u], be[u], b_below, bu[u], k);
                const float lap_c = fmaf(-4.0f, v, (vw[u] + ve[u]) + (v_below + vu[u]));
                pD = fma((double)b, (double)lap_c, pD);
                pk = fma((double)b, (double)v, pk);
                b_below = b;
                b = bu[u];
                v_below = v;
                v = vu[u];
            }
        }
        for (; j < j1; ++j) {
            const size_t at = (size_t)j * nx, up = (size_t)min(j + 1, ny - 1) * nx;
            const float b_up = total(up, 0), v_up = cc[up];
            dst[at] = stencil2d(b, total(at, dw), total(at, de), b_below, b_up, k);
            const float lap_c = fmaf(-4.0f, v, (cc[at + dw] + cc[at + de]) + (v_below + v_up));
            pD = fma((double)b, (double)lap_c, pD);
            pk = fma((double)b, (double)v, pk);
            b_below = b;
            b = b_up;
            v_below = v;
            v = v_up;
        }
    }
    const double sD = block_sum_fp64(pD);
    const double sk = block_sum_fp64(pk);
    if (threadIdx.x == 0) {
        acc_D[box] += sD;
        acc_k[box] += sk;
    }
    if (box == 0)
        for (int m = threadIdx.x; m < n_q; m += kRX)
            acc_q[m] += (double)(a_in[q_cell[m]] + e_in[q_cell[m]]);
}

// Two forward steps of one species per box; the stencil and the separate source add are
// those of the single step, and neighbour indices are clamped grid indices mapped into the
// tile, so the result has the single step's bits.
struct Field2DPairArgs {
    const float* in[2];
    float* out1[2];
    float* out2[2];
    StencilCoef coef[2];
    int nx, ny, n_species, tx, ty, per_xcd;
    const int32_t* src_start;   // [boxes + 1]
    const int32_t* src_pos;     // row * (kRX + 2) + column in the box with its one-cell ring
    const float* src_q;
};


__global__ __launch_bounds__(kRX) void k_field2d_pair(Field2DPairArgs a) {
    const int box = box_of(a.per_xcd);
    if (box >= a.n_species * a.tx * a.ty) return;   // whole workgroup
    const int bx = box % a.tx, by = (box / a.tx) % a.ty, s = box / (a.tx * a.ty);
    const int x0 = bx * kRX, y0 = by * kPY;
    const int nx = a.nx, ny = a.ny;
    const int tid = threadIdx.x;
    const StencilCoef k = a.coef[s];
    __shared__ float T0[kPH][kPW];   // c^n: box and a two-cell ring
    __shared__ float T1[kQH][kQW];   // c^{n+1}: box and a one-cell ring
    __shared__ float T2[kPY][kRX];   // c^{n+2}: box
    auto t0 = [&](int i, int j) { return T0[j - y0 + 2][i - x0 + 2]; };
    auto t1 = [&](int i, int j) { return T1[j - y0 + 1][i - x0 + 1]; };

    // c^n (clamped into the grid; ring copies outside it are never read), this thread's
    // column and, for threads 0..3, the ring columns x0 - 2, x0 - 1, x0 + 256, x0 + 257
    const float* src = a.in[s];
    const int i = x0 + tid;
    const int ci = min(i, nx - 1);
    const int xcol = tid < 2 ? tid : kRX + tid;
    const int xi = min(max(x0 - 2 + xcol, 0), nx - 1);
    float v[kPH], xv[kPH];
#pragma unroll
    for (int u = 0; u < kPH; ++u)
        v[u] = src[(size_t)min(max(y0 - 2 + u, 0), ny - 1) * nx + ci];
    if (tid < 4) {
#pragma unroll
        for (int u = 0; u < kPH; ++u)
            xv[u] = src[(size_t)min(max(y0 - 2 + u, 0), ny - 1) * nx + xi];
    }
#pragma unroll
    for (int u = 0; u < kPH; ++u) T0[u][tid + 2] = v[u];
    if (tid < 4) {
#pragma unroll
        for (int u = 0; u < kPH; ++u) T0[u][xcol] = xv[u];
    }
    __syncthreads();

    // first step on the box and a one-cell ring (in-grid cells)
    auto step1 = [&](int ii, int col) {
        const int w = max(ii - 1, 0), e = min(ii + 1, nx - 1);
#pragma unroll
        for (int r = 0; r < kQH; ++r) {
            const int j = y0 - 1 + r;
            if (j < 0 || j >= ny) continue;
            const int js = max(j - 1, 0), jn = min(j + 1, ny - 1);
            T1[r][col] = stencil2d(t0(ii, j), t0(w, j), t0(e, j), t0(ii, js), t0(ii, jn), k);
        }
    };
    if (i < nx) step1(i, tid + 1);
    if (tid < 2) {
        const int ri = tid == 0 ? x0 - 1 : x0 + kRX;
        if (ri >= 0 && ri < nx) step1(ri, tid == 0 ? 0 : kRX + 1);
    }
    __syncthreads();
    // its sources (every listed cell is in the grid and appears once)
    const int q0 = a.src_start[box], q1 = a.src_start[box + 1];
    for (int q = q0 + tid; q < q1; q += kRX) (&T1[0][0])[a.src_pos[q]] += a.src_q[q];
    __syncthreads();

    // c^{n+1} out, then the second step on the box
    if (i < nx) {
        const int w = max(i - 1, 0), e = min(i + 1, nx - 1);
        const int rows = min(kPY, ny - y0);
        float* out1 = a.out1[s];
#pragma unroll
        for (int r = 0; r < kPY; ++r) {
            if (r >= rows) break;
            const int j = y0 + r;
            const int js = max(j - 1, 0), jn = min(j + 1, ny - 1);
            out1[(size_t)j * nx + i] = T1[r + 1][tid + 1];
            T2[r][tid] = stencil2d(t1(i, j), t1(w, j), t1(e, j), t1(i, js), t1(i, jn), k);
        }
    }
    __syncthreads();
    for (int q = q0 + tid; q < q1; q += kRX) {
        const int r = a.src_pos[q] / kQW, col = a.src_pos[q] % kQW;
        if (r >= 1 && r <= kPY && col >= 1 && col <= kRX) T2[r - 1][col - 1] += a.src_q[q];
    }
    __syncthreads();
    if (i < nx) {
        const int rows = min(kPY, ny - y0);
        float* out2 = a.out2[s];
#pragma unroll
        for (int r = 0; r < kPY; ++r) {
            if (r >= rows) break;
            out2[(size_t)(y0 + r) * nx + i] = T2[r][tid];
        }
    }
}

// Two reverse steps (n, then n - 1) of one species.  Box b of the launch (256 x kPY cells)
// owns acc_D[b] and acc_k[b] (both steps' sums are added) and the sources listed for it.
// Every neighbour index is the clamped grid index mapped into the tile, so the walls are
// exactly those of the single step.
struct FieldAdjointPairArgs {
    const float* a_in;    // a^{n+1}
    const long long* e1;  // e^{n+1}, fixed-point sums of segment step t1
    const long long* e0;  // e^n, of segment step t0
    const uint32_t* step_max;
    int t1, t0;
    const float* c1;      // c^n
    const float* c0;      // c^{n-1}
    float* a_out;         // a^{n-1}
    int nx, ny, tx, ty, per_xcd;
    StencilCoef k;
    double* acc_D;
    double* acc_k;
    const int32_t* q_start;   // [n_boxes + 1] into q_index
    const int32_t* q_index;   // source numbers m
    const int32_t* q_cell;    // cell of source m
    double* acc_q;
    long long* z1;            // sums of two other steps set to zero on the box (may be null)
    long long* z0;
};

__global__ __launch_bounds__(kRX) void k_field_adjoint2d_pair(FieldAdjointPairArgs a) {
    const int box = box_of(a.per_xcd);
    if (box >= a.tx * a.ty) return;   // whole workgroup: the barriers below stay uniform
    const int bx = box % a.tx, by = box / a.tx;
    const int x0 = bx * kRX, y0 = by * kPY;
    const int nx = a.nx, ny = a.ny;
    const int tid = threadIdx.x;
    __shared__ float B1[kPH][kPW];
    __shared__ float B2[kQH][kQW];
    auto b1 = [&](int i, int j) { return B1[j - y0 + 2][i - x0 + 2]; };
    auto b2 = [&](int i, int j) { return B2[j - y0 + 1][i - x0 + 1]; };

    // Every global value this thread needs is requested first.  The thread owns column
    // i = x0 + tid (clamped for loads where past the grid); threads 0..3 also load the
    // ring columns x0 - 2, x0 - 1, x0 + 256, x0 + 257 of b^{n+1}, threads 0 and 1 the ring
    // columns x0 - 1 and x0 + 256 of e^n.
    const int i = x0 + tid;
    const bool live = i < nx;
    const int ci = min(i, nx - 1);
    const int iw = max(ci - 1, 0), ie = min(ci + 1, nx - 1);
    int brow[kPH];   // grid rows of the tile rows y0 - 2 .. y0 + kPY + 1, clamped
#pragma unroll
    for (int u = 0; u < kPH; ++u) brow[u] = min(max(y0 - 2 + u, 0), ny - 1);
    const int xcol = tid < 2 ? tid : kRX + tid;              // tile column, threads 0..3
    const int xi = min(max(x0 - 2 + xcol, 0), nx - 1);
    const int ri = tid == 0 ? x0 - 1 : x0 + kRX;             // ring column, threads 0, 1
    const int rci = min(max(ri, 0), nx - 1);
    const FixedStep e1 = fixed_step(a.e1, a.step_max, a.t1);
    const FixedStep e0 = fixed_step(a.e0, a.step_max, a.t0);
    float va[kPH], ve[kPH], xa[kPH], xe[kPH];
    float en[kQH], xen[kQH], c1v[kQH], c0v[kQH];
    float c1w[kPY], c1e[kPY], c0w[kPY], c0e[kPY];
#pragma unroll
    for (int u = 0; u < kPH; ++u) {
        const size_t at = (size_t)brow[u] * nx;
        va[u] = a.a_in[at + ci];
        ve[u] = e1[at + ci];
    }
    if (tid < 4) {
#pragma unroll
        for (int u = 0; u < kPH; ++u) {
            const size_t at = (size_t)brow[u] * nx;
            xa[u] = a.a_in[at + xi];
            xe[u] = e1[at + xi];
        }
    }
#pragma unroll
    for (int r = 0; r < kQH; ++r) en[r] = e0[(size_t)brow[r + 1] * nx + ci];
    if (tid < 2) {
#pragma unroll
        for (int r = 0; r < kQH; ++r) xen[r] = e0[(size_t)brow[r + 1] * nx + rci];
    }
#pragma unroll
    for (int r = 0; r < kQH; ++r) {
        const size_t at = (size_t)brow[r + 1] * nx;
        c1v[r] = a.c1[at + ci];
        c0v[r] = a.c0[at + ci];
    }
#pragma unroll
    for (int r = 0; r < kPY; ++r) {
        const size_t at = (size_t)brow[r + 2] * nx;
        c1w[r] = a.c1[at + iw];
        c1e[r] = a.c1[at + ie];
        c0w[r] = a.c0[at + iw];
        c0e[r] = a.c0[at + ie];
    }

    // b^{n+1} = a^{n+1} + e^{n+1} on the box and a two-cell ring (ring cells outside the
    // grid hold clamped copies and are never read: every read below uses clamped indices)
#pragma unroll
    for (int u = 0; u < kPH; ++u) B1[u][tid + 2] = va[u] + ve[u];
    if (tid < 4) {
#pragma unroll
        for (int u = 0; u < kPH; ++u) B1[u][xcol] = xa[u] + xe[u];
    }
    __syncthreads();

    // first step on the box and a one-cell ring: a^n = S b^{n+1}, b^n = a^n + e^n; the box
    // cells add b^{n+1} Lap c^n and b^{n+1} c^n
    double pD = 0.0, pk = 0.0;
    if (live) {
        const int w = max(i - 1, 0), e = min(i + 1, nx - 1);
#pragma unroll
        for (int r = 0; r < kQH; ++r) {
            const int j = y0 - 1 + r;
            if (j < 0 || j >= ny) continue;
            const int js = max(j - 1, 0), jn = min(j + 1, ny - 1);
            const float b = b1(i, j);
            B2[r][tid + 1] = stencil2d(b, b1(w, j), b1(e, j), b1(i, js), b1(i, jn), a.k) + en[r];
            if (r >= 1 && r <= kPY) {
                const float v = c1v[r];
                const float lap_c =
                    fmaf(-4.0f, v, (c1w[r - 1] + c1e[r - 1]) + (c1v[r - 1] + c1v[r + 1]));
                pD = fma((double)b, (double)lap_c, pD);
                pk = fma((double)b, (double)v, pk);
            }
        }
    }
    if (tid < 2 && ri >= 0 && ri < nx) {
        const int w = max(ri - 1, 0), e = min(ri + 1, nx - 1);
        const int col = tid == 0 ? 0 : kRX + 1;
#pragma unroll
        for (int r = 0; r < kQH; ++r) {
            const int j = y0 - 1 + r;
            if (j < 0 || j >= ny) continue;
            const int js = max(j - 1, 0), jn = min(j + 1, ny - 1);
            B2[r][col] = stencil2d(b1(ri, j), b1(w, j), b1(e, j), b1(ri, js), b1(ri, jn), a.k) +
                         xen[r];
        }
    }
    __syncthreads();

    // second step on the box: a^{n-1} = S b^n, and b^n Lap c^{n-1}, b^n c^{n-1}
    if (live) {
        const int w = max(i - 1, 0), e = min(i + 1, nx - 1);
        const int rows = min(kPY, ny - y0);
#pragma unroll
        for (int r = 0; r < kPY; ++r) {
            if (r >= rows) break;
            const int j = y0 + r;
            const int js = max(j - 1, 0), jn = min(j + 1, ny - 1);
            const float b = b2(i, j);
            a.a_out[(size_t)j * nx + i] =
                stencil2d(b, b2(w, j), b2(e, j), b2(i, js), b2(i, jn), a.k);
            const float v = c0v[r + 1];
            const float lap_c = fmaf(-4.0f, v, (c0w[r] + c0e[r]) + (c0v[r] + c0v[r + 2]));
            pD = fma((double)b, (double)lap_c, pD);
            pk = fma((double)b, (double)v, pk);
        }
    }
    const double sD = block_sum_fp64(pD);
    const double sk = block_sum_fp64(pk);
    if (tid == 0) {
        a.acc_D[box] += sD;
        a.acc_k[box] += sk;
    }
    // b^{n+1}, then b^n, at this box's source cells (each source is listed by one box)
    for (int q = a.q_start[box] + tid; q < a.q_start[box + 1]; q += kRX) {
        const int m = a.q_index[q];
        const int cell = a.q_cell[m];
        const int ci = cell % nx, cj = cell / nx;
        a.acc_q[m] += (double)b1(ci, cj);
        a.acc_q[m] += (double)b2(ci, cj);
    }
    // the box's cells of two finished steps' sums cleared for their next use (streaming
    // stores: the sums are read again only after a group of steps; 21.8 against 22.5 ms per
    // gradient sweep at 1024^2 with plain stores)
    if (live && a.z1 != nullptr) {
        const int rows = min(kPY, ny - y0);
#pragma unroll
        for (int r = 0; r < kPY; ++r) {
            if (r >= rows) break;
            const size_t at = (size_t)(y0 + r) * nx + i;
            __builtin_nontemporal_store(0LL, &a.z1[at]);
            __builtin_nontemporal_store(0LL, &a.z0[at]);
        }
    }
}

}  // namespace

hipError_t field2d_prepare(Field2DStep& f, int nx, int ny, int n_species,
                           const std::vector<int32_t>* cells, const std::vector<float>* q) {
    field2d_release(f);
    const Tiles2D t = tiles_for(nx, ny);
    const int n_boxes = n_species * t.tx * t.ty;
    // source entries per box, in row order (cells are unique per species)
    std::vector<std::vector<std::pair<int64_t, float>>> per_box(n_boxes);
    for (int s = 0; s < n_species; ++s)
        for (size_t m = 0; m < cells[s].size(); ++m) {
            const int i = cells[s][m] % nx, j = cells[s][m] / nx;
            const int box = (s * t.ty + j / kRY) * t.tx + i / kRX;
            per_box[box].push_back({(int64_t)j * kRX + i % kRX, q[s][m]});
        }
    std::vector<int32_t> start(n_boxes + 1, 0), row_of, col_of;
    std::vector<float> amount;
    for (int box = 0; box < n_boxes; ++box) {
        auto& v = per_box[box];
        std::sort(v.begin(), v.end(),
                  [](const std::pair<int64_t, float>& x, const std::pair<int64_t, float>& y) {
                      return x.first < y.first;
                  });
        for (auto& en : v) {
            row_of.push_back((int32_t)(en.first / kRX));
            col_of.push_back((int32_t)(en.first % kRX));
            amount.push_back(en.second);
        }
        start[box + 1] = (int32_t)row_of.size();
    }
    const size_t n_src = std::max<size_t>(row_of.size(), 1);
    hipError_t e;
    if ((e = hipMalloc((void**)&f.src_start, start.size() * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.src_row, n_src * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.src_col, n_src * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.src_q, n_src * sizeof(float))) != hipSuccess)
        return e;
    if ((e = hipMemcpy(f.src_start, start.data(), start.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (!row_of.empty() &&
        ((e = hipMemcpy(f.src_row, row_of.data(), row_of.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = hipMemcpy(f.src_col, col_of.data(), col_of.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = hipMemcpy(f.src_q, amount.data(), amount.size() * sizeof(float),
                        hipMemcpyHostToDevice)) != hipSuccess))
        return e;
    // two-step boxes: the sources on each box and its one-cell ring (a cell near a box edge
    // is listed by up to four boxes)
    const Tiles2D p = tiles_for(nx, ny, kPY);
    const int n_pair = n_species * p.tx * p.ty;
    std::vector<std::vector<std::pair<int32_t, float>>> per_pair(n_pair);
    for (int s = 0; s < n_species; ++s)
        for (size_t m = 0; m < cells[s].size(); ++m) {
            const int i = cells[s][m] % nx, j = cells[s][m] / nx;
            for (int by = std::max(j / kPY - 1, 0); by <= std::min(j / kPY + 1, p.ty - 1); ++by)
                for (int bx = std::max(i / kRX - 1, 0); bx <= std::min(i / kRX + 1, p.tx - 1);
                     ++bx) {
                    const int r = j - (by * kPY - 1), c = i - (bx * kRX - 1);
                    if (r < 0 || r >= kQH || c < 0 || c >= kQW) continue;
                    per_pair[(s * p.ty + by) * p.tx + bx].push_back({r * kQW + c, q[s][m]});
                }
        }
    std::vector<int32_t> pstart(n_pair + 1, 0), ppos;
    std::vector<float> pq;
    for (int b = 0; b < n_pair; ++b) {
        for (auto& en : per_pair[b]) {
            ppos.push_back(en.first);
            pq.push_back(en.second);
        }
        pstart[b + 1] = (int32_t)ppos.size();
    }
    const size_t n_p = std::max<size_t>(ppos.size(), 1);
    if ((e = hipMalloc((void**)&f.pair_start, pstart.size() * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.pair_pos, n_p * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void**)&f.pair_q, n_p * sizeof(float))) != hipSuccess)
        return e;
    if ((e = hipMemcpy(f.pair_start, pstart.data(), pstart.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if (!ppos.empty() &&
        ((e = hipMemcpy(f.pair_pos, ppos.data(), ppos.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = hipMemcpy(f.pair_q, pq.data(), pq.size() * sizeof(float),
                        hipMemcpyHostToDevice)) != hipSuccess))
        return e;
    f.n_pair_boxes = n_pair;
    f.nx = nx;
    f.ny = ny;
    f.n_species = n_species;
    f.n_boxes = n_boxes;
    return hipSuccess;
}

void field2d_release(Field2DStep& f) {
    if (f.src_start) (void)hipFree(f.src_start);
    if (f.src_row) (void)hipFree(f.src_row);
    if (f.src_col) (void)hipFree(f.src_col);
    if (f.src_q) (void)hipFree(f.src_q);
    if (f.pair_start) (void)hipFree(f.pair_start);
    if (f.pair_pos) (void)hipFree(f.pair_pos);
    if (f.pair_q) (void)hipFree(f.pair_q);
    f = Field2DStep{};
}

hipError_t launch_field2d_rows(const Field2DStep& f, const float* const* in, float* const* out,
                               const StencilCoef* coef, hipStream_t stream, hipEvent_t start,
                               hipEvent_t stop) {
    const Tiles2D t = tiles_for(f.nx, f.ny);
    Field2DStepArgs a = {};
    for (int s = 0; s < f.n_species; ++s) {
        a.in[s] = in[s];
        a.out[s] = out[s];
        a.coef[s] = coef[s];
    }
    a.nx = f.nx;
    a.ny = f.ny;
    a.n_species = f.n_species;
    a.tx = t.tx;
    a.ty = t.ty;
    a.per_xcd = (f.n_boxes + kXcds - 1) / kXcds;
    a.src_start = f.src_start;
    a.src_row = f.src_row;
    a.src_col = f.src_col;
    a.src_q = f.src_q;
    void* args[] = {&a};
    if (!start && !stop)   // a plain launch (also what a graph capture records)
        return hipLaunchKernel((const void*)k_field2d_rows, dim3(a.per_xcd * kXcds), dim3(kRX),
                               args, 0, stream);
    return hipExtLaunchKernel((const void*)k_field2d_rows, dim3(a.per_xcd * kXcds), dim3(kRX),
                              args, 0, stream, start, stop, 0);
}

hipError_t launch_field2d_pair(const Field2DStep& f, const float* const* in, float* const* out1,
                               float* const* out2, const StencilCoef* coef, hipStream_t stream) {
    const Tiles2D t = tiles_for(f.nx, f.ny, kPY);
    Field2DPairArgs a = {};
    for (int s = 0; s < f.n_species; ++s) {
        a.in[s] = in[s];
        a.out1[s] = out1[s];
        a.out2[s] = out2[s];
        a.coef[s] = coef[s];
    }
    a.nx = f.nx;
    a.ny = f.ny;
    a.n_species = f.n_species;
    a.tx = t.tx;
    a.ty = t.ty;
    a.per_xcd = (f.n_pair_boxes + kXcds - 1) / kXcds;
    a.src_start = f.pair_start;
    a.src_pos = f.pair_pos;
    a.src_q = f.pair_q;
    hipLaunchKernelGGL(k_field2d_pair, dim3(a.per_xcd * kXcds), dim3(kRX), 0, stream, a);
    return hipGetLastError();
}

int adjoint_field_blocks(int nx, int ny) {
    const Tiles2D t = tiles_for(nx, ny, kAY);
    return t.tx * t.ty;
}

int adjoint_pair_blocks(int nx, int ny) {
    const Tiles2D t = tiles_for(nx, ny, kPY);
    return t.tx * t.ty;
}

void adjoint_pair_sources(int nx, int ny, const std::vector<int32_t>& cells,
                          std::vector<int32_t>& start, std::vector<int32_t>& index) {
    const Tiles2D t = tiles_for(nx, ny, kPY);
    const int nb = t.tx * t.ty;
    std::vector<std::vector<int32_t>> per_box(nb);
    for (size_t m = 0; m < cells.size(); ++m) {
        const int i = cells[m] % nx, j = cells[m] / nx;
        per_box[(j / kPY) * t.tx + i / kRX].push_back((int32_t)m);
    }
    start.assign(nb + 1, 0);
    index.clear();
    for (int b = 0; b < nb; ++b) {
        start[b] = (int32_t)index.size();
        index.insert(index.end(), per_box[b].begin(), per_box[b].end());
    }
    start[nb] = (int32_t)index.size();
}

hipError_t launch_field_adjoint2d_pair(int nx, int ny, const float* a_in, const long long* e1,
                                       const long long* e0, const uint32_t* step_max, int t1,
                                       int t0, const float* c1, const float* c0, float* a_out,
                                       StencilCoef coef, double* acc_D, double* acc_k,
                                       const int32_t* q_start, const int32_t* q_index,
                                       const int32_t* q_cell, double* acc_q,
                                       long long* z1, long long* z0, hipStream_t stream) {
    if ((z1 == nullptr) != (z0 == nullptr)) return hipErrorInvalidValue;
    const Tiles2D t = tiles_for(nx, ny, kPY);
    FieldAdjointPairArgs a{};
    a.a_in = a_in;
    a.e1 = e1;
    a.e0 = e0;
    a.step_max = step_max;
    a.t1 = t1;
    a.t0 = t0;
    a.c1 = c1;
    a.c0 = c0;
    a.a_out = a_out;
    a.nx = nx;
    a.ny = ny;
    a.tx = t.tx;
    a.ty = t.ty;
    a.per_xcd = (t.tx * t.ty + kXcds - 1) / kXcds;
    a.k = coef;
    a.acc_D = acc_D;
    a.acc_k = acc_k;
    a.q_start = q_start;
    a.q_index = q_index;
    a.q_cell = q_cell;
    a.acc_q = acc_q;
    a.z1 = z1;
    a.z0 = z0;
    hipLaunchKernelGGL(k_field_adjoint2d_pair, dim3(a.per_xcd * kXcds), dim3(kRX), 0, stream,
                       a);
    return hipGetLastError();
}

hipError_t launch_field_adjoint2d(int nx, int ny, const float* a_in, const long long* e_in,
                                  const uint32_t* step_max, int t, const float* c,
                                  float* a_out, StencilCoef coef, double* acc_D, double* acc_k,
                                  const int32_t* q_cell, int n_q, double* acc_q,
                                  hipStream_t stream) {
    const Tiles2D tl = tiles_for(nx, ny, kAY);
    const int per_xcd = (tl.tx * tl.ty + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(k_field_adjoint2d_rows, dim3(per_xcd * kXcds), dim3(kRX), 0, stream,
                       a_in, e_in, step_max, t, c, a_out, nx, ny, tl.tx, tl.ty, per_xcd, coef,
                       acc_D, acc_k, q_cell, n_q, acc_q);
    return hipGetLastError();
}

}  // namespace cuesim
