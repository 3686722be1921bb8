// kernels_sort.hip -- stable sort of (key, value) pairs by counting: per-tile histograms,
// one exclusive scan, stable scatter; least significant 8-bit digit first.
//
// This is the hash -> sort -> cell-start step of the paper's uniform-grid broadphase
// (Sec. 3.5, Table 1): items keyed by their cell end up grouped by cell, in their original
// order within a cell, and the scanned histogram gives every cell's start.  The library
// uses it to order 3D cones by the cell of their tip and to group contact edges by the
// neuron that owns them (Sec. 3.4).
//
// One pass over a digit:
//   histogram  one workgroup per tile of kTile consecutive items counts the tile's digits
//              in LDS and writes them digit-major: hist[digit * n_tiles + tile];
//   scan       one workgroup turns hist into exclusive prefix sums, so entry
//              (digit, tile) is where the tile's first item with that digit goes;
//   scatter    every tile re-reads its items in order, kSortThreads at a time; an item's
//              place among equal digits of the same round comes from wavefront ballots
//              (the lanes whose digit matches, below it), the waves before it and the
//              items of earlier rounds, so equal digits keep their input order.
#include <algorithm>

#include "internal.hpp"

namespace cuesim {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kDigitBits = 8;
constexpr int kBins = 1 << kDigitBits;   // == kSortThreads: one bin per thread
constexpr int kRounds = 8;
constexpr int kTile = kSortThreads * kRounds;
constexpr int kScanThreads = 1024;
static_assert(kBins == kSortThreads, "one digit bin per thread");

int sort_tiles(int n) { return (n + kTile - 1) / kTile; }

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ keys,
                                                            int n, int shift, int n_tiles,
                                                            int32_t* __restrict__ hist) {
    __shared__ int32_t count[kBins];
    const int tid = threadIdx.x, tile = blockIdx.x;
    count[tid] = 0;
    // every round's key first (indices clamped, so nothing branches between the loads)
    uint32_t key[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) key[r] = keys[min(tile * kTile + r * kSortThreads + tid, n - 1)];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
        if (tile * kTile + r * kSortThreads + tid < n)
            atomicAdd(&count[(key[r] >> shift) & (kBins - 1)], 1);
    __syncthreads();
    hist[tid * n_tiles + tile] = count[tid];
}

// Exclusive scan of a[0..n) in place by one workgroup, kScanPer entries per thread at a
// time: each thread loads its run of kScanPer consecutive entries into registers (16-byte
// loads when the run lies inside the array, else loads at clamped indices; either way all
// issued before any is used), the run totals are scanned across each wavefront by lane
// shuffles and across the wavefronts in LDS, and each thread writes its run back; longer
// arrays take several such rounds, carrying the total.
constexpr int kScanPer = 32;
constexpr int kScanWaves = kScanThreads / 64;

__global__ __launch_bounds__(kScanThreads) void k_sort_scan(int32_t* __restrict__ a, int n) {
    __shared__ int32_t wave_total[kScanWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t carry = 0;
    for (int base = 0; base < n; base += kScanThreads * kScanPer) {
        const int lo = base + (int)threadIdx.x * kScanPer;
        int32_t v[kScanPer];
        if (lo + kScanPer <= n && (lo & 3) == 0) {
#pragma unroll
            for (int u = 0; u < kScanPer; u += 4) {
                const int4 q = *(const int4*)(a + lo + u);
                v[u] = q.x;
                v[u + 1] = q.y;
                v[u + 2] = q.z;
                v[u + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int u = 0; u < kScanPer; ++u) v[u] = a[min(lo + u, n - 1)];
#pragma unroll
            for (int u = 0; u < kScanPer; ++u) v[u] = lo + u < n ? v[u] : 0;
        }
        int32_t sum = 0;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) sum += v[u];
        int32_t incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wave_total[wave] = incl;
        __syncthreads();
        int32_t at = carry + incl - sum, round_total = 0;
#pragma unroll
        for (int w = 0; w < kScanWaves; ++w) {
            const int32_t t = wave_total[w];
            at += w < wave ? t : 0;
            round_total += t;
        }
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            if (lo + u < n) a[lo + u] = at;
            at += v[u];
        }
        carry += round_total;
        __syncthreads();   // every thread has read wave_total
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int n, int shift, int n_tiles,
    const int32_t* __restrict__ start) {
    __shared__ int32_t next[kBins];                 // next output position per digit
    __shared__ int32_t wave_count[kSortWaves][kBins];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, tile = blockIdx.x;
    next[tid] = start[tid * n_tiles + tile];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // every round's item first (indices clamped, so nothing branches between the loads)
    uint32_t keys[kRounds];
    int32_t vals[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int i = min(tile * kTile + r * kSortThreads + tid, n - 1);
        keys[r] = kin[i];
        vals[r] = vin[i];
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int i = tile * kTile + r * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? keys[r] : 0u;
        const int32_t val = vals[r];
        const int d = (int)((key >> shift) & (kBins - 1));
        // lanes of this wavefront holding a valid item with the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kDigitBits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t set = __ballot(bit);
            peers &= bit ? set : ~set;
        }
        const int rank = __popcll(peers & below);
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) wave_count[w][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wave_count[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = next[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wave_count[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) add += wave_count[w][tid];
        next[tid] += add;
    }
}

}  // namespace

size_t sort_pairs_scratch_bytes(int n) {
    return (size_t)kBins * (size_t)std::max(sort_tiles(n), 1) * sizeof(int32_t);
}

hipError_t sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                      int n, int key_bits, int32_t* scratch, hipStream_t stream, bool* in_alt) {
    *in_alt = false;
    if (n <= 0 || key_bits <= 0) return hipSuccess;
    const int tiles = sort_tiles(n);
    uint32_t* k[2] = {keys, keys_alt};
    int32_t* v[2] = {vals, vals_alt};
    int cur = 0;
    for (int shift = 0; shift < key_bits; shift += kDigitBits) {
        hipLaunchKernelGGL(k_sort_hist, dim3(tiles), dim3(kSortThreads), 0, stream, k[cur], n,
                           shift, tiles, scratch);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kScanThreads), 0, stream, scratch,
                           kBins * tiles);
        hipLaunchKernelGGL(k_sort_scatter, dim3(tiles), dim3(kSortThreads), 0, stream, k[cur],
                           v[cur], k[cur ^ 1], v[cur ^ 1], n, shift, tiles, scratch);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    *in_alt = cur == 1;
    return hipSuccess;
}

}  // namespace cuesim
