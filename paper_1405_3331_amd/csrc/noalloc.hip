// noalloc.hip -- sim_connectivity_noalloc: the connectivity build (Sec. 3.4, Figs. 4-5) with
// every device buffer it needs taken from one fixed array instead of hipMalloc, for callers
// that cannot allocate device memory.
//
// `scratch` is a file-scope __device__ array: every GPU the library runs on holds its own
// copy, at its own address, until the process ends.  In host code the name is only a
// stand-in for the symbol, so the device address is looked up once per device (with that
// device current) through hipGetSymbolAddress and kept; kernels and copies only ever see
// that address.  All calls on one GPU share the array: calls that overlap on one GPU race.
#include <mutex>

#include "internal.hpp"

namespace cuesim {

namespace {

constexpr int kNoAllocMax = 1 << 18;   // cones, targets and neurons per call
constexpr int kMaxDevices = 64;

// Words of the layout below at the largest sizes.
constexpr size_t words_for(size_t M, size_t T, size_t N) {
    return 7 * M + T + 2 * N + 1 + ((M + 2047) / 2048) * 256;
}
constexpr size_t kScratchWords = words_for(kNoAllocMax, kNoAllocMax, kNoAllocMax);

static __device__ __align__(256) int32_t scratch[kScratchWords];

std::mutex g_lookup_mutex;
int32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `device`'s copy of `scratch`, looked up on first use with that device
// current (the caller's current device is restored).
hipError_t scratch_address(int device, int32_t** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_lookup_mutex);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) e = hipSetDevice(device);
        if (e != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (int32_t*)ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

}  // namespace cuesim

using namespace cuesim;

extern "C" sim_status sim_connectivity_noalloc(sim_handle* h, int32_t n_neurons,
                                               const int32_t* cone_owner,
                                               const int32_t* target_owner,
                                               int32_t* row_start, int32_t* edges,
                                               int64_t edge_capacity, int64_t* n_edges) {
    sim_status st = connectivity_validate(h, n_neurons, cone_owner, target_owner, row_start,
                                          edges, edge_capacity, n_edges);
    if (st != SIM_OK) return st;
    const int M = handle_cones(h), T = handle_targets(h);
    if (M > kNoAllocMax || T > kNoAllocMax || n_neurons > kNoAllocMax)
        return handle_fail(h, SIM_EINVAL,
                           "sim_connectivity_noalloc: more than 262144 cones, targets or "
                           "neurons (the size of its fixed device buffer)");
    int32_t* base = nullptr;
    hipError_t e = scratch_address(handle_device(h), &base);
    if (e != hipSuccess) return handle_fail(h, SIM_EDEVICE, "scratch address lookup failed");
    // carve this call's buffers out of the array, at this call's sizes
    const size_t Ms = (size_t)std::max(M, 1), Ts = (size_t)std::max(T, 1);
    const size_t N = (size_t)n_neurons;
    GraphBuffers g{};
    int32_t* p = base;
    g.owner = p;        p += Ms;
    g.target_owner = p; p += Ts;
    g.key = p;          p += Ms;
    g.cone = p;         p += Ms;
    g.key_sorted = p;   p += Ms;
    g.cone_sorted = p;  p += Ms;
    g.edges = p;        p += Ms;
    g.degree = p;       p += N;
    g.row_start = p;    p += N + 1;
    g.scratch = p;      p += sort_pairs_scratch_bytes(M) / sizeof(int32_t);
    if ((size_t)(p - base) > kScratchWords)
        return handle_fail(h, SIM_EINVAL, "sim_connectivity_noalloc: layout exceeds its buffer");
    g.n_neurons = n_neurons;
    return connectivity_build(h, g, cone_owner, target_owner, row_start, edges, edge_capacity,
                              n_edges);
}
