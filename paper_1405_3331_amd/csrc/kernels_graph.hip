// kernels_graph.hip -- the connectivity the growth produced, as a compact adjacency list,
// and its level-synchronous breadth-first traversal (Sec. 3.4, Figs. 4-5).
//
// A cone that stopped on a target is a connection from the neuron owning the cone to the
// neuron owning the target.  The adjacency list is the paper's pair of arrays: V_a (for
// every neuron the start of its list) and E_a (the lists, neuron after neuron).  Within a
// neuron's list the edges are in increasing cone index, so the list is unique.  It is
// built with the project's stable counting sort of (owner, cone) pairs (kernels_sort.hip;
// non-edges carry the key n_neurons and sort last), a count per neuron and an exclusive
// scan.
//
// The traversal expands one level per launch with one thread per vertex, as in the paper's
// kernel: a vertex at level d labels its unlabelled neighbours d + 1.  Reading the level
// itself as the frontier flag keeps the expansion level-synchronous (a vertex labelled
// d + 1 during the launch is not expanded in it).
#include "internal.hpp"

namespace cuesim {

namespace {

constexpr int kGraphThreads = 256;
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kGraphThreads) void k_edge_keys(const int32_t* __restrict__ status,
                                                             const int32_t* __restrict__ owner,
                                                             int n, int n_neurons,
                                                             int32_t* __restrict__ key,
                                                             int32_t* __restrict__ cone,
                                                             int32_t* __restrict__ degree) {
    const int i = blockIdx.x * kGraphThreads + threadIdx.x;
    if (i >= n) return;
    const bool edge = status[i] == kContact;
    key[i] = edge ? owner[i] : n_neurons;
    cone[i] = i;
    if (edge) atomicAdd(&degree[owner[i]], 1);
}

// Exclusive scan of n counts into row_start[0..n] by one workgroup: each thread sums a
// contiguous chunk, the chunk sums are scanned in LDS, then each thread writes its chunk.
__global__ __launch_bounds__(kScanThreads) void k_row_start(const int32_t* __restrict__ degree,
                                                            int n,
                                                            int32_t* __restrict__ row_start) {
    __shared__ int32_t part[kScanThreads];
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int lo = min((int)threadIdx.x * per, n), hi = min(lo + per, n);
    int32_t sum = 0;
    for (int v = lo; v < hi; ++v) sum += degree[v];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t at = part[threadIdx.x] - sum;
    for (int v = lo; v < hi; ++v) {
        row_start[v] = at;
        at += degree[v];
    }
    if (threadIdx.x == kScanThreads - 1) row_start[n] = part[kScanThreads - 1];
}

__global__ __launch_bounds__(kGraphThreads) void k_fill_edges(
    const int32_t* __restrict__ sorted_cone, const int32_t* __restrict__ target,
    const int32_t* __restrict__ target_owner, const int32_t* __restrict__ row_start,
    int n_neurons, int32_t* __restrict__ edges) {
    const int k = blockIdx.x * kGraphThreads + threadIdx.x;
    if (k >= row_start[n_neurons]) return;
    edges[k] = target_owner[target[sorted_cone[k]]];
}

__global__ __launch_bounds__(kGraphThreads) void k_bfs_level(const int32_t* __restrict__ row_start,
                                                             const int32_t* __restrict__ edges,
                                                             int n, int depth,
                                                             int32_t* __restrict__ level,
                                                             int32_t* __restrict__ grew) {
    const int v = blockIdx.x * kGraphThreads + threadIdx.x;
    if (v >= n || level[v] != depth) return;
    for (int e = row_start[v]; e < row_start[v + 1]; ++e) {
        const int u = edges[e];
        if (level[u] < 0) {
            level[u] = depth + 1;   // every writer writes the same value
            grew[0] = 1;
        }
    }
}

__global__ void k_set_root(int32_t* level, int root) {
    if (threadIdx.x == 0) level[root] = 0;
}

int graph_blocks(int n) { return (n + kGraphThreads - 1) / kGraphThreads; }

int key_bits(int n_neurons) {
    int bits = 1;
    while (bits < 31 && (1 << bits) <= n_neurons) ++bits;
    return bits;
}

}  // namespace

hipError_t launch_adjacency(const GraphBuffers& g, const int32_t* status, const int32_t* target,
                            int n_cones, int n_neurons, hipStream_t stream) {
    hipError_t e = hipMemsetAsync(g.degree, 0, (size_t)n_neurons * sizeof(int32_t), stream);
    if (e != hipSuccess) return e;
    const int32_t* sorted_cone = g.cone;
    if (n_cones > 0) {
        hipLaunchKernelGGL(k_edge_keys, dim3(graph_blocks(n_cones)), dim3(kGraphThreads), 0,
                           stream, status, g.owner, n_cones, n_neurons, g.key, g.cone, g.degree);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        bool in_alt = false;
        e = sort_pairs((uint32_t*)g.key, g.cone, (uint32_t*)g.key_sorted, g.cone_sorted,
                       n_cones, key_bits(n_neurons), g.scratch, stream, &in_alt);
        if (e != hipSuccess) return e;
        if (in_alt) sorted_cone = g.cone_sorted;
    }
    hipLaunchKernelGGL(k_row_start, dim3(1), dim3(kScanThreads), 0, stream, g.degree, n_neurons,
                       g.row_start);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_cones > 0) {
        hipLaunchKernelGGL(k_fill_edges, dim3(graph_blocks(n_cones)), dim3(kGraphThreads), 0,
                           stream, sorted_cone, target, g.target_owner, g.row_start,
                           n_neurons, g.edges);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_bfs_init(int32_t* level, int n, int root, hipStream_t stream) {
    hipError_t e = hipMemsetAsync(level, 0xFF, (size_t)n * sizeof(int32_t), stream);   // -1
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_set_root, dim3(1), dim3(64), 0, stream, level, root);
    return hipGetLastError();
}

hipError_t launch_bfs_level(const int32_t* row_start, const int32_t* edges, int n, int depth,
                            int32_t* level, int32_t* grew, hipStream_t stream) {
    hipLaunchKernelGGL(k_bfs_level, dim3(graph_blocks(n)), dim3(kGraphThreads), 0, stream,
                       row_start, edges, n, depth, level, grew);
    return hipGetLastError();
}

}  // namespace cuesim
