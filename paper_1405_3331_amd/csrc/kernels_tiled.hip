// kernels_tiled.hip -- temporally blocked, LDS-tiled step kernel (not yet enabled: the
// plan reports no usable tiling, so every step runs the plain kernels).
#include "tiled.hpp"

namespace cuesim {

TiledPlan tiled_plan(int dim, int nx, int ny, int nz, int n_species, double step_cells,
                     int block_steps, int n_cones) {
    (void)step_cells;
    (void)block_steps;
    (void)n_cones;
    TiledPlan p;
    p.dim = dim;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.n_species = n_species;
    p.block_steps = 1;
    return p;
}

hipError_t tiled_allocate(const TiledPlan&, TiledState&, int, const ConeRules&,
                          const sim_params*, hipStream_t) {
    return hipErrorNotSupported;
}

void tiled_release(TiledState& st) {
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(st.bucket[b]);
        (void)hipFree(st.count[b]);
        st.bucket[b] = nullptr;
        st.count[b] = nullptr;
    }
    (void)hipFree(st.src_start);
    (void)hipFree(st.src_entry);
    (void)hipFree(st.src_amount);
    st.src_start = nullptr;
    st.src_entry = nullptr;
    st.src_amount = nullptr;
}

hipError_t tiled_bucket(const TiledPlan&, TiledState&, ConeArrays, hipStream_t) {
    return hipErrorNotSupported;
}

hipError_t tiled_unbucket(const TiledPlan&, TiledState&, ConeArrays, hipStream_t) {
    return hipErrorNotSupported;
}

hipError_t tiled_launch(const TiledPlan&, TiledState&, const ConeRules&, float* const[],
                        float* const[], ConeArrays, int, uint32_t, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace cuesim
