// validate_driver.cpp -- runs the library's parameter checks (validate.cpp, host code only)
// on a valid 2D and 3D struct and on one broken field at a time, under the address and
// undefined-behaviour sanitizers; every case must return its documented status.  Exit
// status 0 when all do.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <vector>

#include "validate.hpp"

using cuesim::validate_params;

namespace {

int failures = 0;

struct Case2D {
    std::vector<int32_t> cells{0, 5, 5, 99};
    std::vector<float> q{1.0f, 2.0f, 0.5f, 1.5f};
    std::vector<float> pos{0.0f, 0.0f, 9.99f, 9.99f, 3.5f, 4.5f};
    std::vector<float> dir{0.1f, -2.0f, 3.0f};
    std::vector<float> targets{1.0f, 2.0f, 8.0f, 8.0f};
    std::vector<float> init = std::vector<float>(100, 0.25f);
    sim_params p{};
    Case2D() {
        p.struct_size = sizeof(sim_params);
        p.dim = 2;
        p.nx = p.ny = 10;
        p.nz = 1;
        p.dx = 1.0;
        p.dt = 0.2;
        p.n_species = 1;
        p.D[0] = 1.0;
        p.k[0] = 0.01;
        p.sign[0] = 1.0;
        p.n_sources[0] = 4;
        p.source_cell[0] = cells.data();
        p.source_q[0] = q.data();
        p.init_field[0] = init.data();
        p.n_cones = 3;
        p.cone_pos = pos.data();
        p.cone_dir = dir.data();
        p.n_targets = 2;
        p.target_pos = targets.data();
        p.contact_radius = 1.0;
        p.step_len = 0.5;
        p.turn_gain = 10.0;
        p.max_turn = M_PI / 30.0;
        p.noise_sigma = 0.1;
    }
};

void expect(const char* what, const sim_params& p, sim_status want) {
    char msg[512] = "";
    const sim_status got = validate_params(&p, msg, sizeof msg);
    if (got != want) {
        std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, msg);
        ++failures;
    }
}

void broken(const char* what, sim_status want, const std::function<void(sim_params&)>& edit) {
    Case2D c;
    edit(c.p);
    expect(what, c.p, want);
}

}  // namespace

int main() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const float fnan = std::numeric_limits<float>::quiet_NaN();
    {
        Case2D c;
        expect("valid 2D", c.p, SIM_OK);
    }
    {   // valid 3D, two species, SNR law rejected in 3D
        std::vector<int32_t> cells{0, 63};
        std::vector<float> q{1.0f, 1.0f};
        std::vector<float> pos{0.5f, 0.5f, 0.5f, 3.9f, 3.9f, 3.9f};
        const float s = 1.0f / std::sqrt(3.0f);
        std::vector<float> dir{1.0f, 0.0f, 0.0f, s, s, s};
        sim_params p{};
        p.struct_size = sizeof(sim_params);
        p.dim = 3;
        p.nx = p.ny = p.nz = 4;
        p.dx = 1.0;
        p.dt = 0.15;
        p.n_species = 2;
        for (int sp = 0; sp < 2; ++sp) {
            p.D[sp] = sp ? 0.5 : 1.0;
            p.k[sp] = 0.01;
            p.sign[sp] = sp ? -1.0 : 1.0;
            p.n_sources[sp] = 2;
            p.source_cell[sp] = cells.data();
            p.source_q[sp] = q.data();
        }
        p.n_cones = 2;
        p.cone_pos = pos.data();
        p.cone_dir = dir.data();
        p.max_turn = M_PI / 30.0;
        expect("valid 3D", p, SIM_OK);
        p.turn_law = SIM_TURN_SNR;
        p.kd = 1.0;
        p.c_min = 1e-3;
        p.c_max = 1.0;
        expect("SNR law in 3D", p, SIM_EINVAL);
        p.turn_law = SIM_TURN_VECTOR;
        dir[3] = 2.0f;
        expect("3D heading not unit", p, SIM_EINVAL);
    }
    {
        char msg[64];
        if (validate_params(nullptr, msg, sizeof msg) != SIM_EINVAL) ++failures;
    }
    broken("struct size", SIM_EINVAL, [](sim_params& p) { p.struct_size = 8; });
    broken("dim 4", SIM_EINVAL, [](sim_params& p) { p.dim = 4; });
    broken("one-cell axis", SIM_EINVAL, [](sim_params& p) { p.nx = 1; });
    broken("grid beyond 2^31 cells", SIM_EINVAL, [](sim_params& p) {
        p.nx = 70000;
        p.ny = 70000;
        p.init_field[0] = nullptr;
    });
    broken("dt NaN", SIM_EINVAL, [&](sim_params& p) { p.dt = nan; });
    broken("dx 0", SIM_EINVAL, [](sim_params& p) { p.dx = 0.0; });
    broken("3 species", SIM_EINVAL, [](sim_params& p) { p.n_species = 3; });
    broken("negative D", SIM_EINVAL, [](sim_params& p) { p.D[0] = -1.0; });
    broken("CFL", SIM_ECFL, [](sim_params& p) { p.D[0] = 1.3; });
    broken("positivity", SIM_ECFL, [](sim_params& p) { p.k[0] = 4.0; });
    broken("sources NULL", SIM_EINVAL, [](sim_params& p) { p.source_cell[0] = nullptr; });
    broken("negative sources", SIM_EINVAL, [](sim_params& p) { p.n_sources[0] = -1; });
    broken("source cell", SIM_EINVAL, [](sim_params& p) {
        static const int32_t bad[4] = {0, 1, 100, 2};
        p.source_cell[0] = bad;
    });
    broken("source q", SIM_EINVAL, [&](sim_params& p) {
        static float q[4] = {1.0f, 1.0f, 1.0f, 1.0f};
        q[2] = fnan;
        p.source_q[0] = q;
    });
    broken("init field", SIM_EINVAL, [&](sim_params& p) {
        static std::vector<float> f(100, 0.0f);
        f[99] = std::numeric_limits<float>::infinity();
        p.init_field[0] = f.data();
    });
    broken("cones NULL", SIM_EINVAL, [](sim_params& p) { p.cone_pos = nullptr; });
    broken("cone outside", SIM_EINVAL, [](sim_params& p) {
        static const float pos[6] = {0.0f, 0.0f, 10.0f, 1.0f, 3.0f, 3.0f};
        p.cone_pos = pos;
    });
    broken("cone heading", SIM_EINVAL, [&](sim_params& p) {
        static float dir[3] = {0.0f, 0.0f, 0.0f};
        dir[1] = fnan;
        p.cone_dir = dir;
    });
    broken("targets NULL", SIM_EINVAL, [](sim_params& p) { p.target_pos = nullptr; });
    broken("negative radius", SIM_EINVAL, [](sim_params& p) { p.contact_radius = -1.0; });
    broken("max turn", SIM_EINVAL, [](sim_params& p) { p.max_turn = 4.0; });
    broken("block steps", SIM_EINVAL, [](sim_params& p) { p.block_steps = 33; });
    broken("row width", SIM_EINVAL, [](sim_params& p) { p.tile_cols_per_lane = 3; });
    broken("tile height", SIM_EINVAL, [](sim_params& p) { p.tile_height = -1; });
    broken("turn law", SIM_EINVAL, [](sim_params& p) { p.turn_law = 7; });
    broken("SNR window", SIM_EINVAL, [](sim_params& p) {
        p.turn_law = SIM_TURN_SNR;
        p.kd = 1.0;
        p.c_min = 2.0;
        p.c_max = 1.0;
    });
    broken("SNR valid", SIM_OK, [](sim_params& p) {
        p.turn_law = SIM_TURN_SNR;
        p.kd = 1.0;
        p.c_min = 1e-3;
        p.c_max = 1.0;
    });
    broken("D = 0 allowed", SIM_OK, [](sim_params& p) { p.D[0] = 0.0; });
    broken("no cones, no targets", SIM_OK, [](sim_params& p) {
        p.n_cones = 0;
        p.cone_pos = nullptr;
        p.cone_dir = nullptr;
        p.n_targets = 0;
        p.target_pos = nullptr;
    });
    if (failures) {
        std::fprintf(stderr, "%d cases failed\n", failures);
        return 1;
    }
    std::printf("validate driver: ok\n");
    return 0;
}
