// validate.cpp -- the checks sim_create applies to a parameter struct before it touches
// the device.  Plain host C++ with no HIP dependency, so that it also builds (and is
// exercised) under the address and undefined-behaviour sanitizers on the CPU.
#include "validate.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

namespace cuesim {

namespace {

sim_status bad(char* msg, size_t cap, sim_status st, const char* fmt, ...) {
    if (msg && cap) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(msg, cap, fmt, ap);
        va_end(ap);
    }
    return st;
}

bool finite(double v) { return std::isfinite(v); }

}  // namespace

sim_status validate_params(const sim_params* p, char* msg, size_t cap) {
    if (!p) return bad(msg, cap, SIM_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(sim_params))
        return bad(msg, cap, SIM_EINVAL, "struct_size %u != sizeof(sim_params) %zu",
                    p->struct_size, sizeof(sim_params));
    if (p->dim != 2 && p->dim != 3) return bad(msg, cap, SIM_EINVAL, "dim must be 2 or 3");
    const int nz = p->dim == 3 ? p->nz : 1;
    if (p->nx < 2 || p->ny < 2 || (p->dim == 3 && p->nz < 2))
        return bad(msg, cap, SIM_EINVAL, "every axis needs at least 2 cells");
    const double cells = (double)p->nx * p->ny * nz;
    if (cells > 2147483647.0) return bad(msg, cap, SIM_EINVAL, "grid has more than 2^31-1 cells");
    if (!finite(p->dx) || !finite(p->dt) || p->dx <= 0 || p->dt <= 0)
        return bad(msg, cap, SIM_EINVAL, "dx and dt must be finite and positive");
    if (p->n_species < 1 || p->n_species > SIM_MAX_SPECIES)
        return bad(msg, cap, SIM_EINVAL, "n_species must be 1 or 2");
    for (int s = 0; s < p->n_species; ++s) {
        if (!finite(p->D[s]) || p->D[s] < 0 || !finite(p->k[s]) || p->k[s] < 0 ||
            !finite(p->sign[s]))
            return bad(msg, cap, SIM_EINVAL, "species %d: D, k must be finite >= 0, sign finite", s);
        const double r = p->D[s] * p->dt / (p->dx * p->dx);
        if (r > 1.0 / (2.0 * p->dim))
            return bad(msg, cap, SIM_ECFL, "species %d: D dt / dx^2 = %g exceeds 1/(2 dim) = %g",
                        s, r, 1.0 / (2.0 * p->dim));
        if (2.0 * p->dim * r + p->k[s] * p->dt > 1.0)
            return bad(msg, cap, SIM_ECFL, "species %d: 2 dim r + k dt = %g exceeds 1", s,
                        2.0 * p->dim * r + p->k[s] * p->dt);
        if (p->n_sources[s] < 0 || (p->n_sources[s] > 0 && (!p->source_cell[s] || !p->source_q[s])))
            return bad(msg, cap, SIM_EINVAL, "species %d: bad source arrays", s);
        for (int m = 0; m < p->n_sources[s]; ++m) {
            if (p->source_cell[s][m] < 0 || (double)p->source_cell[s][m] >= cells)
                return bad(msg, cap, SIM_EINVAL, "species %d source %d: cell %d out of range", s,
                            m, p->source_cell[s][m]);
            if (!std::isfinite(p->source_q[s][m]))
                return bad(msg, cap, SIM_EINVAL, "species %d source %d: q not finite", s, m);
        }
        if (p->init_field[s])
            for (int64_t x = 0; x < (int64_t)cells; ++x)
                if (!std::isfinite(p->init_field[s][x]))
                    return bad(msg, cap, SIM_EINVAL, "species %d: init_field not finite", s);
    }
    if (p->n_cones < 0 || (p->n_cones > 0 && (!p->cone_pos || !p->cone_dir)))
        return bad(msg, cap, SIM_EINVAL, "bad cone arrays");
    const double L[3] = {p->nx * p->dx, p->ny * p->dx, nz * p->dx};
    for (int i = 0; i < p->n_cones; ++i) {
        for (int a = 0; a < p->dim; ++a) {
            const float v = p->cone_pos[(int64_t)i * p->dim + a];
            if (!std::isfinite(v) || v < 0.0f || (double)v >= L[a])
                return bad(msg, cap, SIM_EINVAL, "cone %d: position outside the domain", i);
        }
        if (p->dim == 2) {
            if (!std::isfinite(p->cone_dir[i]))
                return bad(msg, cap, SIM_EINVAL, "cone %d: heading not finite", i);
        } else {
            const float* h = p->cone_dir + (int64_t)i * 3;
            const double n2 = (double)h[0] * h[0] + (double)h[1] * h[1] + (double)h[2] * h[2];
            if (!std::isfinite(n2) || std::fabs(n2 - 1.0) > 1e-3)
                return bad(msg, cap, SIM_EINVAL, "cone %d: heading is not a unit vector", i);
        }
    }
    if (p->n_targets < 0 || (p->n_targets > 0 && !p->target_pos))
        return bad(msg, cap, SIM_EINVAL, "bad target arrays");
    for (int64_t t = 0; t < (int64_t)p->n_targets * p->dim; ++t)
        if (!std::isfinite(p->target_pos[t]))
            return bad(msg, cap, SIM_EINVAL, "target coordinates must be finite");
    if (!finite(p->contact_radius) || p->contact_radius < 0 || !finite(p->step_len) ||
        p->step_len < 0 || !finite(p->turn_gain) || !finite(p->max_turn) || p->max_turn < 0 ||
        p->max_turn > M_PI || !finite(p->noise_sigma) || p->noise_sigma < 0)
        return bad(msg, cap, SIM_EINVAL,
                    "contact_radius, step_len >= 0; max_turn in [0, pi]; noise_sigma >= 0");
    if (p->block_steps < 0 || p->block_steps > 32)
        return bad(msg, cap, SIM_EINVAL, "block_steps must be in [0, 32]");
    if (p->tile_cols_per_lane != 0 && p->tile_cols_per_lane != 2 && p->tile_cols_per_lane != 4)
        return bad(msg, cap, SIM_EINVAL, "tile_cols_per_lane must be 0, 2 or 4");
    if (p->tile_height < 0 || p->tile_height > 4096)
        return bad(msg, cap, SIM_EINVAL, "tile_height must be in [0, 4096]");
    if (p->turn_law != SIM_TURN_VECTOR && p->turn_law != SIM_TURN_SNR)
        return bad(msg, cap, SIM_EINVAL, "turn_law must be SIM_TURN_VECTOR or SIM_TURN_SNR");
    if (p->turn_law == SIM_TURN_SNR &&
        (p->dim != 2 || !finite(p->snr_scale) || !finite(p->cone_width) || p->cone_width < 0 ||
         !finite(p->kd) || !(p->kd > 0) || !finite(p->c_min) || !finite(p->c_max) ||
         !(p->c_min > 0) || p->c_max < p->c_min))
        return bad(msg, cap, SIM_EINVAL,
                    "SNR turn law: 2D only; finite snr_scale, cone_width >= 0, kd > 0, "
                    "0 < c_min <= c_max");
    return SIM_OK;
}

}  // namespace cuesim
