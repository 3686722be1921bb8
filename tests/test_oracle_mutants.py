"""Planted mistakes: rebuild the oracle with one plausible error each (a dropped term, a
wrong sign, index or factor, a transposed operand) and require that at least one pin
fails.  This shows the pins constrain every part of the oracle."""
import os
import shutil
import tempfile

import pytest

import pins
from oracle import build as obuild

SRC = os.path.join(os.path.dirname(obuild.SOURCE), "cuesim_oracle.c")

# (name, original text, planted text, pins expected to catch it)
MUTANTS = [
    ("laplacian_centre_weight", "- 2.0 * centre;", "- 1.0 * centre;", ["mass2d", "eigen2d"]),
    ("decay_sign", "+ r * laplacian_sum - kdt * centre;", "+ r * laplacian_sum + kdt * centre;",
     ["mass2d"]),
    ("dirichlet_walls", "        return c[cell_index(p, idx)];\n    return c[cell_index(p, nb)];",
     "        return 0.0;\n    return c[cell_index(p, nb)];", ["mass2d", "eigen2d"]),
    ("source_units", "p->source_q[s][m] / cell_volume", "p->source_q[s][m] / p->dx",
     ["mass2d", "line"]),
    ("source_overwrites", "c_new[p->source_cell[s][m]] +=", "c_new[p->source_cell[s][m]] =",
     ["mass2d"]),
    ("layout_transposed", "return (l * p->ny + idx[1]) * p->nx + idx[0];",
     "return (l * p->nx + idx[1]) * p->ny + idx[0];", ["eigen2d", "mass2d"]),
    ("cell_centre_offset", "double u = point[a] / p->dx - 0.5;", "double u = point[a] / p->dx;",
     ["grad2d"]),
    ("interp_weights_swapped", "weight *= upper ? frac[a] : (1.0 - frac[a]);",
     "weight *= upper ? (1.0 - frac[a]) : frac[a];", ["grad2d"]),
    ("gradient_spacing", "/ (2.0 * p->dx);\n}", "/ p->dx;\n}", ["grad2d"]),
    ("species_sign_dropped", "g[a] += p->sign[sp] * gs[a];", "g[a] += gs[a];", ["turn2d"]),
    ("turn_away", "double cross = hx * g[1] - hy * g[0];", "double cross = hy * g[0] - hx * g[1];",
     ["turn2d"]),
    ("no_turn_cap", "if (delta > p->max_turn) delta = p->max_turn;", "", ["turn2d"]),
    ("turn_3d_away", "h[a] = c * h[a] + s * perp[a] / perp_norm;",
     "h[a] = c * h[a] - s * perp[a] / perp_norm;", ["turn3d"]),
    ("noise_counter_swapped", "(uint32_t)i, (uint32_t)(n >> 1), 0u, p->sim_index",
     "(uint32_t)(n >> 1), (uint32_t)i, 0u, p->sim_index", ["noise"]),
    ("noise_pair_ignored", "z[0] = zz[2 * (n & 1)];", "z[0] = zz[0];", ["noise"]),
    ("noise_3d_counter_swapped", "(uint32_t)i, (uint32_t)n, 0u, p->sim_index",
     "(uint32_t)n, (uint32_t)i, 0u, p->sim_index", ["noise3d", "bruteforce3d"]),
    ("noise_not_tangent", "w[a] = p->noise_sigma * (z[a] - along * h[a]);",
     "w[a] = p->noise_sigma * z[a];", ["noise3d"]),
    ("exit_closed_interval", "if (pos[a] < 0.0 || pos[a] >= domain_length(p, a))",
     "if (pos[a] < 0.0 || pos[a] > domain_length(p, a))", ["edges"]),
    ("contact_not_strict", "best_d2 < R * R", "best_d2 <= R * R", ["edges"]),
    ("tie_to_last", "if (d2 < best_d2) {", "if (d2 <= best_d2) {", ["edges"]),
    ("step_length_twice", "pos[a] += p->step_len * h[a];", "pos[a] += 2.0 * p->step_len * h[a];",
     ["direct2d"]),
    ("philox_round_word", "uint32_t y0 = hi1 ^ x1 ^ k0;", "uint32_t y0 = hi0 ^ x1 ^ k0;", ["philox"]),
    ("philox_key_schedule", "k0 += weyl0;", "k0 += weyl1;", ["philox"]),
    ("box_muller_angle", "z[2 * pair] = radius * cos(2.0 * ORACLE_PI * u_a);",
     "z[2 * pair] = radius * cos(ORACLE_PI * u_a);", ["normals"]),
    ("box_muller_radius", "double radius = sqrt(-2.0 * log(u_r));", "double radius = sqrt(-log(u_r));",
     ["normals"]),
    ("adjoint_no_position_term", "ap[b] += p->sign[sp] * dw / p->dx * sum;", "", ["adjoint"]),
    ("adjoint_scatter_sign", "ac[neighbour_index(p, idx, a, -1)] -= v;",
     "ac[neighbour_index(p, idx, a, -1)] += v;", ["adjoint"]),
    ("adjoint_decay_sign", "aprev[x] = a[x] + r * lap[x] - kdt * a[x];",
     "aprev[x] = a[x] + r * lap[x] + kdt * a[x];", ["adjoint"]),
    ("adjoint_turn_theta", "a_theta += a_y * (-lam * (hx * g[0] + hy * g[1])) + a_x * y;",
     "a_theta += a_x * y;", ["adjoint"]),
    ("adjoint_advance_sign", "(-sin(theta_new) * ap[0] + cos(theta_new) * ap[1])",
     "(sin(theta_new) * ap[0] + cos(theta_new) * ap[1])", ["adjoint"]),
    ("adjoint_species_sign", "double v = p->sign[sp] * w * a_g[a] / (2.0 * p->dx);",
     "double v = w * a_g[a] / (2.0 * p->dx);", ["adjoint2"]),
    ("adjoint_D_units", "dL_dD[sp] += sD * p->dt / (p->dx * p->dx);", "dL_dD[sp] += sD * p->dt;",
     ["adjoint"]),
    ("adjoint_source_units", "dL_dq[q_off[sp] + m] += a[p->source_cell[sp][m]] / vol;",
     "dL_dq[q_off[sp] + m] += a[p->source_cell[sp][m]];", ["adjoint"]),
    ("snr_turn_left", "return x > 0.0 ? theta - p->max_turn : theta + p->max_turn;",
     "return x > 0.0 ? theta + p->max_turn : theta - p->max_turn;", ["snr"]),
    ("snr_no_width", "double snr = p->snr_scale * (p->cone_width / c) *",
     "double snr = p->snr_scale * (1.0 / c) *", ["snr"]),
    ("snr_gamma_power", "sqrt(gamma / pow(1.0 + gamma, 3.0))", "sqrt(gamma / pow(1.0 + gamma, 2.0))",
     ["snr"]),
    ("snr_window_ignored", "if (c < p->c_min || c > p->c_max ||", "if (", ["snr"]),
    ("snr_noise_word", "theta += p->noise_sigma * z[1];", "theta += p->noise_sigma * z[0];",
     ["snr_noise"]),
    ("bfs_level_step", "level[u] = level[v] + 1;", "level[u] = level[v] + 2;", ["graph"]),
    ("adjacency_by_target_owner", "row_start[cone_owner[i] + 1] += 1;",
     "row_start[target_owner[target[i]] + 1] += 1;", ["graph"]),
    ("adjacency_counts_exits", "        if (status[i] == ORACLE_CONTACT)\n            row_start",
     "        if (status[i] != ORACLE_ACTIVE)\n            row_start", ["graph"]),
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mutants")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,orig,planted,catchers", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(workdir, name, orig, planted, catchers):
    text = open(SRC).read()
    assert text.count(orig) == 1, f"mutation anchor not unique/found: {orig!r}"
    src = os.path.join(workdir, f"{name}.c")
    with open(src, "w") as f:
        f.write(text.replace(orig, planted))
    lib = obuild.build(source=src, output=os.path.join(workdir, f"lib_{name}.so"))
    caught = []
    for pin in catchers:
        try:
            pins.ALL_PINS[pin](lib)
        except AssertionError:
            caught.append(pin)
    assert caught, f"planted mistake {name} passed every pin in {catchers}"
