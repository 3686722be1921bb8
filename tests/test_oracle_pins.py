"""The FP64 oracle against exact invariants, closed forms, brute force and an independent
Philox implementation (CPU only)."""
import pytest

import pins


@pytest.fixture(autouse=True)
def _built(oracle_lib):
    return oracle_lib


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_recursion(dim):
    pins.pin_mass_recursion(dim=dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_point_mass_moments(dim):
    pins.pin_moments(dim=dim)


def test_green_function():
    pins.pin_green_function()


def test_steady_state_2d_bessel_k0():
    pins.pin_steady_state_2d()


def test_steady_state_3d_yukawa():
    pins.pin_steady_state_3d()


def test_line_source_exact_discrete_steady_state():
    pins.pin_line_source()


@pytest.mark.parametrize("dim", [2, 3])
def test_cosine_eigenmodes(dim):
    pins.pin_eigenmodes(dim=dim)


def test_unstable_mode_above_stability_limit():
    pins.pin_unstable_mode()


@pytest.mark.parametrize("dim", [2, 3])
def test_max_principle(dim):
    pins.pin_max_principle(dim=dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_exact_for_quadratics(dim):
    pins.pin_gradient_quadratic(dim=dim)


def test_turn_rule_2d_vector_addition():
    pins.pin_turn_rule_2d()


def test_turn_rule_3d_vector_addition():
    pins.pin_turn_rule_3d()


@pytest.mark.parametrize("dim", [2, 3])
def test_direct_guidance_brute_force(dim):
    pins.pin_direct_guidance(dim=dim)


def test_contact_and_exit_edges():
    pins.pin_contact_edges()


def test_noise_stream_plumbing():
    pins.pin_noise_plumbing()


def test_noise_3d_tangent_rotation_statistics():
    pins.pin_noise_3d()


def test_mirror_symmetry():
    pins.pin_mirror()


def test_philox_matches_torch_engine():
    pins.pin_philox_vs_torch()


def test_box_muller_statistics():
    pins.pin_normal_statistics()


@pytest.mark.parametrize("n_species", [1, 2])
def test_adjoint_matches_finite_differences(n_species):
    pins.pin_adjoint_fd(n_species=n_species)


def test_adjoint_zero_without_coupling():
    pins.pin_adjoint_no_coupling()


def test_connectivity_and_bfs():
    pins.pin_connectivity()


def test_snr_turn_law():
    pins.pin_snr_law()


def test_adjoint_summand_magnitudes():
    pins.pin_adjoint_magnitude()
