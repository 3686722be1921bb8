"""Trajectory-loss gradient on the GPU (sim_adjoint_run / sim_adjoint_backward) against
the FP64 oracle's reverse sweep, checkpoint invariance, error paths and the torch binding."""
import math

import numpy as np
import pytest

import oracle
from paper_1405_3331_amd import binding as B, scenarios

pytestmark = pytest.mark.gpu

# FP32 forward + reverse against FP64: the tips agree to ~1e-6 of the domain over these
# runs, and the gradient's relative error stays within 1e-3 of its largest component.
GRAD_TOL = 1e-3


@pytest.fixture(autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _case(n_species=1, n=(96, 80), cones=48, seed=4):
    species = ((1.0, 0.01, 1.0),) if n_species == 1 else ((1.0, 0.01, 1.0), (0.6, 0.02, -1.0))
    return scenarios.make_scenario("adjoint case", 2, n, 1.0, 0.2, species, 4, (2.0, 8.0),
                                   cones, 12, 1.0, 0.5, 10.0, math.pi / 30.0, 0.1, seed=seed)


def _compare(sc, steps, every, block_steps=0):
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    w = np.linspace(0.5, 1.5, M)
    ref = oracle.OracleSim(sc)
    L_ref, dq_ref, dD_ref, dk_ref = ref.adjoint(steps, assign, w)
    sim = B.Simulation(sc, block_steps=block_steps)
    L = sim.adjoint(steps, assign, w, every)
    c = sim.cones()
    # the comparison is meaningful only on the same branch: identical stop events
    np.testing.assert_array_equal(c["status"], ref.status)
    np.testing.assert_array_equal(c["event_step"], ref.event_step)
    dq, dD, dk = sim.adjoint_backward()
    sim.close()
    got = np.concatenate([dq, dD, dk])
    want = np.concatenate([dq_ref, dD_ref, dk_ref])
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"[adjoint] steps={steps} every={every} loss rel {abs(L - L_ref) / L_ref:.2e} "
          f"grad rel {err:.2e}", flush=True)
    assert abs(L - L_ref) <= 1e-5 * L_ref
    assert err <= GRAD_TOL, (got, want)
    return got


@pytest.mark.parametrize("n_species", [1, 2])
def test_gradient_matches_oracle(n_species):
    sc = _case(n_species)
    _compare(sc, 120, 50)   # three segments, the last one ragged


def test_ragged_boxes_two_species():
    """A grid that ends inside the reverse kernels' boxes on both axes (300 x 43: two
    256-column boxes, rows not a multiple of 4 or 8), two species, odd and even segment
    lengths (25, 25, 10): the two-step and the single-step reverse launches both run."""
    sc = _case(2, n=(300, 43), cones=64, seed=9)
    _compare(sc, 60, 25)


def test_sources_on_box_edges():
    """Sources on the cells either side of the two-step kernels' box edges (columns 255/256,
    rows 7/8 and 15/16, edges of 4- and of 8-row boxes), at the walls and duplicated: the
    forward re-run adds them in the one-cell ring of the neighbouring boxes, the reverse
    gathers them per box.  Two species, a segment of odd length."""
    sc = _case(2, n=(300, 24), cones=64, seed=11)
    cells = [(255, 7), (256, 8), (255, 8), (256, 7), (0, 0), (299, 23), (128, 15), (128, 16),
             (255, 16), (0, 8)]
    for s, sp in enumerate(sc.species):
        picked = cells[s::2] + [cells[s]]            # one cell listed twice
        sp.source_cell = np.array([j * 300 + i for i, j in picked], dtype=np.int32)
        sp.source_q = np.linspace(2.0, 6.0, len(picked)).astype(np.float32).astype(np.float64)
    _compare(sc, 45, 15)


def test_tiny_grid():
    """A 7 x 2 grid (short steps, one target far enough for the cones to keep moving):
    every box is ragged and nearly every neighbour index is clamped; segments of 4, 4, 1."""
    sc = scenarios.make_scenario("tiny", 2, (7, 2), 1.0, 0.2, ((1.0, 0.01, 1.0),), 2,
                                 (2.0, 8.0), 4, 1, 0.2, 0.05, 10.0, math.pi / 30.0, 0.1,
                                 seed=12)
    _compare(sc, 9, 4)


def test_checkpoint_spacing_does_not_change_the_gradient():
    sc = _case(1, seed=7)
    a = _compare(sc, 90, 90)   # whole run recorded once
    b = _compare(sc, 90, 7)    # many short segments
    c = _compare(sc, 90, 1)    # one-step segments: single-step kernels only
    assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()
    assert np.abs(a - c).max() <= 1e-5 * np.abs(a).max()


def test_tiled_forward_and_plain_forward_agree():
    sc = _case(1, seed=9)
    a = _compare(sc, 60, 25, block_steps=1)
    b = _compare(sc, 60, 25, block_steps=8)
    assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()


def test_zero_steps_and_zero_weights():
    sc = _case(1)
    M = sc.n_cones
    assign = np.zeros(M, dtype=np.int32)
    with B.Simulation(sc) as sim:
        L = sim.adjoint(0, assign, np.ones(M), 10)
        d = sim.cones()["pos"] - sc.target_pos[0]
        assert abs(L - float((d.astype(np.float64) ** 2).sum())) <= 1e-6 * L
        dq, dD, dk = sim.adjoint_backward()
        assert not dq.any() and not dD.any() and not dk.any()
        sim.adjoint(20, assign, np.zeros(M), 10)
        dq, dD, dk = sim.adjoint_backward()
        assert not dq.any() and not dD.any() and not dk.any()


def test_error_paths():
    sc = _case(1)
    M = sc.n_cones
    with B.Simulation(sc) as sim:
        with pytest.raises(B.SimError) as e:
            sim.adjoint_backward()
        assert e.value.status == B.SIM_ESTATE
        with pytest.raises(B.SimError) as e:
            sim.adjoint(10, np.full(M, 99, dtype=np.int32), np.ones(M), 5)
        assert e.value.status == B.SIM_EINVAL
        with pytest.raises(B.SimError) as e:
            sim.adjoint(10, np.zeros(M, dtype=np.int32), np.ones(M), 0)
        assert e.value.status == B.SIM_EINVAL
        sim.adjoint(10, np.zeros(M, dtype=np.int32), np.ones(M), 5)
        sim.step(1)
        with pytest.raises(B.SimError) as e:
            sim.adjoint_backward()
        assert e.value.status == B.SIM_ESTATE
    sc3 = scenarios.make_scenario("3d", 3, (16, 16, 16), dt=0.1, n_cones=8, n_targets=4,
                                  n_sources=2)
    with B.Simulation(sc3) as sim:
        with pytest.raises(B.SimError) as e:
            sim.adjoint(5, np.zeros(8, dtype=np.int32), np.ones(8), 5)
        assert e.value.status == B.SIM_EINVAL


def test_torch_autograd_function():
    import torch
    from paper_1405_3331_amd.autograd import trajectory_loss
    sc = _case(1, seed=11)
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    w = np.ones(M)
    q = torch.tensor(sc.species[0].source_q, dtype=torch.float64, requires_grad=True)
    D = torch.tensor([sc.species[0].D], dtype=torch.float64, requires_grad=True)
    k = torch.tensor([sc.species[0].k], dtype=torch.float64, requires_grad=True)
    loss = trajectory_loss(q, D, k, sc, 40, assign, w, checkpoint_every=16)
    (2.0 * loss).backward()
    with B.Simulation(sc) as sim:
        L = sim.adjoint(40, assign, w, 16)
        dq, dD, dk = sim.adjoint_backward()
    assert abs(float(loss.detach()) - L) <= 1e-12 * L
    np.testing.assert_allclose(q.grad.numpy(), 2.0 * dq, rtol=1e-5, atol=1e-9 * np.abs(dq).max())
    np.testing.assert_allclose(D.grad.numpy(), 2.0 * dD, rtol=1e-5)
    np.testing.assert_allclose(k.grad.numpy(), 2.0 * dk, rtol=1e-5)


def test_full_size_gradient_matches_oracle():
    """The gradient workload at full size (1024^2, 8192 cones, 32 sources, 256 targets) in the
    launch configuration bench.py times, over 60 steps in three checkpoint segments (the last
    ragged), against the oracle's FP64 reverse sweep of the same run.  (Finite differences of
    the FP32 forward run are no check at this size: rounding noise in 8192 tips outweighs the
    loss change of any perturbation small enough to stay linear.)"""
    _compare(scenarios.adjoint(), 60, 25)
