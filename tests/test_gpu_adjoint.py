"""Trajectory-loss gradient on the GPU (sim_adjoint_run / sim_adjoint_backward) against
the FP64 oracle's reverse sweep, checkpoint invariance, error paths and the torch binding."""
import copy
import math

import numpy as np
import pytest

import oracle
from paper_1405_3331_amd import binding as B, scenarios

pytestmark = pytest.mark.gpu

# Gradient tolerance, per component (FP32 forward + reverse against the FP64 oracle):
#   |got_i - want_i| <= GRAD_TOL * magnitude_i + GRAD_FLOOR * max_group magnitude
#                       + COND_K * sensitivity_i
# magnitude_i is the oracle's sum of the absolute values of the terms component i adds up
# (over steps and cells: |a c|, |a Lap c|, or |a| at the source cell): a sum of terms each
# correct to a relative error e is correct to e * magnitude, so every component is held to
# 1e-4 of its own terms however much they cancel (dL/dk of one species can be a thousand
# times smaller than its terms).  Components far smaller than their group's terms (a source
# far from every cone, in the diffusion tail of the cones' sample adjoints) are held to an
# absolute floor of GRAD_FLOOR (the FP32 epsilon) times the group's largest term scale.
#
# sensitivity_i is the conditioning of the component, measured on the oracle alone: the
# largest change of the FP64 gradient when every cone's initial tip and heading move (either
# way) by as many FP32 rounding steps (relative 2^-23 each) as it takes for the oracle's tips
# to move as far as the FP32 run's tips are from the oracle's (their median distance, over
# the compared cones, rounded up to a power of two).  The response of the gradient to such
# moves is far from linear -- the interpolated gradient the cones sample is only continuous,
# so its derivative jumps where a tip crosses a line of cell centres, and a moved trajectory
# crosses some of them on the other side -- so the probe is taken at the FP32 run's own
# distance, and COND_K covers the spread between two such probes and the FP32 run.  Before
# that, the cones whose own trajectories are chaotic at this length (their FP64 tip moves
# more than CHAOS_CELLS under a one-step move, ~16x the move), that the oracle flagged as
# near-ties, or that stop differently on the two sides, are given weight 0 on both sides:
# they leave the loss and the gradient (cones do not interact), and at most MAX_EXCLUDED of
# the cones may be left out.
GRAD_TOL = 1e-4
GRAD_FLOOR = 1e-7
COND_K = 4.0
CHAOS_CELLS = 1e-3
MAX_EXCLUDED = 0.1
# near-tie margin of the stop events here: 1e-5 of the longest side (0.01 cell at 1024^2),
# ten times the chaos threshold above and above the FP32 tips' distance from the oracle's
NEAR_TIE = 1e-5


def _groups(n_q, ns):
    g = [("dL/dq", slice(0, n_q))]
    for s in range(ns):
        g.append((f"dL/dD[{s}]", slice(n_q + s, n_q + s + 1)))
        g.append((f"dL/dk[{s}]", slice(n_q + ns + s, n_q + ns + s + 1)))
    return g


def check_gradient(got, want, magnitude, sensitivity, n_q, ns, where=""):
    """Per-component check; prints each group's worst component."""
    for name, sl in _groups(n_q, ns):
        g, w, mag, sens = got[sl], want[sl], magnitude[sl], sensitivity[sl]
        err = np.abs(g - w)
        bound = GRAD_TOL * mag + GRAD_FLOOR * mag.max() + COND_K * sens
        i = int(np.argmax(err / np.maximum(bound, 1e-300)))
        limited = int((COND_K * sens > GRAD_TOL * mag).sum())
        print(f"[adjoint] {where} {name}: worst component {i}: got {g[i]:.6e} want {w[i]:.6e}, "
              f"error {err[i] / max(mag[i], 1e-300):.2e} of its terms ({mag[i]:.3e}), "
              f"{err[i] / max(abs(w[i]), 1e-300):.2e} of its value, "
              f"{err[i] / max(bound[i], 1e-300):.2f} of its bound; oracle 1-ulp sensitivity "
              f"{sens[i] / max(mag[i], 1e-300):.1e} of its terms; {limited} of {len(g)} "
              f"components conditioning-limited; largest error / sensitivity "
              f"{np.max(err / np.maximum(sens, 1e-300)):.2e}", flush=True)
        assert np.all(err <= bound), (where, name, i, g[i], w[i], mag[i], sens[i])


def _perturbed(sc, sign, ulps=1):
    """Oracle started with every cone's tip and heading `ulps` FP32 rounding steps away (in
    the direction `sign`; 0 = unperturbed); its near-tie margin is NEAR_TIE x the longest
    side."""
    r = oracle.OracleSim(sc, flag_tol=NEAR_TIE * sc.side)
    if sign:
        f = sign * ulps * 2.0 ** -23
        r.set_state(fields=[x.copy() for x in r.fields], pos=r.pos * (1.0 + f),
                    dir=r.dir * (1.0 - f), status=r.status.copy(), target=r.target.copy(),
                    event_step=r.event_step.copy(), step=0)
    return r


def oracle_exclusions(sc, steps):
    """Cones left out of a gradient comparison (weight 0): chaotic at this run length, or
    near-ties the oracle flagged.  Also returns the oracle's final tips and the median tip
    move of the kept cones under a one-step move of every initial tip."""
    runs = [_perturbed(sc, sign).step(steps) for sign in (0.0, 1.0, -1.0)]
    base = runs[0]
    dtip = np.zeros(sc.n_cones)
    for r in runs[1:]:
        dtip = np.maximum(dtip, np.abs(r.pos - base.pos).max(axis=1) / sc.dx)
    excluded = (dtip > CHAOS_CELLS) | (base.flag_step >= 0)
    kept = ~excluded
    return excluded, base, float(np.median(dtip[kept])) if kept.any() else 0.0


def oracle_reference(sc, steps, assign, w, ulps):
    """The oracle's loss and gradient with their summand magnitudes, and each component's
    change under an `ulps`-step move of every initial tip and heading (either way)."""
    grads = []
    for sign in (0.0, 1.0, -1.0):
        out = _perturbed(sc, sign, ulps).adjoint(steps, assign, w, magnitude=(sign == 0.0))
        grads.append((np.concatenate(out[1:4]), out[4] if sign == 0.0 else None, out[0]))
    g0, mag, L0 = grads[0]
    sens = np.maximum(np.abs(grads[1][0] - g0), np.abs(grads[2][0] - g0))
    return L0, g0, mag, sens


@pytest.fixture(autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _case(n_species=1, n=(96, 80), cones=48, seed=4):
    species = ((1.0, 0.01, 1.0),) if n_species == 1 else ((1.0, 0.01, 1.0), (0.6, 0.02, -1.0))
    return scenarios.make_scenario("adjoint case", 2, n, 1.0, 0.2, species, 4, (2.0, 8.0),
                                   cones, 12, 1.0, 0.5, 10.0, math.pi / 30.0, 0.1, seed=seed)


def _run_gpu(sc, steps, every, assign, w, block_steps, tape_limit):
    sim = B.Simulation(sc, block_steps=block_steps)
    if tape_limit:
        sim.set_tape_limit(tape_limit)
    L = sim.adjoint(steps, assign, w, every)
    c = sim.cones()
    dq, dD, dk = sim.adjoint_backward()
    sim.close()
    return L, c, np.concatenate([dq, dD, dk])


def _compare(sc, steps, every, block_steps=0, tape_limit=0):
    """GPU gradient against the oracle's on the same branch of the run, each component
    within its own bound (see GRAD_TOL above).  A cone that stops differently on the two
    sides must be one the oracle flagged, and so already has weight 0."""
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    excluded, ref, move_1 = oracle_exclusions(sc, steps)
    assert excluded.sum() <= max(1, MAX_EXCLUDED * M), excluded.sum()
    w = np.where(excluded, 0.0, np.linspace(0.5, 1.5, M))
    L, c, got = _run_gpu(sc, steps, every, assign, w, block_steps, tape_limit)
    differ = np.nonzero((c["status"] != ref.status) | (c["event_step"] != ref.event_step) |
                        (c["target"] != ref.target))[0]
    assert np.all(excluded[differ]), (differ, ref.flag_step[differ])
    kept = ~excluded
    gpu_move = float(np.median(np.abs(c["pos"][kept] - ref.pos[kept]).max(axis=1))) / sc.dx \
        if kept.any() else 0.0
    ulps = 1
    while ulps * move_1 < gpu_move and ulps < 1 << 12:
        ulps *= 2
    L_ref, want, mag, sens = oracle_reference(sc, steps, assign, w, ulps)
    where = f"steps={steps} every={every} tape_limit={tape_limit}"
    print(f"[adjoint] {where}: {int(excluded.sum())} of {M} cones weighted 0 (chaotic or "
          f"near-tie), {len(differ)} stop differently; FP32 tips {gpu_move:.1e} cells from "
          f"the oracle's (median), a one-step move {move_1:.1e}: probe {ulps} steps; loss rel "
          f"{abs(L - L_ref) / L_ref:.2e}", flush=True)
    assert abs(L - L_ref) <= 1e-5 * L_ref
    n_q = len(want) - 2 * len(sc.species)
    check_gradient(got, want, mag, sens, n_q, len(sc.species), where)
    return got, mag


def _same_gradient(a, b, tol):
    """Two GPU gradients of the same run, per component against the size of its terms."""
    (ga, mag), (gb, _) = a, b
    assert np.all(np.abs(ga - gb) <= tol * mag), np.max(np.abs(ga - gb) / mag)


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
    _same_gradient(a, b, 1e-9)
    _same_gradient(a, c, 1e-9)


@pytest.mark.parametrize("n_species", [1, 2])
def test_segment_rerun_path_matches_whole_run_path(n_species):
    """A one-byte tape limit forces the checkpoint-and-recompute sweep (each segment's
    fields and cone steps re-run from its own checkpoint, just before it is reversed) on a
    run of four ragged segments (35, 35, 35, 25): the same gradient as the sweep that re-runs
    the whole run once, and as the oracle."""
    sc = _case(n_species, seed=13)
    a = _compare(sc, 130, 35)
    b = _compare(sc, 130, 35, tape_limit=1)
    _same_gradient(a, b, 1e-9)


@pytest.mark.parametrize("n_species", [1, 2])
def test_gradient_is_bitwise_reproducible(n_species):
    """The samples' adjoints are summed as integers (fixed point, scaled per step), so two
    runs of the same gradient agree bit for bit, in both sweeps (whole run re-run once, and
    segment by segment), on a crowded grid where many cones sample the same cells."""
    sc = _case(n_species, n=(64, 48), cones=400, seed=21)
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    w = np.linspace(0.5, 1.5, M)
    runs = []
    for tape_limit in (0, 0, 1, 1):
        L, _, g = _run_gpu(sc, 90, 30, assign, w, 0, tape_limit)
        runs.append((L, g))
    for L, g in runs[1:]:
        assert L == runs[0][0]
        np.testing.assert_array_equal(g, runs[0][1])


def test_tiled_forward_and_plain_forward_agree():
    sc = _case(1, seed=9)
    a = _compare(sc, 60, 25, block_steps=1)
    b = _compare(sc, 60, 25, block_steps=8)
    _same_gradient(a, b, 1e-9)


def test_deep_tiled_forward_agrees():
    """The recording forward run at the depth and tile height the autotuner chose for the
    gradient workload (16 steps per launch, 110-row tiles), on a grid of several tiles with
    checkpoints that do not fall on launch boundaries, gives the gradient of the per-step
    run."""
    sc = _case(1, n=(300, 260), cones=160, seed=10)
    deep = copy.copy(sc)
    deep.tile = (2, 110)
    with B.Simulation(deep, block_steps=16) as sim:
        assert sim.tiling()["block_steps"] == 16
    a = _compare(sc, 70, 30, block_steps=1)
    b = _compare(deep, 70, 30, block_steps=16)
    _same_gradient(a, b, 1e-9)


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
    launch configuration bench.py times, over 400 steps in four checkpoint segments of 100,
    against the oracle's FP64 reverse sweep of the same run, each component on its own scale.
    (Finite differences of the FP32 forward run are no check at this size: rounding noise in
    8192 tips outweighs the loss change of any perturbation small enough to stay linear.)"""
    _compare(scenarios.adjoint(), 400, 100)
