"""Contact search across target-grid cell boundaries (GPU against the FP64 oracle).

The library bins targets into cubic cells (side max(R, longest side / 512 in 2D or / 128 in
3D)) and, for a tip p, searches only the cells between those of p - R and p + R on every
axis.  Here every target sits within 1% of a cell boundary and a cone's tip lands, after one
straight step (no steering, no noise), on the far side of that boundary at distance
R - 0.05 R (must stop on it) or R + 0.05 R (must not), so a search that missed a
neighbouring cell, or took one too few, would change the events.  Both the cell = R case and
the cell > R case are covered, in 2D (tiled and un-blocked paths) and 3D.
"""
import numpy as np
import pytest

import parity
from paper_1405_3331_amd import scenarios as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _edge_scenario(dim, n, R, seed):
    rng = np.random.default_rng(seed)
    dt = 0.2 if dim == 2 else 0.15   # within the explicit step's stability limit
    sc = S.make_scenario("contact edges", dim, n, 1.0, dt, ((1.0, 0.01, 1.0),), 1,
                         (1.0, 1.0), 0, 0, contact_radius=R, turn_gain=0.0, noise_sigma=0.0,
                         step_len=0.5, seed=seed)
    n = np.array(n, dtype=np.float64)
    cell = max(R, n.max() / (512 if dim == 2 else 128))
    lo, hi = 2.0 * R + 1.0, n - 2.0 * R - 1.0
    targets, cones, dirs = [], [], []
    for _ in range(4000):
        if len(targets) == 120:
            break
        # a target within 1% of a cell boundary on a random subset of axes
        t = lo + rng.random(dim) * (hi - lo)
        for a in range(dim):
            if rng.random() < 0.7:
                k = np.round(t[a] / cell)
                t[a] = k * cell + rng.uniform(-0.01, 0.01) * cell
        if any(np.linalg.norm(t - u) < 4.0 * R + 1.0 for u in targets):
            continue
        targets.append(t)
        for d in (0.95 * R, 1.05 * R):
            # tip after the step: across the boundary from the target where it has one
            u = rng.normal(size=dim)
            for a in range(dim):
                edge = np.round(t[a] / cell) * cell
                if abs(t[a] - edge) < 0.02 * cell:
                    u[a] = -abs(u[a]) if t[a] > edge else abs(u[a])
            u /= np.linalg.norm(u)
            tip = t + d * u
            h = rng.normal(size=dim)
            h /= np.linalg.norm(h)
            cones.append(tip - 0.5 * h)
            dirs.append(np.arctan2(h[1], h[0]) if dim == 2 else h)
    assert len(targets) >= 6
    f32 = lambda v: np.asarray(v, dtype=np.float32).astype(np.float64)
    sc.target_pos = f32(targets)
    sc.cone_pos = f32(cones)
    sc.cone_dir = f32(dirs)
    if dim == 3:   # headings renormalised in FP32 the way the inputs are
        sc.cone_dir = f32(sc.cone_dir / np.linalg.norm(sc.cone_dir, axis=1, keepdims=True))
    return sc


@pytest.mark.parametrize("block", [1, 0])
@pytest.mark.parametrize("n,R", [((64, 48), 1.0), ((64, 48), 2.5), ((1024, 40), 1.0)])
def test_contact_across_cell_boundaries_2d(n, R, block):
    sc = _edge_scenario(2, n, R, seed=31)
    _say(f"2D {n} R={R} block_steps={block}: {sc.n_targets} targets, {sc.n_cones} cones")
    run = parity.FullRun(sc, block)
    run.advance(1, where="step 1")
    status = run.sim.cones()["status"]
    # the inner cone of each pair stops on its target at the first step, the outer does not
    assert (status[0::2] == 1).all() and not (status[1::2] == 1).any()
    run.advance(2, where="step 3")
    run.sim.close()


@pytest.mark.parametrize("n,R", [((24, 20, 18), 1.0), ((256, 16, 16), 1.0)])
def test_contact_across_cell_boundaries_3d(n, R):
    sc = _edge_scenario(3, n, R, seed=32)
    _say(f"3D {n} R={R}: {sc.n_targets} targets, {sc.n_cones} cones")
    run = parity.FullRun(sc, 1)
    run.advance(1, where="step 1")
    status = run.sim.cones()["status"]
    assert (status[0::2] == 1).all() and not (status[1::2] == 1).any()
    run.advance(2, where="step 3")
    run.sim.close()
