"""3D cones held in spatial order on the GPU.

The ordered state (tips sorted by the Morton code of their cell, refreshed every few steps)
changes which thread steps which cone, never a cone's arithmetic, so:

* parity with the FP64 oracle holds at a size spanning many workgroups, with cones that
  stop (contacts and exits) between refreshes;
* the result is bit-identical however the steps are split into calls, with reads of the
  state (which bring the ordered copy back to caller order) in between;
* a write of cone state between calls (which rebuilds the order) continues exactly as a
  fresh simulation started from that state.
"""
import numpy as np
import pytest

import parity
from paper_1405_3331_amd import binding as B
from paper_1405_3331_amd import scenarios as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _scenario(seed=11):
    # 64 x 48 x 40 cells, two species, 8000 cones (32 workgroups), dense targets
    return S.make_scenario("3d ordered", 3, (64, 48, 40), 1.0, 0.15,
                           ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), [8, 8], (1.0, 2.0),
                           8000, 600, seed=seed)


def _same(a, b):
    for k in ("pos", "dir", "status", "target", "event_step"):
        assert np.array_equal(a[k], b[k]), k


def test_ordered_cones_parity():
    sc = _scenario()
    _say("3D 64x48x40, 8000 cones, 80 steps, checked every 20")
    run = parity.FullRun(sc, 1)
    for k in range(4):
        run.advance(20, where=f"step {20 * (k + 1)}")
    counts = run.sim.counts()
    _say(f"counts {counts.tolist()} worst field {run.worst['field']:.2e} "
         f"tip {run.worst['tip']:.2e}")
    summary = run.summary()
    _say(parity.describe(summary))
    parity.check_exclusions(summary)
    assert counts[1] > 0 and counts[2] > 0   # contacts and exits both happened
    run.sim.close()


def test_ordered_cones_call_split_invariance():
    sc = _scenario(seed=12)
    _say("3D 64x48x40: 70 steps in one call vs in calls of 1..9 with reads between")
    one = B.Simulation(sc, block_steps=1)
    one.step(70)
    ref = one.cones()
    split = B.Simulation(sc, block_steps=1)
    done, n = 0, 1
    while done < 70:
        k = min(n, 70 - done)
        split.step(k)
        split.cones()           # brings the ordered copy back to caller order
        done += k
        n = n % 9 + 1
    _same(split.cones(), ref)
    assert np.array_equal(split.field(0), one.field(0))
    assert np.array_equal(split.field(1), one.field(1))
    one.close()
    split.close()


def test_ordered_cones_state_write_restarts_order():
    sc = _scenario(seed=13)
    _say("3D 64x48x40: write cone state mid-run, continue; compare with a fresh simulation "
         "loaded with the same state")
    sim = B.Simulation(sc, block_steps=1)
    sim.step(25)
    c = sim.cones()
    # send the first 100 cones back to their start and reactivate them
    c["pos"][:100] = sc.cone_pos[:100]
    c["status"][:100] = 0
    c["target"][:100] = -1
    c["event_step"][:100] = -1
    sim.write(B.CONE_POS, c["pos"]).write(B.CONE_STATUS, c["status"])
    sim.write(B.CONE_TARGET, c["target"]).write(B.CONE_EVENT_STEP, c["event_step"])
    fields = [sim.field(0), sim.field(1)]
    fresh = B.Simulation(sc, block_steps=1)
    for s, f in enumerate(fields):
        fresh.write(B.FIELD, f, s)
    for item, key in ((B.CONE_POS, "pos"), (B.CONE_DIR, "dir"), (B.CONE_STATUS, "status"),
                      (B.CONE_TARGET, "target"), (B.CONE_EVENT_STEP, "event_step")):
        fresh.write(item, c[key])
    fresh.write(B.STEP, np.array([25], dtype=np.int64))
    sim.step(30)
    fresh.step(30)
    got = sim.cones()
    _same(fresh.cones(), got)
    moved = np.linalg.norm(got["pos"][:100] - sc.cone_pos[:100], axis=1)
    assert (moved > 0).all()   # the reactivated cones were stepped
    sim.close()
    fresh.close()


@pytest.mark.parametrize("shape", [(70, 9, 37), (2, 2, 2), (65, 5, 33)])
def test_field3d_ragged_boxes_and_dense_sources(shape):
    """The one-launch 3D field step on grids that end inside a box on every axis (x past a
    64-column tile, y past a 4-row tile, z past a 32-plane chunk and a 4-plane group), with
    hundreds of sources per species so that boxes hold many (some cells drawn twice)."""
    n = shape[0] * shape[1] * shape[2]
    sc = S.make_scenario("3d field", 3, shape, 1.0, 0.15,
                         ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), [min(300, 2 * n)] * 2,
                         (0.5, 2.0), 0, 0, seed=21)
    _say(f"3D field {shape}, {len(sc.species[0].source_q)} sources per species, 40 steps")
    run = parity.FullRun(sc, 1)
    run.advance(20, where="step 20")
    run.advance(20, where="step 40")
    run.sim.close()


def test_volume_full_size_short_run_elementwise():
    """The 3D workload at full size (256^3, two species, 262,144 cones, 4096 targets) in the
    configuration bench.py times: 40 steps compared element by element with the oracle,
    across the refresh of the cones' spatial order at step 32.  Stop events and tips are
    compared over ALL cones, flagged ones included: at most 0.01% may differ."""
    sc = S.volume()
    _say("volume 256^3 two species, 262144 cones, 40 steps")
    run = parity.FullRun(sc, 1)
    for n in (2, 30, 34, 40):   # before and after the order refresh at step 32
        run.advance(n - run.ref.step_count, where=f"step {n}")
    summary = run.summary()
    _say(parity.describe(summary))
    parity.check_exclusions(summary)
    _say(f"worst field {run.worst['field']:.2e} tip {run.worst['tip']:.2e}")
    run.sim.close()


def test_volume_full_size_mass():
    """At full size over 400 steps, each species' FP64-accumulated mass follows the exact
    recursion M <- (1 - k dt) M + sum q."""
    sc = S.volume()
    sim = B.Simulation(sc, block_steps=1)
    M = np.zeros(2)
    kdt = np.array([s.k * sc.dt for s in sc.species])
    Q = np.array([float(np.sum(s.source_q)) for s in sc.species])
    for blk in range(4):
        sim.step(100)
        for _ in range(100):
            M = (1 - kdt) * M + Q
        got = sim.mass()
        assert np.all(np.abs(got - M) <= 1e-5 * M), (blk, got, M)
    assert sim.counts().sum() == sc.n_cones
    sim.close()
