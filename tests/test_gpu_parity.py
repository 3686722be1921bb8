"""GPU (gfx950) path against the FP64 oracle through the C ABI.

Bars: field max-abs / max <= 1e-5 per species; tips <= 1e-4 x longest side for cones the
oracle did not flag as near-ties; identical events (status, target, step) for those cones.
"""
import math
import os

import numpy as np
import pytest

import oracle
import parity
from paper_1405_3331_amd import autotune
from paper_1405_3331_amd import binding as B
from paper_1405_3331_amd import scenarios as S

pytestmark = pytest.mark.gpu

# one kernel sequence per step; library default (tiled, 8 steps per launch); 3 and 12 steps
BLOCKS = [1, 0, 3, 12]


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def run_pair(sc, steps, block_steps=0, check_every=None, max_differ=None, max_amplified=None):
    """Advance oracle and GPU side by side without restarts; check parity at every
    checkpoint (cones whose tip error grows by the dynamics are classified by a windowed
    re-run, see parity.FullRun).  Events and tips are compared over all cones; the flagged
    cones that differ and the amplified ones are counted, printed and bounded
    (parity.check_exclusions)."""
    run = parity.FullRun(sc, block_steps)
    check_every = check_every or steps
    done = 0
    while done < steps:
        n = min(check_every, steps - done)
        run.advance(n, where=f"step {done + n}")
        done += n
    if run.amplified.any():
        _say(f"amplified cones (windowed parity held): {np.nonzero(run.amplified)[0].tolist()}")
    summary = run.summary()
    _say(parity.describe(summary))
    parity.check_exclusions(summary, max_differ, max_amplified)
    return run.sim, run.ref, run.worst


@pytest.mark.parametrize("block", BLOCKS)
def test_small_2d_full_run(block):
    """The 128^2 small workload, 1000 steps, checked every 100 steps."""
    sc = S.small()
    _say(f"small 2D 128^2 1000 steps block_steps={block}")
    sim, ref, worst = run_pair(sc, 1000, block, 100)
    _say(f"worst field {worst['field']:.2e} tip {worst['tip']:.2e}")
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
def test_small_2d_windowed_tips(block):
    """Windowed tip parity: restart the GPU from the oracle every 100 steps and compare
    every 10 steps (removes dynamical amplification of rounding differences)."""
    sc = S.small(seed=1)
    ref = oracle.OracleSim(sc)
    sim = B.Simulation(sc, block_steps=block)
    for window in range(10):
        parity.restart_from_oracle(sim, ref)
        for _ in range(10):
            ref.step(10)
            sim.step(10)
            m = parity.compare(sim, ref, sc)
            parity.assert_parity(m, where=f"window {window} step {ref.step_count}")
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("shape", [(100, 37), (37, 100), (2, 2), (3, 130), (257, 65)])
def test_ragged_grids(shape, block):
    n = shape[0] * shape[1]
    sc = S.make_scenario("ragged", 2, shape, 1.0, 0.2, ((1.0, 0.01, 1.0),),
                         min(3, n), (0.5, 2.0), 40, 6, seed=3)
    _say(f"ragged {shape} block_steps={block}")
    sim, ref, _ = run_pair(sc, 120, block, 40)
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
def test_two_species_2d(block):
    sc = S.make_scenario("2sp", 2, (90, 70), 0.5, 0.04, ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)),
                         [4, 3], (0.5, 2.0), 80, 10, seed=4)
    sim, ref, _ = run_pair(sc, 300, block, 100)
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
def test_volume_3d_two_species(block):
    sc = S.make_scenario("3d", 3, (24, 20, 18), 1.0, 0.15,
                         ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), [6, 6], (1.0, 1.0), 500, 40,
                         seed=5)
    _say(f"3D 24x20x18 two species block_steps={block}")
    sim, ref, _ = run_pair(sc, 200, block, 50)
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("shape", [(300, 21), (513, 9)])
def test_dense_sources_2d(shape, block):
    """Hundreds of sources per species (some cells drawn twice), on grids that end inside a
    workgroup's box on both axes (the un-blocked step's 256-column x 8-row boxes)."""
    sc = S.make_scenario("dense sources", 2, shape, 1.0, 0.2,
                         ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), [400, 300], (0.5, 2.0), 0, 0,
                         seed=22)
    _say(f"dense sources {shape} block_steps={block}")
    sim, ref, _ = run_pair(sc, 60, block, 30)
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
def test_degenerate_cases(block):
    # no cones, no targets, no sources: the field just decays
    sc = S.make_scenario("empty", 2, (33, 17), 1.0, 0.2, ((1.0, 0.05, 1.0),), 0, (1, 1), 0, 0)
    sc.init_field = [np.random.default_rng(0).random(sc.shape)]
    sim, ref, _ = run_pair(sc, 50, block, 25)
    assert sim.counts().tolist() == [0, 0, 0]
    assert sim.events().shape == (0, 4)
    sim.close()
    # zero step length: cones never move; zero contact radius: no contacts
    sc = S.make_scenario("still", 2, (40, 40), 1.0, 0.2, ((1.0, 0.01, 1.0),), 2, (1, 1), 30, 5,
                         contact_radius=0.0, step_len=0.0)
    sim, ref, _ = run_pair(sc, 30, block, 30)
    c = sim.cones()
    assert np.array_equal(c["pos"], sc.cone_pos.astype(np.float32))
    sim.close()
    # zero steps is a no-op
    sim = B.Simulation(sc, block_steps=block)
    sim.step(0)
    assert sim.step_count == 0
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
def test_crowded_tiles(block):
    """Thousands of cones per tile: a crowded tile is stepped by several workgroups (its cones
    shared evenly among parts of at most 512, one cone per thread, each part recomputing the
    tile's stencil), and cones cross tile borders."""
    sc = S.make_scenario("crowded", 2, (200, 180), 1.0, 0.2, ((1.0, 0.01, 1.0),), 5,
                         (0.5, 2.0), 7000, 30, seed=8)
    _say(f"crowded 200x180, 7000 cones, block_steps={block}")
    sim, ref, _ = run_pair(sc, 120, block, 40)
    sim.close()


@pytest.mark.parametrize("block", [3, 12])
def test_one_crowded_tile_in_small_parts(block):
    """All 900 cones start within a 24-cell square, so one or two tiles hold them.  The list
    build then has room for three parts beyond one per tile and shares each crowded tile's
    cones among parts well under 512 (four of 225 if one tile holds them all, two of 225 each
    if two do); as the cones spread the part size changes from launch to launch.  The tiled
    path stays bitwise equal to the un-blocked per-step path."""
    sc = S.make_scenario("cluster", 2, (512, 448), 1.0, 0.2, ((1.0, 0.01, 1.0),), 6,
                         (0.5, 2.0), 900, 24, seed=12)
    rng = np.random.default_rng(12)
    sc.cone_pos = (np.array([250.0, 230.0]) +
                   rng.uniform(-12.0, 12.0, size=(900, 2))).astype(sc.cone_pos.dtype)
    _say(f"one crowded tile, 512x448, 900 cones in a 24-cell square, block_steps={block}")
    tiled = B.Simulation(sc, block_steps=block).step(150)
    plain = B.Simulation(sc, block_steps=1).step(150)
    assert tiled.tiling()["block_steps"] == block
    assert np.array_equal(tiled.field(), plain.field())
    ct, cp = tiled.cones(), plain.cones()
    for k in ct:
        assert np.array_equal(ct[k], cp[k]), k
    tiled.close()
    plain.close()


def test_mass_recursion_on_gpu():
    """M^{n+1} = (1 - k dt) M^n + sum q, with the GPU's FP64-accumulated mass."""
    sc = S.make_scenario("mass", 2, (200, 150), 1.0, 0.2, ((1.0, 0.01, 1.0),), 5, (0.5, 2.0),
                         0, 0)
    sim = B.Simulation(sc)
    M = 0.0
    kdt = sc.species[0].k * sc.dt
    Q = float(np.sum(sc.species[0].source_q))
    for n in range(10):
        sim.step(100)
        for _ in range(100):
            M = (1 - kdt) * M + Q
        got = sim.mass()[0]
        assert abs(got - M) <= 2e-6 * M, (n, got, M)
    sim.close()


@pytest.mark.parametrize("block", BLOCKS)
def test_bitwise_determinism_and_resume(block):
    sc = S.make_scenario("det", 2, (120, 90), 1.0, 0.2, ((1.0, 0.01, 1.0),), 4, (0.5, 2.0),
                         300, 20, seed=6)
    a = B.Simulation(sc, block_steps=block).step(250)
    b = B.Simulation(sc, block_steps=block).step(250)
    fa, fb = a.field(), b.field()
    assert np.array_equal(fa, fb)
    ca, cb = a.cones(), b.cones()
    for k in ca:
        assert np.array_equal(ca[k], cb[k]), k
    # resume: save at 100, restore into a fresh simulation, continue to 250
    c = B.Simulation(sc, block_steps=block).step(100)
    saved = dict(field=c.field(), **c.cones())
    d = B.Simulation(sc, block_steps=block)
    d.write(B.FIELD, saved["field"])
    d.write(B.CONE_POS, saved["pos"])
    d.write(B.CONE_DIR, saved["dir"])
    d.write(B.CONE_STATUS, saved["status"])
    d.write(B.CONE_TARGET, saved["target"])
    d.write(B.CONE_EVENT_STEP, saved["event_step"])
    d.write(B.STEP, np.array([100], dtype=np.int64))
    d.step(150)
    assert np.array_equal(d.field(), fa)
    cd = d.cones()
    for k in ca:
        assert np.array_equal(ca[k], cd[k]), k
    for s in (a, b, c, d):
        s.close()


def test_events_sorted_and_consistent():
    sc = S.small(seed=2)
    sim = B.Simulation(sc).step(1000)
    ev = sim.events()
    c = sim.cones()
    stopped = np.nonzero(c["status"] != B.ACTIVE)[0]
    assert len(ev) == len(stopped)
    assert np.all(np.diff(ev[:, 2]) >= 0)
    for cone, target, step, kind in ev:
        assert c["status"][cone] == kind and c["event_step"][cone] == step
        assert c["target"][cone] == target
        if kind == B.CONTACT:
            d = np.linalg.norm(c["pos"][cone] - sc.target_pos[target])
            assert d < sc.contact_radius * (1 + 1e-6)
    counts = sim.counts()
    assert counts.sum() == sc.n_cones
    sim.close()


def test_headline_size_short_run_elementwise():
    """The 2048^2 headline workload at full size in the default launch configuration: 30
    steps compared element by element with the oracle.  At this size tau = 1e-4 L is 0.2
    cells, so most stop events fall within tau of a tie; they are compared over ALL cones,
    flagged ones included, and at most 0.01% of the cones may differ."""
    sc = S.headline()
    block = autotune.apply(sc)   # the depth and tile shape bench.py uses
    _say(f"headline 2048^2, 65536 cones, 30 steps, block_steps {block}")
    sim, ref, worst = run_pair(sc, 30, block, 15)
    _say(f"worst field {worst['field']:.2e} tip {worst['tip']:.2e}")
    sim.close()


def test_headline_size_long_run_tiled_equals_per_step():
    """At full size over 4000 steps -- long enough for ~16K cones to gather around the
    sources, so that a handful of tiles are each stepped by several workgroups (parts of at
    most 512 cones) -- the tiled path in bench.py's launch configuration gives bitwise the state of the
    un-blocked per-step path (separate field and cone kernels, caller-order cones)."""
    sc = S.headline()
    block = autotune.apply(sc)
    _say(f"headline 2048^2, 4000 steps, tiled (block_steps {block}) vs per-step")
    tiled = B.Simulation(sc, block_steps=block).step(4000)
    plain = B.Simulation(sc, block_steps=1).step(4000)
    assert np.array_equal(tiled.field(), plain.field())
    ct, cp = tiled.cones(), plain.cones()
    for k in ct:
        assert np.array_equal(ct[k], cp[k]), k
    counts = tiled.counts()
    _say(f"active {counts[0]}, contact {counts[1]}, exited {counts[2]}")
    tiled.close()
    plain.close()


def test_headline_size_long_run_mass():
    """At full size over 2000 steps, the GPU field obeys the exact mass recursion."""
    sc = S.headline()
    sim = B.Simulation(sc)
    kdt = sc.species[0].k * sc.dt
    Q = float(np.sum(sc.species[0].source_q))
    M = 0.0
    for blk in range(4):
        sim.step(500)
        for _ in range(500):
            M = (1 - kdt) * M + Q
        got = sim.mass()[0]
        assert abs(got - M) <= 1e-5 * M, (blk, got, M)
    counts = sim.counts()
    assert counts.sum() == sc.n_cones
    sim.close()
