"""Batched simulations (one persistent launch per block of steps for many uneven 2D
simulations) against the same simulations run alone, graph replay against eager launches,
and a batch member against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import parity
from paper_1405_3331_amd import autotune
from paper_1405_3331_amd import binding as B
from paper_1405_3331_amd import scenarios as S

pytestmark = pytest.mark.gpu


def uneven(count=10, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = int(rng.integers(40, 230))
        ny = int(rng.integers(30, 230))
        cones = int(rng.integers(5, 1500))
        out.append(S.make_scenario(f"b{i}", 2, (side, ny), 1.0, 0.2,
                                   ((float(rng.uniform(0.5, 1.2)), float(rng.uniform(0.001, 0.02)), 1.0),),
                                   int(rng.integers(1, 8)), (0.5, 2.0), cones,
                                   int(rng.integers(2, 30)), seed=seed, sim_index=i))
    return out


def assert_same(sim_state, ref_state, what):
    for k in ref_state:
        assert np.array_equal(sim_state[k], ref_state[k]), (what, k)


def test_batch_equals_single_runs_bitwise():
    scs = uneven()
    print(f"[gpu] batch of {len(scs)} uneven simulations, 100 steps", flush=True)
    with B.Batch(scs) as bt:
        bt.step(37)
        bt.step(63)
        for i, sc in enumerate(scs):
            with B.Simulation(sc) as one:
                one.step(100)
                assert np.array_equal(bt.field(i), one.field()), i
                assert_same(bt.cones(i), one.cones(), i)


def test_batch_graph_replays_match_eager():
    scs = uneven(6, seed=4)
    eager = B.Batch(scs, graph_launches=0, block_steps=8)
    graph = B.Batch(scs, graph_launches=3, block_steps=8)
    for replay in range(4):   # each call replays the 3-launch graph once (24 steps)
        eager.step(24)
        graph.step(24)
        graph.synchronize()
        for i in range(len(scs)):
            assert np.array_equal(eager.field(i), graph.field(i)), (replay, i)
            assert_same(graph.cones(i), eager.cones(i), (replay, i))
    eager.close()
    graph.close()


def test_batch_member_matches_oracle():
    scs = uneven(5, seed=5)
    with B.Batch(scs, graph_launches=2) as bt:
        refs = [oracle.OracleSim(sc) for sc in scs]
        for chunk in range(3):
            bt.step(40)
            for i, sc in enumerate(scs):
                refs[i].step(40)
                f = bt.field(i)
                r = refs[i].fields[0]
                assert np.abs(f - r).max() <= 1e-5 * np.abs(r).max(), (chunk, i)
                c = bt.cones(i)
                ok = refs[i].flag_step < 0
                tip = np.abs(c["pos"][ok] - refs[i].pos[ok]).max() / sc.side if ok.any() else 0
                assert tip <= 1e-4, (chunk, i, tip)
                same = ((c["status"] == refs[i].status) & (c["target"] == refs[i].target) &
                        (c["event_step"] == refs[i].event_step))
                assert np.all(same[ok]), (chunk, i)


def test_plain_and_tiled_paths_are_bitwise_identical():
    """The stencil, source and cone arithmetic is the same in the per-step kernels and the
    tiled kernel, so both paths give bitwise identical states."""
    sc = S.make_scenario("cross", 2, (150, 110), 1.0, 0.2, ((1.0, 0.01, 1.0),), 4, (0.5, 2.0),
                         400, 20, seed=9)
    a = B.Simulation(sc, block_steps=1).step(90)
    b = B.Simulation(sc, block_steps=8).step(90)
    assert np.array_equal(a.field(), b.field())
    assert_same(a.cones(), b.cones(), "plain vs tiled")
    a.close()
    b.close()


def test_full_size_batch():
    """The batched workload at full size (512 simulations, sides 64..512, 16..4096 cones) in
    bench.py's launch configuration (10 launches per graph replay): after 80 steps every member
    equals the same simulation run alone bit for bit, and eight of those single runs (the
    smallest, the largest, the most and the fewest cones, four more) match the FP64 oracle
    (full-run parity with the classification of dynamically amplified cones)."""
    scs = S.batched()
    block = autotune.apply_batch(scs)   # the launch shape bench.py uses
    print(f"[gpu] full-size batch: {len(scs)} simulations, 80 steps, block_steps {block}, "
          f"tile hint {getattr(scs[0], 'tile', None)}", flush=True)
    with B.Batch(scs, graph_launches=10, block_steps=block) as bt:
        bt.step(80)
        for i, sc in enumerate(scs):
            with B.Simulation(sc) as one:
                one.step(80)
                assert np.array_equal(bt.field(i), one.field()), i
                assert_same(bt.cones(i), one.cones(), i)
    sides = np.array([sc.nx for sc in scs])
    cones = np.array([sc.n_cones for sc in scs])
    picks = sorted({int(sides.argmin()), int(sides.argmax()), int(cones.argmax()),
                    int(cones.argmin()), 7, 100, 301, 511})
    for i in picks:
        run = parity.FullRun(scs[i])
        run.advance(40, where=f"member {i} step 40")
        run.advance(40, where=f"member {i} step 80")
        print(f"[gpu] member {i}: side {scs[i].nx}, {scs[i].n_cones} cones, worst field "
              f"{run.worst['field']:.2e} tip {run.worst['tip']:.2e}, amplified "
              f"{int(run.amplified.sum())}", flush=True)
        summary = run.summary()
        print(f"[gpu] member {i}: {parity.describe(summary)}", flush=True)
        parity.check_exclusions(summary, where=f"member {i}")
        run.sim.close()
