"""The SNR turn law (Sec. 3.5, Eq. 5) on the GPU against the FP64 oracle: full and windowed
runs on every path (plain, tiled at several depths, batched), with the decision's
near-ties (|SNR + Z0| <= 1e-4, concentration within 1e-4 of a window edge) flagged by the
oracle and excluded from the exact comparison like every other near-tie."""
import numpy as np
import pytest

import oracle
import parity
from paper_1405_3331_amd import binding as B
from paper_1405_3331_amd import scenarios as S

pytestmark = pytest.mark.gpu

LAW = (50.0, 1.0, 0.5, 1e-3, 1e3)   # snr_scale, cone_width, kd, c_min, c_max


def _scenario(seed=0, window=(1e-3, 1e3), sigma=0.1):
    sc = S.small(seed=seed)
    sc.snr_law = LAW[:3] + window
    sc.noise_sigma = sigma
    return sc


@pytest.mark.parametrize("block", [1, 0, 12])
def test_snr_full_run(block):
    sc = _scenario()
    ref = oracle.OracleSim(sc)
    sim = B.Simulation(sc, block_steps=block)
    turned = 0
    for _ in range(10):
        before = ref.dir.copy()
        ref.step(100)
        sim.step(100)
        turned += int(np.sum(np.abs(ref.dir - before) > 1e-9))
        parity.assert_parity(parity.compare(sim, ref, sc), where=f"step {ref.step_count}")
    sim.close()
    assert turned > 0


@pytest.mark.parametrize("block", [1, 12])
def test_snr_windowed_tips(block):
    sc = _scenario(seed=3)
    ref = oracle.OracleSim(sc)
    sim = B.Simulation(sc, block_steps=block)
    for window in range(5):
        parity.restart_from_oracle(sim, ref)
        for _ in range(5):
            ref.step(20)
            sim.step(20)
            parity.assert_parity(parity.compare(sim, ref, sc),
                                 where=f"window {window} step {ref.step_count}")
    sim.close()


def test_snr_window_gates_the_turn():
    # a window no concentration reaches: no cone turns, so with sigma = 0 they go straight
    sc = _scenario(seed=5, window=(1e6, 1e7), sigma=0.0)
    with B.Simulation(sc) as sim:
        sim.step(40)
        c = sim.cones()
    active = c["status"] == B.ACTIVE
    np.testing.assert_allclose(c["dir"][active], sc.cone_dir[active], atol=0, rtol=0)


def test_snr_plain_tiled_batch_bitwise():
    sc = _scenario(seed=7)
    runs = []
    for block in (1, 8):
        with B.Simulation(sc, block_steps=block) as sim:
            sim.step(200)
            runs.append(sim.cones())
    with B.Batch([sc, S.small(seed=8)], block_steps=8) as bt:
        bt.step(200)
        runs.append(bt.cones(0))
    for r in runs[1:]:
        for key in ("pos", "dir", "status", "target", "event_step"):
            np.testing.assert_array_equal(r[key], runs[0][key])


def test_snr_rejects_3d_and_bad_parameters():
    sc = S.make_scenario("3d", 3, (16, 16, 16), dt=0.1, n_cones=8, n_targets=4, n_sources=2)
    sc.snr_law = LAW
    with pytest.raises(B.SimError) as e:
        B.Simulation(sc)
    assert e.value.status == B.SIM_EINVAL
    sc = _scenario()
    sc.snr_law = (50.0, 1.0, 0.0, 1e-3, 1e3)   # kd = 0
    with pytest.raises(B.SimError) as e:
        B.Simulation(sc)
    assert e.value.status == B.SIM_EINVAL
    sc = _scenario()
    with B.Simulation(sc) as sim:
        with pytest.raises(B.SimError) as e:
            sim.adjoint(10, np.zeros(sc.n_cones, np.int32), np.ones(sc.n_cones), 5)
        assert e.value.status == B.SIM_EINVAL
