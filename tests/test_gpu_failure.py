"""Failure handling forced from the host: a NaN written into the field through
sim_write_state is caught by the next mass check (a SIM_MASS read, or the periodic check
that sim_set_mass_check enables inside sim_step), the handle then refuses to step with the
sticky SIM_ENONFINITE until a finite state has been written back and a mass read clears it.
Every kernel runs normally on finite or non-finite data; nothing here faults the GPU."""
import numpy as np
import pytest

from paper_1405_3331_amd import binding as B
from paper_1405_3331_amd import scenarios as S

pytestmark = pytest.mark.gpu


def _scenario(dim):
    if dim == 2:
        return S.make_scenario("nan", 2, (64, 48), 1.0, 0.2, ((1.0, 0.01, 1.0),), 3,
                               (0.5, 2.0), 40, 6, seed=3)
    return S.make_scenario("nan3d", 3, (20, 16, 12), 1.0, 0.15,
                           ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), [3, 3], (0.5, 2.0), 30, 6,
                           seed=3)


def _status(fn):
    try:
        fn()
    except B.SimError as e:
        return e.status
    return B.SIM_OK


@pytest.mark.parametrize("dim,block", [(2, 1), (2, 0), (3, 1)])
def test_mass_read_catches_nan_and_is_sticky(dim, block):
    sc = _scenario(dim)
    with B.Simulation(sc, block_steps=block) as sim:
        sim.step(5)
        good = sim.field(0)
        bad = good.copy()
        bad[sc.shape[0] // 2].flat[3] = np.nan
        sim.write(B.FIELD, bad, 0)
        assert _status(sim.mass) == B.SIM_ENONFINITE
        # sticky: no stepping, and synchronise reports it, until a finite state is back
        assert _status(lambda: sim.step(1)) == B.SIM_ENONFINITE
        assert _status(sim.synchronize) == B.SIM_ENONFINITE
        assert sim.step_count == 5
        assert _status(sim.cones) == B.SIM_OK          # reads stay usable
        sim.write(B.FIELD, good, 0)
        assert _status(lambda: sim.step(1)) == B.SIM_ENONFINITE   # not cleared by the write
        assert np.all(np.isfinite(sim.mass()))          # a finite mass check clears it
        sim.step(3)
        assert sim.step_count == 8


@pytest.mark.parametrize("dim,block", [(2, 1), (2, 0), (3, 1)])
def test_periodic_mass_check_catches_nan(dim, block):
    sc = _scenario(dim)
    with B.Simulation(sc, block_steps=block) as sim:
        sim.set_mass_check(10)
        sim.step(25)
        sim.synchronize()                               # finite run: no report
        f = sim.field(sc.species.__len__() - 1)
        f.flat[7] = np.inf
        sim.write(B.FIELD, f, len(sc.species) - 1)
        sim.step(7)                                     # crosses the check at step 30
        assert _status(sim.synchronize) == B.SIM_ENONFINITE
        assert _status(lambda: sim.step(1)) == B.SIM_ENONFINITE
        assert sim.step_count == 32
        with pytest.raises(B.SimError) as e:
            sim.set_mass_check(-1)
        assert e.value.status == B.SIM_EINVAL


def test_mass_check_does_not_change_the_run():
    sc = _scenario(2)
    a = B.Simulation(sc).step(60)
    b = B.Simulation(sc).set_mass_check(7).step(60)
    assert np.array_equal(a.field(), b.field())
    for k, v in a.cones().items():
        assert np.array_equal(v, b.cones()[k]), k
    a.close()
    b.close()
