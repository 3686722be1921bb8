"""The FP64 oracle against a second, naive pure-Python implementation on tiny scenarios
(grids of at most 8 x 6 or 4 x 5 x 3 cells, a few cones, tens of steps), CPU only.  The
two share only the seeded input generator; the naive side draws its deviates from
PyTorch's Philox engine."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import naive
import oracle
from paper_1405_3331_amd import scenarios


@pytest.fixture(autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _compare(sc, steps):
    a = oracle.OracleSim(sc).step(steps)
    b = naive.NaiveSim(sc).step(steps)
    for s in range(len(sc.species)):
        fa = a.fields[s].ravel()
        fb = np.array(b.fields[s])
        scale = max(np.abs(fa).max(), 1e-300)
        assert np.abs(fa - fb).max() <= 1e-12 * scale, (s, np.abs(fa - fb).max(), scale)
    np.testing.assert_array_equal(a.status, np.array(b.status))
    np.testing.assert_array_equal(a.target, np.array(b.target))
    np.testing.assert_array_equal(a.event_step, np.array(b.event_step))
    L = sc.side
    assert np.abs(a.pos - np.array(b.pos)).max() <= 1e-10 * L
    if sc.dim == 2:
        d = np.angle(np.exp(1j * (a.dir - np.array(b.dir))))
        assert np.abs(d).max() <= 1e-10
    else:
        assert np.abs(a.dir - np.array(b.dir)).max() <= 1e-10
    return a


def _tiny(dim, n, species, n_cones, n_targets, seed, step_len=0.2, radius=1.0,
          rate=(5.0, 20.0), n_sources=3, gain=10.0, sigma=0.1):
    return scenarios.make_scenario("tiny", dim, n, 1.0, 0.2 if dim == 2 else 0.12, species,
                                   n_sources, rate, n_cones, n_targets, radius, step_len,
                                   gain, math.pi / 30.0, sigma, seed=seed)


def test_bruteforce_2d_one_species():
    sc = _tiny(2, (8, 6), ((1.0, 0.01, 1.0),), 4, 4, seed=3)
    a = _compare(sc, 40)
    # the case exercises the rules it is meant to pin: cones move, some stop
    assert (a.status != oracle.ACTIVE).any() or np.ptp(a.pos) > 1.0


def test_bruteforce_2d_two_species_with_events():
    sc = _tiny(2, (8, 6), ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), 4, 6, seed=11,
               step_len=0.3, radius=1.2)
    a = _compare(sc, 50)
    assert (a.status != oracle.ACTIVE).any()


def test_bruteforce_3d_two_species():
    sc = _tiny(3, (4, 5, 3), ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), 3, 3, seed=5,
               step_len=0.15)
    _compare(sc, 30)


@settings(max_examples=8, deadline=None)
@given(seed=st.integers(0, 2 ** 31 - 1), dim=st.sampled_from([2, 3]),
       two=st.booleans(), gain=st.sampled_from([0.0, 1.0, 10.0]),
       sigma=st.sampled_from([0.0, 0.1, 0.4]))
def test_bruteforce_hypothesis(seed, dim, two, gain, sigma):
    species = ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)) if two else ((0.8, 0.005, 1.0),)
    n = (7, 5) if dim == 2 else (4, 4, 3)
    sc = _tiny(dim, n, species, 3, 3, seed=seed, gain=gain, sigma=sigma)
    _compare(sc, 20)


@pytest.mark.parametrize("seed", [2, 9])
def test_bruteforce_snr_law(seed):
    sc = _tiny(2, (8, 6), ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), 4, 3, seed=seed, sigma=0.05)
    sc.snr_law = (30.0, 1.0, 2.0, 0.05, 50.0)
    a = _compare(sc, 40)
    assert np.ptp(a.pos) > 0.5
