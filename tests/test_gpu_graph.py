"""Connectivity on the GPU (sim_connectivity, sim_bfs_levels) against the oracle's
definition, bit-exact (integer work), on the GPU run's own contact record."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1405_3331_amd import binding as B, scenarios

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _built(oracle_lib):
    return oracle_lib


def _check(sim, sc, n_neurons, owner, towner, roots):
    row, edges = sim.connectivity(n_neurons, owner, towner)
    c = sim.cones()
    row_ref, edges_ref = oracle.connectivity(n_neurons, c["status"], c["target"], owner, towner)
    np.testing.assert_array_equal(row, row_ref)
    np.testing.assert_array_equal(edges, edges_ref)
    for root in roots:
        np.testing.assert_array_equal(sim.bfs_levels(root, n_neurons),
                                      oracle.bfs_levels(row_ref, edges_ref, root))
    return len(edges)


def test_small_run_connectivity_and_levels():
    sc = scenarios.make_scenario("graph", 2, (128, 128), 1.0, 0.2, ((1.0, 0.01, 1.0),), 6,
                                 (2.0, 8.0), 600, 80, 2.0, 0.5, 10.0, seed=3)
    n = 150
    owner = np.arange(sc.n_cones) % n
    towner = (np.arange(80) * 7) % n
    with B.Simulation(sc) as sim:
        sim.step(400)
        e = _check(sim, sc, n, owner, towner, roots=[0, 1, 17, 149])
    assert e > 20   # the case has connections to traverse


def test_headline_size_connectivity():
    sc = scenarios.headline()
    n = 4096
    owner = np.arange(sc.n_cones) // 16
    towner = np.arange(sc.target_pos.shape[0]) * 4
    with B.Simulation(sc) as sim:
        sim.step(600)
        e = _check(sim, sc, n, owner, towner, roots=[0, 2048, 4095])
    assert e > 0


def test_degenerate_graphs():
    sc = scenarios.make_scenario("graph", 2, (64, 64), n_cones=0, n_targets=4, n_sources=1)
    with B.Simulation(sc) as sim:
        row, edges = sim.connectivity(3, np.zeros(0, np.int32), np.zeros(4, np.int32))
        assert row.tolist() == [0, 0, 0, 0] and edges.size == 0
        assert sim.bfs_levels(1, 3).tolist() == [-1, 0, -1]
    sc = scenarios.make_scenario("graph", 2, (64, 64), n_cones=32, n_targets=4, n_sources=1)
    with B.Simulation(sc) as sim:   # no steps: no contacts yet
        row, edges = sim.connectivity(1, np.zeros(32, np.int32), np.zeros(4, np.int32))
        assert row.tolist() == [0, 0] and edges.size == 0
        assert sim.bfs_levels(0, 1).tolist() == [0]


def test_error_paths():
    sc = scenarios.make_scenario("graph", 2, (64, 64), 1.0, 0.2, ((1.0, 0.01, 1.0),), 4,
                                 (2.0, 8.0), 200, 40, 3.0, 0.5, 10.0, seed=1)
    M, T = sc.n_cones, sc.target_pos.shape[0]
    with B.Simulation(sc) as sim:
        with pytest.raises(B.SimError) as e:
            sim.bfs_levels(0, 4)
        assert e.value.status == B.SIM_ESTATE
        with pytest.raises(B.SimError) as e:
            sim.connectivity(4, np.full(M, 4, np.int32), np.zeros(T, np.int32))
        assert e.value.status == B.SIM_EINVAL
        sim.step(300)
        owner = np.zeros(M, np.int32)
        towner = np.zeros(T, np.int32)
        row, edges = sim.connectivity(1, owner, towner)
        assert len(edges) > 0
        # an edge buffer that is too small: SIM_ERANGE with the needed count
        ip = C.POINTER(C.c_int32)
        rs = np.zeros(2, np.int32)
        n_edges = C.c_int64(0)
        st = B.load().sim_connectivity(sim.h, 1, owner.ctypes.data_as(ip),
                                       towner.ctypes.data_as(ip), rs.ctypes.data_as(ip), None, 0,
                                       C.byref(n_edges))
        assert st == B.SIM_ERANGE and n_edges.value == len(edges)
        with pytest.raises(B.SimError) as e:
            sim.bfs_levels(1, 1)
        assert e.value.status == B.SIM_EINVAL
