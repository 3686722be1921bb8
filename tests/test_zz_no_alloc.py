"""sim_connectivity_noalloc (the connectivity build from one fixed device array, for
callers that cannot allocate) against sim_connectivity, bit for bit, through the C ABI:
two calls in a row on one GPU, the second with fewer cones, targets and neurons (the array
keeps the first call's contents), and the size limit rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

from paper_1405_3331_amd import binding as B, scenarios

pytestmark = pytest.mark.gpu

_ip = C.POINTER(C.c_int32)
MAX_ITEMS = 1 << 18


def _noalloc(h, n_neurons, cone_owner, target_owner):
    """Status and outputs of one sim_connectivity_noalloc call through the C ABI."""
    fn = B.load().sim_connectivity_noalloc
    owner = np.ascontiguousarray(cone_owner, dtype=np.int32)
    towner = np.ascontiguousarray(target_owner, dtype=np.int32)
    row_start = np.full(n_neurons + 1, -7, dtype=np.int32)
    cap = max(int(owner.size), 1)
    edges = np.full(cap, -7, dtype=np.int32)
    n_edges = C.c_int64(-1)
    st = fn(h, int(n_neurons), owner.ctypes.data_as(_ip), towner.ctypes.data_as(_ip),
            row_start.ctypes.data_as(_ip), edges.ctypes.data_as(_ip), cap, C.byref(n_edges))
    return st, row_start, edges[: max(n_edges.value, 0)].copy()


def _scenario(cones, targets, seed):
    return scenarios.make_scenario("graph", 2, (128, 128), 1.0, 0.2, ((1.0, 0.01, 1.0),), 6,
                                   (2.0, 8.0), cones, targets, 2.0, 0.5, 10.0, seed=seed)


def test_noalloc_matches_allocating_call_twice_in_a_row():
    cases = [(_scenario(3000, 120, 3), 400, 500), (_scenario(700, 40, 5), 90, 300)]
    for sc, n, steps in cases:        # the second call is smaller than the first
        owner = (np.arange(sc.n_cones) * 13) % n
        towner = (np.arange(sc.target_pos.shape[0]) * 7) % n
        with B.Simulation(sc) as sim:
            sim.step(steps)
            row, edges = sim.connectivity(n, owner, towner)
            st, row2, edges2 = _noalloc(sim.h, n, owner, towner)
            assert st == B.SIM_OK, B.load().sim_last_error(sim.h)
            np.testing.assert_array_equal(row2, row)
            np.testing.assert_array_equal(edges2, edges)
            assert len(edges) > 10   # the case has connections
            print(f"[noalloc] {sc.n_cones} cones, {n} neurons: {len(edges)} edges equal",
                  flush=True)


def test_noalloc_rejects_sizes_beyond_its_array():
    sc = _scenario(40, 8, 7)
    with B.Simulation(sc) as sim:
        st, _, _ = _noalloc(sim.h, MAX_ITEMS + 1, np.zeros(40), np.zeros(8))
        assert st == B.SIM_EINVAL
        assert b"262144" in B.load().sim_last_error(sim.h)
