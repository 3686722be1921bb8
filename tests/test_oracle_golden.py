"""The oracle against values the paper prints (CPU only)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            key, val = line.split("=", 1)
            out[key.strip()] = [tuple(int(v) for v in item.split()) for item in val.split(",")]
    return out


def test_table1_cell_sort(oracle_lib):
    """Sec. 3.5, Table 1: particles keyed by cell, stably sorted, with cell start/end.  The
    oracle's adjacency construction is the same operation: owner = cell, payload = particle
    (every particle 'contacts' its own payload, which its owner maps to itself)."""
    g = _read("table1_cell_sort.txt")
    cells = np.array([c for c, _ in g["pairs"]], dtype=np.int32)
    particles = np.array([p for _, p in g["pairs"]], dtype=np.int32)
    n_cells = 10
    status = np.ones(len(cells), dtype=np.int32)             # contact
    target = np.arange(len(cells), dtype=np.int32)
    row, payload = oracle.connectivity(n_cells, status, target, cells, particles)
    assert [(int(cells[i]), int(p)) for i, p in zip(np.argsort(cells, kind="stable"), payload)] \
        == [tuple(x) for x in g["sorted"]]
    for c, start in g["cell_start"]:
        assert row[c] == start
    for c, end in g["cell_end"]:
        assert row[c + 1] == end
    occupied = {c for c, _ in g["cell_start"]}
    for c in range(n_cells):
        if c not in occupied:
            assert row[c] == row[c + 1]   # empty cell
