"""Host-side checks of the C-ABI library that need no GPU: every symbol the header declares
is exported, the binding's struct matches the header's, and parameter validation rejects bad
input (validation runs before any HIP call)."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1405_3331_amd import binding as B
from paper_1405_3331_amd import scenarios as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cuesim.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIBRARY):
        from paper_1405_3331_amd import build
        build.build()
    return B.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:sim_status|const char\*)\s+(sim_\w+)\s*\(", text, re.M)))


def test_header_declares_the_abi():
    assert declared_functions() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIBRARY], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(sim_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_params_struct_matches_header():
    """Compile a host program that prints sizeof/offsetof of sim_params from the header."""
    src = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "cuesim.h"
    int main(void) {
      printf("%zu %zu %zu %zu %zu %zu\n", sizeof(sim_params), offsetof(sim_params, dx),
             offsetof(sim_params, source_cell), offsetof(sim_params, n_cones),
             offsetof(sim_params, seed), offsetof(sim_params, block_steps));
      return 0;
    }
    """
    import tempfile
    d = tempfile.mkdtemp()
    with open(os.path.join(d, "t.c"), "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), os.path.join(d, "t.c"), "-o",
                    os.path.join(d, "t")], check=True)
    vals = [int(v) for v in subprocess.run([os.path.join(d, "t")], capture_output=True,
                                           text=True, check=True).stdout.split()]
    P = B.SimParams
    assert vals == [C.sizeof(P), P.dx.offset, P.source_cell.offset, P.n_cones.offset,
                    P.seed.offset, P.block_steps.offset]


def _params(**over):
    sc = S.make_scenario("v", 2, (16, 12), 1.0, 0.2, ((1.0, 0.01, 1.0),), 2, (1.0, 1.0), 4, 2)
    for k, v in over.items():
        setattr(sc, k, v)
    return sc


def _create_status(sc, mutate=None):
    p, keep = B.make_params(sc)
    if mutate:
        mutate(p)
    st, h = B.sim_create_raw(p)
    if st == B.SIM_OK:          # only on a machine with a GPU
        B.sim_destroy(h)
    return st


@pytest.mark.parametrize("mutate,expect", [
    (lambda p: setattr(p, "struct_size", 12), B.SIM_EINVAL),
    (lambda p: setattr(p, "dim", 4), B.SIM_EINVAL),
    (lambda p: setattr(p, "nx", 1), B.SIM_EINVAL),
    (lambda p: setattr(p, "dx", 0.0), B.SIM_EINVAL),
    (lambda p: setattr(p, "dt", float("nan")), B.SIM_EINVAL),
    (lambda p: setattr(p, "n_species", 3), B.SIM_EINVAL),
    (lambda p: p.D.__setitem__(0, -1.0), B.SIM_EINVAL),
    (lambda p: p.k.__setitem__(0, -0.1), B.SIM_EINVAL),
    (lambda p: p.D.__setitem__(0, 1.26), B.SIM_ECFL),          # r = 0.252 > 1/4
    (lambda p: p.k.__setitem__(0, 1.1), B.SIM_ECFL),           # 4 r + k dt = 1.02 > 1
    (lambda p: setattr(p, "contact_radius", -1.0), B.SIM_EINVAL),
    (lambda p: setattr(p, "max_turn", 4.0), B.SIM_EINVAL),
    (lambda p: setattr(p, "noise_sigma", -0.1), B.SIM_EINVAL),
    (lambda p: setattr(p, "block_steps", 99), B.SIM_EINVAL),
    (lambda p: setattr(p, "n_cones", -1), B.SIM_EINVAL),
])
def test_validation_rejects(lib, mutate, expect):
    sc = _params()
    assert _create_status(sc, mutate) == expect
    assert B.sim_last_error(None) != ""


def test_validation_rejects_bad_arrays(lib):
    sc = _params()
    sc.cone_pos = sc.cone_pos.copy()
    sc.cone_pos[0, 0] = 16.0            # on the upper face: outside [0, L)
    assert _create_status(sc) == B.SIM_EINVAL
    sc = _params()
    sc.species[0].source_cell = np.array([0, 16 * 12], dtype=np.int32)
    sc.species[0].source_q = np.array([1.0, 1.0])
    assert _create_status(sc) == B.SIM_EINVAL
    sc = _params()
    sc.target_pos = sc.target_pos.copy()
    sc.target_pos[1, 1] = np.inf
    assert _create_status(sc) == B.SIM_EINVAL
    sc = S.make_scenario("v3", 3, (4, 4, 4), 1.0, 0.1, ((1.0, 0.0, 1.0),), 1, (1, 1), 2, 1)
    sc.cone_dir = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])   # not unit
    assert _create_status(sc) == B.SIM_EINVAL


def test_stability_limit_is_inclusive(lib):
    # r exactly 1/4 with k = 0 is allowed; validation passes and only the device step can
    # fail here (no GPU in this container), which is reported as a device error, not CFL.
    sc = _params()
    sc.dt = 0.25
    sc.species[0].k = 0.0
    st = _create_status(sc)
    assert st != B.SIM_ECFL and st != B.SIM_EINVAL


def test_null_handle_calls_are_errors(lib):
    assert lib.sim_step(None, 1) == B.SIM_EINVAL
    assert lib.sim_destroy(None) == B.SIM_OK
    assert lib.sim_synchronize(None) == B.SIM_EINVAL
