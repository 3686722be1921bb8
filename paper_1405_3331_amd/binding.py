"""Python binding of the C ABI in ``include/cuesim.h`` (argument marshalling only).

Every step of the simulation runs in the HIP library ``libcuesim.so``; this module only
converts a scenario (``paper_1405_3331_amd.scenarios.Scenario`` or any object with the same
attributes) into ``sim_params``, and host buffers into numpy arrays.  Loading fails loudly
when the library has not been built: there is no fallback.

PyTorch is optional: a ``torch.cuda.Stream`` (or a raw ``hipStream_t`` integer) can be
passed as the stream every operation is enqueued on.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libcuesim.so")

SIM_OK, SIM_EINVAL, SIM_ECFL, SIM_ENOMEM, SIM_EDEVICE, SIM_ERANGE, SIM_ESTATE = 0, -1, -2, -3, -4, -5, -6
SIM_ENONFINITE = -7
STATUS_NAMES = {0: "SIM_OK", -1: "SIM_EINVAL", -2: "SIM_ECFL", -3: "SIM_ENOMEM",
                -4: "SIM_EDEVICE", -5: "SIM_ERANGE", -6: "SIM_ESTATE", -7: "SIM_ENONFINITE"}
ACTIVE, CONTACT, EXITED = 0, 1, 2
SIM_TURN_VECTOR, SIM_TURN_SNR = 0, 1

FIELD, CONE_POS, CONE_DIR, CONE_STATUS, CONE_TARGET, CONE_EVENT_STEP, EVENTS, MASS, STEP, \
    COUNTS, KERNEL_TIME, TILING = range(12)

EXPORTED = ["sim_create", "sim_step", "sim_set_mass_check", "sim_read_state",
            "sim_write_state", "sim_device_ptr", "sim_set_timing", "sim_synchronize", "sim_destroy", "sim_last_error",
            "sim_batch_create", "sim_batch_step", "sim_batch_read_state",
            "sim_batch_synchronize", "sim_batch_destroy", "sim_batch_last_error",
            "sim_adjoint_run", "sim_adjoint_backward", "sim_adjoint_set_tape_limit",
            "sim_connectivity", "sim_connectivity_noalloc", "sim_bfs_levels"]


class SimError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)


class SimParams(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double),
        ("n_species", C.c_int32),
        ("D", C.c_double * 2), ("k", C.c_double * 2), ("sign", C.c_double * 2),
        ("n_sources", C.c_int32 * 2),
        ("source_cell", _ip * 2), ("source_q", _fp * 2), ("init_field", _fp * 2),
        ("n_cones", C.c_int32), ("cone_pos", _fp), ("cone_dir", _fp),
        ("n_targets", C.c_int32), ("target_pos", _fp), ("contact_radius", C.c_double),
        ("step_len", C.c_double), ("turn_gain", C.c_double), ("max_turn", C.c_double),
        ("noise_sigma", C.c_double),
        ("seed", C.c_uint64), ("sim_index", C.c_uint32), ("block_steps", C.c_int32),
        ("tile_cols_per_lane", C.c_int32), ("tile_height", C.c_int32),
        ("turn_law", C.c_int32), ("snr_scale", C.c_double), ("cone_width", C.c_double),
        ("kd", C.c_double), ("c_min", C.c_double), ("c_max", C.c_double),
    ]


_lib = None


def load(path: str = LIBRARY):
    """Load ``libcuesim.so``; raises if it is missing (build it with ``build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} -- run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(path)
    H = C.c_void_p
    lib.sim_create.argtypes = [C.POINTER(SimParams), C.c_void_p, C.POINTER(H)]
    lib.sim_step.argtypes = [H, C.c_int64]
    lib.sim_set_mass_check.argtypes = [H, C.c_int64]
    lib.sim_read_state.argtypes = [H, C.c_int, C.c_int32, C.c_void_p, C.c_size_t,
                                   C.POINTER(C.c_size_t)]
    lib.sim_write_state.argtypes = [H, C.c_int, C.c_int32, C.c_void_p, C.c_size_t]
    lib.sim_device_ptr.argtypes = [H, C.c_int, C.c_int32, C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_size_t)]
    lib.sim_set_timing.argtypes = [H, C.c_int32]
    lib.sim_synchronize.argtypes = [H]
    lib.sim_destroy.argtypes = [H]
    lib.sim_last_error.argtypes = [H]
    lib.sim_last_error.restype = C.c_char_p
    lib.sim_batch_create.argtypes = [C.POINTER(C.POINTER(SimParams)), C.c_int32, C.c_void_p,
                                     C.c_int32, C.POINTER(H)]
    lib.sim_batch_step.argtypes = [H, C.c_int64]
    lib.sim_batch_read_state.argtypes = [H, C.c_int32, C.c_int, C.c_int32, C.c_void_p,
                                         C.c_size_t, C.POINTER(C.c_size_t)]
    lib.sim_batch_synchronize.argtypes = [H]
    lib.sim_batch_destroy.argtypes = [H]
    lib.sim_batch_last_error.argtypes = [H]
    lib.sim_batch_last_error.restype = C.c_char_p
    _dp = C.POINTER(C.c_double)
    lib.sim_adjoint_run.argtypes = [H, C.c_int64, C.c_int32, _ip, _fp, _dp]
    lib.sim_adjoint_backward.argtypes = [H, _dp, _dp, _dp]
    lib.sim_adjoint_set_tape_limit.argtypes = [H, C.c_int64]
    lib.sim_connectivity.argtypes = [H, C.c_int32, _ip, _ip, _ip, _ip, C.c_int64,
                                     C.POINTER(C.c_int64)]
    lib.sim_connectivity_noalloc.argtypes = [H, C.c_int32, _ip, _ip, _ip, _ip, C.c_int64,
                                             C.POINTER(C.c_int64)]
    lib.sim_bfs_levels.argtypes = [H, C.c_int32, _ip]
    for name in EXPORTED:
        if not name.endswith("last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status, handle=None):
    if status != SIM_OK:
        msg = load().sim_last_error(handle)
        raise SimError(status, msg.decode() if msg else "")


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def make_params(sc, block_steps: int = 0):
    """sim_params for a scenario; returns (params, keep-alive list of arrays)."""
    keep = []

    def f32(a, shape=None):
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        if shape is not None:
            arr = arr.reshape(shape)
        keep.append(arr)
        return arr.ctypes.data_as(_fp)

    p = SimParams()
    p.struct_size = C.sizeof(SimParams)
    p.dim = sc.dim
    p.nx, p.ny, p.nz = sc.nx, sc.ny, (sc.nz if sc.dim == 3 else 1)
    p.dx, p.dt = sc.dx, sc.dt
    p.n_species = len(sc.species)
    for s, spc in enumerate(sc.species):
        p.D[s], p.k[s], p.sign[s] = spc.D, spc.k, spc.sign
        cells = np.ascontiguousarray(spc.source_cell, dtype=np.int32)
        keep.append(cells)
        p.n_sources[s] = cells.size
        p.source_cell[s] = cells.ctypes.data_as(_ip)
        p.source_q[s] = f32(spc.source_q)
        init = None if sc.init_field is None else sc.init_field[s]
        p.init_field[s] = f32(init) if init is not None else None
    M = sc.n_cones
    p.n_cones = M
    p.cone_pos = f32(sc.cone_pos, (M, sc.dim))
    p.cone_dir = f32(sc.cone_dir, (M,) if sc.dim == 2 else (M, 3))
    p.n_targets = sc.n_targets
    p.target_pos = f32(sc.target_pos, (sc.n_targets, sc.dim))
    p.contact_radius = sc.contact_radius
    p.step_len, p.turn_gain = sc.step_len, sc.turn_gain
    p.max_turn, p.noise_sigma = sc.max_turn, sc.noise_sigma
    p.seed, p.sim_index = sc.seed, sc.sim_index
    p.block_steps = block_steps
    tile = getattr(sc, "tile", None) or (0, 0)   # (cols per lane, height) hint, 0 = planner
    p.tile_cols_per_lane, p.tile_height = int(tile[0]), int(tile[1])
    law = getattr(sc, "snr_law", None)   # (snr_scale, cone_width, kd, c_min, c_max)
    if law is not None:
        p.turn_law = SIM_TURN_SNR
        p.snr_scale, p.cone_width, p.kd, p.c_min, p.c_max = (float(v) for v in law)
    return p, keep


# -- the C ABI, one Python function per entry point ------------------------------------

def sim_create(sc, stream=None, block_steps: int = 0):
    lib = load()
    params, keep = make_params(sc, block_steps)
    h = C.c_void_p()
    _check(lib.sim_create(C.byref(params), _stream_handle(stream), C.byref(h)))
    del keep
    return h


def sim_create_raw(params: SimParams, stream=None):
    """sim_create on an explicit SimParams (for tests of argument validation)."""
    lib = load()
    h = C.c_void_p()
    st = lib.sim_create(C.byref(params), _stream_handle(stream), C.byref(h))
    return st, h


def sim_step(h, n_steps: int):
    _check(load().sim_step(h, int(n_steps)), h)


def _item_bytes(h, what, index):
    need = C.c_size_t(0)
    st = load().sim_read_state(h, what, index, None, 0, C.byref(need))
    if st not in (SIM_OK, SIM_ERANGE):
        _check(st, h)
    return need.value


def sim_read_state(h, what: int, index: int = 0, shape=None) -> np.ndarray:
    dtype = {MASS: np.float64, STEP: np.int64, KERNEL_TIME: np.float64,
             CONE_STATUS: np.int32, CONE_TARGET: np.int32, CONE_EVENT_STEP: np.int32,
             EVENTS: np.int32, COUNTS: np.int32, TILING: np.int32}.get(what, np.float32)
    need = _item_bytes(h, what, index)
    out = np.empty(need // np.dtype(dtype).itemsize, dtype=dtype)
    written = C.c_size_t(0)
    _check(load().sim_read_state(h, what, index, out.ctypes.data_as(C.c_void_p), out.nbytes,
                                 C.byref(written)), h)
    if what == EVENTS:
        out = out.reshape(-1, 4)
    if shape is not None:
        out = out.reshape(shape)
    return out


def sim_write_state(h, what: int, index: int, array) -> None:
    dtype = {STEP: np.int64, CONE_STATUS: np.int32, CONE_TARGET: np.int32,
             CONE_EVENT_STEP: np.int32}.get(what, np.float32)
    arr = np.ascontiguousarray(np.asarray(array, dtype=dtype))
    _check(load().sim_write_state(h, what, index, arr.ctypes.data_as(C.c_void_p), arr.nbytes), h)


def sim_device_ptr(h, what: int = FIELD, index: int = 0):
    ptr = C.c_void_p()
    nbytes = C.c_size_t()
    _check(load().sim_device_ptr(h, what, index, C.byref(ptr), C.byref(nbytes)), h)
    return ptr.value, nbytes.value


def sim_set_timing(h, enable: bool):
    _check(load().sim_set_timing(h, 1 if enable else 0), h)


def sim_synchronize(h):
    _check(load().sim_synchronize(h), h)


def sim_destroy(h):
    _check(load().sim_destroy(h))


def sim_last_error(h=None) -> str:
    msg = load().sim_last_error(h)
    return msg.decode() if msg else ""


def sim_adjoint_run(h, n_steps: int, checkpoint_every: int, assign, weight) -> float:
    assign = np.ascontiguousarray(assign, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float32)
    loss = C.c_double(0.0)
    _check(load().sim_adjoint_run(h, int(n_steps), int(checkpoint_every),
                                  assign.ctypes.data_as(_ip), weight.ctypes.data_as(_fp),
                                  C.byref(loss)), h)
    return float(loss.value)


def sim_adjoint_backward(h, n_q: int, n_species: int):
    """(dL/dq [n_q], dL/dD [n_species], dL/dk [n_species]) of the last sim_adjoint_run."""
    dq = np.zeros(max(n_q, 1))
    dD = np.zeros(n_species)
    dk = np.zeros(n_species)
    dp = C.POINTER(C.c_double)
    _check(load().sim_adjoint_backward(h, dq.ctypes.data_as(dp), dD.ctypes.data_as(dp),
                                       dk.ctypes.data_as(dp)), h)
    return dq[:n_q], dD, dk


def sim_connectivity(h, n_neurons: int, cone_owner, target_owner, noalloc: bool = False):
    """(row_start [n_neurons + 1], edges [n_edges]) of the connections made so far
    (noalloc: through sim_connectivity_noalloc, which allocates no device memory)."""
    owner = np.ascontiguousarray(cone_owner, dtype=np.int32)
    towner = np.ascontiguousarray(target_owner, dtype=np.int32)
    row_start = np.zeros(n_neurons + 1, dtype=np.int32)
    n_edges = C.c_int64(0)
    cap = max(int(owner.size), 1)
    edges = np.zeros(cap, dtype=np.int32)
    fn = load().sim_connectivity_noalloc if noalloc else load().sim_connectivity
    _check(fn(h, int(n_neurons), owner.ctypes.data_as(_ip), towner.ctypes.data_as(_ip),
              row_start.ctypes.data_as(_ip), edges.ctypes.data_as(_ip), cap,
              C.byref(n_edges)), h)
    return row_start, edges[: n_edges.value].copy()


def sim_bfs_levels(h, root: int, n_neurons: int) -> np.ndarray:
    level = np.zeros(n_neurons, dtype=np.int32)
    _check(load().sim_bfs_levels(h, int(root), level.ctypes.data_as(_ip)), h)
    return level


class Simulation:
    """Owning wrapper around a handle with numpy views of the state."""

    def __init__(self, sc, stream=None, block_steps: int = 0):
        self.sc = sc
        self.dim = sc.dim
        self.shape = sc.shape
        self.h = sim_create(sc, stream, block_steps)

    def step(self, n: int = 1):
        sim_step(self.h, n)
        return self

    def field(self, s: int = 0) -> np.ndarray:
        return sim_read_state(self.h, FIELD, s, self.shape)

    def cones(self):
        M = self.sc.n_cones
        pos = sim_read_state(self.h, CONE_POS, 0, (M, self.dim))
        dir_ = sim_read_state(self.h, CONE_DIR, 0, (M,) if self.dim == 2 else (M, 3))
        return dict(pos=pos, dir=dir_,
                    status=sim_read_state(self.h, CONE_STATUS),
                    target=sim_read_state(self.h, CONE_TARGET),
                    event_step=sim_read_state(self.h, CONE_EVENT_STEP))

    def events(self) -> np.ndarray:
        return sim_read_state(self.h, EVENTS)

    def set_mass_check(self, every: int):
        """Periodic mass check every `every` steps (0: off); see sim_set_mass_check."""
        _check(load().sim_set_mass_check(self.h, int(every)), self.h)
        return self

    def mass(self) -> np.ndarray:
        return sim_read_state(self.h, MASS)

    def counts(self) -> np.ndarray:
        return sim_read_state(self.h, COUNTS)

    def tiling(self) -> dict:
        v = sim_read_state(self.h, TILING)
        keys = ["block_steps", "halo", "core_x", "core_y", "tiles", "cols_per_lane",
                "height", "lds_bytes"]
        return dict(zip(keys, (int(x) for x in v)))

    @property
    def step_count(self) -> int:
        return int(sim_read_state(self.h, STEP)[0])

    def write(self, what, array, index=0):
        sim_write_state(self.h, what, index, array)
        return self

    def adjoint(self, n_steps: int, assign, weight, checkpoint_every: int = 100):
        """Run n_steps with checkpoints and return the trajectory loss
        sum_i weight[i] |p_i^N - target[assign[i]]|^2; gradients via adjoint_backward()."""
        return sim_adjoint_run(self.h, n_steps, checkpoint_every, assign, weight)

    def connectivity(self, n_neurons: int, cone_owner, target_owner):
        return sim_connectivity(self.h, n_neurons, cone_owner, target_owner)

    def bfs_levels(self, root: int, n_neurons: int):
        return sim_bfs_levels(self.h, root, n_neurons)

    def set_tape_limit(self, max_bytes: int):
        """Bytes the reverse sweep may record (0: library default); see the header."""
        _check(load().sim_adjoint_set_tape_limit(self.h, int(max_bytes)), self.h)
        return self

    def adjoint_backward(self):
        n_q = sum(len(s.source_q) for s in self.sc.species)
        return sim_adjoint_backward(self.h, n_q, len(self.sc.species))

    def synchronize(self):
        sim_synchronize(self.h)

    def close(self):
        if self.h is not None:
            sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# -- batches ----------------------------------------------------------------------------

def _check_batch(status, handle=None):
    if status != SIM_OK:
        msg = load().sim_batch_last_error(handle)
        raise SimError(status, msg.decode() if msg else "")


def sim_batch_create(scenarios, stream=None, graph_launches: int = 0, block_steps: int = 0):
    lib = load()
    made = [make_params(sc, block_steps) for sc in scenarios]
    arr = (C.POINTER(SimParams) * len(made))(*[C.pointer(p) for p, _ in made])
    h = C.c_void_p()
    _check_batch(lib.sim_batch_create(arr, len(made), _stream_handle(stream), graph_launches,
                                      C.byref(h)))
    del made
    return h


def sim_batch_step(b, n_steps: int):
    _check_batch(load().sim_batch_step(b, int(n_steps)), b)


def sim_batch_read_state(b, sim: int, what: int, index: int = 0, shape=None) -> np.ndarray:
    dtype = {MASS: np.float64, STEP: np.int64, KERNEL_TIME: np.float64,
             CONE_STATUS: np.int32, CONE_TARGET: np.int32, CONE_EVENT_STEP: np.int32,
             EVENTS: np.int32, COUNTS: np.int32, TILING: np.int32}.get(what, np.float32)
    lib = load()
    need = C.c_size_t(0)
    st = lib.sim_batch_read_state(b, sim, what, index, None, 0, C.byref(need))
    if st not in (SIM_OK, SIM_ERANGE):
        _check_batch(st, b)
    out = np.empty(need.value // np.dtype(dtype).itemsize, dtype=dtype)
    _check_batch(lib.sim_batch_read_state(b, sim, what, index,
                                          out.ctypes.data_as(C.c_void_p), out.nbytes,
                                          C.byref(need)), b)
    if what == EVENTS:
        out = out.reshape(-1, 4)
    if shape is not None:
        out = out.reshape(shape)
    return out


def sim_batch_synchronize(b):
    _check_batch(load().sim_batch_synchronize(b), b)


def sim_batch_destroy(b):
    _check_batch(load().sim_batch_destroy(b))


def sim_batch_last_error(b=None) -> str:
    msg = load().sim_batch_last_error(b)
    return msg.decode() if msg else ""


class Batch:
    """Owning wrapper around a batch of simulations."""

    def __init__(self, scenarios, stream=None, graph_launches: int = 0, block_steps: int = 0):
        self.scenarios = list(scenarios)
        self.h = sim_batch_create(self.scenarios, stream, graph_launches, block_steps)

    def step(self, n: int = 1):
        sim_batch_step(self.h, n)
        return self

    def field(self, i: int, s: int = 0) -> np.ndarray:
        return sim_batch_read_state(self.h, i, FIELD, s, self.scenarios[i].shape)

    def cones(self, i: int):
        sc = self.scenarios[i]
        M = sc.n_cones
        return dict(pos=sim_batch_read_state(self.h, i, CONE_POS, 0, (M, sc.dim)),
                    dir=sim_batch_read_state(self.h, i, CONE_DIR, 0, (M,)),
                    status=sim_batch_read_state(self.h, i, CONE_STATUS),
                    target=sim_batch_read_state(self.h, i, CONE_TARGET),
                    event_step=sim_batch_read_state(self.h, i, CONE_EVENT_STEP))

    def tiling(self, i: int) -> dict:
        v = sim_batch_read_state(self.h, i, TILING)
        keys = ["block_steps", "halo", "core_x", "core_y", "tiles", "cols_per_lane",
                "height", "lds_bytes"]
        return dict(zip(keys, (int(x) for x in v)))

    def synchronize(self):
        sim_batch_synchronize(self.h)

    def close(self):
        if self.h is not None:
            sim_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
