"""FP64 CPU oracle of the cue-diffusion / growth-cone time step -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  The product path (the HIP library and its binding) never does, and this
package imports nothing from the product path: it takes any object with the attributes of
a scenario (grid, species, cones, targets, rule constants) and copies its arrays.

The simulation rules are in ``cuesim_oracle.c``; this file is argument marshalling.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libcuesim_oracle.so")

ACTIVE, CONTACT, EXITED = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double),
        ("n_species", C.c_int32),
        ("D", C.c_double * 2), ("k", C.c_double * 2), ("sign", C.c_double * 2),
        ("n_sources", C.c_int32 * 2),
        ("source_cell", _ip * 2), ("source_q", _dp * 2),
        ("n_targets", C.c_int32), ("target_pos", _dp), ("contact_radius", C.c_double),
        ("step_len", C.c_double), ("turn_gain", C.c_double), ("max_turn", C.c_double),
        ("noise_sigma", C.c_double),
        ("seed", C.c_uint64), ("sim_index", C.c_uint32),
        ("noise_sign", C.c_double), ("flag_tol", C.c_double),
        ("turn_law", C.c_int32), ("snr_scale", C.c_double), ("cone_width", C.c_double),
        ("kd", C.c_double), ("c_min", C.c_double), ("c_max", C.c_double),
    ]


class _State(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("field", _dp * 2), ("n_cones", C.c_int32),
        ("pos", _dp), ("dir", _dp), ("status", _ip), ("target", _ip),
        ("event_step", _ip), ("flag_step", _ip), ("cap_margin", _dp),
    ]


_lib = None


def load(path: str = LIBRARY):
    """Load the compiled oracle (build it with ``python oracle/build.py``)."""
    global _lib
    if _lib is not None and path == LIBRARY:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library not built: {path} (run python oracle/build.py)")
    lib = C.CDLL(path)
    lib.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32)]
    lib.oracle_normals4.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.c_uint32, _dp]
    lib.oracle_sample_gradient.argtypes = [C.POINTER(_Params), _dp, _dp, _dp]
    lib.oracle_field_step.argtypes = [C.POINTER(_Params), C.POINTER(_dp), C.POINTER(_dp)]
    lib.oracle_cone_step.argtypes = [C.POINTER(_Params), C.POINTER(_State)]
    lib.oracle_run.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.c_int64]
    lib.oracle_run.restype = C.c_int
    lib.oracle_mass.argtypes = [C.POINTER(_Params), _dp]
    lib.oracle_mass.restype = C.c_double
    lib.oracle_num_threads.restype = C.c_int
    if hasattr(lib, "oracle_connectivity"):
        _i32p = C.POINTER(C.c_int32)
        lib.oracle_connectivity.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p,
                                            _i32p, _i32p]
        lib.oracle_connectivity.restype = C.c_int64
        lib.oracle_bfs_levels.argtypes = [C.c_int32, _i32p, _i32p, C.c_int32, _i32p]
        lib.oracle_bfs_levels.restype = C.c_int
    if hasattr(lib, "oracle_adjoint"):
        lib.oracle_adjoint.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.c_int64,
                                       C.POINTER(C.c_int32), _dp, _dp, _dp, _dp, _dp, _dp,
                                       _dp]
        lib.oracle_adjoint.restype = C.c_int
    if path == LIBRARY:
        _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox4x32_10(ctr, key, lib=None) -> np.ndarray:
    lib = lib or load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def normals4(seed, c0, c1, c2, c3, lib=None) -> np.ndarray:
    lib = lib or load()
    z = np.zeros(4)
    lib.oracle_normals4(C.c_uint64(seed), c0, c1, c2, c3, _ptr(z, C.c_double))
    return z


def num_threads(lib=None) -> int:
    return int((lib or load()).oracle_num_threads())


def connectivity(n_neurons, status, target, cone_owner, target_owner, lib=None):
    """(row_start [n_neurons + 1], edges) of the contacts: cone i with status CONTACT is an
    edge cone_owner[i] -> target_owner[target[i]], lists in increasing cone index."""
    lib = lib or load()
    st = np.ascontiguousarray(status, dtype=np.int32)
    tg = np.ascontiguousarray(target, dtype=np.int32)
    ow = np.ascontiguousarray(cone_owner, dtype=np.int32)
    to = np.ascontiguousarray(target_owner, dtype=np.int32)
    row = np.zeros(int(n_neurons) + 1, dtype=np.int32)
    edges = np.zeros(max(st.size, 1), dtype=np.int32)
    p = lambda a: _ptr(a, C.c_int32)
    n = lib.oracle_connectivity(int(n_neurons), st.size, p(st), p(tg), p(ow), p(to), p(row),
                                p(edges))
    if n < 0:
        raise MemoryError("oracle_connectivity")
    return row, edges[:n].copy()


def bfs_levels(row_start, edges, root, lib=None):
    lib = lib or load()
    row = np.ascontiguousarray(row_start, dtype=np.int32)
    e = np.ascontiguousarray(edges if len(edges) else np.zeros(1), dtype=np.int32)
    level = np.zeros(row.size - 1, dtype=np.int32)
    if lib.oracle_bfs_levels(row.size - 1, _ptr(row, C.c_int32), _ptr(e, C.c_int32), int(root),
                             _ptr(level, C.c_int32)) != 0:
        raise MemoryError("oracle_bfs_levels")
    return level


class OracleSim:
    """FP64 simulation of one scenario, state held in numpy arrays.

    ``noise_sign`` = -1 negates every normal deviate (used by the mirror-symmetry check);
    ``flag_tol`` is the near-tie margin tau (default 1e-4 x the longest side).
    """

    def __init__(self, sc, noise_sign: float = 1.0, flag_tol: float | None = None,
                 lib_path: str = LIBRARY):
        self.lib = load(lib_path)
        self.sc = sc
        self.dim = sc.dim
        self.shape = sc.shape
        n_species = len(sc.species)
        assert n_species in (1, 2) and sc.dim in (2, 3)
        self._keep = []
        p = _Params()
        p.dim, p.nx, p.ny, p.nz = sc.dim, sc.nx, sc.ny, sc.nz if sc.dim == 3 else 1
        p.dx, p.dt = sc.dx, sc.dt
        p.n_species = n_species
        for s, spc in enumerate(sc.species):
            p.D[s], p.k[s], p.sign[s] = spc.D, spc.k, spc.sign
            cells = np.ascontiguousarray(spc.source_cell, dtype=np.int32)
            q = np.ascontiguousarray(spc.source_q, dtype=np.float64)
            self._keep += [cells, q]
            p.n_sources[s] = cells.size
            p.source_cell[s] = _ptr(cells, C.c_int32)
            p.source_q[s] = _ptr(q, C.c_double)
        tgt = np.ascontiguousarray(sc.target_pos, dtype=np.float64).reshape(-1, sc.dim)
        self._keep.append(tgt)
        p.n_targets = tgt.shape[0]
        p.target_pos = _ptr(tgt, C.c_double)
        p.contact_radius = sc.contact_radius
        p.step_len, p.turn_gain = sc.step_len, sc.turn_gain
        p.max_turn, p.noise_sigma = sc.max_turn, sc.noise_sigma
        p.seed, p.sim_index = sc.seed, sc.sim_index
        p.noise_sign = noise_sign
        p.flag_tol = 1e-4 * sc.side if flag_tol is None else flag_tol
        law = getattr(sc, "snr_law", None)   # (snr_scale, cone_width, kd, c_min, c_max)
        if law is not None:
            p.turn_law = 1
            p.snr_scale, p.cone_width, p.kd, p.c_min, p.c_max = (float(v) for v in law)
        self.params = p
        self.flag_tol = p.flag_tol

        M = sc.n_cones
        self.fields = []
        for s in range(n_species):
            if sc.init_field is not None and sc.init_field[s] is not None:
                f = np.array(sc.init_field[s], dtype=np.float64).reshape(self.shape)
            else:
                f = np.zeros(self.shape, dtype=np.float64)
            self.fields.append(np.ascontiguousarray(f))
        self.pos = np.array(sc.cone_pos, dtype=np.float64).reshape(M, sc.dim).copy()
        if sc.dim == 2:
            self.dir = np.array(sc.cone_dir, dtype=np.float64).reshape(M).copy()
        else:
            self.dir = np.array(sc.cone_dir, dtype=np.float64).reshape(M, 3).copy()
        self.status = np.zeros(M, dtype=np.int32)
        self.target = np.full(M, -1, dtype=np.int32)
        self.event_step = np.full(M, -1, dtype=np.int32)
        self.flag_step = np.full(M, -1, dtype=np.int32)
        self.cap_margin = np.full(M, np.inf)
        self.step_count = 0
        self._bind_state()

    def _bind_state(self):
        st = _State()
        st.step = self.step_count
        for s, f in enumerate(self.fields):
            st.field[s] = _ptr(f, C.c_double)
        st.n_cones = self.pos.shape[0]
        st.pos = _ptr(self.pos, C.c_double)
        st.dir = _ptr(self.dir, C.c_double)
        st.status = _ptr(self.status, C.c_int32)
        st.target = _ptr(self.target, C.c_int32)
        st.event_step = _ptr(self.event_step, C.c_int32)
        st.flag_step = _ptr(self.flag_step, C.c_int32)
        st.cap_margin = _ptr(self.cap_margin, C.c_double)
        self.state = st

    # -- stepping --------------------------------------------------------------------
    def step(self, n: int = 1):
        self.state.step = self.step_count
        rc = self.lib.oracle_run(C.byref(self.params), C.byref(self.state), int(n))
        if rc != 0:
            raise MemoryError("oracle_run: allocation failed")
        self.step_count = int(self.state.step)
        return self

    def field_step_only(self):
        """F1 + F2 of one step without moving cones (does not advance the step count)."""
        out = [np.empty_like(f) for f in self.fields]
        ins = (_dp * 2)(*[_ptr(f, C.c_double) for f in self.fields] + [None] * (2 - len(out)))
        outs = (_dp * 2)(*[_ptr(f, C.c_double) for f in out] + [None] * (2 - len(out)))
        self.lib.oracle_field_step(C.byref(self.params), ins, outs)
        for s in range(len(out)):
            self.fields[s][...] = out[s]
        return self

    def adjoint(self, n_steps: int, assign, weight, magnitude=False, cone_adjoint=False):
        """Run n_steps forward (advancing this simulation) and return the trajectory loss
        sum_i weight[i] |p_i^N - target[assign[i]]|^2 with its gradient along the run's
        branch: (loss, dL/dq [all sources, species 0 first], dL/dD [species], dL/dk).  With
        magnitude=True a fifth item holds, for every component in the order
        (dL/dq..., dL/dD..., dL/dk...), the same sum over the absolute values of its terms;
        with cone_adjoint=True a further item holds dL/d(x, y, theta) of every cone at the
        start of the run ([M, 3])."""
        assign = np.ascontiguousarray(assign, dtype=np.int32)
        weight = np.ascontiguousarray(weight, dtype=np.float64)
        assert assign.shape == (self.pos.shape[0],) and weight.shape == assign.shape
        nq = int(sum(self.params.n_sources[s] for s in range(self.params.n_species)))
        dq = np.zeros(max(nq, 1))
        dD = np.zeros(2)
        dk = np.zeros(2)
        loss = np.zeros(1)
        ns = self.params.n_species
        mag = np.zeros(nq + 2 * ns)
        acone = np.zeros((max(self.pos.shape[0], 1), 3))
        self.state.step = self.step_count
        rc = self.lib.oracle_adjoint(C.byref(self.params), C.byref(self.state), int(n_steps),
                                     _ptr(assign, C.c_int32), _ptr(weight, C.c_double),
                                     _ptr(loss, C.c_double), _ptr(dq, C.c_double),
                                     _ptr(dD, C.c_double), _ptr(dk, C.c_double),
                                     _ptr(mag, C.c_double) if magnitude else None,
                                     _ptr(acone, C.c_double) if cone_adjoint else None)
        if rc == -2:
            raise ValueError("oracle_adjoint: 2D only")
        if rc != 0:
            raise MemoryError("oracle_adjoint: allocation failed")
        self.step_count = int(self.state.step)
        out = (float(loss[0]), dq[:nq].copy(), dD[:ns].copy(), dk[:ns].copy())
        if magnitude:
            out += (mag,)
        if cone_adjoint:
            out += (acone[: self.pos.shape[0]].copy(),)
        return out

    # -- reading ---------------------------------------------------------------------
    def mass(self, s: int = 0) -> float:
        return float(self.lib.oracle_mass(C.byref(self.params), _ptr(self.fields[s], C.c_double)))

    def sample_gradient(self, s: int, point) -> np.ndarray:
        pt = np.zeros(3)
        pt[: self.dim] = point
        g = np.zeros(3)
        self.lib.oracle_sample_gradient(C.byref(self.params), _ptr(self.fields[s], C.c_double),
                                        _ptr(pt, C.c_double), _ptr(g, C.c_double))
        return g[: self.dim]

    def events(self) -> np.ndarray:
        """Events (cone, target, step, kind) sorted by (step, cone); kind 1 contact, 2 exit."""
        idx = np.nonzero(self.status != ACTIVE)[0]
        ev = np.stack([idx, self.target[idx], self.event_step[idx], self.status[idx]], axis=1)
        order = np.lexsort((ev[:, 0], ev[:, 2])) if len(ev) else np.zeros(0, dtype=np.int64)
        return ev[order].astype(np.int32).reshape(-1, 4)

    def headings_vec(self) -> np.ndarray:
        if self.dim == 2:
            return np.stack([np.cos(self.dir), np.sin(self.dir)], axis=1)
        return self.dir.copy()

    # -- writing (restart from a given state) -----------------------------------------
    def set_state(self, fields=None, pos=None, dir=None, status=None, target=None,
                  event_step=None, step=None):
        if fields is not None:
            for s, f in enumerate(fields):
                self.fields[s][...] = np.asarray(f, dtype=np.float64).reshape(self.shape)
        if pos is not None:
            self.pos[...] = np.asarray(pos, dtype=np.float64).reshape(self.pos.shape)
        if dir is not None:
            self.dir[...] = np.asarray(dir, dtype=np.float64).reshape(self.dir.shape)
        if status is not None:
            self.status[...] = status
        if target is not None:
            self.target[...] = target
        if event_step is not None:
            self.event_step[...] = event_step
        if step is not None:
            self.step_count = int(step)
        self._bind_state()
        return self


def wrap_angle(theta):
    """Map angles to [-pi, pi) (for comparing headings modulo 2 pi)."""
    return np.asarray(theta) - 2.0 * math.pi * np.floor((np.asarray(theta) + math.pi) / (2.0 * math.pi))
