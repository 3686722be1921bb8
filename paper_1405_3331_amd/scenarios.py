"""Seeded synthetic inputs for the cue-diffusion / growth-cone simulation.

This module only *draws inputs*: grid sizes, coefficients, source cells and rates, cone
positions and headings, target positions.  It holds none of the simulation's arithmetic,
and it is the only code that the FP64 oracle and the GPU library have in common: both are
handed the arrays it produces.

Every floating-point array is rounded to a value exactly representable in FP32, so the
FP64 oracle and the FP32 GPU path start from bit-identical inputs.  Scalars that enter
through the parameter struct as doubles (dx, dt, D, k, radii, gains) are passed as-is to
both sides.

The named workloads mirror the paper's setting (Sec. 3.4-3.5: neurons with growth cones
advancing a fixed distance per step, turning at most pi/30, diffusing guidance cues from
sources) at the sizes this implementation is measured on:

  small     2D 128^2, dt 0.2, k 0.01, 4 sources emitting 1.0/step, 64 cones, 16 targets,
            1000 steps (parity workload)
  headline  2D 2048^2, dt 0.2, k 0.005, 16 sources with rates U(0.5, 2), 65,536 cones,
            1024 targets, 10,000 steps
  volume    3D 256^3, dt 0.15, attractant (D 1.0, k 0.01) and repellent (D 0.5, k 0.02)
            species with 64 sources each, 262,144 cones, 4096 targets, 2000 steps
  adjoint   2D 1024^2, dt 0.2, k 0.005, 32 sources U(0.5, 2), 8192 cones, 256 targets,
            2000 steps
  batched   512 independent 2D simulations, side U{64..512}, cones log-uniform [16, 4096],
            D U(0.5, 1.5), k U(0.001, 0.02), 4-32 sources, dt 0.8 x the stability limit
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Stream tags: every kind of input draws from its own seeded stream.
_TAG_SOURCE_CELL = 1
_TAG_SOURCE_RATE = 2
_TAG_CONE_POS = 3
_TAG_CONE_DIR = 4
_TAG_TARGET_POS = 5
_TAG_BATCH = 6

DEFAULT_MAX_TURN = math.pi / 30.0  # turn magnitude per step fixed in Sec. 3.5


def _f32(a) -> np.ndarray:
    """Round to FP32 and hand back as float64 holding the same values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rng(seed: int, tag: int, species: int = 0, sim_index: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(tag), int(species), int(sim_index)])


@dataclasses.dataclass
class Species:
    D: float
    k: float
    sign: float
    source_cell: np.ndarray   # int32 [S] linear cell index
    source_q: np.ndarray      # float64 (FP32-exact) [S], amount per step


@dataclasses.dataclass
class Scenario:
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    species: List[Species]
    cone_pos: np.ndarray      # [M][dim]
    cone_dir: np.ndarray      # 2D: [M] angle in [-pi, pi); 3D: [M][3] unit vectors
    target_pos: np.ndarray    # [T][dim]
    contact_radius: float
    step_len: float
    turn_gain: float
    max_turn: float
    noise_sigma: float
    seed: int
    sim_index: int
    n_steps: int
    init_field: Optional[List[np.ndarray]] = None
    # SNR turn law of Sec. 3.5, Eq. 5 (2D) instead of vector addition: (snr_scale,
    # cone_width, kd, c_min, c_max); None = vector addition
    snr_law: Optional[tuple] = None

    @property
    def shape(self):
        """Field array shape, slowest axis first."""
        return (self.ny, self.nx) if self.dim == 2 else (self.nz, self.ny, self.nx)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * (self.nz if self.dim == 3 else 1)

    @property
    def n_cones(self) -> int:
        return int(self.cone_pos.shape[0])

    @property
    def n_targets(self) -> int:
        return int(self.target_pos.shape[0])

    @property
    def extent(self) -> np.ndarray:
        n = [self.nx, self.ny, self.nz][: self.dim]
        return np.array(n, dtype=np.float64) * self.dx

    @property
    def side(self) -> float:
        """Longest domain side L (the scale of the tip tolerance)."""
        return float(self.extent.max())


def uniform_points(seed, tag, count, extent, species=0, sim_index=0) -> np.ndarray:
    """FP32-exact points uniform in [0, extent) per axis."""
    u = _rng(seed, tag, species, sim_index).random((count, len(extent)))
    pts = _f32(u * np.asarray(extent, dtype=np.float64))
    # Rounding to FP32 can land exactly on the upper face; pull such points inside.
    for a, e in enumerate(extent):
        hi = np.nextafter(np.float32(e), np.float32(0.0)).astype(np.float64)
        pts[:, a] = np.minimum(pts[:, a], hi)
    return pts


def headings(seed, count, dim, sim_index=0) -> np.ndarray:
    """Initial headings: 2D uniform angles; 3D by the normal-deviate method (Sec. 3.2)."""
    g = _rng(seed, _TAG_CONE_DIR, 0, sim_index)
    if dim == 2:
        theta = _f32(2.0 * math.pi * g.random(count) - math.pi)
        return np.clip(theta, -math.pi, np.nextafter(np.float32(math.pi), 0).astype(np.float64))
    z = g.standard_normal((count, 3))
    norm = np.linalg.norm(z, axis=1, keepdims=True)
    norm[norm == 0.0] = 1.0
    return _f32(z / norm)


def source_cells(seed, count, n_axes, species=0, sim_index=0) -> np.ndarray:
    """Linear indices of cells drawn uniformly over the grid."""
    u = _rng(seed, _TAG_SOURCE_CELL, species, sim_index).random((count, len(n_axes)))
    idx = np.minimum((u * np.asarray(n_axes)).astype(np.int64), np.asarray(n_axes) - 1)
    lin = np.zeros(count, dtype=np.int64)
    stride = 1
    for a, n in enumerate(n_axes):
        lin += idx[:, a] * stride
        stride *= n
    return lin.astype(np.int32)


def source_rates(seed, count, lo, hi, species=0, sim_index=0) -> np.ndarray:
    if lo == hi:
        return _f32(np.full(count, lo))
    return _f32(lo + (hi - lo) * _rng(seed, _TAG_SOURCE_RATE, species, sim_index).random(count))


def make_scenario(name="custom", dim=2, n=(128, 128), dx=1.0, dt=0.2,
                  species=((1.0, 0.01, 1.0),), n_sources=4, rate=(1.0, 1.0),
                  n_cones=64, n_targets=16, contact_radius=1.0, step_len=0.5,
                  turn_gain=10.0, max_turn=DEFAULT_MAX_TURN, noise_sigma=0.1,
                  seed=0, sim_index=0, n_steps=1000) -> Scenario:
    """Build a seeded scenario.  ``n`` is (nx, ny) or (nx, ny, nz); ``species`` is a
    sequence of (D, k, sign); ``n_sources`` an int or one int per species."""
    n = tuple(int(v) for v in n)
    assert len(n) == dim
    extent = np.array(n, dtype=np.float64) * dx
    if isinstance(n_sources, int):
        n_sources = [n_sources] * len(species)
    sp = []
    for s, ((D, k, sign), ns) in enumerate(zip(species, n_sources)):
        sp.append(Species(D=float(D), k=float(k), sign=float(sign),
                          source_cell=source_cells(seed, ns, n, s, sim_index),
                          source_q=source_rates(seed, ns, rate[0], rate[1], s, sim_index)))
    return Scenario(
        name=name, dim=dim, nx=n[0], ny=n[1], nz=n[2] if dim == 3 else 1, dx=float(dx),
        dt=float(dt), species=sp,
        cone_pos=uniform_points(seed, _TAG_CONE_POS, n_cones, extent, 0, sim_index),
        cone_dir=headings(seed, n_cones, dim, sim_index),
        target_pos=uniform_points(seed, _TAG_TARGET_POS, n_targets, extent, 0, sim_index),
        contact_radius=float(contact_radius), step_len=float(step_len),
        turn_gain=float(turn_gain), max_turn=float(max_turn), noise_sigma=float(noise_sigma),
        seed=int(seed), sim_index=int(sim_index), n_steps=int(n_steps))


def small(seed=0) -> Scenario:
    return make_scenario("small 2D 128^2", 2, (128, 128), 1.0, 0.2, ((1.0, 0.01, 1.0),),
                         4, (1.0, 1.0), 64, 16, seed=seed, n_steps=1000)


def headline(seed=0) -> Scenario:
    return make_scenario("headline 2D 2048^2", 2, (2048, 2048), 1.0, 0.2,
                         ((1.0, 0.005, 1.0),), 16, (0.5, 2.0), 65536, 1024,
                         seed=seed, n_steps=10000)


def volume(seed=0) -> Scenario:
    return make_scenario("volume 3D 256^3 two species", 3, (256, 256, 256), 1.0, 0.15,
                         ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), 64, (1.0, 1.0),
                         262144, 4096, seed=seed, n_steps=2000)


def adjoint(seed=0) -> Scenario:
    return make_scenario("adjoint 2D 1024^2", 2, (1024, 1024), 1.0, 0.2,
                         ((1.0, 0.005, 1.0),), 32, (0.5, 2.0), 8192, 256,
                         seed=seed, n_steps=2000)


def batched(seed=0, count=512) -> List[Scenario]:
    """Independent 2D simulations of uneven size for the batched workload."""
    g = _rng(seed, _TAG_BATCH)
    out = []
    for b in range(count):
        side = int(g.integers(64, 513))
        cones = int(math.floor(math.exp(g.uniform(math.log(16), math.log(4096)))))
        D = float(g.uniform(0.5, 1.5))
        k = float(g.uniform(0.001, 0.02))
        ns = int(g.integers(4, 33))
        dt = 0.8 * 1.0 / (2 * 2 * D)   # 0.8 x the limit dt * D / dx^2 <= 1 / (2 dim)
        out.append(make_scenario(f"batched[{b}]", 2, (side, side), 1.0, dt,
                                 ((D, k, 1.0),), ns, (0.5, 2.0), cones,
                                 max(4, side * side // 1024), seed=seed, sim_index=b,
                                 n_steps=2000))
    return out


NAMED = {"small": small, "headline": headline, "volume": volume, "adjoint": adjoint}
