"""Pins of the FP64 oracle against what the mathematics and the paper fix.

Each ``pin_*`` function runs the oracle (optionally a rebuilt variant at ``lib_path``) on a
small case and raises AssertionError when the oracle disagrees with an independent fact:
an exact invariant, a closed-form solution, a geometric construction of the turn rule,
the published Philox bijection as implemented by another library, or brute force.  The
same functions back the ordinary tests and the planted-mistake tests, which rebuild the
oracle with one deliberate error and require that some pin fails.
"""
from __future__ import annotations

import math
import os
import subprocess
import tempfile

import numpy as np
import scipy.special
import scipy.stats

import oracle
from oracle import OracleSim
from paper_1405_3331_amd.scenarios import Scenario, Species, make_scenario

LIB = oracle.LIBRARY


def _blank(dim=2, n=(32, 24), dx=1.0, dt=0.2, species=((1.0, 0.0, 1.0),), **kw):
    """Scenario with no sources, cones or targets unless given."""
    kw.setdefault("n_sources", 0)
    kw.setdefault("n_cones", 0)
    kw.setdefault("n_targets", 0)
    return make_scenario("pin", dim, n, dx, dt, species, **kw)


def _centres(sc, a):
    n = [sc.nx, sc.ny, sc.nz][a]
    return (np.arange(n) + 0.5) * sc.dx


def _mesh(sc):
    """Cell-centre coordinates broadcast to the field shape (slowest axis first)."""
    axes = [_centres(sc, a) for a in range(sc.dim)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    return grids[::-1]   # x, y[, z] each shaped like the field


# ---------------------------------------------------------------------------------------
# P1: mass recursion M^{n+1} = (1 - k dt) M^n + sum(q), exact with zero-flux walls.
# ---------------------------------------------------------------------------------------
def pin_mass_recursion(lib_path=LIB, dim=2):
    if dim == 2:
        sc = make_scenario("p1", 2, (37, 29), 0.5, 0.05, ((1.0, 0.02, 1.0), (0.5, 0.01, -1.0)),
                           n_sources=[3, 5], rate=(0.5, 2.0), n_cones=6, n_targets=3)
    else:
        sc = make_scenario("p1", 3, (11, 9, 7), 0.5, 0.04, ((1.0, 0.02, 1.0), (0.5, 0.03, -1.0)),
                           n_sources=[4, 2], rate=(0.5, 2.0), n_cones=6, n_targets=3)
    # Two sources sharing a cell must both add.
    sp0 = sc.species[0]
    sp0.source_cell = np.concatenate([sp0.source_cell, sp0.source_cell[:1]]).astype(np.int32)
    sp0.source_q = np.concatenate([sp0.source_q, [0.75]])
    o = OracleSim(sc, lib_path=lib_path)
    M = [0.0] * len(sc.species)
    for n in range(120):
        o.step(1)
        for s, spc in enumerate(sc.species):
            M[s] = (1.0 - spc.k * sc.dt) * M[s] + float(np.sum(spc.source_q))
            got = o.mass(s)
            assert abs(got - M[s]) <= 1e-12 * abs(M[s]), (n, s, got, M[s])


# ---------------------------------------------------------------------------------------
# P2: from a unit point mass, before any mass reaches a wall, the mean stays at the
# centre and the variance per axis grows by exactly 2 D dt / (1 - k dt) per step: the
# Laplacian adds 2 dx^2 r M to the second moment (sum x^2 Lap c = 2 dx^2 sum c) while the
# explicit decay scales the mass by (1 - k dt).
# ---------------------------------------------------------------------------------------
def pin_moments(lib_path=LIB, dim=2):
    steps = 12 if dim == 2 else 5
    side = 2 * steps + 5
    dx, D, k = 0.5, 0.8, 0.03
    dt = 0.2 * dx * dx / D
    n = (side,) * dim
    sc = _blank(dim, n, dx, dt, ((D, k, 1.0),))
    f = np.zeros(sc.shape)
    centre = (side // 2,) * dim
    f[centre] = 1.0 / dx ** dim
    sc.init_field = [f]
    o = OracleSim(sc, lib_path=lib_path)
    o.step(steps)
    c = o.fields[0]
    mass = c.sum() * dx ** dim
    assert abs(mass - (1.0 - k * dt) ** steps) <= 1e-13, mass
    coords = _mesh(sc)
    x0 = (side // 2 + 0.5) * dx
    for a in range(dim):
        mean = (c * coords[a]).sum() * dx ** dim / mass
        var = (c * (coords[a] - x0) ** 2).sum() * dx ** dim / mass
        assert abs(mean - x0) <= 1e-12 * x0, (a, mean, x0)
        expect = 2.0 * D * dt * steps / (1.0 - k * dt)
        assert abs(var - expect) <= 1e-11 * expect, (a, var, expect)


# ---------------------------------------------------------------------------------------
# P3: far from walls the point-source solution approaches the free-space Green's function
# M / (4 pi D t)^(d/2) exp(-|x|^2 / (4 D t)); the discrete error falls like 1/t.
# ---------------------------------------------------------------------------------------
def pin_green_function(lib_path=LIB):
    side, D, dt = 161, 1.0, 0.2
    sc = _blank(2, (side, side), 1.0, dt, ((D, 0.0, 1.0),))
    f = np.zeros(sc.shape)
    f[side // 2, side // 2] = 1.0
    sc.init_field = [f]
    o = OracleSim(sc, lib_path=lib_path)
    x, y = _mesh(sc)
    r2 = (x - (side // 2 + 0.5)) ** 2 + (y - (side // 2 + 0.5)) ** 2
    errs = []
    done = 0
    for steps in (50, 200, 400):
        o.step(steps - done)
        done = steps
        t = steps * dt
        g = np.exp(-r2 / (4 * D * t)) / (4 * math.pi * D * t)
        errs.append(np.abs(o.fields[0] - g).max() / g.max())
    assert errs[0] < 2.0e-2 and errs[1] < 5.0e-3 and errs[2] < 2.5e-3, errs
    assert errs[0] > errs[1] > errs[2], errs
    # error ~ 1/t: quadrupling t cuts it by at least 3
    assert errs[0] / errs[1] > 3.0, errs


# ---------------------------------------------------------------------------------------
# P4: steady state of a point source with decay.  2D: (q/dt)/(2 pi D) K0(r/l);
# 3D: (q/dt)/(4 pi D r) exp(-r/l); l = sqrt(D/k).
# ---------------------------------------------------------------------------------------
def pin_steady_state_2d(lib_path=LIB):
    side, D, k, dt, q = 121, 1.0, 0.04, 0.2, 1.0
    sc = _blank(2, (side, side), 1.0, dt, ((D, k, 1.0),))
    sc.species[0].source_cell = np.array([(side // 2) * side + side // 2], dtype=np.int32)
    sc.species[0].source_q = np.array([q])
    o = OracleSim(sc, lib_path=lib_path)
    o.step(2500)
    ell = math.sqrt(D / k)
    c = o.fields[0]
    mid = side // 2
    worst = 0.0
    for d in range(4, 26):
        expect = (q / dt) / (2 * math.pi * D) * scipy.special.k0(d / ell)
        for got in (c[mid, mid + d], c[mid, mid - d], c[mid + d, mid], c[mid - d, mid]):
            worst = max(worst, abs(got - expect) / expect)
    assert worst < 0.02, worst
    # the total is at the fixed point of the mass recursion
    assert abs(o.mass() - q / (k * dt)) < 1e-6 * q / (k * dt)


def pin_steady_state_3d(lib_path=LIB):
    side, D, k, dt, q = 41, 1.0, 1.0 / 9.0, 0.15, 1.0
    sc = _blank(3, (side, side, side), 1.0, dt, ((D, k, 1.0),))
    mid = side // 2
    sc.species[0].source_cell = np.array([(mid * side + mid) * side + mid], dtype=np.int32)
    sc.species[0].source_q = np.array([q])
    o = OracleSim(sc, lib_path=lib_path)
    o.step(700)
    ell = math.sqrt(D / k)
    c = o.fields[0]
    worst = 0.0
    # the lattice differs from the continuum by a few per cent at l = 3 cells (second-order
    # in dx / l); a wrong factor anywhere would be off by tens of per cent
    for d in range(5, 13):
        expect = (q / dt) / (4 * math.pi * D * d) * math.exp(-d / ell)
        for got in (c[mid, mid, mid + d], c[mid, mid - d, mid], c[mid + d, mid, mid]):
            worst = max(worst, abs(got - expect) / expect)
    assert worst < 0.045, worst


# ---------------------------------------------------------------------------------------
# P5: a line of sources (one per row, same column) has the exact discrete steady state
# c_j = c_0 * lam^|j|, lam = 1 + a/2 - sqrt(a + a^2/4), a = k dx^2 / D,
# c_0 = (q / dx^dim) / (2 r (1 - lam) + k dt); each row holds q / (k dt) / dx^(dim-1).
# ---------------------------------------------------------------------------------------
def pin_line_source(lib_path=LIB):
    nx, ny, dx, D, k, q = 241, 3, 2.0, 1.0, 0.025, 1.0
    dt = 0.2 * dx * dx / D
    sc = _blank(2, (nx, ny), dx, dt, ((D, k, 1.0),))
    col = nx // 2
    sc.species[0].source_cell = np.array([j * nx + col for j in range(ny)], dtype=np.int32)
    sc.species[0].source_q = np.full(ny, q)
    o = OracleSim(sc, lib_path=lib_path)
    o.step(2500)
    a = k * dx * dx / D
    r = D * dt / (dx * dx)
    lam = 1.0 + a / 2.0 - math.sqrt(a + a * a / 4.0)
    c0 = (q / dx ** 2) / (2.0 * r * (1.0 - lam) + k * dt)
    c = o.fields[0]
    for j in range(ny):
        for off in range(0, 60):
            expect = c0 * lam ** off
            for i in (col + off, col - off):
                assert abs(c[j, i] - expect) <= 1e-11 * c0, (j, i, c[j, i], expect)


# ---------------------------------------------------------------------------------------
# P6: cosine eigenmodes of the zero-flux lattice decay by exactly
# G = 1 - k dt - 2 r sum_a (1 - cos(pi m_a / n_a)) per step; above r = 1/(2 dim) the top
# mode has |G| > 1 and grows.
# ---------------------------------------------------------------------------------------
def _mode_field(sc, modes):
    coords = _mesh(sc)
    f = np.ones(sc.shape)
    for a, m in enumerate(modes):
        n = [sc.nx, sc.ny, sc.nz][a]
        f = f * np.cos(math.pi * m * (coords[a] / sc.dx) / n)   # (i + 1/2) = x / dx
    return f


def pin_eigenmodes(lib_path=LIB, dim=2, r_value=0.2, steps=40):
    if dim == 2:
        n, modes = (23, 17), (3, 5)
    else:
        n, modes = (9, 7, 6), (2, 1, 3)
    dx, D, k = 1.0, 1.0, 0.01
    dt = r_value * dx * dx / D
    sc = _blank(dim, n, dx, dt, ((D, k, 1.0),))
    f0 = _mode_field(sc, modes)
    sc.init_field = [f0]
    o = OracleSim(sc, lib_path=lib_path)
    o.step(steps)
    r = D * dt / dx ** 2
    G = 1.0 - k * dt - 2.0 * r * sum(1.0 - math.cos(math.pi * m / nn) for m, nn in zip(modes, n))
    err = np.abs(o.fields[0] - G ** steps * f0).max()
    assert err <= 1e-12 * max(1.0, abs(G) ** steps), (err, G)
    return G


def pin_unstable_mode(lib_path=LIB):
    n = (12, 10)
    modes = (11, 9)
    G = pin_eigenmodes_custom(lib_path, n, modes, r_value=0.26, steps=30)
    assert G < -1.0


def pin_eigenmodes_custom(lib_path, n, modes, r_value, steps, k=0.0):
    dx, D = 1.0, 1.0
    dt = r_value * dx * dx / D
    sc = _blank(len(n), n, dx, dt, ((D, k, 1.0),))
    f0 = _mode_field(sc, modes)
    sc.init_field = [f0]
    o = OracleSim(sc, lib_path=lib_path)
    o.step(steps)
    r = D * dt / dx ** 2
    G = 1.0 - k * dt - 2.0 * r * sum(1.0 - math.cos(math.pi * m / nn) for m, nn in zip(modes, n))
    err = np.abs(o.fields[0] - G ** steps * f0).max()
    assert err <= 1e-12 * max(1.0, abs(G) ** steps), (err, G)
    return G


# ---------------------------------------------------------------------------------------
# Maximum principle: for 2 dim r + k dt <= 1 and no sources, the field stays within
# [0, previous max] and the max never increases.
# ---------------------------------------------------------------------------------------
def pin_max_principle(lib_path=LIB, dim=2):
    n = (19, 13) if dim == 2 else (7, 6, 5)
    dt = 0.25 if dim == 2 else 1.0 / 6.0
    sc = _blank(dim, n, 1.0, dt, ((1.0, 0.0, 1.0),))
    f = np.random.default_rng(3).random(sc.shape)
    sc.init_field = [f]
    o = OracleSim(sc, lib_path=lib_path)
    prev = f.max()
    for _ in range(30):
        o.step(1)
        assert o.fields[0].min() >= 0.0
        assert o.fields[0].max() <= prev * (1 + 1e-15)
        prev = o.fields[0].max()


# ---------------------------------------------------------------------------------------
# C1: the interpolated central-difference gradient is exact for quadratic fields in the
# interior (central differences are exact for quadratics; multilinear interpolation is
# exact for their linear derivatives); within half a cell of a wall it is the wall cell's
# one-sided half difference (zero-flux ghost).
# ---------------------------------------------------------------------------------------
def pin_gradient_quadratic(lib_path=LIB, dim=2):
    rng = np.random.default_rng(11)
    n = (14, 11) if dim == 2 else (9, 8, 7)
    dx = 0.5
    sc = _blank(dim, n, dx, 0.01, ((0.0, 0.0, 1.0),))
    coords = _mesh(sc)
    coef = rng.uniform(-1, 1, size=(dim, dim))
    coef = coef + coef.T                       # symmetric Hessian H: c = x^T H x / 2 + b.x
    b = rng.uniform(-1, 1, size=dim)
    c = sum(b[a] * coords[a] for a in range(dim))
    for a in range(dim):
        for bb in range(dim):
            c = c + 0.5 * coef[a, bb] * coords[a] * coords[bb]
    sc.init_field = [c]
    o = OracleSim(sc, lib_path=lib_path)
    ext = sc.extent
    for _ in range(200):
        p = rng.uniform(2.0 * dx, ext - 2.0 * dx)
        g = o.sample_gradient(0, p)
        expect = b + coef @ p
        assert np.allclose(g, expect, rtol=0, atol=1e-12), (p, g, expect)
    # Within half a cell of the x = 0 wall, the x component is the first cell's ghost
    # value (c[1] - c[0]) / (2 dx) interpolated along the other axes only.
    p = rng.uniform(2.0 * dx, ext - 2.0 * dx)
    p[0] = 0.2 * dx
    g = o.sample_gradient(0, p)
    q = p.copy()
    q[0] = 0.5 * dx                                 # the first cell centre along x
    interior = b + coef @ q                          # exact centred gradient there
    # one-sided half difference of the quadratic along x at the first centre:
    step = np.zeros(dim)
    step[0] = dx
    cx0 = float(b @ q + 0.5 * q @ coef @ q)
    q1 = q + step
    cx1 = float(b @ q1 + 0.5 * q1 @ coef @ q1)
    # the other coordinates are interpolated linearly, where the half difference of a
    # quadratic is linear as well, so the mixed terms interpolate exactly
    assert abs(g[0] - (cx1 - cx0) / (2 * dx)) <= 1e-12, (g[0], (cx1 - cx0) / (2 * dx))
    for a in range(1, dim):
        assert abs(g[a] - interior[a]) <= 1e-12


# ---------------------------------------------------------------------------------------
# C2: in a static linear field (D = 0, k = 0, no sources) the interior gradient is the
# constant slope g, and each step the heading turns toward the direction of the vector
# sum h + gain * g (Sec. 3.5, vector-addition steering), by at most pi/30 (Sec. 3.5).
# Reproduced here with complex arithmetic / Rodrigues rotations, not the dot/cross form.
# ---------------------------------------------------------------------------------------
def _static_linear_scenario(dim, slope, sign, theta0, gain, steps, n=200):
    sc = make_scenario("p9", dim, (n,) * dim, 1.0, 0.1, ((0.0, 0.0, sign),), n_sources=0,
                       n_cones=len(theta0), n_targets=0, turn_gain=gain, noise_sigma=0.0,
                       n_steps=steps)
    coords = _mesh(sc)
    sc.init_field = [sum(slope[a] * coords[a] for a in range(dim))]
    mid = n * 0.5
    sc.cone_pos = np.full((len(theta0), dim), mid)
    sc.cone_dir = np.array(theta0, dtype=np.float64)
    return sc


def pin_turn_rule_2d(lib_path=LIB):
    rng = np.random.default_rng(5)
    cap = math.pi / 30.0
    for slope, sign, gain in (((0.01, 0.0), 1.0, 10.0), ((0.3, -0.2), 1.0, 10.0),
                              ((0.002, 0.004), -1.0, 10.0), ((0.05, 0.0), 1.0, 1.0)):
        theta0 = rng.uniform(-math.pi, math.pi, 12)
        steps = 40
        sc = _static_linear_scenario(2, slope, sign, theta0, gain, steps)
        o = OracleSim(sc, lib_path=lib_path)
        g = sign * complex(*slope)
        h = np.exp(1j * theta0)
        pos = sc.cone_pos[:, 0] + 1j * sc.cone_pos[:, 1]
        for n in range(steps):
            o.step(1)
            resultant = h + gain * g
            want = np.angle(resultant / h)            # signed angle from h to h + gain g
            turn = np.clip(want, -cap, cap)
            h = h * np.exp(1j * turn)
            pos = pos + sc.step_len * h
            got = np.exp(1j * o.dir)
            assert np.abs(got - h).max() < 1e-11, (slope, n, np.abs(got - h).max())
            assert np.abs(o.pos[:, 0] + 1j * o.pos[:, 1] - pos).max() < 1e-10


def _rotate_towards(h, v, angle):
    """Rotate unit h toward direction v (in their common plane) by ``angle``."""
    vn = v / np.linalg.norm(v)
    axis = np.cross(h, vn)
    s = np.linalg.norm(axis)
    if s == 0.0:
        return h
    axis = axis / s
    # Rodrigues' rotation about axis
    return (h * math.cos(angle) + np.cross(axis, h) * math.sin(angle)
            + axis * np.dot(axis, h) * (1 - math.cos(angle)))


def pin_turn_rule_3d(lib_path=LIB):
    rng = np.random.default_rng(6)
    cap = math.pi / 30.0
    for slope, sign, gain in (((0.01, 0.02, -0.01), 1.0, 10.0), ((0.5, 0.0, 0.0), 1.0, 10.0),
                              ((0.0, 0.01, 0.01), -1.0, 10.0)):
        h0 = rng.standard_normal((6, 3))
        h0 /= np.linalg.norm(h0, axis=1, keepdims=True)
        steps = 30
        sc = _static_linear_scenario(3, slope, sign, h0, gain, steps, n=60)
        o = OracleSim(sc, lib_path=lib_path)
        g = sign * np.array(slope)
        h = h0.copy()
        pos = sc.cone_pos.copy()
        for n in range(steps):
            o.step(1)
            for i in range(len(h)):
                v = h[i] + gain * g
                want = math.atan2(np.linalg.norm(np.cross(h[i], v)), np.dot(h[i], v))
                h[i] = _rotate_towards(h[i], v, min(want, cap))
                h[i] /= np.linalg.norm(h[i])
            pos = pos + sc.step_len * h
            assert np.abs(o.dir - h).max() < 1e-10, (slope, n, np.abs(o.dir - h).max())
            assert np.abs(o.pos - pos).max() < 1e-9


# ---------------------------------------------------------------------------------------
# C4-C6 (P7, direct guidance, Sec. 3.4): with gain 0 and no noise each cone moves in a
# straight line, p^n = p^0 + n s h^0, until it first leaves [0, L) on some axis or first
# comes strictly within R of a target (nearest target, lowest index on a tie) -- found
# here by brute force over steps and targets.
# ---------------------------------------------------------------------------------------
def pin_direct_guidance(lib_path=LIB, dim=2):
    n = (40, 30) if dim == 2 else (16, 14, 12)
    sc = make_scenario("p7", dim, n, 1.0, 0.1, ((1.0, 0.01, 1.0),), n_sources=2,
                       n_cones=300, n_targets=25 if dim == 2 else 60, contact_radius=1.3,
                       turn_gain=0.0, noise_sigma=0.0, seed=9)
    steps = 120
    o = OracleSim(sc, lib_path=lib_path)
    o.step(steps)
    if dim == 2:
        h0 = np.stack([np.cos(sc.cone_dir), np.sin(sc.cone_dir)], axis=1)
    else:
        # 3D headings are renormalised every step; the FP32-rounded inputs are unit to ~1e-8
        h0 = sc.cone_dir / np.linalg.norm(sc.cone_dir, axis=1, keepdims=True)
    L = sc.extent
    R2 = sc.contact_radius ** 2
    checked = 0
    for i in range(sc.n_cones):
        status, target, ev = 0, -1, -1
        margin = np.inf
        for k in range(1, steps + 1):
            p = sc.cone_pos[i] + k * sc.step_len * h0[i]
            margin = min(margin, np.abs(p).min(), np.abs(L - p).min())
            if np.any(p < 0) or np.any(p >= L):
                status, ev = 2, k
                break
            d2 = ((sc.target_pos - p) ** 2).sum(axis=1)
            margin = min(margin, np.abs(np.sqrt(d2) - sc.contact_radius).min())
            if d2.min() < R2:
                status, target, ev = 1, int(np.argmin(d2)), k
                break
        if status == 0:
            p = sc.cone_pos[i] + steps * sc.step_len * h0[i]
        if margin < 1e-9:
            continue
        checked += 1
        assert (o.status[i], o.target[i], o.event_step[i]) == (status, target, ev), \
            (i, (o.status[i], o.target[i], o.event_step[i]), (status, target, ev))
        assert np.abs(o.pos[i] - p).max() < 1e-9, (i, o.pos[i], p)
    assert checked > 0.9 * sc.n_cones
    counts = np.bincount(o.status, minlength=3)
    assert counts[1] > 0 and counts[2] > 0, counts


def pin_contact_edges(lib_path=LIB):
    """Strict '<' at exactly R; exact ties go to the lowest target index; exit at exactly
    x = L (outside, [0, L) is half-open) and not at x = 0."""
    base = dict(dim=2, n=(20, 20), dx=1.0, dt=0.1, species=((1.0, 0.0, 1.0),),
                n_sources=0, n_targets=0, turn_gain=0.0, noise_sigma=0.0)
    sc = make_scenario("edges", n_cones=4, **base)
    sc.cone_pos = np.array([[10.0, 10.0], [5.0, 5.0], [19.5, 3.0], [0.5, 7.0]])
    sc.cone_dir = np.array([0.0, 0.0, 0.0, math.pi])
    # cone 0 ends at (10.5, 10): target 0 at exactly R = 1 (no contact),
    # cone 1 ends at (5.5, 5): targets 1 and 2 both at distance 0.5 -> index 1 wins
    sc.target_pos = np.array([[11.5, 10.0], [5.5, 5.5], [5.5, 4.5]])
    sc.contact_radius = 1.0
    o = OracleSim(sc, lib_path=lib_path, flag_tol=0.0)
    o.step(1)
    assert o.status[0] == 0, o.status
    assert (o.status[1], o.target[1], o.event_step[1]) == (1, 1, 1)
    # cone 2 reaches x = 20.0 = L exactly -> exited; cone 3 reaches x = 0.0 -> inside
    assert (o.status[2], o.event_step[2]) == (2, 1)
    assert o.status[3] == 0 and o.pos[3, 0] == 0.0


# ---------------------------------------------------------------------------------------
# C3 (P8): with gain 0 the heading is a random walk of the Philox/Box-Muller stream
# keyed (cone, step, tag 0, simulation): theta^n = theta^0 + sigma sum_k Z0(cone, k).
# ---------------------------------------------------------------------------------------
def pin_noise_plumbing(lib_path=LIB):
    seed = (7 << 32) | 12345
    sc = make_scenario("p8", 2, (400, 400), 1.0, 0.1, ((1.0, 0.0, 1.0),), n_sources=0,
                       n_cones=10, n_targets=0, turn_gain=0.0, noise_sigma=0.07,
                       seed=seed, sim_index=3)
    sc.cone_pos = np.full((10, 2), 200.0)
    steps = 50
    o = OracleSim(sc, lib_path=lib_path)
    o.step(steps)
    lib = oracle.load(lib_path)
    for i in range(sc.n_cones):
        theta = sc.cone_dir[i]
        p = sc.cone_pos[i].copy()
        for k in range(steps):
            # 2D: one Philox block per two steps, first pair for even k, second for odd k
            z = oracle.normals4(seed, i, k // 2, 0, 3, lib=lib)
            theta = theta + sc.noise_sigma * z[2 * (k % 2)]
            p = p + sc.step_len * np.array([math.cos(theta), math.sin(theta)])
        d = (o.dir[i] - theta + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-12, (i, o.dir[i], theta)
        assert np.abs(o.pos[i] - p).max() < 1e-10


def pin_noise_3d(lib_path=LIB):
    """3D noise is a rotation by |w| (w the tangent part of sigma z, two Gaussian degrees
    of freedom): the angle between successive headings is sigma times a Rayleigh(1)
    variable (mean square 2 sigma^2), with no preferred direction; headings stay unit."""
    sigma = 0.4
    sc = make_scenario("p8-3d", 3, (8, 8, 8), 1.0, 0.1, ((1.0, 0.0, 1.0),),
                       n_sources=0, n_cones=4000, n_targets=0, turn_gain=0.0,
                       noise_sigma=sigma, seed=4)
    sc.cone_pos = np.full((sc.n_cones, 3), 4.0)
    o = OracleSim(sc, lib_path=lib_path)
    prev = o.dir.copy()
    ang2 = []
    drift = np.zeros(3)
    for _ in range(5):
        o.step(1)
        cosang = np.clip((o.dir * prev).sum(axis=1), -1, 1)
        ang2.append(np.arccos(cosang) ** 2)
        drift += (o.dir - prev).sum(axis=0)
        prev = o.dir.copy()
    angles = np.sqrt(np.concatenate(ang2))
    ms = (angles ** 2).mean()
    assert abs(ms / (2 * sigma ** 2) - 1.0) < 0.04, ms / (2 * sigma ** 2)
    ks = scipy.stats.kstest(angles / sigma, "rayleigh")
    assert ks.pvalue > 1e-4, ks
    assert np.abs(np.linalg.norm(o.dir, axis=1) - 1.0).max() < 1e-14
    assert np.abs(drift).max() / (sc.n_cones * 5 * sigma) < 0.03


# ---------------------------------------------------------------------------------------
# P10: mirror symmetry x -> L - x (sources, cones, headings, targets mirrored; noise
# negated) mirrors the whole run.
# ---------------------------------------------------------------------------------------
def pin_mirror(lib_path=LIB):
    sc = make_scenario("p10", 2, (40, 30), 1.0, 0.2, ((1.0, 0.01, 1.0),), n_sources=3,
                       rate=(0.5, 2.0), n_cones=40, n_targets=8, seed=2)
    nx, L = sc.nx, sc.extent[0]
    m = make_scenario("p10m", 2, (40, 30), 1.0, 0.2, ((1.0, 0.01, 1.0),), n_sources=3,
                      rate=(0.5, 2.0), n_cones=40, n_targets=8, seed=2)
    cells = sc.species[0].source_cell
    m.species[0].source_cell = ((cells // nx) * nx + (nx - 1 - cells % nx)).astype(np.int32)
    m.cone_pos = sc.cone_pos.copy()
    m.cone_pos[:, 0] = L - sc.cone_pos[:, 0]
    m.cone_dir = oracle.wrap_angle(math.pi - sc.cone_dir)
    m.target_pos = sc.target_pos.copy()
    m.target_pos[:, 0] = L - sc.target_pos[:, 0]
    a = OracleSim(sc, lib_path=lib_path)
    b = OracleSim(m, noise_sign=-1.0, lib_path=lib_path)
    a.step(150)
    b.step(150)
    fa, fb = a.fields[0], b.fields[0][:, ::-1]
    assert np.abs(fa - fb).max() <= 1e-12 * np.abs(fa).max()
    ok = (a.flag_step < 0) & (b.flag_step < 0)
    assert ok.sum() > 30
    assert np.array_equal(a.status[ok], b.status[ok])
    assert np.array_equal(a.event_step[ok], b.event_step[ok])
    assert np.array_equal(a.target[ok], b.target[ok])
    assert np.abs(a.pos[ok, 0] - (L - b.pos[ok, 0])).max() < 1e-8
    assert np.abs(a.pos[ok, 1] - b.pos[ok, 1]).max() < 1e-8


# ---------------------------------------------------------------------------------------
# P12: Philox4x32-10 equals the independent implementation shipped with PyTorch
# (ATen/core/PhiloxRNGEngine.h, used as a black box: key = seed, counter = (offset,
# subsequence)); Box-Muller deviates have mean 0, variance 1 and pass a KS test.
# ---------------------------------------------------------------------------------------
_PX_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    at::Philox4_32 eng(strtoull(argv[a], 0, 0), strtoull(argv[a + 1], 0, 0),
                       strtoull(argv[a + 2], 0, 0));
    for (int i = 0; i < 4; ++i) printf("%u ", (unsigned)eng());
    printf("\n");
  }
}
"""


_PX_EXE = []


def _torch_philox_tool():
    if _PX_EXE and os.path.exists(_PX_EXE[0]):
        return _PX_EXE[0]
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    d = tempfile.mkdtemp(prefix="pxref")
    src = os.path.join(d, "px.cpp")
    exe = os.path.join(d, "px")
    with open(src, "w") as f:
        f.write(_PX_SRC)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, src, "-o", exe], check=True)
    _PX_EXE[:] = [exe]
    return exe


def pin_philox_vs_torch(lib_path=LIB, cases=None):
    rng = np.random.default_rng(0)
    if cases is None:
        cases = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1)]
        cases += [tuple(int(v) for v in rng.integers(0, 2 ** 63, 3, dtype=np.int64)) for _ in range(40)]
        cases += [(int(s), int(c), int(o)) for s, c, o in rng.integers(0, 2 ** 32, (20, 3), dtype=np.int64)]
    exe = _torch_philox_tool()
    args = [str(v) for c in cases for v in c]
    out = subprocess.run([exe] + args, check=True, capture_output=True, text=True).stdout.split("\n")
    lib = oracle.load(lib_path)
    for (seed, sub, off), line in zip(cases, out):
        want = [int(v) for v in line.split()]
        ctr = [off & 0xffffffff, off >> 32, sub & 0xffffffff, sub >> 32]
        key = [seed & 0xffffffff, seed >> 32]
        got = [int(v) for v in oracle.philox4x32_10(ctr, key, lib=lib)]
        assert got == want, ((seed, sub, off), got, want)


def pin_normal_statistics(lib_path=LIB, n_blocks=100_000):
    lib = oracle.load(lib_path)
    z = np.empty((n_blocks, 4))
    for i in range(n_blocks):
        z[i] = oracle.normals4(42, i, 7, 0, 0, lib=lib)
    flat = z.ravel()
    assert abs(flat.mean()) < 5.0 / math.sqrt(flat.size), flat.mean()
    assert abs(flat.var() - 1.0) < 5.0 * math.sqrt(2.0 / flat.size), flat.var()
    for col in range(4):
        ks = scipy.stats.kstest(z[:, col], "norm")
        assert ks.pvalue > 1e-4, (col, ks)
    # the two deviates of a pair are uncorrelated; neighbouring counters are uncorrelated
    bound = 5.0 / math.sqrt(n_blocks)
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < bound
    assert abs(np.corrcoef(z[:-1, 0], z[1:, 0])[0, 1]) < bound


# ---------------------------------------------------------------------------------------
# Reverse-mode gradient of the trajectory loss L = sum_i w_i |p_i^N - t_a(i)|^2 against
# central finite differences of the forward run (the definition of the derivative).  The
# derivative is taken along the forward run's branch, so a cone whose exit/contact record
# differs between the +h and -h runs is given weight 0 before comparing.
# ---------------------------------------------------------------------------------------
def _adjoint_case(n_species):
    species = ((1.0, 0.01, 1.0),) if n_species == 1 else ((1.0, 0.01, 1.0), (0.6, 0.02, -1.0))
    # dx != 1 so that every dx factor of the gradient is exercised
    return make_scenario("adjoint pin", 2, (40, 32), 0.5, 0.05, species, 3, (1.0, 4.0), 12, 6,
                         0.5, 0.25, 10.0, math.pi / 30.0, 0.1, seed=2)


def _perturbed(sc, kind, s, m, h):
    import copy
    out = copy.deepcopy(sc)
    spc = out.species[s]
    if kind == "q":
        spc.source_q = spc.source_q.copy()
        spc.source_q[m] += h
    elif kind == "D":
        spc.D += h
    else:
        spc.k += h
    return out


def pin_adjoint_fd(lib_path=LIB, n_species=1, steps=60):
    sc = _adjoint_case(n_species)
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]

    def forward(s2):
        o = OracleSim(s2, lib_path=lib_path).step(steps)
        d = o.pos - s2.target_pos[assign]
        return (d * d).sum(1), np.stack([o.status, o.target, o.event_step], 1)

    checks = []
    for s, spc in enumerate(sc.species):
        for m in range(len(spc.source_q)):
            checks.append(("q", s, m, 1e-5 * spc.source_q[m]))
        checks.append(("D", s, 0, 1e-6 * spc.D))
        checks.append(("k", s, 0, 1e-5 * spc.k))
    nq0 = len(sc.species[0].source_q)
    for kind, s, m, h in checks:
        (la, ea), (lb, eb) = forward(_perturbed(sc, kind, s, m, +h)), forward(_perturbed(sc, kind, s, m, -h))
        w = np.where((ea == eb).all(1), 1.0, 0.0)
        assert w.sum() >= M // 2, "too many event changes for a meaningful check"
        fd = float((w * (la - lb)).sum()) / (2.0 * h)
        _, dq, dD, dk = OracleSim(sc, lib_path=lib_path).adjoint(steps, assign, w)
        got = {"q": dq[(nq0 if s else 0) + m], "D": dD[s], "k": dk[s]}[kind]
        scale = max(abs(fd), 1e-3 * max(np.abs(dq).max(), np.abs(dD).max(), np.abs(dk).max()))
        assert abs(got - fd) <= 2e-5 * scale, (kind, s, m, got, fd)


def pin_adjoint_magnitude(lib_path=LIB):
    """The summand magnitudes the oracle reports with its gradient (the scale of the terms
    each component cancels, used as the GPU comparison's tolerance scale): at least the
    component's absolute value (triangle inequality), exactly homogeneous in the loss
    weights, and zero where the gradient has no terms at all (gain 0)."""
    sc = _adjoint_case(2)
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    w = np.linspace(0.5, 1.5, M)
    _, dq, dD, dk, mag = OracleSim(sc, lib_path=lib_path).adjoint(50, assign, w, magnitude=True)
    g = np.concatenate([dq, dD, dk])
    assert mag.shape == g.shape and np.all(mag >= np.abs(g) * (1 - 1e-12))
    assert np.all(mag > 0)
    _, _, _, _, mag2 = OracleSim(sc, lib_path=lib_path).adjoint(50, assign, 2.0 * w,
                                                                magnitude=True)
    assert np.allclose(mag2, 2.0 * mag, rtol=1e-12, atol=0.0)
    sc.turn_gain = 0.0
    _, _, _, _, mag0 = OracleSim(sc, lib_path=lib_path).adjoint(30, assign, w, magnitude=True)
    assert not mag0.any()


def pin_adjoint_no_coupling(lib_path=LIB):
    """With gain 0 the tips do not feel the field: every gradient is exactly zero, while
    the loss itself is the direct-guidance one."""
    sc = _adjoint_case(2)
    sc.turn_gain = 0.0
    M = sc.n_cones
    assign = np.arange(M) % sc.target_pos.shape[0]
    loss, dq, dD, dk = OracleSim(sc, lib_path=lib_path).adjoint(40, assign, np.ones(M))
    assert not dq.any() and not dD.any() and not dk.any()
    ref = OracleSim(sc, lib_path=lib_path).step(40)
    d = ref.pos - sc.target_pos[assign]
    assert abs(loss - float((d * d).sum())) <= 1e-12 * loss


# ---------------------------------------------------------------------------------------
# Connectivity (Sec. 3.4, Figs. 4-5): the adjacency list against its definition written out
# as Python lists, the breadth-first levels against scipy's unweighted shortest paths and a
# hand-built graph.
# ---------------------------------------------------------------------------------------
def pin_connectivity(lib_path=LIB):
    import scipy.sparse
    import scipy.sparse.csgraph
    lib = oracle.load(lib_path)
    # hand-built: edges 0->1, 0->3, 1->2, 2->0 (cycle), 3->3 (self loop), 4 isolated
    status = np.array([1, 1, 1, 1, 0, 1, 2], dtype=np.int32)
    target = np.array([0, 1, 2, 3, -1, 4, -1], dtype=np.int32)
    owner = np.array([0, 1, 2, 0, 4, 3, 4], dtype=np.int32)
    towner = np.array([1, 2, 0, 3, 3], dtype=np.int32)
    row, edges = oracle.connectivity(5, status, target, owner, towner, lib=lib)
    assert row.tolist() == [0, 2, 3, 4, 5, 5] and edges.tolist() == [1, 3, 2, 0, 3]
    assert oracle.bfs_levels(row, edges, 0, lib=lib).tolist() == [0, 1, 2, 1, -1]
    assert oracle.bfs_levels(row, edges, 2, lib=lib).tolist() == [1, 2, 0, 2, -1]
    rng = np.random.default_rng(5)
    for trial in range(20):
        N = int(rng.integers(1, 60))
        M = int(rng.integers(0, 400))
        T = int(rng.integers(1, 50))
        status = rng.integers(0, 3, M).astype(np.int32)
        target = np.where(status == 1, rng.integers(0, T, M), -1).astype(np.int32)
        owner = rng.integers(0, N, M).astype(np.int32)
        towner = rng.integers(0, N, T).astype(np.int32)
        row, edges = oracle.connectivity(N, status, target, owner, towner, lib=lib)
        lists = [[int(towner[target[i]]) for i in range(M) if status[i] == 1 and owner[i] == v]
                 for v in range(N)]
        assert row.tolist() == [0] + list(np.cumsum([len(x) for x in lists]))
        assert edges.tolist() == [u for x in lists for u in x]
        adj = scipy.sparse.csr_matrix((np.ones(len(edges)), edges, row), shape=(N, N))
        root = int(rng.integers(0, N))
        dist = scipy.sparse.csgraph.shortest_path(adj, directed=True, unweighted=True,
                                                  indices=root)
        want = np.where(np.isinf(dist), -1, dist).astype(np.int32)
        assert oracle.bfs_levels(row, edges, root, lib=lib).tolist() == want.tolist(), trial


# ---------------------------------------------------------------------------------------
# SNR turn law (Sec. 3.5, Eq. 5).  In a frozen linear field (D = k = 0, no sources) every
# cone placed at the same interior point with the same heading sees the same concentration
# c and gradient (G, 0), so SNR is a closed form and each cone turns right (by -max_turn)
# with probability Phi(SNR), independently (its own Philox stream).  Outside the detection
# window no cone turns.
# ---------------------------------------------------------------------------------------
def _snr_case(theta0, law, n_cones=20000, c0=0.4, G=0.02, x0=20.3, y0=15.6):
    sc = make_scenario("snr pin", 2, (48, 32), 1.0, 0.2, ((0.0, 0.0, 1.0),), 0, (1.0, 1.0),
                       n_cones, 0, 1.0, 0.1, 10.0, math.pi / 30.0, 0.0, seed=7)
    xs = (np.arange(sc.nx) + 0.5) * sc.dx
    field = np.tile(c0 + G * xs, (sc.ny, 1))
    sc.init_field = [np.asarray(field, dtype=np.float32).astype(np.float64)]
    sc.cone_pos = np.tile([x0, y0], (n_cones, 1)).astype(np.float64)
    sc.cone_dir = np.full(n_cones, theta0)
    sc.snr_law = law
    return sc, c0 + G * x0, G   # interpolation of a linear field is exact


def pin_snr_law(lib_path=LIB):
    law = (40.0, 1.5, 0.6, 0.05, 5.0)     # snr_scale, cone_width, kd, c_min, c_max
    A, w, kd, cmin, cmax = law
    for theta0 in (math.pi / 3, -math.pi / 4, 0.0, 2.5):
        sc, c, G = _snr_case(theta0, law)
        gamma = c / kd
        snr = A * (w / c) * math.sqrt(gamma / (1.0 + gamma) ** 3) * (math.sin(theta0) * G)
        o = OracleSim(sc, lib_path=lib_path).step(1)
        d = np.angle(np.exp(1j * (o.dir - theta0)))
        assert np.all(np.abs(np.abs(d) - sc.max_turn) < 1e-12), "every cone turns by the cap"
        right = float(np.mean(d < 0))
        p = float(scipy.stats.norm.cdf(snr))
        sd = math.sqrt(max(p * (1 - p), 1e-12) / sc.n_cones)
        assert abs(right - p) <= 5 * sd + 1e-9, (theta0, right, p, snr)
    # below the window: no turn at all
    sc, c, G = _snr_case(1.0, (40.0, 1.5, 0.6, 2.0, 5.0), n_cones=500)
    o = OracleSim(sc, lib_path=lib_path).step(3)
    assert np.all(np.abs(o.dir - 1.0) < 1e-12)


def pin_snr_bruteforce(lib_path=LIB):
    """The SNR law's whole step against the naive implementation (its deviates from
    PyTorch's Philox): angular noise included, two species, 30 steps."""
    import naive
    sc = make_scenario("snr brute force", 2, (8, 6), 1.0, 0.2,
                       ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), 3, (5.0, 20.0), 4, 3, 1.0, 0.2,
                       10.0, math.pi / 30.0, 0.3, seed=9)
    sc.snr_law = (30.0, 1.0, 2.0, 0.05, 50.0)
    a = OracleSim(sc, lib_path=lib_path).step(30)
    b = naive.NaiveSim(sc).step(30)
    assert np.abs(a.pos - np.array(b.pos)).max() <= 1e-10 * sc.side
    assert np.abs(np.angle(np.exp(1j * (a.dir - np.array(b.dir))))).max() <= 1e-10


def pin_bruteforce_3d(lib_path=LIB):
    """The whole 3D step against the naive implementation (deviates from PyTorch's
    Philox): two species, noise, 20 steps."""
    import naive
    sc = make_scenario("3d brute force", 3, (4, 5, 3), 1.0, 0.12,
                       ((1.0, 0.01, 1.0), (0.5, 0.02, -1.0)), 3, (5.0, 20.0), 3, 3, 1.0, 0.15,
                       10.0, math.pi / 30.0, 0.2, seed=5)
    a = OracleSim(sc, lib_path=lib_path).step(20)
    b = naive.NaiveSim(sc).step(20)
    assert np.abs(a.pos - np.array(b.pos)).max() <= 1e-10 * sc.side
    assert np.abs(a.dir - np.array(b.dir)).max() <= 1e-10


ALL_PINS = {
    "mass2d": lambda p: pin_mass_recursion(p, 2),
    "mass3d": lambda p: pin_mass_recursion(p, 3),
    "moments2d": lambda p: pin_moments(p, 2),
    "moments3d": lambda p: pin_moments(p, 3),
    "eigen2d": lambda p: pin_eigenmodes(p, 2),
    "eigen3d": lambda p: pin_eigenmodes(p, 3),
    "line": pin_line_source,
    "grad2d": lambda p: pin_gradient_quadratic(p, 2),
    "grad3d": lambda p: pin_gradient_quadratic(p, 3),
    "turn2d": pin_turn_rule_2d,
    "turn3d": pin_turn_rule_3d,
    "direct2d": lambda p: pin_direct_guidance(p, 2),
    "direct3d": lambda p: pin_direct_guidance(p, 3),
    "edges": pin_contact_edges,
    "noise": pin_noise_plumbing,
    "noise3d": pin_noise_3d,
    "philox": lambda p: pin_philox_vs_torch(p, cases=[(0, 0, 0), (12345, 7, 99), (2 ** 40 + 3, 2 ** 33 + 1, 2 ** 35 + 5)]),
    "normals": lambda p: pin_normal_statistics(p, 20_000),
    "adjoint": lambda p: pin_adjoint_fd(p, 1, 40),
    "adjoint2": lambda p: pin_adjoint_fd(p, 2, 40),
    "graph": pin_connectivity,
    "snr": pin_snr_law,
    "snr_noise": pin_snr_bruteforce,
    "bruteforce3d": pin_bruteforce_3d,
}
