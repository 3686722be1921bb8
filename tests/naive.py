"""A second, deliberately naive implementation of the simulation step, for tiny cases.

Pure Python over scalars (the ``math`` module and nested loops; no numpy arithmetic), written
independently of the C oracle from the same rules, so that the two can pin each other: a
mistake in either (a dropped term, a wrong index or sign, a swapped operand) shows as a
disagreement far above FP64 rounding.  The Gaussian deviates come from PyTorch's own
Philox4x32-10 engine used as a black box, not from the oracle's generator.

Rules, per step n -> n + 1 (paper Sec. 3.4-3.5 for the cone rules; the field rules are the
explicit finite-difference diffusion with first-order decay and point sources):

* field: c' = c + r * sum over axes (c[+] + c[-] - 2c) - k dt c, r = D dt / dx^2, a
  neighbour outside the grid replaced by the cell itself; then each source adds q / dx^dim;
* gradient: central differences at cell centres (same wall rule), interpolated
  multilinearly at u = p / dx - 1/2 (clamped), summed over species with their signs;
* turn: toward h + gain * g by at most max_turn (2D: atan2 of cross and 1 + dot; 3D: in
  the plane of h and g);
* noise: Box-Muller deviates from Philox(key = seed); 3D: counter (cone, n, 0, sim), rotate h
  about the tangent-plane vector sigma * (z - (z.h) h) and renormalise; 2D: counter
  (cone, n // 2, 0, sim), the block's first pair for even n and second for odd n, sigma
  times the pair's first deviate added to the angle, wrapped to [-pi, pi);
* advance by step_len along h; exit (outside [0, n dx) on any axis) before contact; contact
  when the squared distance to a target is strictly below R^2, nearest (lowest index on a
  tie) wins.
"""
from __future__ import annotations

import math
import subprocess

import pins


def philox_words(seed: int, counters):
    """Philox4x32-10 outputs for counters (c0, c1, c2, c3) under key = seed, from PyTorch's
    engine: offset = c0 + 2^32 c1, subsequence = c2 + 2^32 c3."""
    exe = pins._torch_philox_tool()
    args = []
    for c0, c1, c2, c3 in counters:
        args += [str(seed), str(c2 | (c3 << 32)), str(c0 | (c1 << 32))]
    out = subprocess.run([exe] + args, check=True, capture_output=True, text=True).stdout
    return [tuple(int(v) for v in line.split()) for line in out.strip().split("\n")]


def _uniform(x: int) -> float:
    # top 23 bits of the word, centred in their interval: ((x >> 9) + 1/2) / 2^23
    return ((x >> 9) + 0.5) / 8388608.0


def _deviates(words):
    u = [_uniform(w) for w in words]
    r0 = math.sqrt(-2.0 * math.log(u[0]))
    r1 = math.sqrt(-2.0 * math.log(u[2]))
    return (r0 * math.cos(2.0 * math.pi * u[1]), r0 * math.sin(2.0 * math.pi * u[1]),
            r1 * math.cos(2.0 * math.pi * u[3]), r1 * math.sin(2.0 * math.pi * u[3]))


class NaiveSim:
    def __init__(self, sc):
        self.sc = sc
        self.dim = sc.dim
        self.n = [sc.nx, sc.ny] + ([sc.nz] if sc.dim == 3 else [])
        cells = 1
        for v in self.n:
            cells *= v
        self.fields = []
        for s in range(len(sc.species)):
            if sc.init_field is not None and sc.init_field[s] is not None:
                self.fields.append([float(v) for v in list(sc.init_field[s].ravel())])
            else:
                self.fields.append([0.0] * cells)
        M = sc.n_cones
        self.pos = [[float(sc.cone_pos[i][a]) for a in range(sc.dim)] for i in range(M)]
        if sc.dim == 2:
            self.dir = [float(sc.cone_dir[i]) for i in range(M)]
        else:
            self.dir = [[float(sc.cone_dir[i][a]) for a in range(3)] for i in range(M)]
        self.status = [0] * M
        self.target = [-1] * M
        self.event_step = [-1] * M
        self.step_count = 0

    # linear index, x fastest
    def _lin(self, idx):
        if self.dim == 2:
            return idx[1] * self.n[0] + idx[0]
        return (idx[2] * self.n[1] + idx[1]) * self.n[0] + idx[0]

    def _value(self, c, idx, axis, offset):
        j = list(idx)
        j[axis] += offset
        if j[axis] < 0 or j[axis] >= self.n[axis]:
            j = list(idx)
        return c[self._lin(j)]

    def _cells(self):
        if self.dim == 2:
            for y in range(self.n[1]):
                for x in range(self.n[0]):
                    yield (x, y)
        else:
            for z in range(self.n[2]):
                for y in range(self.n[1]):
                    for x in range(self.n[0]):
                        yield (x, y, z)

    def _field_step(self):
        sc = self.sc
        for s, spc in enumerate(sc.species):
            c = self.fields[s]
            r = spc.D * sc.dt / (sc.dx * sc.dx)
            new = [0.0] * len(c)
            for idx in self._cells():
                here = c[self._lin(idx)]
                lap = 0.0
                for a in range(self.dim):
                    lap += self._value(c, idx, a, +1) + self._value(c, idx, a, -1) - 2.0 * here
                new[self._lin(idx)] = here + r * lap - spc.k * sc.dt * here
            vol = sc.dx ** self.dim
            for cell, q in zip(spc.source_cell, spc.source_q):
                new[int(cell)] += float(q) / vol
            self.fields[s] = new

    def _gradient(self, c, p):
        sc = self.sc
        base, frac = [], []
        for a in range(self.dim):
            u = min(max(p[a] / sc.dx - 0.5, 0.0), float(self.n[a] - 1))
            i0 = min(int(math.floor(u)), self.n[a] - 2)
            base.append(i0)
            frac.append(u - i0)
        g = [0.0] * self.dim
        for corner in range(2 ** self.dim):
            idx, w = [], 1.0
            for a in range(self.dim):
                up = (corner >> a) & 1
                idx.append(base[a] + up)
                w *= frac[a] if up else 1.0 - frac[a]
            for a in range(self.dim):
                d = (self._value(c, idx, a, +1) - self._value(c, idx, a, -1)) / (2.0 * sc.dx)
                g[a] += w * d
        return g

    def _value_at(self, c, p):
        """Multilinear interpolation of cell-centre values at p (same corners as _gradient)."""
        base, frac = [], []
        for a in range(self.dim):
            u = min(max(p[a] / self.sc.dx - 0.5, 0.0), float(self.n[a] - 1))
            i0 = min(int(math.floor(u)), self.n[a] - 2)
            base.append(i0)
            frac.append(u - i0)
        v = 0.0
        for corner in range(2 ** self.dim):
            idx, w = [], 1.0
            for a in range(self.dim):
                up = (corner >> a) & 1
                idx.append(base[a] + up)
                w *= frac[a] if up else 1.0 - frac[a]
            v += w * c[self._lin(idx)]
        return v

    def step(self, n_steps: int = 1):
        sc = self.sc
        for _ in range(n_steps):
            self._field_step()
            active = [i for i in range(sc.n_cones) if self.status[i] == 0]
            n = self.step_count
            if not active:
                self.step_count += 1
                continue
            if self.dim == 2:
                # one block per two steps: the first Box-Muller pair for even n, the second
                # for odd n
                words = philox_words(sc.seed, [(i, n // 2, 0, sc.sim_index) for i in active])
                zs = [_deviates(wd)[2 * (n % 2):2 * (n % 2) + 2] for wd in words]
            else:
                words = philox_words(sc.seed, [(i, n, 0, sc.sim_index) for i in active])
                zs = [_deviates(wd) for wd in words]
            for i, z in zip(active, zs):
                self._cone(i, z)
            self.step_count += 1
        return self

    def _cone(self, i, z):
        sc = self.sc
        p = self.pos[i]
        g = [0.0] * self.dim
        for s, spc in enumerate(sc.species):
            gs = self._gradient(self.fields[s], p)
            for a in range(self.dim):
                g[a] += spc.sign * gs[a]
        if self.dim == 2 and getattr(sc, "snr_law", None) is not None:
            # Sec. 3.5, Eq. 5: turn right when N(SNR, 1) > 0, inside the detection window
            A, width, kd, cmin, cmax = sc.snr_law
            th = self.dir[i]
            c = self._value_at(self.fields[0], p)
            if cmin <= c <= cmax and (g[0] != 0.0 or g[1] != 0.0):
                theta_g = math.atan2(g[1], g[0])
                mu = width * math.hypot(g[0], g[1]) / c
                gamma = c / kd
                snr = A * mu * math.sqrt(gamma / (1.0 + gamma) ** 3) * math.sin(th - theta_g)
                th = th - sc.max_turn if snr + z[0] > 0.0 else th + sc.max_turn
            th = th + sc.noise_sigma * z[1]
            th = th - 2.0 * math.pi * math.floor((th + math.pi) / (2.0 * math.pi))
            self.dir[i] = th
            h = [math.cos(th), math.sin(th)]
        elif self.dim == 2:
            th = self.dir[i]
            hx, hy = math.cos(th), math.sin(th)
            cross = sc.turn_gain * (hx * g[1] - hy * g[0])
            if cross == 0.0:
                cross = 0.0
            turn = math.atan2(cross, 1.0 + sc.turn_gain * (hx * g[0] + hy * g[1]))
            turn = max(-sc.max_turn, min(sc.max_turn, turn))
            th = th + turn + sc.noise_sigma * z[0]
            th = th - 2.0 * math.pi * math.floor((th + math.pi) / (2.0 * math.pi))
            self.dir[i] = th
            h = [math.cos(th), math.sin(th)]
        else:
            h = list(self.dir[i])
            gh = sum(g[a] * h[a] for a in range(3))
            perp = [g[a] - gh * h[a] for a in range(3)]
            pn = math.sqrt(sum(v * v for v in perp))
            if pn > 0.0:
                phi = min(math.atan2(sc.turn_gain * pn, 1.0 + sc.turn_gain * gh), sc.max_turn)
                h = [math.cos(phi) * h[a] + math.sin(phi) * perp[a] / pn for a in range(3)]
            zh = sum(z[a] * h[a] for a in range(3))
            w = [sc.noise_sigma * (z[a] - zh * h[a]) for a in range(3)]
            wn = math.sqrt(sum(v * v for v in w))
            if wn > 0.0:
                h = [math.cos(wn) * h[a] + math.sin(wn) * w[a] / wn for a in range(3)]
            hn = math.sqrt(sum(v * v for v in h))
            h = [v / hn for v in h]
            self.dir[i] = h
        for a in range(self.dim):
            p[a] += sc.step_len * h[a]
        if any(p[a] < 0.0 or p[a] >= self.n[a] * sc.dx for a in range(self.dim)):
            self.status[i], self.event_step[i] = 2, self.step_count + 1
            return
        best, best_d2 = -1, math.inf
        for j, t in enumerate(sc.target_pos):
            d2 = sum((p[a] - float(t[a])) ** 2 for a in range(self.dim))
            if d2 < best_d2:
                best, best_d2 = j, d2
        if best >= 0 and best_d2 < sc.contact_radius ** 2:
            self.status[i], self.target[i], self.event_step[i] = 1, best, self.step_count + 1
