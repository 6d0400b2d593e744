"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws initial states, box shapes and request traces.  It holds
none of the method's arithmetic (no forces, no integration, no binning):
both the GPU library and the CPU oracle receive exactly the arrays it
returns.

Workload recipe (the paper's benchmark fluids are uniform DPD solvents at
number density rho in periodic boxes, Sec. 5.1):
  - positions uniform on [0, L) per axis, placed on the FP32 grid of the
    box's largest edge (the spacing of FP32 numbers just below L_max), so a
    position survives storage in the GPU's fixed position grid unchanged;
  - velocities Maxwellian, N(0, kT/m) per component, with the centre-of-mass
    velocity removed (no rescale);
  - everything drawn in FP64 from numpy's PCG64 with an explicit seed, then
    rounded to FP32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def position_grid(cells) -> float:
    """Spacing of FP32 numbers at the largest box edge: 2**(floor(log2 L_max) - 23)."""
    lmax = int(max(int(c) for c in cells))
    return float(np.spacing(np.float32(lmax)))


def _positions_on_grid(rng, cells, n, grid):
    L = np.asarray(cells, dtype=np.float64)
    u = rng.random((n, 3))
    k = np.floor(u * (L / grid))                      # integer grid index in [0, L/grid)
    k = np.minimum(k, L / grid - 1.0)
    return (k * grid).astype(np.float32)


def _maxwell(rng, n, kT, mass):
    v = rng.normal(0.0, math.sqrt(kT / mass), size=(n, 3)) if kT > 0 else np.zeros((n, 3))
    if n > 0:
        v -= v.mean(axis=0, keepdims=True)
    return v.astype(np.float32)


def uniform_state(cells, n=None, density=None, kT=1.0, mass=1.0, seed=0, grid=None):
    """Uniform positions and Maxwellian velocities, FP32, rows in id order.
    Exactly one of n or density must be given; n = round(density * volume)."""
    cells = tuple(int(c) for c in cells)
    vol = cells[0] * cells[1] * cells[2]
    if n is None:
        n = int(round(density * vol))
    grid = position_grid(cells) if grid is None else grid
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = _positions_on_grid(rng, cells, n, grid)
    vel = _maxwell(rng, n, kT, mass)
    return pos, vel


def offgrid_state(cells, n, kT=1.0, mass=1.0, seed=0):
    """Uniform positions rounded to the nearest FP32 number (not to the
    position grid of the box: most coordinates below L_max / 2 have bits
    finer than it), each strictly inside [0, L), and Maxwellian velocities."""
    cells = tuple(int(c) for c in cells)
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(cells, dtype=np.float64)
    pos = (rng.random((n, 3)) * L).astype(np.float32)
    top = np.nextafter(L.astype(np.float32), np.float32(0.0))
    pos = np.minimum(pos, top[None, :])                 # FP32 rounding can reach L itself
    return pos, _maxwell(rng, n, kT, mass)


def clumped_state(cells, n, centre, radius=0.5, kT=1.0, mass=1.0, seed=0, grid=None):
    """n particles packed into a small ball (cells of 40+ particles): the stress
    case for per-cell capacity and work balance."""
    cells = tuple(int(c) for c in cells)
    grid = position_grid(cells) if grid is None else grid
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True) + 1e-300
    rad = radius * rng.random(n) ** (1.0 / 3.0)
    x = np.asarray(centre, dtype=np.float64) + d * rad[:, None]
    L = np.asarray(cells, dtype=np.float64)
    x = np.mod(x, L)
    k = np.minimum(np.floor(x / grid), L / grid - 1.0)
    pos = (k * grid).astype(np.float32)
    return pos, _maxwell(rng, n, kT, mass)


def face_state(cells, n, kT=1.0, mass=1.0, seed=0, grid=None):
    """Uniform state in which about a third of the coordinates sit exactly on a
    cell face (integer values, including 0) and a few sit at L - grid, the
    largest coordinate inside the box."""
    cells = tuple(int(c) for c in cells)
    grid = position_grid(cells) if grid is None else grid
    pos, vel = uniform_state(cells, n=n, kT=kT, mass=mass, seed=seed, grid=grid)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    p = pos.astype(np.float64)
    mask = rng.random(p.shape) < 1.0 / 3.0
    p[mask] = np.floor(p[mask])
    top = rng.random(p.shape) < 0.02
    L = np.broadcast_to(np.asarray(cells, dtype=np.float64), p.shape)
    p[top] = L[top] - grid
    return p.astype(np.float32), vel


def species_types(n, fractions, seed=0):
    """Species of n particles (id order), drawn independently with the given
    probabilities (normalised), as int32."""
    f = np.asarray(fractions, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    return rng.choice(len(f), size=int(n), p=f / f.sum()).astype(np.int32)


# Two fluids of different viscosity in one domain (the plasma / cytoplasm
# pair of Sec. 5.2-5.3, cytoplasm five times more viscous): the same
# conservative a = 25 for every pair, gamma 4.5 within the solvent, 22.5
# within the second fluid and 0 across, where only the conservative part
# acts (the cross-membrane rule of Sec. 2.3).  Half the particles of each.
MIXTURE_TABLES = {
    "a": [[25.0, 25.0], [25.0, 25.0]],
    "gamma": [[4.5, 0.0], [0.0, 22.5]],
    "fractions": [0.5, 0.5],
}


# ---------------------------------------------------------------------------
# The workloads (uniform DPD solvents; Sec. 5.1 uses L = 64, rho = 8 per GPU)
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    cells: tuple
    density: float
    a: float
    gamma: float
    kT: float
    dt: float
    steps: int
    seed: int
    body_f: float = 0.0
    profile_bins: int = 0
    mass: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(round(self.density * self.cells[0] * self.cells[1] * self.cells[2]))


WORKLOADS = {
    # small parity case: 8^3 cells, rho = 3, 1 536 particles, 100 steps
    "cube8_rho3": Workload("cube8_rho3", (8, 8, 8), 3.0, 25.0, 4.5, 1.0, 0.01, 100, 0),
    # single box 48^3, rho = 3, 331 776 particles, 1 000 steps
    "cube48_rho3": Workload("cube48_rho3", (48, 48, 48), 3.0, 25.0, 4.5, 1.0, 0.01, 1000, 1),
    # one GPU's share of a large periodic-Poiseuille run: 192 x 96 x 96, rho = 8,
    # 14 155 776 particles, reverse-Poiseuille body force 0.05 along x, gradient y
    "pp192x96x96_rho8": Workload("pp192x96x96_rho8", (192, 96, 96), 8.0, 10.0, 10.0, 1.0, 0.005,
                                 2000, 2, body_f=0.05, profile_bins=96),
}


def batch_boxes(nboxes=64, lo=8, hi=32, density=3.0, rng_seed=4):
    """Edges drawn log-uniform in [lo, hi] per axis and rounded to integers;
    particle count round(density * volume); per-box seed 1000 + b."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    e = np.exp(rng.uniform(math.log(lo), math.log(hi), size=(nboxes, 3)))
    edges = np.clip(np.rint(e).astype(int), 3, None)
    out = []
    for b in range(nboxes):
        c = tuple(int(x) for x in edges[b])
        out.append({"cells": c, "n": int(round(density * c[0] * c[1] * c[2])), "seed": 1000 + b})
    return out


def request_trace(nreq=1000, rate=200.0, lo=8, hi=48, rng_seed=5, steps=500):
    """Poisson arrivals (exponential gaps of mean 1/rate seconds), edges
    log-uniform in [lo, hi], density 3 or 8 with probability 1/2, body force
    amplitude uniform in [0, 0.1], per-request seed 100000 + r."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    gaps = rng.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    e = np.clip(np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=(nreq, 3)))).astype(int), 3, None)
    dens = np.where(rng.random(nreq) < 0.5, 3.0, 8.0)
    fb = rng.uniform(0.0, 0.1, size=nreq)
    reqs = []
    for r in range(nreq):
        c = tuple(int(x) for x in e[r])
        rho = float(dens[r])
        # the trace names no a, gamma: the rho = 3 and rho = 8 fluids of the
        # other workloads are reused (a = 25, gamma = 4.5 and a = 10, gamma = 10)
        a, g = (25.0, 4.5) if rho == 3.0 else (10.0, 10.0)
        reqs.append({"t_arrival": float(t[r]), "cells": c, "density": rho,
                     "n": int(round(rho * c[0] * c[1] * c[2])), "a": a, "gamma": g, "kT": 1.0,
                     "dt": 0.01, "body_f": float(fb[r]), "steps": int(steps), "seed": 100000 + r})
    return reqs
