"""Seeded synthetic workloads shared by the oracle-side tests and the GPU path.

This module only *describes* problems: grid sizes, physical parameters, body point
sets and initial fields drawn from ``numpy.random.default_rng``.  It holds none of
the method's arithmetic (no operators, no solves, no structural updates), so both
the CPU oracle and the HIP library can be fed from it without sharing code.

The paper's own problems (flapping plates, NACA0012 with flap, tandem airfoils)
need geometry and reference data that are not available; these synthetic setups
stand in for them with the same kinds of bodies (rigid, torsionally hinged,
deformable), the same grid hierarchy (nested levels that double in extent) and the
same body-point spacing rules (Sec. 5: body spacing twice the finest grid spacing
for the plates; a cylinder sampled at about the grid spacing).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Flow:
    n: int               # cells per side of every level
    levels: int          # number of nested levels (level 0 is the finest)
    h: float             # finest grid spacing
    dt: float
    re: float
    cx: float = 0.0      # common centre of all levels
    cy: float = 0.0
    u_inf: tuple = (1.0, 0.0)


@dataclasses.dataclass
class Rigid:
    xy: np.ndarray                      # (n, 2) body point positions
    ds: float                           # body point spacing (arc length per point)
    u_b: Optional[np.ndarray] = None    # (n, 2) prescribed velocity, None = stationary


@dataclasses.dataclass
class Torsional:
    n: int                # number of points, j = 0 .. n-1, j = 0 at the hinge
    hinge: tuple
    length: float
    theta0: float         # undeformed angle from the x axis (radians)
    inertia: float
    stiffness: float
    damping: float
    theta: float = 0.0    # initial deflection from theta0
    phi: float = 0.0      # initial angular velocity

    @property
    def ds(self) -> float:
        return self.length / (self.n - 1)


@dataclasses.dataclass
class Deformable:
    xy_ref: np.ndarray    # (n, 2) stress-free straight configuration, node 0 clamped
    mass: float           # mass per unit length (mass ratio with rho_f = 1, L = 1)
    ei: float             # bending stiffness
    ea: float             # stretching stiffness
    xy0: np.ndarray       # (n, 2) initial node positions
    rot0: np.ndarray      # (n,) initial node rotations relative to the reference

    @property
    def ds(self) -> float:
        d = np.diff(self.xy_ref, axis=0)
        return float(np.hypot(d[:, 0], d[:, 1]).mean())


@dataclasses.dataclass
class Problem:
    name: str
    flow: Flow
    bodies: list
    subdomain: Optional[tuple] = None          # (x0, x1, y0, y1) or None = exact operators
    vorticity0: Optional[List[np.ndarray]] = None  # per level, (n-1, n-1) interior omega
    steps: int = 1


def cylinder(center, diameter, h):
    """Points on a circle at angle 2*pi*j/n with spacing close to h."""
    n = int(round(math.pi * diameter / h))
    ang = 2.0 * math.pi * np.arange(n) / n
    xy = np.stack([center[0] + 0.5 * diameter * np.cos(ang),
                   center[1] + 0.5 * diameter * np.sin(ang)], axis=1)
    return Rigid(xy=xy, ds=math.pi * diameter / n)


def cylinder_problem(n=128, seed=1, steps=50, noise=1e-3):
    """Stationary rigid cylinder (D = 1) on one 2.56 x 2.56 level, Re = 100.

    At n = 128: h = 0.02, dt = 0.004, 157 body points (ds ~ h), seeded
    N(0, noise) vorticity on the interior vertices.
    """
    width = 2.56
    h = width / n
    flow = Flow(n=n, levels=1, h=h, dt=0.2 * h, re=100.0, cx=0.0, cy=0.0)
    rng = np.random.default_rng(seed)
    w0 = [rng.normal(0.0, noise, size=(n - 1, n - 1))]
    return Problem("cylinder", flow, [cylinder((0.0, 0.0), 1.0, h)], None, w0, steps)


def plate_problem(n=512, levels=3, seed=2, steps=400, subdomain=True):
    """Torsionally hinged flat plate (L = 1, ds = 2h) at 20 degrees attack, Re = 200.

    Finest level 5.12 x 5.12 centred at (0.5, 0); at n = 512: h = 0.01 and 51 points.
    """
    width = 5.12
    h = width / n
    flow = Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=200.0, cx=0.5, cy=0.0)
    npts = int(round(1.0 / (2.0 * h))) + 1
    body = Torsional(n=npts, hinge=(0.0, 0.0), length=1.0, theta0=-math.radians(20.0),
                     inertia=5.0, stiffness=1.0, damping=0.1)
    sd = (-0.05, 1.05, -1.05, 1.05) if subdomain else None
    return Problem("plate", flow, [body], sd, None, steps)


def flag_problem(n=1024, levels=4, seed=3, steps=1000, subdomain=True):
    """Deformable flag clamped at (0, 0) along +x (L = 1, ds = 2h), Re = 500.

    Mass ratio 0.2, bending stiffness 1e-3, stretching stiffness 1e3; seeded initial
    deflection w(s) = a (s/L)^2 with a ~ U[0.05, 0.1], nodes placed at equal arc
    length along that curve, at rest.
    """
    width = 5.12
    h = width / n
    flow = Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=500.0, cx=0.5, cy=0.0)
    npts = int(round(1.0 / (2.0 * h))) + 1
    rng = np.random.default_rng(seed)
    a = float(rng.uniform(0.05, 0.1))
    ds = 1.0 / (npts - 1)
    xy_ref = np.stack([np.arange(npts) * ds, np.zeros(npts)], axis=1)
    # equal arc length along y = a x^2 (fine tabulation of the arc length)
    xs = np.linspace(0.0, 1.2, 240001)
    seg = np.hypot(np.diff(xs), np.diff(a * xs * xs))
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    sx = np.interp(np.arange(npts) * ds, arc, xs)
    xy0 = np.stack([sx, a * sx * sx], axis=1)
    rot0 = np.arctan(2.0 * a * sx)
    body = Deformable(xy_ref=xy_ref, mass=0.2, ei=1e-3, ea=1e3, xy0=xy0, rot0=rot0)
    sd = (-0.02, 1.02, -0.6, 0.6) if subdomain else None
    return Problem("flag", flow, [body], sd, None, steps)


def batch_problems(count=64, seed=4, steps=200, sizes=(128, 256, 384, 512, 768)):
    """Independent instances: seeded grid size, level count, Re and 1-3 bodies each.

    Bodies are rigid circles (D ~ U[0.3, 0.8]) or torsional plates (L ~ U[0.3, 0.8],
    theta0 ~ U[-30, 30] degrees, inertia 5, stiffness 1, damping 0.1) placed without
    overlap in [-1.2, 1.2]^2 on a finest level of side 4.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(1000 * seed + i)
        n = int(rng.choice(sizes))
        levels = int(rng.integers(1, 4))
        re = float(rng.uniform(50.0, 400.0))
        h = 4.0 / n
        flow = Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=re)
        nb = int(rng.integers(1, 4))
        bodies, boxes = [], []
        tries = 0
        while len(bodies) < nb and tries < 200:
            tries += 1
            size = float(rng.uniform(0.3, 0.8))
            c = rng.uniform(-1.2 + size / 2, 1.2 - size / 2, size=2)
            box = (c[0] - size / 2 - 4 * h, c[0] + size / 2 + 4 * h,
                   c[1] - size / 2 - 4 * h, c[1] + size / 2 + 4 * h)
            if any(not (box[1] < b[0] or b[1] < box[0] or box[3] < b[2] or b[3] < box[2])
                   for b in boxes):
                continue
            boxes.append(box)
            if rng.uniform() < 0.5:
                bodies.append(cylinder((float(c[0]), float(c[1])), size, h))
            else:
                npts = int(round(size / (2.0 * h))) + 1
                th0 = math.radians(float(rng.uniform(-30.0, 30.0)))
                hinge = (float(c[0] - 0.5 * size * math.cos(th0)),
                         float(c[1] - 0.5 * size * math.sin(th0)))
                bodies.append(Torsional(n=npts, hinge=hinge, length=size, theta0=th0,
                                        inertia=5.0, stiffness=1.0, damping=0.1))
        # sub-domain: bounding box of all bodies' reach, when any body moves
        sd = None
        if any(isinstance(b, Torsional) for b in bodies):
            sd = (-1.3, 1.3, -1.3, 1.3)
        out.append(Problem(f"batch{i}", flow, bodies, sd, None, steps))
    return out
