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
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Flow:
    n: int               # cells along x of every level (and along y unless ny is set)
    levels: int          # number of nested levels (level 0 is the finest)
    h: float             # finest grid spacing
    dt: float
    re: float
    cx: float = 0.0      # common centre of all levels
    cy: float = 0.0
    u_inf: tuple = (1.0, 0.0)
    delta: str = "roma3"  # discrete delta kernel: "roma3" (3-point) or "peskin4" (4-point)
    ny: int = 0          # cells along y of every level; 0: ny = n (square levels)

    @property
    def nx_ny(self):
        return self.n, (self.ny if self.ny else self.n)


@dataclasses.dataclass
class Rigid:
    xy: np.ndarray                      # (n, 2) body point positions
    ds: float                           # body point spacing (arc length per point)
    u_b: Optional[np.ndarray] = None    # (n, 2) prescribed velocity, None = stationary


@dataclasses.dataclass
class MovingRigid:
    """Rigid body with prescribed motion: points xy_ref in the body frame, and
    motion(t) -> (x, y, angle, vx, vy, omega), the pose of the body frame at time t and
    its rates (an input of the problem).  accel(t) -> (ax, ay, alpha_dd), the frame's
    accelerations, is needed only when a MountedTorsional body rides on it."""
    xy_ref: np.ndarray                  # (n, 2) body-frame point coordinates
    ds: float
    motion: Callable[[float], tuple]
    accel: Optional[Callable[[float], tuple]] = None

    def pose(self, t):
        return tuple(float(v) for v in self.motion(t))

    def accelerations(self, t):
        if self.accel is None:
            raise ValueError("this driver has no accelerations")
        return tuple(float(v) for v in self.accel(t))


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
class MountedTorsional:
    """A torsional body whose hinge rides on a rigid body in prescribed motion (Sec. 5.1: the
    passive plate hinged to the driven plate).  The hinge sits at `hinge_body` in the
    driver's body frame; at zero deflection the plate points at the driver's angle plus
    `theta_rel`.  inertia is about the hinge; mass and cg (hinge to centre of mass, along the
    plate) give the pseudo-moments of the hinge's acceleration.  driver: index of the
    MovingRigid in the problem's body list."""
    driver: int
    n: int
    hinge_body: tuple
    theta_rel: float
    length: float
    inertia: float
    stiffness: float
    damping: float
    mass: float
    cg: float
    theta: float = 0.0
    phi: float = 0.0

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
    subdomain: Optional[object] = None         # (x0, x1, y0, y1), a list of such rectangles,
                                               # or None = exact operators
    vorticity0: Optional[List[np.ndarray]] = None  # per level, (ny-1, nx-1) interior omega
    steps: int = 1


def flapping_motion(a0=1.4, beta=math.pi / 4, sigma_t=0.628, sigma_r=0.628, freq=1.0,
                    center=(0.0, 0.0)):
    """Driven-plate kinematics of Sec. 5.1 (lengths in chords, time in 1/freq units):
    X(t) = (A0/2) G_t(ft)/max G_t C(ft), Y = 0, alpha(t) = -beta G_r(ft)/max G_r, with
    G_t(t) = int_0^t tanh(sigma_t cos 2 pi t') dt', G_r(t) = tanh(sigma_r cos 2 pi t) and the
    start-up conditioner C(t) = (tanh(8t - 2) + tanh 2)/(1 + tanh 2).  Returns
    motion(t) -> (x, y, angle, vx, vy, omega) with the rates in closed form (G_t by
    Gauss-Legendre quadrature; max G_t = G_t(1/4), max G_r = tanh sigma_r)."""
    xg, wg = np.polynomial.legendre.leggauss(48)

    def g_t(t):
        # integrate over whole quarter periods and the remainder, 48 points each
        q = math.floor(4.0 * t)
        total = 0.0
        for a, b in [(k / 4.0, (k + 1) / 4.0) for k in range(int(q))] + [(q / 4.0, t)]:
            if b <= a:
                continue
            u = 0.5 * (b - a) * xg + 0.5 * (b + a)
            total += 0.5 * (b - a) * float(np.sum(wg * np.tanh(sigma_t * np.cos(2 * math.pi * u))))
        return total

    gt_max = g_t(0.25)
    gr_max = math.tanh(sigma_r)
    th2 = math.tanh(2.0)

    def motion(t):
        ft = freq * t
        cnd = (math.tanh(8.0 * ft - 2.0) + th2) / (1.0 + th2)
        dcnd = 8.0 * freq * (1.0 - math.tanh(8.0 * ft - 2.0) ** 2) / (1.0 + th2)
        gt = g_t(ft) if ft >= 0 else -g_t(-ft)
        dgt = freq * math.tanh(sigma_t * math.cos(2 * math.pi * ft))
        x = 0.5 * a0 * gt / gt_max * cnd
        vx = 0.5 * a0 / gt_max * (dgt * cnd + gt * dcnd)
        gr = math.tanh(sigma_r * math.cos(2 * math.pi * ft))
        dgr = (1.0 - gr * gr) * sigma_r * (-2 * math.pi * freq * math.sin(2 * math.pi * ft))
        ang = -beta * gr / gr_max
        om = -beta * dgr / gr_max
        return (center[0] + x, center[1], ang, vx, 0.0, om)

    def accel(t):
        ft = freq * t
        w = 2 * math.pi * freq
        tc = math.tanh(8.0 * ft - 2.0)
        cnd = (tc + th2) / (1.0 + th2)
        dcnd = 8.0 * freq * (1.0 - tc * tc) / (1.0 + th2)
        ddcnd = -2.0 * tc * 8.0 * freq * dcnd
        gt = g_t(ft) if ft >= 0 else -g_t(-ft)
        tt = math.tanh(sigma_t * math.cos(w * t))
        dgt = freq * tt
        ddgt = freq * (1.0 - tt * tt) * sigma_t * (-w * math.sin(w * t))
        ax = 0.5 * a0 / gt_max * (ddgt * cnd + 2.0 * dgt * dcnd + gt * ddcnd)
        gr = math.tanh(sigma_r * math.cos(w * t))
        u = sigma_r * (-w * math.sin(w * t))           # d/dt of the argument
        du = sigma_r * (-w * w * math.cos(w * t))
        dgr = (1.0 - gr * gr) * u
        ddgr = -2.0 * gr * dgr * u + (1.0 - gr * gr) * du
        return (ax, 0.0, -beta * ddgr / gr_max)

    motion.accel = accel
    return motion


def driven_plate_problem(n=256, levels=2, steps=50, case=2, subdomain=True):
    """A flat plate of chord 1.05 (its centre at the origin) driven by the Sec. 5.1
    flapping kinematics (Table kineparams case 1 or 2, f = 1) in fluid at rest; ds = 2h.
    Re = f c^2 / nu from the rotational Reynolds number 100 of the table.  Finest level
    6.4 x 6.4; sub-domain [-1.95, 1.95] x [-0.85, 0.85] holds every plate position."""
    sigma = 3.770 if case == 1 else 0.628
    beta = math.pi / 4
    re = 100.0 * math.tanh(sigma) / (2 * math.pi * beta * sigma)
    width = 6.4
    h = width / n
    flow = Flow(n=n, levels=levels, h=h, dt=0.05 * h, re=re, cx=0.0, cy=0.0, u_inf=(0.0, 0.0))
    chord = 1.05
    npts = int(round(chord / (2.0 * h))) + 1
    xs = np.linspace(-0.5 * chord, 0.5 * chord, npts)
    body = MovingRigid(xy_ref=np.stack([xs, np.zeros(npts)], axis=1), ds=chord / (npts - 1),
                       motion=flapping_motion(sigma_t=sigma, sigma_r=sigma))
    sd = (-1.95, 1.95, -0.85, 0.85) if subdomain else None
    return Problem("driven_plate", flow, [body], sd, None, steps)


def two_plate_problem(n=256, levels=2, steps=50, case=2, subdomain=True, dt_scale=0.11):
    """Sec. 5.1's flapping of two torsionally connected plates: a driven plate (chord 1.05,
    centre of mass 0.55 above the hinge) in the Table kineparams motion, and a passive plate
    of chord 1.05 hinged at its lower end.  At zero angles both hang along -y (the driver's
    body frame points along -y; the paper's angles are measured from that direction, which
    its coefficient cos(alpha_1 + theta) of the hinge acceleration implies).  Spring
    K = 456, damper C = 3.95, inertia about the hinge 0.2886 (f = c = rho_f = 1); the
    passive plate's mass pi/4 and its centre-of-mass distance 0.55 are those of the 5:1
    ellipse of density ratio 5 that the paper's inertia stands for (m ((c/2)^2 + (c/10)^2)/4
    + m 0.55^2 = 0.2886).  Finest level 6.3 x 6.3 centred at (0, -1.5); sub-domain
    [-1.89, 1.89] x [-1.66, 0.65]; ds = 2h.  Time step dt = dt_scale (h/c) tau_r with the
    rotational time tau_r = c / U_r, U_r = 2 pi beta sigma_r f c / tanh sigma_r (the scale of
    Re_r): the paper's grid study keeps dt / tau_r = 0.466 dx / c; on the coarser grids used
    here the explicit advection needs about a quarter of that."""
    sigma = 3.770 if case == 1 else 0.628
    beta = math.pi / 4
    re = 100.0 * math.tanh(sigma) / (2 * math.pi * beta * sigma)
    tau_r = math.tanh(sigma) / (2 * math.pi * beta * sigma)
    width = 6.3
    h = width / n
    flow = Flow(n=n, levels=levels, h=h, dt=dt_scale * h * tau_r, re=re, cx=0.0, cy=-1.5,
                u_inf=(0.0, 0.0))
    chord = 1.05
    npts = int(round(chord / (2.0 * h))) + 1
    # the hinge point belongs to the passive plate (its point 0), so the driver stops one
    # spacing above it (coincident points would make the Schur matrix singular)
    ys = np.linspace(0.5, -0.55, npts)[:-1]
    driver = MovingRigid(xy_ref=np.stack([np.zeros(npts - 1), ys], axis=1), ds=chord / (npts - 1),
                         motion=flapping_motion(sigma_t=sigma, sigma_r=sigma))
    driver.accel = driver.motion.accel
    passive = MountedTorsional(driver=0, n=npts, hinge_body=(0.0, -0.55), theta_rel=-math.pi / 2,
                               length=chord, inertia=0.2886, stiffness=456.0, damping=3.95,
                               mass=math.pi / 4, cg=0.55)
    sd = (-1.89, 1.89, -1.66, 0.65) if subdomain else None
    return Problem("two_plates", flow, [driver, passive], sd, None, steps)


def cylinder(center, diameter, h, spacing=1.0):
    """Points on a circle at angle 2*pi*j/n with spacing close to spacing*h."""
    n = int(round(math.pi * diameter / (spacing * h)))
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


def flag_body(hinge, length, h, mass=0.2, ei=1e-3, ea=1e3, a=0.075, spacing=2.0):
    """Deformable flag clamped at `hinge` along +x with node spacing about spacing*h and an
    initial deflection w(s) = a (s/L)^2 L, nodes at equal arc length, at rest."""
    npts = max(3, int(round(length / (spacing * h))) + 1)
    ds = length / (npts - 1)
    xy_ref = np.stack([hinge[0] + np.arange(npts) * ds, np.full(npts, float(hinge[1]))], axis=1)
    k = a / length
    xs = np.linspace(0.0, 1.2 * length, 240001)
    seg = np.hypot(np.diff(xs), np.diff(k * xs * xs))
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    sx = np.interp(np.arange(npts) * ds, arc, xs)
    xy0 = np.stack([hinge[0] + sx, hinge[1] + k * sx * sx], axis=1)
    rot0 = np.arctan(2.0 * k * sx)
    return Deformable(xy_ref=xy_ref, mass=mass, ei=ei, ea=ea, xy0=xy0, rot0=rot0)


def plate_box(hinge, length, theta0, spread=math.radians(55.0), margin=0.05):
    """Bounding box of the sector a hinged plate can sweep (theta0 +- spread)."""
    angs = [theta0 - spread, theta0 + spread]
    for k in range(-4, 5):
        a = k * math.pi / 2.0
        if theta0 - spread < a < theta0 + spread:
            angs.append(a)
    xs = [hinge[0]] + [hinge[0] + length * math.cos(a) for a in angs]
    ys = [hinge[1]] + [hinge[1] + length * math.sin(a) for a in angs]
    return (min(xs) - margin, max(xs) + margin, min(ys) - margin, max(ys) + margin)


def _place(rng, sizes_wanted, h, lim=1.2, boxes=None):
    """Centres for bodies of the given sizes inside [-lim, lim]^2 without overlap."""
    boxes = [] if boxes is None else boxes
    out = []
    for size in sizes_wanted:
        for _ in range(400):
            c = rng.uniform(-lim + size / 2, lim - size / 2, size=2)
            box = (c[0] - size / 2 - 4 * h, c[0] + size / 2 + 4 * h,
                   c[1] - size / 2 - 4 * h, c[1] + size / 2 + 4 * h)
            if all(box[1] < b[0] or b[1] < box[0] or box[3] < b[2] or b[3] < box[2] for b in boxes):
                boxes.append(box)
                out.append((float(c[0]), float(c[1])))
                break
    return out


def batch_problems(count=64, seed=4, steps=200, sizes=(128, 256, 384, 512, 768)):
    """Independent instances: seeded grid size, level count, Re and 1-3 bodies each.

    Bodies are rigid circles (D ~ U[0.3, 0.8]) or torsional plates (L ~ U[0.3, 0.8],
    theta0 ~ U[-30, 30] degrees, inertia 5, stiffness 1, damping 0.1), each kind with
    probability 1/2, placed without overlap in [-1.2, 1.2]^2 on a finest level of side 4
    (h = 4/n, dt = 0.2 h), Re ~ U[50, 400]; body points 2h apart (Sec. 5).  Every plate
    has a sub-domain rectangle of its own, the box of the sector it can sweep; instances with
    only circles use the exact stationary operator.
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
        kinds = ["plate" if rng.uniform() < 0.5 else "circle" for k in range(nb)]
        sizes_ = [float(rng.uniform(0.3, 0.8)) for _ in range(nb)]
        centres = _place(rng, sizes_, h)
        bodies, boxes = [], []
        for kind, size, c in zip(kinds, sizes_, centres):
            if kind == "circle":
                bodies.append(cylinder(c, size, h, spacing=2.0))
            else:
                npts = int(round(size / (2.0 * h))) + 1
                th0 = math.radians(float(rng.uniform(-30.0, 30.0)))
                hinge = (c[0] - 0.5 * size * math.cos(th0), c[1] - 0.5 * size * math.sin(th0))
                bodies.append(Torsional(n=npts, hinge=hinge, length=size, theta0=th0,
                                        inertia=5.0, stiffness=1.0, damping=0.1))
                boxes.append(plate_box(hinge, size, th0))
        out.append(Problem(f"batch{i}", flow, bodies, boxes or None, None, steps))
    return out


# Families of the serving trace: grid, levels, Re, stationary circles (centre, D) and
# the moving body, whose geometry (and so the offline operator) the requests of a family
# share; a request varies the moving body's parameters, the initial noise and the steps.
SERVE_FAMILIES = (
    dict(n=256, levels=1, re=100.0, circles=[((0.0, 0.0), 0.8)], moving=None, weight=3),
    dict(n=384, levels=2, re=200.0, circles=[((0.6, 0.5), 0.4)],
         moving=("plate", (-0.6, 0.0), 0.6, -0.35), weight=3),
    dict(n=512, levels=3, re=300.0, circles=[], moving=("flag", (-0.4, 0.0), 0.6), weight=2),
    dict(n=768, levels=2, re=150.0, circles=[((0.7, 0.7), 0.4), ((0.7, -0.7), 0.4)],
         moving=("plate", (-0.8, 0.0), 0.6, 0.0), weight=2),
    dict(n=1024, levels=4, re=500.0, circles=[], moving=("flag", (-0.3, 0.0), 0.6), weight=1),
    dict(n=512, levels=1, re=250.0, circles=[((-0.5, 0.3), 0.5), ((0.5, -0.3), 0.5)],
         moving=None, weight=2),
)


def serve_request(family, rng, steps, noise=1e-3):
    """One request of a family (see SERVE_FAMILIES)."""
    n, levels = family["n"], family["levels"]
    h = 4.0 / n
    flow = Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=family["re"])
    bodies = [cylinder(c, d, h, spacing=2.0) for c, d in family["circles"]]
    sd = None
    mv = family["moving"]
    if mv is not None and mv[0] == "plate":
        _, hinge, length, th0c = mv
        npts = int(round(length / (2.0 * h))) + 1
        th0 = th0c + math.radians(float(rng.uniform(-10.0, 10.0)))
        bodies.append(Torsional(n=npts, hinge=hinge, length=length, theta0=th0,
                                inertia=float(rng.uniform(2.0, 8.0)),
                                stiffness=float(rng.uniform(0.5, 2.0)), damping=0.1))
        sd = plate_box(hinge, length, th0c, spread=math.radians(65.0))
    elif mv is not None:
        _, hinge, length = mv
        bodies.append(flag_body(hinge, length, h, mass=float(rng.uniform(0.1, 0.4)),
                                ei=float(rng.uniform(5e-4, 2e-3)),
                                a=float(rng.uniform(0.05, 0.1)) * length))
        sd = (hinge[0] - 0.02, hinge[0] + length + 0.02, hinge[1] - 0.6 * length,
              hinge[1] + 0.6 * length)
    w0 = [rng.normal(0.0, noise, size=(n - 1, n - 1))] + [None] * (levels - 1)
    return Problem("serve", flow, bodies, sd, w0, steps)


def serve_trace(count=48, rate=40.0, seed=5, steps=(200, 2000), families=SERVE_FAMILIES):
    """Poisson arrivals (mean rate per second) of requests drawn from the families by
    weight, steps ~ U{steps[0] .. steps[1]}: a list of (arrival seconds, Problem)."""
    rng = np.random.default_rng(seed)
    w = np.array([f["weight"] for f in families], dtype=float)
    w /= w.sum()
    t, out = 0.0, []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        fam = families[int(rng.choice(len(families), p=w))]
        st = int(rng.integers(steps[0], steps[1] + 1))
        out.append((t, serve_request(fam, rng, st)))
    return out


def drawn_request(rng, steps=(200, 2000), sizes=(256, 384, 512, 768, 1024), noise=1e-3):
    """One request with everything drawn: N ~ U{sizes}, G ~ U{1..4}, Re ~ U[50, 400] and 1-3
    bodies, each a rigid circle, a torsional plate or a deformable flag with equal probability,
    steps ~ U{steps[0] .. steps[1]}.  Sizes and placement as in batch_problems (circles
    D ~ U[0.3, 0.8]; plates L ~ U[0.3, 0.8], theta0 ~ U[-30, 30] degrees, inertia 5,
    stiffness 1, damping 0.1; flags L ~ U[0.3, 0.8] clamped along +x, mass ratio 0.2, bending
    stiffness 1e-3, stretching stiffness 1e3, initial deflection a ~ U[0.05, 0.1] L), finest
    level of side 4 (h = 4/N, dt = 0.2 h), body points 2h apart.  Every plate and flag has a
    sub-domain rectangle of its own: the box of the sector a plate can sweep, or the strip
    [x_c - 0.02, x_c + L + 0.02] x [y_c - 0.6 L, y_c + 0.6 L] of a flag clamped at (x_c, y_c)."""
    n = int(rng.choice(sizes))
    levels = int(rng.integers(1, 5))
    re = float(rng.uniform(50.0, 400.0))
    h = 4.0 / n
    flow = Flow(n=n, levels=levels, h=h, dt=0.2 * h, re=re)
    nb = int(rng.integers(1, 4))
    kinds = [("circle", "plate", "flag")[int(rng.integers(0, 3))] for _ in range(nb)]
    sizes_ = [float(rng.uniform(0.3, 0.8)) for _ in range(nb)]
    centres = _place(rng, sizes_, h)
    bodies, boxes = [], []
    for kind, size, c in zip(kinds, sizes_, centres):
        if kind == "circle":
            bodies.append(cylinder(c, size, h, spacing=2.0))
        elif kind == "plate":
            npts = int(round(size / (2.0 * h))) + 1
            th0 = math.radians(float(rng.uniform(-30.0, 30.0)))
            hinge = (c[0] - 0.5 * size * math.cos(th0), c[1] - 0.5 * size * math.sin(th0))
            bodies.append(Torsional(n=npts, hinge=hinge, length=size, theta0=th0,
                                    inertia=5.0, stiffness=1.0, damping=0.1))
            boxes.append(plate_box(hinge, size, th0))
        else:
            clamp = (c[0] - 0.5 * size, c[1])
            a = float(rng.uniform(0.05, 0.1)) * size
            bodies.append(flag_body(clamp, size, h, a=a))
            boxes.append((clamp[0] - 0.02, clamp[0] + size + 0.02, clamp[1] - 0.6 * size,
                          clamp[1] + 0.6 * size))
    w0 = [rng.normal(0.0, noise, size=(n - 1, n - 1))] + [None] * (levels - 1)
    st = int(rng.integers(steps[0], steps[1] + 1))
    return Problem("drawn", flow, bodies, boxes or None, w0, st)


def drawn_trace(count=500, rate=40.0, seed=6, steps=(200, 2000)):
    """Poisson arrivals (mean rate per second) of requests drawn one by one (drawn_request):
    a list of (arrival seconds, Problem)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        out.append((t, drawn_request(rng, steps)))
    return out
