"""Pins of the oracle's torsional body mounted on a driven rigid body (Sec. 5.1's passive
plate hinged to the driven plate).

The mount enters through the hinge position and reference angle at t_{n+1}, the driver's
velocity at the points, and the pseudo-moment g of the hinge's acceleration.  Pinned by:
the driver at rest reduces exactly to a fixed hinge; the structural trajectory with no
fluid force satisfies the Newton-Euler equations about the plate's centre of mass (a
formulation independent of the hinge-moment form the oracle uses) to second order in dt;
the pseudo-moment reproduces the paper's two-plate equation term by term; the coupled step
satisfies the no-slip constraint at round-off; and the kinematics' accelerations match
their velocities."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import structure
from oracle.step import Oracle


def _flow():
    n = 16
    return W.Flow(n=n, levels=1, h=0.1, dt=0.02, re=50.0, cx=0.0, cy=0.0, u_inf=(1.0, 0.2))


def _w0(n):
    rng = np.random.default_rng(5)
    return [0.5 * rng.normal(size=(n - 1, n - 1))]


DRIVER_REF = np.array([[0.0, 0.25], [0.0, 0.15], [0.0, 0.05], [0.0, -0.05]])


class _Motion:
    """Smooth prescribed motion with closed-form rates and accelerations."""

    def __init__(self, ax=0.3, wx=2.0, ay=0.1, aa=0.4, wa=3.0, x0=0.0, y0=0.0, a0=0.2):
        self.p = (ax, wx, ay, aa, wa, x0, y0, a0)

    def __call__(self, t):
        ax, wx, ay, aa, wa, x0, y0, a0 = self.p
        return (x0 + ax * math.sin(wx * t), y0 + ay * t * t, a0 + aa * math.sin(wa * t),
                ax * wx * math.cos(wx * t), 2 * ay * t, aa * wa * math.cos(wa * t))

    def accel(self, t):
        ax, wx, ay, aa, wa, *_ = self.p
        return (-ax * wx * wx * math.sin(wx * t), 2 * ay, -aa * wa * wa * math.sin(wa * t))


def _mount(driver=0, **kw):
    # the hinge one spacing below the driver's last point (a point of the mounted body;
    # coincident points would make the Schur matrix singular)
    args = dict(driver=driver, n=5, hinge_body=(0.0, -0.15), theta_rel=-math.pi / 2 + 0.2,
                length=0.3, inertia=0.05, stiffness=0.8, damping=0.02, mass=0.3, cg=0.15,
                theta=0.05, phi=0.0)
    args.update(kw)
    return W.MountedTorsional(**args)


def test_driver_at_rest_reduces_to_a_fixed_hinge():
    """A driver at rest: the mounted body is a torsional body with a fixed hinge at the
    driver's hinge point and reference angle driver angle + theta_rel, and the driver a
    stationary rigid body (results identical to round-off)."""
    x0, y0, a0 = 0.1, 0.2, 0.3
    rest = W.MovingRigid(xy_ref=DRIVER_REF, ds=0.1, motion=lambda t: (x0, y0, a0, 0, 0, 0),
                         accel=lambda t: (0.0, 0.0, 0.0))
    mb = _mount()
    c, s = math.cos(a0), math.sin(a0)
    hx = x0 + c * mb.hinge_body[0] - s * mb.hinge_body[1]
    hy = y0 + s * mb.hinge_body[0] + c * mb.hinge_body[1]
    pts = DRIVER_REF @ np.array([[c, s], [-s, c]]) + np.array([x0, y0])
    fixed = W.Torsional(n=mb.n, hinge=(hx, hy), length=mb.length, theta0=a0 + mb.theta_rel,
                        inertia=mb.inertia, stiffness=mb.stiffness, damping=mb.damping,
                        theta=mb.theta, phi=mb.phi)
    flow = _flow()
    a = Oracle(W.Problem("a", flow, [rest, mb], None, _w0(flow.n), 3), fixed_iters=4)
    b = Oracle(W.Problem("b", flow, [W.Rigid(xy=pts, ds=0.1), fixed], None, _w0(flow.n), 3),
               fixed_iters=4)
    for _ in range(3):
        a.step()
        b.step()
    assert np.max(np.abs(a.s[0] - b.s[0])) < 1e-12 * np.max(np.abs(b.s[0]))
    assert np.max(np.abs(a.f - b.f)) < 1e-10 * np.max(np.abs(b.f))
    assert abs(a.bodies[1][1].theta - b.bodies[1][1].theta) < 1e-13


def _trajectory(dt, t_end, mb, motion):
    """Structure alone (no fluid force) under the mount's pseudo-moment: Newmark average
    acceleration, each step's implicit g resolved by fixed-point iteration."""
    driver = W.MovingRigid(xy_ref=DRIVER_REF, ds=0.1, motion=motion, accel=motion.accel)
    st = structure.MountedState(mb, driver, dt)
    out = []

    def record(t):
        ph = st.ang0 + st.theta
        g = (st.hinge[0] + mb.cg * math.cos(ph), st.hinge[1] + mb.cg * math.sin(ph))
        out.append((t, st.theta, ph, g[0], g[1], st.hinge[0], st.hinge[1]))

    record(0.0)
    steps = int(round(t_end / dt))
    jt = st.jac()
    for k in range(steps):
        st.set_time((k + 1) * dt)
        st.theta_k = st.theta
        for _ in range(100):
            th = st.r_phi() / jt
            done = abs(th - st.theta_k) < 1e-15
            st.theta_k = th
            if done:
                break
        st.finish(st.theta_k)
        record((k + 1) * dt)
    return np.array(out)


def _newton_euler_residual(tr, dt, mb):
    """max over interior times of |I_G phi'' - (H - G) x m G'' + k theta + c theta'|, the
    angular balance about the centre of mass with the hinge reaction m G''."""
    t, th, ph, gx, gy, hx, hy = tr.T
    d2 = lambda v: (v[2:] - 2 * v[1:-1] + v[:-2]) / dt ** 2
    d1 = lambda v: (v[2:] - v[:-2]) / (2 * dt)
    ig = mb.inertia - mb.mass * mb.cg ** 2
    axg, ayg = d2(gx), d2(gy)
    rx, ry = hx[1:-1] - gx[1:-1], hy[1:-1] - gy[1:-1]
    torque_reaction = mb.mass * (rx * ayg - ry * axg)
    res = ig * d2(ph) - torque_reaction + mb.stiffness * th[1:-1] + mb.damping * d1(th)
    scale = np.max(np.abs(ig * d2(ph))) + np.max(np.abs(torque_reaction))
    return float(np.max(np.abs(res))), float(scale)


def test_pseudo_moment_obeys_newton_euler_about_the_centre_of_mass():
    """The oracle integrates the hinge-moment form I_H theta'' + c theta' + k theta = g with
    g = -I_H alpha'' - m r_G x a_H.  Its trajectory must satisfy the balance about the
    centre of mass, I_G phi'' = (H - G) x m G'' - k theta - c theta' (the hinge reaction is
    m G''), to second order in dt: a dropped or mis-signed term of g leaves an O(1) residual."""
    mb = _mount(inertia=0.3, stiffness=2.0, damping=0.1, mass=0.8, cg=0.55, theta=0.1,
                hinge_body=(0.2, -0.5), theta_rel=-math.pi / 2 + 0.3)
    motion = _Motion()
    r1, scale = _newton_euler_residual(_trajectory(2e-3, 1.5, mb, motion), 2e-3, mb)
    r2, _ = _newton_euler_residual(_trajectory(1e-3, 1.5, mb, motion), 1e-3, mb)
    print(f"residual {r1:.3e} -> {r2:.3e}, scale {scale:.3e}")
    assert r2 < 1e-4 * scale
    assert 3.0 < r1 / r2 < 5.0  # second order


def test_pseudo_moment_is_the_papers_two_plate_equation():
    """For Sec. 5.1's geometry (driver along -y at zero angle, hinge L1 below the driver's
    centre of mass, theta_rel = -pi/2) g equals the paper's right-hand side
    -m L2 cos(a1 + th) X1'' - [I_H + m L1 L2 cos th] a1'' - m L1 L2 sin th a1'^2
    for any state."""
    rng = np.random.default_rng(3)
    l1, l2, m, ih = 0.55, 0.55, math.pi / 4, 0.2886
    for _ in range(20):
        x, a1, v, w, ax, al, th = rng.normal(size=7)
        driver = W.MovingRigid(xy_ref=DRIVER_REF, ds=0.1, motion=lambda t: (x, 0.0, a1, v, 0.0, w),
                               accel=lambda t: (ax, 0.0, al))
        mb = W.MountedTorsional(driver=0, n=5, hinge_body=(0.0, -l1), theta_rel=-math.pi / 2,
                                length=1.05, inertia=ih, stiffness=456.0, damping=3.95, mass=m,
                                cg=l2)
        st = structure.MountedState(mb, driver, 0.01)
        st.set_time(0.0)
        paper = (-m * l2 * math.cos(a1 + th) * ax - (ih + m * l1 * l2 * math.cos(th)) * al
                 - m * l1 * l2 * math.sin(th) * w * w)
        assert abs(st.pseudo_moment(th) - paper) < 1e-12 * max(1.0, abs(paper))


def test_mounted_step_satisfies_no_slip():
    """Coupled steps with a driven hinge (exact operators): the constraint velocity of the
    mounted points (driver's velocity at the point plus the deflection rate) is met at
    round-off, and the mount changes the answer against a fixed hinge."""
    motion = _Motion(ax=0.1, ay=0.05, aa=0.2)
    drv = W.MovingRigid(xy_ref=DRIVER_REF, ds=0.1, motion=motion, accel=motion.accel)
    flow = _flow()
    o = Oracle(W.Problem("m", flow, [drv, _mount(inertia=0.5, mass=0.8)], None, _w0(flow.n), 3))
    for _ in range(3):
        o.step()
        assert o.noslip_residual() < 1e-11
    assert o.last_iters >= 2


@pytest.mark.parametrize("sigma", [3.770, 0.628])
def test_flapping_accelerations_match_the_velocities(sigma):
    mo = W.flapping_motion(sigma_t=sigma, sigma_r=sigma)
    for t in (0.05, 0.3, 0.77, 1.2, 2.45):
        e = 1e-5
        p, m = mo(t + e), mo(t - e)
        acc = mo.accel(t)
        for k, q in ((0, 3), (1, 4), (2, 5)):
            fd = (p[q] - m[q]) / (2 * e)
            assert abs(acc[k] - fd) < 1e-6 * max(1.0, abs(fd))
