"""Pins of the oracle's rigid bodies in prescribed motion (Sec. 2.1, eq. (5): rigid bodies
move with a prescribed velocity; Sec. 5.1's driven plate): the motion enters only through
the point positions and the prescribed velocity at the new time level, so special motions
reduce exactly to the stationary-body path, and the driven-plate kinematics match their
definitions."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle.step import Oracle


def _flow():
    n = 16
    return W.Flow(n=n, levels=1, h=0.1, dt=0.02, re=50.0, cx=0.0, cy=0.0, u_inf=(1.0, 0.2))


def _w0(n):
    rng = np.random.default_rng(5)
    return [0.5 * rng.normal(size=(n - 1, n - 1))]


REF = np.array([[-0.1, 0.0], [-0.05, 0.02], [0.0, 0.03], [0.05, 0.02], [0.1, 0.0]])
DS = 0.055


def _run(body, steps=3):
    flow = _flow()
    o = Oracle(W.Problem("m", flow, [body], None, _w0(flow.n), steps))
    for _ in range(steps):
        o.step()
    return o


@pytest.mark.parametrize("case", ["still", "slip", "spin"])
def test_special_motions_equal_the_stationary_path(case):
    """A pose fixed in time with given rates is a stationary rigid body whose points carry
    that velocity: identical positions, prescribed velocities and hence identical steps."""
    ang, om, v = {"still": (0.0, 0.0, (0.0, 0.0)), "slip": (0.3, 0.0, (0.4, -0.2)),
                  "spin": (-0.5, 1.7, (0.0, 0.0))}[case]
    x0, y0 = 0.12, -0.07
    mover = W.MovingRigid(xy_ref=REF, ds=DS, motion=lambda t: (x0, y0, ang, v[0], v[1], om))
    c, s = math.cos(ang), math.sin(ang)
    r = np.stack([c * REF[:, 0] - s * REF[:, 1], s * REF[:, 0] + c * REF[:, 1]], axis=1)
    ub = np.stack([v[0] - om * r[:, 1], v[1] + om * r[:, 0]], axis=1)
    still = W.Rigid(xy=r + np.array([x0, y0]), ds=DS, u_b=ub if case != "still" else None)
    a, b = _run(mover), _run(still)
    assert np.array_equal(a.s[0], b.s[0])
    assert np.array_equal(a.f, b.f)


def test_positions_follow_the_pose_at_the_new_time_level():
    """An accelerating, turning body: the constraint of step n uses the pose and rates at
    t_{n+1}, so the no-slip residual evaluated there with the last operator is at
    round-off (it would be of order acc * dt at any other time level)."""
    acc, om = 3.0, 0.9
    mover = W.MovingRigid(xy_ref=REF, ds=DS,
                          motion=lambda t: (-0.2 + 0.5 * acc * t * t, 0.05, 0.2 + om * t,
                                            acc * t, 0.0, om))
    flow = _flow()
    o = Oracle(W.Problem("m", flow, [mover], None, _w0(flow.n), 3))
    for _ in range(3):
        o.step()
        assert o.noslip_residual() < 1e-11


def test_moving_body_changes_the_answer():
    """Motion is not ignored: the same body moving differs from it at rest."""
    mover = W.MovingRigid(xy_ref=REF, ds=DS, motion=lambda t: (0.1 * t, 0.0, 0.3 * t, 0.1, 0.0, 0.3))
    rest = W.MovingRigid(xy_ref=REF, ds=DS, motion=lambda t: (0.0, 0.0, 0.0, 0.0, 0.0, 0.0))
    a, b = _run(mover), _run(rest)
    assert np.max(np.abs(a.f - b.f)) > 1e-3 * np.max(np.abs(b.f))


@pytest.mark.parametrize("sigma", [3.770, 0.628])
def test_flapping_kinematics_match_their_definitions(sigma):
    """Sec. 5.1 kinematics: G_t against adaptive quadrature, the extremes of X and alpha,
    the start-up conditioner, and the rates against central differences."""
    a0, beta = 1.4, math.pi / 4
    mo = W.flapping_motion(a0=a0, beta=beta, sigma_t=sigma, sigma_r=sigma, freq=1.0)
    gmax = integrate.quad(lambda u: math.tanh(sigma * math.cos(2 * math.pi * u)), 0, 0.25,
                          epsabs=1e-14, epsrel=1e-13)[0]
    for t in (0.13, 0.61, 1.37, 2.9):
        g = integrate.quad(lambda u: math.tanh(sigma * math.cos(2 * math.pi * u)), 0, t,
                           epsabs=1e-14, epsrel=1e-13, limit=200)[0]
        cnd = (math.tanh(8 * t - 2) + math.tanh(2)) / (1 + math.tanh(2))
        x = mo(t)[0]
        assert abs(x - 0.5 * a0 * g / gmax * cnd) < 1e-13
    # once the conditioner has settled, X peaks at A0/2 a quarter period into a cycle and
    # alpha is -beta at whole periods
    assert abs(mo(3.25)[0] - 0.5 * a0) < 1e-10
    assert abs(mo(3.0)[2] + beta) < 1e-13
    assert abs(mo(3.5)[2] - beta) < 1e-13
    for t in (0.07, 0.4, 1.9):
        e = 1e-5
        p, m = mo(t + e), mo(t - e)
        vx_fd = (p[0] - m[0]) / (2 * e)
        om_fd = (p[2] - m[2]) / (2 * e)
        assert abs(mo(t)[3] - vx_fd) < 1e-7 * max(1.0, abs(vx_fd))
        assert abs(mo(t)[5] - om_fd) < 1e-7 * max(1.0, abs(om_fd))
        assert mo(t)[1] == 0.0 and mo(t)[4] == 0.0
