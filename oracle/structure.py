"""Structural models for the FSI iteration (FP64 oracle).

Torsional body (Appendix A, eqs. (A.2)-(A.4), (A.10)-(A.11)): points j = 0..n-1 at
hinge + j ds (cos, sin)(theta0 + theta).  The normal stress is (R f)_j =
-f_x sin + f_y cos, the moment is Q R f ds with Q = [0, 1, .., n-1] ds (rectangle
weights including the tip, as written in eq. (A.3)), and Newmark average
acceleration gives

    J theta_{n+1} - Q R f ds = r_phi,     J = 4 I/dt^2 + 2 c/dt + k,
    (2/dt) theta_{n+1} - phi_{n+1} = r_theta,

r_phi = I (4 theta/dt^2 + 4 phi/dt + phidot) + c (2 theta/dt + phi) + g and
r_theta = phi + 2 theta / dt.  f is the stress the fluid exerts on the body.
Reading: the initial angular acceleration is (g - c phi - k theta) / I (f_0 = 0).

Deformable body (eqs. (A.5), (A.12)-(A.13); the paper defers the finite elements to
Goza & Colonius 2017, which is not available).  Reading: a 2-D corotational
Euler-Bernoulli beam, nodes = body points, DOFs (x, y, rotation) per node, node 0
clamped.  Element internal force f = B^T [N, M1, M2] with N = EA (L - L0)/L0 and
[M1, M2] = (2 EI / L0) [[2, 1], [1, 2]] [tb1, tb2], tb = nodal rotation minus the
chord rotation; tangent K = B^T D B + (N/L) z z^T + ((M1 + M2)/L^2)(r z^T + z r^T).
Lumped mass: m L0 / 2 per element end for x and y, m L0^3 / 105 rotary.  The fluid
load on a node is f ds (the same point quadrature the regularisation uses).  Newmark
average acceleration as for the torsional body, with J_d = 4 M/dt^2 + K(chi).
"""
import math

import numpy as np


class TorsionalState:
    def __init__(self, body, dt):
        self.b = body
        self.dt = dt
        self.theta = float(body.theta)
        self.phi = float(body.phi)
        self.g = 0.0
        self.phidot = (self.g - body.damping * self.phi - body.stiffness * self.theta) / body.inertia
        self.theta_k = self.theta

    @property
    def npts(self):
        return self.b.n

    @property
    def ds(self):
        return self.b.ds

    def jac(self):
        b, dt = self.b, self.dt
        return 4.0 * b.inertia / dt ** 2 + 2.0 * b.damping / dt + b.stiffness

    def r_phi(self):
        b, dt = self.b, self.dt
        return (b.inertia * (4.0 * self.theta / dt ** 2 + 4.0 * self.phi / dt + self.phidot)
                + b.damping * (2.0 * self.theta / dt + self.phi) + self.g)

    def r_theta(self):
        return self.phi + 2.0 * self.theta / self.dt

    def positions(self, theta):
        b = self.b
        ang = b.theta0 + theta
        j = np.arange(b.n) * b.ds
        return np.stack([b.hinge[0] + j * math.cos(ang), b.hinge[1] + j * math.sin(ang)], axis=1)

    def s_row(self, theta):
        """S = Q R over this body's [f_x (n), f_y (n)] block: S f = sum_j j ds (R f)_j."""
        ang = self.b.theta0 + theta
        j = np.arange(self.b.n) * self.b.ds
        return np.concatenate([-j * math.sin(ang), j * math.cos(ang)])

    def finish(self, theta_new):
        dt = self.dt
        phi_new = 2.0 * theta_new / dt - self.r_theta()
        phidot_new = 4.0 * (theta_new - self.theta) / dt ** 2 - 4.0 * self.phi / dt - self.phidot
        self.theta, self.phi, self.phidot = theta_new, phi_new, phidot_new


class MountedState(TorsionalState):
    """Torsional body whose hinge rides on a rigid body in prescribed motion (Sec. 5.1's
    passive plate).  Reading (the paper gives the equation for its two-plate case only, with
    a garbled inertia symbol): with the hinge H(t) fixed in the driver's frame, the
    driver's angle alpha(t), and the plate's absolute angle phi = alpha + theta_rel + theta,
    the angular momentum balance about the moving hinge is

        I_H (alpha_dd + theta_dd) + m r_G x a_H = M_fluid - k theta - c theta_dot,

    r_G = cg (cos phi, sin phi), so the torsional equation of Sec. 2.1 holds for the
    relative deflection theta with g = -I_H alpha_dd - m cg (cos phi a_Hy - sin phi a_Hx).
    For the two-plate case (angles measured from the driver's -y direction) this is term
    by term the paper's equation.  g is evaluated at the current iterate and at t_{n+1}
    (Newmark average acceleration, as for the other torsional terms); the points carry the
    hinge's velocity plus the driver's rotation on top of the deflection rate."""

    def __init__(self, body, driver, dt):
        self.mount = body
        self.driver = driver
        self.frame_t = None
        base = _Plain(n=body.n, length=body.length, inertia=body.inertia,
                      stiffness=body.stiffness, damping=body.damping, theta=body.theta,
                      phi=body.phi)
        self.b = base
        self.dt = dt
        self.theta = float(body.theta)
        self.phi = float(body.phi)
        self.set_time(0.0)
        self.g = self.pseudo_moment(self.theta)
        self.phidot = (self.g - body.damping * self.phi - body.stiffness * self.theta) / body.inertia
        self.theta_k = self.theta

    def set_time(self, t):
        """Hinge, reference angle, and the driver's rates and accelerations at time t."""
        x, y, ang, vx, vy, om = self.driver.pose(t)
        ax, ay, al = self.driver.accelerations(t)
        hb = self.mount.hinge_body
        c, sn = math.cos(ang), math.sin(ang)
        rx, ry = c * hb[0] - sn * hb[1], sn * hb[0] + c * hb[1]
        self.hinge = (x + rx, y + ry)
        self.vh = (vx - om * ry, vy + om * rx)
        self.ah = (ax - al * ry - om * om * rx, ay + al * rx - om * om * ry)
        self.omega = om
        self.alpha_dd = al
        self.ang0 = ang + self.mount.theta_rel
        self.frame_t = t

    def pseudo_moment(self, theta):
        mb = self.mount
        ph = self.ang0 + theta
        return (-mb.inertia * self.alpha_dd
                - mb.mass * mb.cg * (math.cos(ph) * self.ah[1] - math.sin(ph) * self.ah[0]))

    def r_phi(self):
        b, dt = self.b, self.dt
        return (b.inertia * (4.0 * self.theta / dt ** 2 + 4.0 * self.phi / dt + self.phidot)
                + b.damping * (2.0 * self.theta / dt + self.phi) + self.pseudo_moment(self.theta_k))

    def positions(self, theta):
        ang = self.ang0 + theta
        j = np.arange(self.b.n) * self.b.ds
        return np.stack([self.hinge[0] + j * math.cos(ang), self.hinge[1] + j * math.sin(ang)], axis=1)

    def s_row(self, theta):
        ang = self.ang0 + theta
        j = np.arange(self.b.n) * self.b.ds
        return np.concatenate([-j * math.sin(ang), j * math.cos(ang)])

    def mount_velocity(self, theta):
        """Velocity of the points from the driver alone: v_H + omega e_z x (p - H)."""
        p = self.positions(theta) - np.array(self.hinge)
        return np.stack([self.vh[0] - self.omega * p[:, 1], self.vh[1] + self.omega * p[:, 0]], axis=1)


class _Plain:
    """The torsional constants a MountedState shares with a fixed-hinge body."""

    def __init__(self, n, length, inertia, stiffness, damping, theta, phi):
        self.n, self.length = n, length
        self.inertia, self.stiffness, self.damping = inertia, stiffness, damping
        self.theta, self.phi = theta, phi

    @property
    def ds(self):
        return self.length / (self.n - 1)


def _wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


class Beam:
    """Corotational Euler-Bernoulli beam; chi = [x0, y0, r0, x1, y1, r1, ...]."""

    def __init__(self, body):
        self.b = body
        ref = np.asarray(body.xy_ref, dtype=np.float64)
        self.n = ref.shape[0]
        d = np.diff(ref, axis=0)
        self.l0 = np.hypot(d[:, 0], d[:, 1])
        self.beta0 = np.arctan2(d[:, 1], d[:, 0])
        self.mass = np.zeros(3 * self.n)
        for e in range(self.n - 1):
            me = body.mass * self.l0[e]
            for node in (e, e + 1):
                self.mass[3 * node] += 0.5 * me
                self.mass[3 * node + 1] += 0.5 * me
                self.mass[3 * node + 2] += me * self.l0[e] ** 2 / 105.0

    def internal(self, chi):
        """Internal force R(chi) (3n) and tangent K = dR/dchi (3n x 3n)."""
        n, ea, ei = self.n, self.b.ea, self.b.ei
        r_int = np.zeros(3 * n)
        k = np.zeros((3 * n, 3 * n))
        for e in range(n - 1):
            idx = np.array([3 * e, 3 * e + 1, 3 * e + 2, 3 * e + 3, 3 * e + 4, 3 * e + 5])
            x1, y1, t1, x2, y2, t2 = chi[idx]
            dx, dy = x2 - x1, y2 - y1
            length = math.hypot(dx, dy)
            c, s = dx / length, dy / length
            alpha = _wrap(math.atan2(dy, dx) - self.beta0[e])
            l0 = self.l0[e]
            tb1 = _wrap(t1 - alpha)
            tb2 = _wrap(t2 - alpha)
            nax = ea * (length - l0) / l0
            m1 = 2.0 * ei / l0 * (2.0 * tb1 + tb2)
            m2 = 2.0 * ei / l0 * (tb1 + 2.0 * tb2)
            r = np.array([-c, -s, 0.0, c, s, 0.0])
            z = np.array([s, -c, 0.0, -s, c, 0.0])
            bmat = np.vstack([r,
                              np.array([0, 0, 1.0, 0, 0, 0]) - z / length,
                              np.array([0, 0, 0, 0, 0, 1.0]) - z / length])
            dmat = np.array([[ea / l0, 0.0, 0.0],
                             [0.0, 4.0 * ei / l0, 2.0 * ei / l0],
                             [0.0, 2.0 * ei / l0, 4.0 * ei / l0]])
            fe = bmat.T @ np.array([nax, m1, m2])
            ke = (bmat.T @ dmat @ bmat + (nax / length) * np.outer(z, z)
                  + ((m1 + m2) / length ** 2) * (np.outer(r, z) + np.outer(z, r)))
            r_int[idx] += fe
            k[np.ix_(idx, idx)] += ke
        return r_int, k


class BeamState:
    """Newmark state of a clamped beam; node 0's three DOFs are held fixed."""

    def __init__(self, body, dt):
        self.b = body
        self.beam = Beam(body)
        self.dt = dt
        n = self.beam.n
        chi = np.zeros(3 * n)
        chi[0::3] = body.xy0[:, 0]
        chi[1::3] = body.xy0[:, 1]
        chi[2::3] = body.rot0
        self.chi = chi
        self.zeta = np.zeros(3 * n)
        r_int, _ = self.beam.internal(chi)
        acc = -r_int / self.beam.mass
        acc[:3] = 0.0
        self.zetadot = acc
        self.free = np.arange(3, 3 * n)
        self.chi_k = chi.copy()

    @property
    def npts(self):
        return self.beam.n

    @property
    def ds(self):
        return self.b.ds

    def positions(self, chi):
        return np.stack([chi[0::3], chi[1::3]], axis=1)

    def r_zeta(self):
        dt = self.dt
        return self.beam.mass * (4.0 * self.chi / dt ** 2 + 4.0 * self.zeta / dt + self.zetadot)

    def r_chi(self):
        return self.zeta + 2.0 * self.chi / self.dt

    def jacobian(self, chi):
        """J_d over the free DOFs and the residual r_zeta - 4 M chi/dt^2 - R(chi)."""
        dt = self.dt
        r_int, k = self.beam.internal(chi)
        jd = k + np.diag(4.0 * self.beam.mass / dt ** 2)
        res = self.r_zeta() - 4.0 * self.beam.mass * chi / dt ** 2 - r_int
        fr = self.free
        return jd[np.ix_(fr, fr)], res[fr]

    def t_matrix(self):
        """T: (2 n, free DOFs) picking each node's translational DOFs in the body's
        [x block, y block] stress order; the clamped node maps to nothing."""
        n = self.beam.n
        t = np.zeros((2 * n, 3 * n))
        for p in range(n):
            t[p, 3 * p] = 1.0
            t[n + p, 3 * p + 1] = 1.0
        return t[:, self.free]

    def finish(self, chi_new):
        dt = self.dt
        zeta_new = 2.0 * chi_new / dt - self.r_chi()
        zetadot_new = 4.0 * (chi_new - self.chi) / dt ** 2 - 4.0 * self.zeta / dt - self.zetadot
        zeta_new[:3] = 0.0
        zetadot_new[:3] = 0.0
        self.chi, self.zeta, self.zetadot = chi_new, zeta_new, zetadot_new
