"""Pins of the oracle's structural models: Newmark closed forms and beam textbook cases."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import structure


def _torsional(inertia=2.0, stiffness=3.0, damping=0.0, theta=0.3, phi=-0.2, dt=0.05):
    b = W.Torsional(n=5, hinge=(0.0, 0.0), length=1.0, theta0=0.1, inertia=inertia,
                    stiffness=stiffness, damping=damping, theta=theta, phi=phi)
    return structure.TorsionalState(b, dt)


def _advance(st, moment):
    st.finish((st.r_phi() + moment) / st.jac())


def test_newmark_amplification_matrix():
    """f = 0: one step equals the closed-form trapezoidal amplification matrix of
    i th'' + c th' + k th = 0 (Newmark beta = 1/4, gamma = 1/2)."""
    i, k, c, dt = 2.0, 3.0, 0.4, 0.05
    st = _torsional(inertia=i, stiffness=k, damping=c, dt=dt)
    # average acceleration == trapezoidal rule on y' = A y, y = (theta, phi)
    a = np.array([[0.0, 1.0], [-k / i, -c / i]])
    amp = np.linalg.solve(np.eye(2) - 0.5 * dt * a, np.eye(2) + 0.5 * dt * a)
    y = np.array([st.theta, st.phi])
    for _ in range(5):
        _advance(st, 0.0)
        y = amp @ y
        np.testing.assert_allclose([st.theta, st.phi], y, atol=1e-14)


def test_newmark_energy_conserved_without_damping():
    st = _torsional(damping=0.0)
    e0 = 0.5 * st.b.inertia * st.phi ** 2 + 0.5 * st.b.stiffness * st.theta ** 2
    for _ in range(200):
        _advance(st, 0.0)
    e1 = 0.5 * st.b.inertia * st.phi ** 2 + 0.5 * st.b.stiffness * st.theta ** 2
    assert abs(e1 - e0) < 1e-13


def test_constant_moment_static_limit():
    st = _torsional(damping=1.5, theta=0.0, phi=0.0)
    for _ in range(3000):
        _advance(st, 0.6)
    assert abs(st.theta - 0.6 / st.b.stiffness) < 1e-9


def _beam(nel=20, length=1.0, ei=2.0, ea=1e4, mass=1.0):
    n = nel + 1
    xy = np.stack([np.linspace(0, length, n), np.zeros(n)], axis=1)
    body = W.Deformable(xy_ref=xy, mass=mass, ei=ei, ea=ea, xy0=xy.copy(), rot0=np.zeros(n))
    return structure.Beam(body), xy


def test_beam_tangent_is_derivative_of_internal_force():
    beam, xy = _beam(nel=6)
    rng = np.random.default_rng(4)
    chi = np.zeros(3 * beam.n)
    chi[0::3] = xy[:, 0] + 0.02 * rng.normal(size=beam.n)
    chi[1::3] = 0.1 * xy[:, 0] ** 2 + 0.02 * rng.normal(size=beam.n)
    chi[2::3] = 0.3 * rng.normal(size=beam.n)
    _, k = beam.internal(chi)
    eps = 1e-6
    fd = np.zeros_like(k)
    for j in range(chi.size):
        d = np.zeros_like(chi)
        d[j] = eps
        fd[:, j] = (beam.internal(chi + d)[0] - beam.internal(chi - d)[0]) / (2 * eps)
    np.testing.assert_allclose(k, fd, atol=1e-5 * np.abs(k).max())


def _static(beam, xy, load, steps=1):
    """Newton solve of R(chi) = load on the free DOFs (node 0 clamped)."""
    chi = np.zeros(3 * beam.n)
    chi[0::3], chi[1::3] = xy[:, 0], xy[:, 1]
    free = np.arange(3, 3 * beam.n)
    for s in range(1, steps + 1):
        for _ in range(50):
            r, k = beam.internal(chi)
            res = (s / steps) * load[free] - r[free]
            d = np.linalg.solve(k[np.ix_(free, free)], res)
            chi[free] += d
            if np.max(np.abs(d)) < 1e-13:
                break
    return chi


def test_cantilever_uniform_load_tip_deflection():
    """Small uniform load q: tip deflection q L^4 / (8 EI) (lumped nodal loads)."""
    nel, length, ei = 40, 1.0, 2.0
    beam, xy = _beam(nel=nel, ei=ei, ea=1e7)
    q = 1e-4
    load = np.zeros(3 * beam.n)
    le = length / nel
    load[1::3] = q * le
    load[1] = 0.5 * q * le
    load[-2] = 0.5 * q * le
    chi = _static(beam, xy, load)
    tip = chi[-2]
    assert abs(tip / (q * length ** 4 / (8 * ei)) - 1.0) < 2e-3


def test_end_moment_gives_circular_arc():
    """Pure end moment M: every element carries the same moment, so the nodes lie on a
    circle whose chords have the element length, R = L0 / (2 sin(M L0 / 2 EI)) -> EI/M
    as the mesh is refined, and the tip rotates by M L / EI."""
    nel, ei, m = 20, 1.0, 1.5
    beam, xy = _beam(nel=nel, ei=ei, ea=1e9)
    load = np.zeros(3 * beam.n)
    load[-1] = m
    chi = _static(beam, xy, load, steps=5)
    x, y = chi[0::3], chi[1::3]
    l0 = 1.0 / nel
    rad = l0 / (2.0 * math.sin(m * l0 / (2.0 * ei)))
    np.testing.assert_allclose(np.hypot(x, y - rad), rad, rtol=1e-7)
    assert abs(rad * m / ei - 1.0) < (m * l0 / ei) ** 2 / 20
    np.testing.assert_allclose(chi[-1], m * 1.0 / ei, rtol=1e-9)


def test_first_bending_frequency():
    nel, length, ei, mass = 60, 1.0, 2.0, 0.7
    beam, xy = _beam(nel=nel, ei=ei, ea=1e6, mass=mass)
    chi = np.zeros(3 * beam.n)
    chi[0::3], chi[1::3] = xy[:, 0], xy[:, 1]
    _, k = beam.internal(chi)
    free = np.arange(3, 3 * beam.n)
    kf = k[np.ix_(free, free)]
    mf = beam.mass[free]
    w2 = np.linalg.eigvals(kf / np.sqrt(mf)[:, None] / np.sqrt(mf)[None, :])
    w1 = math.sqrt(np.sort(np.real(w2))[0])
    exact = 1.875104 ** 2 * math.sqrt(ei / (mass * length ** 4))
    assert abs(w1 / exact - 1.0) < 5e-3


def test_beam_newmark_free_vibration_energy():
    """Linear regime, no fluid: total energy stays bounded and near its start value."""
    nel = 10
    n = nel + 1
    xy = np.stack([np.linspace(0, 1, n), np.zeros(n)], axis=1)
    a = 0.01
    body = W.Deformable(xy_ref=xy, mass=0.5, ei=1.0, ea=1e4,
                        xy0=np.stack([xy[:, 0], a * xy[:, 0] ** 2], axis=1),
                        rot0=np.arctan(2 * a * xy[:, 0]))
    st = structure.BeamState(body, dt=1e-3)

    def energy():
        # element strain energy in the corotated frame plus kinetic energy
        e = 0.0
        bm = st.beam
        for k in range(bm.n - 1):
            x1, y1, t1, x2, y2, t2 = st.chi[3 * k:3 * k + 6]
            ln = math.hypot(x2 - x1, y2 - y1)
            al = math.atan2(y2 - y1, x2 - x1) - bm.beta0[k]
            a1, a2 = t1 - al, t2 - al
            e += 0.5 * body.ea * (ln - bm.l0[k]) ** 2 / bm.l0[k]
            e += body.ei / bm.l0[k] * (2 * a1 * a1 + 2 * a1 * a2 + 2 * a2 * a2)
        return e + 0.5 * np.sum(st.beam.mass * st.zeta ** 2)

    e0 = energy()
    for _ in range(100):
        jd, res = st.jacobian(st.chi)
        chi = st.chi.copy()
        for _ in range(20):
            jd, res = st.jacobian(chi)
            d = np.linalg.solve(jd, res)
            chi[st.free] += d
            if np.max(np.abs(d)) < 1e-14:
                break
        st.finish(chi)
    assert abs(energy() / e0 - 1.0) < 2e-3
