"""Pins of the oracle's coupled step: the block-LU path against a dense solve of the
un-factored linear system, the no-slip residual, the Schur matrix's structure, the
sub-domain operators, and the nested-level far field against one large grid."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import delta, dst, grid, subdomain
from oracle.step import Oracle


def _dense_l5(n):
    m = n - 1
    a = np.zeros((m * m, m * m))
    for j in range(m):
        for i in range(m):
            r = j * m + i
            a[r, r] = 4.0
            for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                jj, ii = j + dj, i + di
                if 0 <= jj < m and 0 <= ii < m:
                    a[r, jj * m + ii] = -1.0
    return a


def _small_problem(with_beam=False):
    n = 16
    flow = W.Flow(n=n, levels=1, h=0.1, dt=0.02, re=50.0, cx=0.0, cy=0.0, u_inf=(1.0, 0.2))
    rng = np.random.default_rng(11)
    w0 = [0.5 * rng.normal(size=(n - 1, n - 1))]
    rigid = W.Rigid(xy=np.array([[0.25, 0.3], [0.3, 0.33], [0.35, 0.3], [0.31, 0.24]]), ds=0.06)
    bodies = [rigid]
    if with_beam:
        m = 5
        xy = np.stack([-0.35 + 0.1 * np.arange(m), -0.25 + 0 * np.arange(m)], axis=1)
        def_xy = xy + np.stack([0 * xy[:, 0], 0.2 * (xy[:, 0] + 0.35) ** 2], axis=1)
        bodies.append(W.Deformable(xy_ref=xy, mass=0.3, ei=0.05, ea=20.0, xy0=def_xy,
                                   rot0=np.arctan(0.4 * (xy[:, 0] + 0.35))))
    else:
        bodies.append(W.Torsional(n=6, hinge=(-0.3, -0.2), length=0.5, theta0=0.4, inertia=0.7,
                                  stiffness=2.0, damping=0.1, theta=0.05, phi=0.3))
    return W.Problem("small", flow, bodies, None, w0, 1)


@pytest.mark.parametrize("with_beam", [False, True])
def test_block_lu_equals_dense_coupled_solve(with_beam):
    """Appendix A eq. (A.17) with the interpolation at the current iterate, assembled
    densely and solved by LU, equals one FSI iteration of the factored path."""
    p = _small_problem(with_beam)
    o = Oracle(p, fixed_iters=1, subdomain_mode=False)
    lv = o.levels[0]
    n, h, dt, alpha = lv.n, lv.h, lv.dt, lv.alpha
    # explicit right-hand side (first step: AB2 uses N_0 twice), computed directly
    s0 = o.s[0].copy()
    gam = grid.pad(grid.l5(s0))
    qx, qy = lv.flux(s0)
    ctn = grid.curl_t_nonlinear(*grid.nonlinear(qx, qy, gam, h))
    r = (gam[1:-1, 1:-1] - alpha * grid.l5(gam) + dt * ctn).ravel()
    kinds = [k for k, _ in o.bodies]
    struct = o.bodies[1][1]
    pos = [o.bodies[0][1].xy,
           struct.positions(struct.theta if kinds[1] == "torsional" else struct.chi)]
    e = np.vstack([delta.interpolation_matrix(lv, x).toarray() for x in pos])
    ds = o.ds_vector()
    c = grid.dense_curl(n)
    lap = _dense_l5(n)
    m = (n - 1) ** 2
    nf = e.shape[0]
    qinf = grid.flatten_faces(np.full((n, n + 1), lv.u_inf[0] * h), np.full((n + 1, n), lv.u_inf[1] * h))
    nr = 8
    if kinds[1] == "torsional":
        nst = 2
        tot = m + nst + nf
        a = np.zeros((tot, tot))
        b = np.zeros(tot)
        a[:m, :m] = (np.eye(m) + alpha * lap) @ lap
        a[:m, m + nst:] = dt / h * c.T @ e.T @ np.diag(ds)
        b[:m] = r
        srow = struct.s_row(struct.theta)
        jt = struct.jac()
        ft = slice(m + nst + nr, m + nst + nf)
        a[m, m] = jt
        a[m, ft] = -struct.ds * srow
        b[m] = struct.r_phi()
        a[m + 1, m] = 2.0 / dt
        a[m + 1, m + 1] = -1.0
        b[m + 1] = struct.r_theta()
        a[m + nst:, :m] = e @ c / h
        a[m + nst + nr:, m + 1] = -srow
        b[m + nst:] = -(e @ qinf) / h
        x = np.linalg.solve(a, b)
        o.step()
        np.testing.assert_allclose(o.bodies[1][1].theta, x[m], rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(o.bodies[1][1].phi, x[m + 1], rtol=1e-10, atol=1e-12)
    else:
        jd, res = struct.jacobian(struct.chi)
        t = struct.t_matrix()
        nd = jd.shape[0]
        tot = m + nd + nf
        a = np.zeros((tot, tot))
        b = np.zeros(tot)
        a[:m, :m] = (np.eye(m) + alpha * lap) @ lap
        a[:m, m + nd:] = dt / h * c.T @ e.T @ np.diag(ds)
        b[:m] = r
        fd = slice(m + nd + nr, m + nd + nf)
        a[m:m + nd, m:m + nd] = jd
        a[m:m + nd, fd] = -struct.ds * t.T
        b[m:m + nd] = res
        a[m + nd:, :m] = e @ c / h
        a[m + nd + nr:, m:m + nd] = -(2.0 / dt) * t
        b[m + nd:] = -(e @ qinf) / h
        b[m + nd + nr:] += t @ ((2.0 / dt) * struct.chi[struct.free] - struct.r_chi()[struct.free])
        x = np.linalg.solve(a, b)
        chi_before = struct.chi.copy()
        o.step()
        np.testing.assert_allclose(o.bodies[1][1].chi[struct.free] - chi_before[struct.free],
                                   x[m:m + nd], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(o.f, x[-nf:], rtol=1e-9, atol=1e-10 * np.abs(x[-nf:]).max())
    np.testing.assert_allclose(o.s[0][1:-1, 1:-1].ravel(), x[:m], rtol=1e-9,
                               atol=1e-11 * np.abs(x[:m]).max())


def test_noslip_residual_exact_mode():
    p = W.cylinder_problem(n=32, steps=2)
    o = Oracle(p)
    for _ in range(2):
        o.step()
        assert o.noslip_residual() < 1e-12


def test_noslip_residual_moving_exact_mode():
    o = Oracle(_small_problem(), subdomain_mode=False, newton_tol=1e-13)
    for _ in range(2):
        o.step()
        assert o.noslip_residual() < 1e-11


def test_stationary_schur_block_is_spd():
    p = W.cylinder_problem(n=32, steps=1)
    o = Oracle(p)
    o.prepare()
    g = o.g_static
    assert np.max(np.abs(g - g.T)) < 1e-13 * np.max(np.abs(g))
    np.linalg.cholesky(g)


def _sd_level():
    return grid.Level(W.Flow(n=32, levels=1, h=0.1, dt=0.02, re=100.0), 0)


def test_b_symmetric_and_filter_limits():
    lv = _sd_level()
    pts = subdomain.point_set(lv, (-0.3, 0.3, -0.2, 0.2))
    e0 = subdomain.sub_e0(lv, pts)
    b = subdomain.build_b(lv, e0)
    assert np.max(np.abs(b - b.T)) < 1e-13 * np.max(np.abs(b))
    np.testing.assert_array_equal(subdomain.filter_b(b, 0.0), b.T * (b.T != 0))
    bf = subdomain.filter_b(b, 0.007)
    assert 0 < np.count_nonzero(bf) < b.size
    # every kept entry clears the threshold of its row's diagonal, every dropped one does not
    d = np.abs(np.diag(b))
    kept = bf != 0
    assert np.all(np.abs(b.T)[kept] > 0.007 * np.repeat(d, b.shape[0]).reshape(b.shape)[kept])
    assert np.all(np.abs(b.T)[~kept] <= 0.007 * np.repeat(d, b.shape[0]).reshape(b.shape)[~kept])


def test_hat_interpolation_bilinear_exact_and_second_order():
    lv = _sd_level()
    box = (-0.5, 0.5, -0.4, 0.4)
    pts = subdomain.point_set(lv, box)
    rng = np.random.default_rng(5)
    body = np.stack([rng.uniform(-0.45, 0.45, 9), rng.uniform(-0.35, 0.35, 9)], axis=1)
    nsd = pts.shape[0]
    rows = subdomain.hat_rows(lv, box, nsd, nsd, body, 0)[:, :nsd]
    f = 0.3 + 2 * pts[:, 0] - pts[:, 1] + 1.7 * pts[:, 0] * pts[:, 1]
    np.testing.assert_allclose(rows @ f, 0.3 + 2 * body[:, 0] - body[:, 1] + 1.7 * body[:, 0] * body[:, 1],
                               atol=1e-13)
    errs = []
    many = np.stack([rng.uniform(-0.45, 0.45, 2000), rng.uniform(-0.35, 0.35, 2000)], axis=1)
    for hh in (0.1, 0.05):
        lv2 = grid.Level(W.Flow(n=int(round(3.2 / hh)), levels=1, h=hh, dt=0.02, re=100.0), 0)
        pts2 = subdomain.point_set(lv2, box)
        ns2 = pts2.shape[0]
        rows2 = subdomain.hat_rows(lv2, box, ns2, ns2, many, 0)[:, :ns2]
        g = np.sin(2 * pts2[:, 0]) * np.cos(3 * pts2[:, 1])
        err = rows2 @ g - np.sin(2 * many[:, 0]) * np.cos(3 * many[:, 1])
        errs.append(np.sqrt(np.mean(err ** 2)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_subdomain_without_filter_on_vertices_equals_exact():
    """eps = 0 and body points on sub-domain vertices: P E0 = E and P B P^T = E C K C^T E^T,
    so one step of both modes agrees to round-off."""
    flow = W.Flow(n=32, levels=1, h=0.1, dt=0.02, re=100.0, u_inf=(1.0, 0.0))
    rng = np.random.default_rng(6)
    w0 = [0.3 * rng.normal(size=(31, 31))]
    body = W.Torsional(n=4, hinge=(-0.2, 0.0), length=0.6, theta0=0.0, inertia=1.0,
                       stiffness=1.0, damping=0.0)
    p = W.Problem("v", flow, [body], (-0.4, 0.6, -0.3, 0.3), w0, 1)
    a = Oracle(p, fixed_iters=1, drop_tol=0.0, subdomain_mode=True)
    b = Oracle(p, fixed_iters=1, subdomain_mode=False)
    a.step()
    b.step()
    np.testing.assert_allclose(a.f, b.f, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(a.s[0], b.s[0], atol=1e-12)


def test_multidomain_matches_single_large_grid():
    """A compact vortex advected for a few steps: the level-0 vorticity of a 3-level
    32^2 hierarchy matches one 128^2 grid spanning the coarsest extent at level-0
    spacing (the nested levels only coarsen the far field)."""
    h, dt, re = 0.1, 0.02, 200.0
    nc = 32
    x = -0.5 * nc * h + h * np.arange(1, nc)
    yy, xx = np.meshgrid(x, x, indexing="ij")
    w = 5.0 * np.exp(-((xx + 0.3) ** 2 + yy ** 2) / 0.1)
    small = W.Problem("md", W.Flow(n=nc, levels=3, h=h, dt=dt, re=re, u_inf=(1.0, 0.0)), [],
                      vorticity0=[w, None, None])
    nb = 4 * nc
    xb = -0.5 * nb * h + h * np.arange(1, nb)
    yyb, xxb = np.meshgrid(xb, xb, indexing="ij")
    wb = 5.0 * np.exp(-((xxb + 0.3) ** 2 + yyb ** 2) / 0.1)
    big = W.Problem("big", W.Flow(n=nb, levels=1, h=h, dt=dt, re=re, u_inf=(1.0, 0.0)), [],
                    vorticity0=[wb])
    a, b = Oracle(small), Oracle(big)
    for _ in range(5):
        a.step()
        b.step()
    wa = a.vorticity(0)
    c0 = (nb - nc) // 2
    wbig = b.vorticity(0)[c0:c0 + nc - 1, c0:c0 + nc - 1]
    rel = np.linalg.norm(wa - wbig) / np.linalg.norm(wbig)
    assert rel < 2e-3, rel


def test_fsi_iterations_and_converged_residual():
    """FSI iterations stay within a few per step (Sec. 5 reports at most 3), and the
    converged state satisfies the torsional equation (A.10) with the final stresses."""
    p = W.plate_problem(n=32, levels=2, steps=3)
    o = Oracle(p, newton_tol=1e-10)
    for _ in range(3):
        o.step()
        assert o.last_iters <= 6
    b = o.bodies[0][1]
    assert o.last_delta <= 1e-10
