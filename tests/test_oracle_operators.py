"""Pins of the oracle's flow operators against the mathematics and the paper.

Each test checks an oracle function against something other than itself: a dense
assembly, a closed form, a value printed in the paper, or a convergence order.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import delta, dst, grid, multidomain as md

import json
import os

PAPER = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def dense_l5(n):
    """5-point Laplacian on the interior by its stencil, assembled entry by entry."""
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


@pytest.mark.parametrize("n", [8, 12])
def test_ctc_is_five_point_laplacian(n):
    c = grid.dense_curl(n)
    np.testing.assert_allclose(c.T @ c, dense_l5(n), atol=1e-14)


@pytest.mark.parametrize("n", [8, 16])
def test_curl_transpose_is_adjoint(n):
    rng = np.random.default_rng(0)
    c = grid.dense_curl(n)
    nqx, nqy = grid.face_count(n)
    q = rng.normal(size=nqx + nqy)
    s = rng.normal(size=(n - 1) ** 2)
    lhs = q @ (c @ s)
    qx, qy = grid.unflatten_faces(q, n)
    rhs = grid.curl_t(qx, qy).ravel() @ s
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("n", [8, 16, 20])
def test_laplacian_eigenvalues_closed_form(n):
    ev = np.sort(np.linalg.eigvalsh(dense_l5(n)))
    closed = np.sort(dst.eigenvalues(n).ravel())
    np.testing.assert_allclose(ev, closed, atol=1e-13)


@pytest.mark.parametrize("n", [8, 16, 20, 24])
def test_sine_matrix_orthonormal_and_involutory(n):
    s = dst.sine_matrix(n)
    np.testing.assert_allclose(s @ s, np.eye(n - 1), atol=1e-14)
    np.testing.assert_allclose(s, s.T, atol=0)


@pytest.mark.parametrize("n", [8, 16])
def test_sine_transform_diagonalises_laplacian(n):
    s = dst.sine_matrix(n)
    s2 = np.kron(s, s)
    d = s2 @ dense_l5(n) @ s2
    np.testing.assert_allclose(d, np.diag(dst.eigenvalues(n).ravel()), atol=1e-12)


@pytest.mark.parametrize("n,alpha", [(8, 0.05), (16, 0.3), (20, 0.1)])
def test_cac_solve_matches_dense_solve(n, alpha):
    """(C^T A C) from the dense curl and A = I/dt + C C^T/(2 Re h^2) (Sec. 2.2),
    solved by LU; the oracle uses the sine diagonalisation (Sec. 3.2.1)."""
    c = grid.dense_curl(n)
    dt, re, h = 0.01, 7.0, math.sqrt(0.01 / (2 * 7.0 * alpha))
    lap_vec = -c @ c.T / (re * h * h)
    amat = np.eye(c.shape[0]) / dt - 0.5 * lap_vec
    cac = c.T @ amat @ c
    rng = np.random.default_rng(1)
    r = rng.normal(size=(n - 1, n - 1))
    ref = np.linalg.solve(cac, r.ravel()).reshape(n - 1, n - 1)
    got = dt * dst.solve_cac(r, alpha)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_single_mode_solve():
    n, alpha = 16, 0.2
    s = dst.sine_matrix(n)
    k, l = 3, 5
    mode = np.outer(s[:, l - 1], s[:, k - 1])
    lam = 4 * math.sin(math.pi * k / (2 * n)) ** 2 + 4 * math.sin(math.pi * l / (2 * n)) ** 2
    np.testing.assert_allclose(dst.solve_cac(mode, alpha), mode / (lam * (1 + alpha * lam)), atol=1e-14)


def test_condition_number_near_two():
    """Sec. 3.2.1: alpha = 0.125 gives cond(I + alpha Lambda) of about 2."""
    ref = PAPER["condition_number"]
    lam = dst.eigenvalues(512)
    v = 1.0 + ref["alpha"] * lam
    assert abs(v.max() / v.min() - ref["value"]) < 1e-3


def test_sparsity_of_sine_cosine_product():
    """Sec. 3.2.1, Fig. (sparsity): column 250 of |S_x C_x^T| on a 500 grid keeps about
    60 entries at a relative drop tolerance of 1e-2 (the discrete part relative to 1)."""
    n = 500
    j = np.arange(1, n)
    s = math.sqrt(2.0 / n) * np.sin(math.pi * np.outer(j, j) / n)        # DST-I, size n-1
    i = np.arange(n)
    c = math.sqrt(2.0 / n) * np.cos(math.pi * np.outer(i + 0.5, j) / n)  # DCT-II without the constant
    ref = PAPER["sparsity_column_nnz"]
    prod = np.abs(s @ c.T)
    kept = int(np.sum(prod[:, ref["column"] - 1] > ref["tolerance"]))
    assert abs(kept - ref["value"]) <= 10, kept


def test_free_stream_preserved_exactly():
    """No vorticity and no body: the discrete step keeps s = 0 exactly, on all levels."""
    from oracle.step import Oracle
    p = W.Problem("fs", W.Flow(n=16, levels=3, h=0.1, dt=0.02, re=100.0, u_inf=(1.0, 0.3)), [])
    o = Oracle(p)
    for _ in range(3):
        o.step()
    for s in o.s:
        assert np.all(s == 0.0)


def test_crank_nicolson_mode_factor():
    """U = 0, one small sine mode of gamma, one level: every step multiplies it by
    (1 - alpha lam) / (1 + alpha lam) (nonlinear term is O(amplitude^2))."""
    from oracle.step import Oracle
    n, amp = 16, 1e-7
    flow = W.Flow(n=n, levels=1, h=0.1, dt=0.05, re=10.0, u_inf=(0.0, 0.0))
    s = dst.sine_matrix(n)
    k, l = 2, 3
    mode = np.outer(s[:, l - 1], s[:, k - 1])
    h = flow.h
    p = W.Problem("cn", flow, [], vorticity0=[amp * mode / (h * h)])
    o = Oracle(p)
    alpha = flow.dt / (2 * flow.re * h * h)
    lam = 4 * math.sin(math.pi * k / (2 * n)) ** 2 + 4 * math.sin(math.pi * l / (2 * n)) ** 2
    fac = (1 - alpha * lam) / (1 + alpha * lam)
    g0 = grid.l5(o.s[0])
    for step in range(1, 4):
        o.step()
        np.testing.assert_allclose(grid.l5(o.s[0]), g0 * fac ** step, atol=1e-12 * amp)


def _advection_error(n):
    """|C^T N / h^2 + u . grad(omega)| at interior vertices for an analytic field."""
    lv = grid.Level(W.Flow(n=n, levels=1, h=2.0 / n, dt=0.01, re=1.0, cx=0.0, cy=0.0,
                           u_inf=(0.7, 0.2)), 0)
    x = lv.x0 + lv.h * np.arange(n + 1)
    y = lv.y0 + lv.h * np.arange(n + 1)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    sig2 = 0.08
    s = np.exp(-(xx ** 2 + 1.3 * yy ** 2) / sig2)
    # analytic derivatives of s = exp(-q/sig2), q = x^2 + 1.3 y^2
    sx = -2 * xx / sig2 * s
    sy = -2.6 * yy / sig2 * s
    sxx = (4 * xx ** 2 / sig2 ** 2 - 2 / sig2) * s
    syy = (6.76 * yy ** 2 / sig2 ** 2 - 2.6 / sig2) * s
    omega = -(sxx + syy)
    # d omega / dx, d omega / dy analytically
    sxxx = (-8 * xx ** 3 / sig2 ** 3 + 12 * xx / sig2 ** 2) * s
    syyx = (6.76 * yy ** 2 / sig2 ** 2 - 2.6 / sig2) * (-2 * xx / sig2) * s
    sxxy = (4 * xx ** 2 / sig2 ** 2 - 2 / sig2) * (-2.6 * yy / sig2) * s
    syyy = (-2.6 ** 3 * yy ** 3 / sig2 ** 3 + 3 * 2.6 ** 2 * yy / sig2 ** 2) * s
    wx = -(sxxx + syyx)
    wy = -(sxxy + syyy)
    u = sy + 0.7
    v = -sx + 0.2
    exact = -(u * wx + v * wy)[1:-1, 1:-1]
    gam = grid.pad(grid.l5(s), grid.ring_only(lv.h ** 2 * omega))
    qx, qy = lv.flux(s)
    got = grid.curl_t_nonlinear(*grid.nonlinear(qx, qy, gam, lv.h)) / lv.h ** 2
    return np.max(np.abs(got - exact)) / np.max(np.abs(exact))


def test_nonlinear_term_second_order():
    e1, e2 = _advection_error(64), _advection_error(128)
    assert e2 < 0.02
    assert 3.3 < e1 / e2 < 4.7, (e1, e2)


def test_roma_kernel_moments():
    rng = np.random.default_rng(2)
    for shift in rng.uniform(-0.5, 0.5, size=20):
        r = np.arange(-3, 4) - shift
        w = delta.roma3(r)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((r * w).sum()) < 1e-14
        assert abs((w * w).sum() - 0.5) < 1e-14


def test_peskin_kernel_moments():
    """Peskin's 4-point kernel: for any shift the weights sum to 1, have zero first moment,
    split evenly between even and odd offsets (1/2 each), and their squares sum to 3/8."""
    rng = np.random.default_rng(4)
    for shift in rng.uniform(-0.5, 0.5, size=20):
        j = np.arange(-4, 5)
        r = j - shift
        w = delta.peskin4(r)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((r * w).sum()) < 1e-14
        assert abs(w[j % 2 == 0].sum() - 0.5) < 1e-14
        assert abs((w * w).sum() - 0.375) < 1e-14
    assert delta.peskin4(np.array([2.0, -2.0, 2.5]))[:].max() == 0.0
    np.testing.assert_allclose(delta.peskin4(np.array([0.0, 1.0])), [0.5, 0.25], atol=1e-15)


@pytest.mark.parametrize("kernel", ["roma3", "peskin4"])
def test_interpolation_reproduces_linear_fields_and_conserves_force(kernel):
    lv = grid.Level(W.Flow(n=32, levels=1, h=0.1, dt=0.01, re=1.0), 0)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-0.8, 0.8, size=(7, 2))
    e = delta.interpolation_matrix(lv, pts, kernel)
    (xfx, xfy), (yfx, yfy) = lv.face_coords()
    ux = 0.3 + 1.1 * xfx[None, :] - 0.7 * xfy[:, None]
    uy = -0.2 + 0.4 * yfx[None, :] + 0.9 * yfy[:, None]
    u = e @ grid.flatten_faces(ux, uy)
    np.testing.assert_allclose(u[:7], 0.3 + 1.1 * pts[:, 0] - 0.7 * pts[:, 1], atol=1e-13)
    np.testing.assert_allclose(u[7:], -0.2 + 0.4 * pts[:, 0] + 0.9 * pts[:, 1], atol=1e-13)
    lam = rng.normal(size=14)
    qx, qy = grid.unflatten_faces(e.T @ lam, 32)
    assert abs(qx.sum() - lam[:7].sum()) < 1e-13
    assert abs(qy.sum() - lam[7:].sum()) < 1e-13


def test_support_check_rejects_points_near_the_edge():
    lv = grid.Level(W.Flow(n=16, levels=1, h=0.1, dt=0.01, re=1.0), 0)
    e = delta.interpolation_matrix(lv, np.array([[0.0, 0.0]]))
    delta.check_support(lv, e)
    e = delta.interpolation_matrix(lv, np.array([[0.75, 0.0]]))
    with pytest.raises(ValueError):
        delta.check_support(lv, e)
    # the 4-point kernel reaches half a cell further: accepted with the 3-point one only
    e = delta.interpolation_matrix(lv, np.array([[0.6, 0.0]]))
    delta.check_support(lv, e)
    e = delta.interpolation_matrix(lv, np.array([[0.6, 0.0]]), "peskin4")
    with pytest.raises(ValueError):
        delta.check_support(lv, e)


def test_ring_interpolation_exact_for_cubics():
    n = 16
    pts = np.arange(n + 1)
    for f in (lambda x, y: 1 + 0 * x, lambda x, y: x * x * x - 2 * y * y + x * y,
              lambda x, y: 0.3 * y ** 3 - x):
        yy, xx = np.meshgrid(pts * 2.0, pts * 2.0, indexing="ij")   # coarse coordinates
        vc = f(xx, yy)
        ring = md.ring_from_coarse(vc, n)
        yyf, xxf = np.meshgrid(pts + n / 2, pts + n / 2, indexing="ij")
        ref = f(xxf, yyf)
        mask = np.ones_like(ring, dtype=bool)
        mask[1:-1, 1:-1] = False
        np.testing.assert_allclose(ring[mask], ref[mask], atol=1e-10)


# ---- extended precision (numpy.longdouble, 64-bit significand: eps = 2^-63 ~ 1.1e-19) ----

LD = np.longdouble
EPS_LD = float(np.finfo(LD).eps)


def test_longdouble_is_wider_than_double():
    assert EPS_LD < 1e-18


@pytest.mark.parametrize("n", [16, 64, 96])
def test_extended_sine_transform_equals_dense_extended_matrix(n):
    """The library DST-I used in extended precision equals the dense orthonormal sine matrix
    S[j-1, k-1] = sqrt(2/n) sin(pi j k / n) built and multiplied in long double, and S S = I
    there (Sec. 3.2.1).  A transform done in double anywhere would miss by ~1e-16."""
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n - 1, n - 1)).astype(LD)
    s = dst.sine_matrix(n, LD)
    assert s.dtype == LD
    dense = s @ x @ s
    fast = dst.dst2(x)
    assert fast.dtype == LD
    assert float(np.max(np.abs(fast - dense))) < 100 * EPS_LD * float(np.max(np.abs(dense)))
    eye = s @ s
    assert float(np.max(np.abs(eye - np.eye(n - 1, dtype=LD)))) < 50 * EPS_LD


@pytest.mark.parametrize("n", [32, 96])
def test_extended_eigenvalues_closed_form(n):
    """In long double, the 5-point stencil applied to a sine mode returns the mode times
    4 sin^2(pi k/2n) + 4 sin^2(pi l/2n) (the diagonalisation of C^T C, Sec. 3.2.1)."""
    k, l = 3, n // 3
    s = dst.sine_matrix(n, LD)
    mode = np.outer(s[:, l - 1], s[:, k - 1])
    lam = dst.eigenvalues(n, LD)[l - 1, k - 1]
    res = grid.l5(grid.pad(mode)) - lam * mode
    assert float(np.max(np.abs(res))) < 50 * EPS_LD * float(np.max(np.abs(mode)))


def test_extended_solve_residual():
    """The extended-precision solve of L (I + alpha L) s = r leaves a long-double residual
    when the operator is applied back by its stencils."""
    n, alpha = 48, 0.31
    rng = np.random.default_rng(3)
    r = rng.normal(size=(n - 1, n - 1)).astype(LD)
    x = dst.solve_cac(r, alpha)
    lx = grid.l5(grid.pad(x))
    back = lx + alpha * grid.l5(grid.pad(lx))
    assert float(np.max(np.abs(back - r))) < 1e3 * EPS_LD * float(np.max(np.abs(r)))


def _smooth_flow(n, levels):
    flow = W.Flow(n=n, levels=levels, h=3.2 / n, dt=0.2 * 3.2 / n, re=150.0, cx=0.1, cy=-0.05,
                  u_inf=(1.0, 0.3))
    x = flow.cx - 0.5 * n * flow.h + flow.h * np.arange(1, n)
    y = flow.cy - 0.5 * n * flow.h + flow.h * np.arange(1, n)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    rng = np.random.default_rng(7)
    w = 4.0 * np.exp(-((xx + 0.2) ** 2 + (yy - 0.1) ** 2) / 0.08) + 0.05 * rng.normal(size=xx.shape)
    return W.Problem("flow", flow, [], vorticity0=[w] + [None] * (levels - 1))


def test_extended_oracle_agrees_with_double_where_double_is_accurate():
    """One level (no circulation handed between levels): the double oracle holds s to a few
    ulps, so the extended run agrees with it to 1e-14 in s; its vorticity, C^T C s, to the
    (n/pi)^2 / 2 amplified double rounding.  Every array of the extended run stays long
    double."""
    from oracle.step import Oracle
    p = _smooth_flow(64, 1)
    a, b = Oracle(p), Oracle(p, dtype=LD)
    for _ in range(3):
        a.step()
        b.step()
    assert b.s[0].dtype == LD and b.vorticity(0).dtype == LD
    es = float(np.linalg.norm((a.s[0] - b.s[0]).astype(np.float64)) / np.linalg.norm(a.s[0]))
    ew = float(np.linalg.norm((a.vorticity(0) - b.vorticity(0)).astype(np.float64))
               / np.linalg.norm(a.vorticity(0)))
    assert es < 1e-14, es
    assert ew < 40 * 2.0 ** -52 * 0.5 * (64 / math.pi) ** 2, ew


def test_extended_oracle_rejects_bodies():
    from oracle.step import Oracle
    with pytest.raises(ValueError):
        Oracle(W.cylinder_problem(n=32, steps=1), dtype=LD)
