"""Pins of the oracle on rectangular levels (nx cells along x, ny along y), CPU only.

The paper's largest run (Sec. 5.3) uses levels of 4000 x 2000 cells; the operators of Sec. 3.2.1
are the same on a rectangle, with one sine transform per axis: C^T C = (S_y (x) S_x)
diag(lam_x + lam_y) (S_y (x) S_x).  These tests pin the oracle's rectangular form to closed forms,
to a dense solve, to a single large grid, and to the mirror symmetry of the equations.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dst, grid, multidomain as md
from oracle.step import Oracle


def test_sine_modes_are_eigenvectors_on_a_rectangle():
    """l5 of sin(pi k i / nx) sin(pi l j / ny) (zero ring) is (lam_x(k) + lam_y(l)) times it."""
    nx, ny = 12, 8
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    for k, l in ((1, 1), (3, 5), (11, 7), (6, 2)):
        mode = np.sin(np.pi * l * j / ny)[:, None] * np.sin(np.pi * k * i / nx)[None, :]
        lam = 4 * np.sin(np.pi * k / (2 * nx)) ** 2 + 4 * np.sin(np.pi * l / (2 * ny)) ** 2
        np.testing.assert_allclose(grid.l5(mode), lam * mode[1:-1, 1:-1], atol=1e-13)
        assert abs(dst.eigenvalues(nx, np.float64, ny)[l - 1, k - 1] - lam) < 1e-14


def test_rectangular_solve_matches_dense_solve():
    """[C^T C (I + alpha C^T C)]^{-1} r by the two sine transforms equals the dense solve."""
    nx, ny, alpha = 12, 8, 0.3
    m = (nx - 1) * (ny - 1)
    lmat = np.zeros((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        lmat[:, c] = grid.l5(grid.pad(e.reshape(ny - 1, nx - 1))).ravel()
    r = np.random.default_rng(0).normal(size=(ny - 1, nx - 1))
    want = np.linalg.solve(lmat @ (np.eye(m) + alpha * lmat), r.ravel()).reshape(ny - 1, nx - 1)
    np.testing.assert_allclose(dst.solve_cac(r, alpha), want, atol=1e-12)
    want_p = np.linalg.solve(lmat, r.ravel()).reshape(ny - 1, nx - 1)
    np.testing.assert_allclose(dst.solve_poisson(r), want_p, atol=1e-12)
    # the extended-precision path (library transforms) agrees
    ld = dst.solve_cac(r.astype(np.longdouble), alpha)
    np.testing.assert_allclose(ld.astype(np.float64), want, atol=1e-12)


def _vortex(nx, ny, h, x0, y0, width, amp=5.0):
    x = -0.5 * nx * h + h * np.arange(1, nx)
    y = -0.5 * ny * h + h * np.arange(1, ny)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    return amp * np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / width)


@pytest.mark.parametrize("nx,ny", [(32, 16), (16, 32)])
def test_rectangular_hierarchy_matches_single_large_grid(nx, ny):
    """A vortex advected for 5 steps on a 3-level nx x ny hierarchy (every level seeded from the
    same field) matches one 4nx x 4ny grid spanning the coarsest extent at level-0 spacing, on
    level 0 and, at their own vertices, on levels 1 and 2 (measured at most 0.1 %, 0.6 % and
    1.6 %).  With the ring's coarse lines or the coarsification window taken along the wrong
    axis the levels disagree."""
    h, dt, re = 0.1, 0.02, 200.0
    w = [_vortex(nx, ny, h * 2 ** g, -0.3, 0.1, 0.3) for g in range(3)]
    small = W.Problem("r", W.Flow(n=nx, ny=ny, levels=3, h=h, dt=dt, re=re, u_inf=(1.0, 0.0)), [],
                      vorticity0=w)
    bx, by = 4 * nx, 4 * ny
    big = W.Problem("b", W.Flow(n=bx, ny=by, levels=1, h=h, dt=dt, re=re, u_inf=(1.0, 0.0)), [],
                    vorticity0=[_vortex(bx, by, h, -0.3, 0.1, 0.3)])
    a, b = Oracle(small), Oracle(big)
    for _ in range(5):
        a.step()
        b.step()
    wb = b.vorticity(0)
    for g, bar in ((0, 2e-3), (1, 0.01), (2, 0.03)):
        st = 2 ** g                        # level-g vertex spacing in big-grid vertices
        cx, cy = (bx - st * nx) // 2, (by - st * ny) // 2
        ref = wb[cy + st - 1:cy + st * ny - 1:st, cx + st - 1:cx + st * nx - 1:st]
        wa = a.vorticity(g)
        assert wa.shape == ref.shape == (ny - 1, nx - 1)
        rel = np.linalg.norm(wa - ref) / np.linalg.norm(ref)
        assert rel < bar, (g, rel)


def test_transposed_problem_is_the_mirror_image():
    """Reflecting the plane across y = x maps vorticity to its negative and swaps the velocity
    components, so the nx x ny problem with vorticity w and free stream (1, 0) and the ny x nx
    problem with vorticity -w^T and free stream (0, 1) give s' = -s^T on every level.  Any
    place where the rectangular code uses nx for ny (or the reverse) breaks the mirror."""
    h, dt, re = 0.1, 0.02, 150.0
    nx, ny, levels = 24, 16, 3
    rng = np.random.default_rng(5)
    w = _vortex(nx, ny, h, -0.2, 0.15, 0.08) + 0.05 * rng.normal(size=(ny - 1, nx - 1))
    p = W.Problem("a", W.Flow(n=nx, ny=ny, levels=levels, h=h, dt=dt, re=re, u_inf=(1.0, 0.0)),
                  [], vorticity0=[w] + [None] * (levels - 1))
    q = W.Problem("b", W.Flow(n=ny, ny=nx, levels=levels, h=h, dt=dt, re=re, u_inf=(0.0, 1.0)),
                  [], vorticity0=[-w.T] + [None] * (levels - 1))
    a, b = Oracle(p), Oracle(q)
    for _ in range(4):
        a.step()
        b.step()
    for g in range(levels):
        scale = np.max(np.abs(a.s[g]))
        np.testing.assert_allclose(b.s[g], -a.s[g].T, atol=1e-12 * scale, rtol=0)


def test_square_given_as_rectangle_is_the_same():
    """ny = n equals the square default bit for bit."""
    h = 0.1
    w = _vortex(16, 16, h, 0.0, 0.0, 0.1)
    p = W.Problem("s", W.Flow(n=16, levels=2, h=h, dt=0.02, re=100.0), [], vorticity0=[w, None])
    q = W.Problem("r", W.Flow(n=16, ny=16, levels=2, h=h, dt=0.02, re=100.0), [],
                  vorticity0=[w, None])
    a, b = Oracle(p), Oracle(q)
    for _ in range(3):
        a.step()
        b.step()
    for g in range(2):
        assert np.array_equal(a.s[g], b.s[g])


def test_rectangular_levels_refuse_bodies():
    flow = W.Flow(n=32, ny=16, levels=1, h=0.1, dt=0.02, re=100.0)
    body = W.cylinder((0.0, 0.0), 0.5, 0.1)
    with pytest.raises(ValueError):
        Oracle(W.Problem("c", flow, [body]))


def test_ring_lines_follow_their_axes():
    """The fine ring reads the coarse rows ny/4, 3ny/4 for its bottom and top edges and the
    coarse columns nx/4, 3nx/4 for its left and right edges (linear data: exact)."""
    nx, ny = 16, 8
    jj, ii = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    coarse = 3.0 * ii + 7.0 * jj + 1.0          # coarse vertex (I, J) -> 3 I + 7 J + 1
    ring = md.ring_from_coarse(coarse, nx, ny)
    # fine vertex (i, j) sits at coarse ((i + nx/2) / 2, (j + ny/2) / 2)
    fine = 3.0 * (np.arange(nx + 1) + nx / 2) / 2
    np.testing.assert_allclose(ring[0, :], fine + 7.0 * (ny / 4) + 1.0)
    np.testing.assert_allclose(ring[ny, :], fine + 7.0 * (3 * ny / 4) + 1.0)
    fj = 7.0 * (np.arange(ny + 1) + ny / 2) / 2
    np.testing.assert_allclose(ring[:, 0], fj + 3.0 * (nx / 4) + 1.0)
    np.testing.assert_allclose(ring[:, nx], fj + 3.0 * (3 * nx / 4) + 1.0)
