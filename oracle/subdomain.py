"""Sub-domain operators: E0, hat interpolation P, B and its drop-tolerance filter.

Sec. 3.1 (eqs. (22)-(29)): E ~= P E0 with E0 the IB interpolation at a fixed set of
sub-domain points and P a sparse interpolation onto the moving body points.
Sec. 3.1.1: sub-domain points are the vertices (vorticity points) of the finest
level inside a user rectangle.  Reading for several bodies far apart: the sub-domain may be
a union of rectangles (one per body, say); its points are the rectangles' vertex grids one
after another (row-major each, the rectangles in the order given), and each moving body is
interpolated through P on the first rectangle that contains it at the start.  Sec. 3.1.2: P uses the two-point hat
d_p(r) = 1 - |r|/dr with the 4 tensor neighbours (eq. (29)).  Sec. 5.2: exact body
points of stationary bodies may be appended to the sub-domain point set; reading:
each appended point is one more row/column of B and its body point takes P weight 1.

B = E0 C (C^T A C)^{-1} C^T E0^T is built column by column (eq. (35), Algorithm 1)
and filtered by eq. (34): b'_ij = b_ij if |b_ij| > eps |b_ii|, else 0.  Reading:
B is symmetric, so row i of B' is formed from column i of B with the threshold
eps |b_ii| of that same column; each column is then filtered on its own, as the
paper's column-by-column construction requires.  The stored value of b'_ij is the
entry (j, i) of the computed B.

Here B omits the scalar dt * ds / h^2 that turns it into the flow block of the Schur
matrix; ``step`` applies that factor.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import delta, dst, grid

TOL = 1e-9


def grid_points(level, box):
    """Vertex index range (i0, i1, j0, j1) of the smallest vertex rectangle that
    contains box = (x0, x1, y0, y1)."""
    x0, x1, y0, y1 = box
    h = level.h
    i0 = int(math.floor((x0 - level.x0) / h + TOL))
    i1 = int(math.ceil((x1 - level.x0) / h - TOL))
    j0 = int(math.floor((y0 - level.y0) / h + TOL))
    j1 = int(math.ceil((y1 - level.y0) / h - TOL))
    return i0, i1, j0, j1


def boxes_of(sub):
    """The rectangles of a sub-domain given as one (x0, x1, y0, y1) or a list of them."""
    if sub is None:
        return []
    if len(sub) == 4 and all(np.isscalar(v) for v in sub):
        return [tuple(float(v) for v in sub)]
    return [tuple(float(v) for v in b) for b in sub]


def box_offsets(level, boxes):
    """First sub-domain point of each rectangle and the total count of grid points."""
    offs, tot = [], 0
    for box in boxes:
        i0, i1, j0, j1 = grid_points(level, box)
        offs.append(tot)
        tot += (i1 - i0 + 1) * (j1 - j0 + 1)
    return offs, tot


def point_set(level, box, appended=None):
    """Coordinates of the sub-domain points: each rectangle's grid vertices row-major (y
    outer), rectangle after rectangle, followed by the appended exact points."""
    parts = []
    for b in boxes_of(box):
        i0, i1, j0, j1 = grid_points(level, b)
        ii, jj = np.meshgrid(np.arange(i0, i1 + 1), np.arange(j0, j1 + 1))
        parts.append(np.stack([level.x0 + ii.ravel() * level.h, level.y0 + jj.ravel() * level.h],
                              axis=1))
    pts = np.concatenate(parts, axis=0)
    if appended is not None and len(appended):
        pts = np.concatenate([pts, np.asarray(appended, dtype=np.float64)], axis=0)
    return pts


def box_containing(level, boxes, positions):
    """Index of the first rectangle whose vertex grid contains every point (the body's
    rectangle); ValueError when none does."""
    for k, box in enumerate(boxes):
        i0, i1, j0, j1 = grid_points(level, box)
        rx = (positions[:, 0] - (level.x0 + i0 * level.h)) / level.h
        ry = (positions[:, 1] - (level.y0 + j0 * level.h)) / level.h
        if (np.all(rx >= -TOL) and np.all(ry >= -TOL) and np.all(rx <= i1 - i0 + TOL)
                and np.all(ry <= j1 - j0 + TOL)):
            return k
    raise ValueError("body outside every sub-domain rectangle")


def apply_b_column(level, e0, col):
    """B e_col by the chain E0 C K C^T E0^T e_col, K = [C^T C (I + alpha C^T C)]^{-1}."""
    n = level.n
    lam = np.zeros(e0.shape[0])
    lam[col] = 1.0
    qx, qy = grid.unflatten_faces(e0.T @ lam, n)
    src = grid.curl_t(qx, qy)
    s = grid.pad(dst.solve_cac(src, level.alpha))
    qx, qy = grid.curl(s)
    return e0 @ grid.flatten_faces(qx, qy)


def build_b(level, e0):
    """Dense B, one column at a time (small problems only)."""
    m = e0.shape[0]
    return np.array([apply_b_column(level, e0, j) for j in range(m)]).T


def filter_b(b, eps):
    """B' as a dense array: row i keeps column i's entries above eps |b_ii|."""
    m = b.shape[0]
    out = np.zeros_like(b)
    for i in range(m):
        col = b[:, i]
        keep = np.abs(col) > eps * abs(b[i, i])
        out[i, keep] = col[keep]
    return out


def hat_rows(level, box, npts_grid, n_sd_total, positions, comp_offset, appended_index=None,
             box_offset=0):
    """Rows of P for one component of a body's points.

    ``positions`` (m, 2); ``comp_offset`` is 0 (x) or n_sd_total (y); ``box`` the body's
    rectangle, whose first grid point is ``box_offset``.  With ``appended_index`` (m,) the
    rows are unit rows on appended points instead.
    """
    m = positions.shape[0]
    rows = np.zeros((m, 2 * n_sd_total))
    if appended_index is not None:
        for a in range(m):
            rows[a, comp_offset + npts_grid + appended_index[a]] = 1.0
        return rows
    i0, i1, j0, j1 = grid_points(level, box)
    npx, npy = i1 - i0 + 1, j1 - j0 + 1
    xs0 = level.x0 + i0 * level.h
    ys0 = level.y0 + j0 * level.h
    for a in range(m):
        rx = (positions[a, 0] - xs0) / level.h
        ry = (positions[a, 1] - ys0) / level.h
        if rx < -TOL or ry < -TOL or rx > npx - 1 + TOL or ry > npy - 1 + TOL:
            raise ValueError("body point outside the sub-domain")
        ix = min(max(int(math.floor(rx)), 0), npx - 2)
        iy = min(max(int(math.floor(ry)), 0), npy - 2)
        fx, fy = rx - ix, ry - iy
        for dxi, wx in ((0, 1.0 - fx), (1, fx)):
            for dyi, wy in ((0, 1.0 - fy), (1, fy)):
                rows[a, comp_offset + box_offset + (iy + dyi) * npx + (ix + dxi)] += wx * wy
    return rows


def sub_e0(level, pts, kernel="roma3"):
    """E0 (2 n_sd x n_faces): x rows of all points, then y rows."""
    return delta.interpolation_matrix(level, pts, kernel)


def as_sparse(b):
    return sp.csr_matrix(b)
