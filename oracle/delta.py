"""Discrete delta functions and the IB interpolation E / regularisation E^T (FP64 oracle).

Sec. 3.1, eq. (24): E_ij = d(x_j - xi_i) d(y_j - eta_i).  The paper does not name the
kernel d; the reading adopted here is the 3-point kernel of Roma, Peskin & Berger
(1999) in grid units r = distance / h:

    d(r) = (1 + sqrt(1 - 3 r^2)) / 3                      |r| <= 1/2
    d(r) = (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6       1/2 <= |r| <= 3/2
    d(r) = 0                                              otherwise

Peskin's 4-point kernel (Peskin 2002) is the alternative, selected per problem:

    d(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8        |r| <= 1
    d(r) = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8       1 <= |r| <= 2
    d(r) = 0                                              otherwise

The scaling the paper leaves open ("to within a scaling factor") is fixed by the
physics: interpolated velocity = E q / h on the flux q = u h, and the body force
enters the circulation equation as C^T E^T (ds / h) f, which keeps the spread the
exact transpose of the interpolation.

E rows for a body point are ordered x-component (acting on x-faces) then
y-component (acting on y-faces); per body, all x rows precede all y rows.
"""
import numpy as np
import scipy.sparse as sp

from . import grid


def roma3(r):
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 0.5
    m2 = (a > 0.5) & (a <= 1.5)
    out[m1] = (1.0 + np.sqrt(1.0 - 3.0 * a[m1] ** 2)) / 3.0
    out[m2] = (5.0 - 3.0 * a[m2] - np.sqrt(np.maximum(0.0, 1.0 - 3.0 * (1.0 - a[m2]) ** 2))) / 6.0
    return out


def peskin4(r):
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a <= 2.0)
    out[m1] = (3.0 - 2.0 * a[m1] + np.sqrt(1.0 + 4.0 * a[m1] - 4.0 * a[m1] ** 2)) / 8.0
    out[m2] = (5.0 - 2.0 * a[m2] - np.sqrt(np.maximum(0.0, -7.0 + 12.0 * a[m2] - 4.0 * a[m2] ** 2))) / 8.0
    return out


KERNELS = {"roma3": roma3, "peskin4": peskin4}


def interpolation_matrix(level, points, kernel="roma3"):
    """Sparse E (2 m x n_faces) for m points (x rows then y rows), by the definition:
    the tensor product of the kernel over every face of the level."""
    phi = KERNELS[kernel]
    (xfx, xfy), (yfx, yfy) = level.face_coords()
    h = level.h
    n = level.n
    nqx, nqy = grid.face_count(n)
    m = points.shape[0]
    rows, cols, vals = [], [], []
    for a in range(m):
        px, py = points[a]
        wx = phi((xfx - px) / h)
        wy = phi((xfy - py) / h)
        w = np.outer(wy, wx)                     # x-faces [j, i]
        jj, ii = np.nonzero(w)
        rows.append(np.full(jj.size, a))
        cols.append(jj * (n + 1) + ii)
        vals.append(w[jj, ii])
        wx = phi((yfx - px) / h)
        wy = phi((yfy - py) / h)
        w = np.outer(wy, wx)                     # y-faces [j, i]
        jj, ii = np.nonzero(w)
        rows.append(np.full(jj.size, m + a))
        cols.append(nqx + jj * n + ii)
        vals.append(w[jj, ii])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * m, nqx + nqy))


def reorder_rows_per_body(counts):
    """Row permutation from (all x rows, all y rows) to per-body (x block, y block)."""
    total = sum(counts)
    perm = []
    start = 0
    for c in counts:
        perm.extend(range(start, start + c))
        perm.extend(range(total + start, total + start + c))
        start += c
    return np.array(perm, dtype=np.int64)


def check_support(level, e):
    """The faces touched by E must have both end vertices in the level interior, so
    that the regularised force acts on unknowns only (the support stays at least
    about two cells away from the level edge).  Raises ValueError otherwise."""
    n = level.n
    nqx, _ = grid.face_count(n)
    cols = np.unique(e.indices)
    cx = cols[cols < nqx]
    jx, ix = cx // (n + 1), cx % (n + 1)
    cy = cols[cols >= nqx] - nqx
    jy, iy = cy // n, cy % n
    ok = (np.all((ix >= 1) & (ix <= n - 1) & (jx >= 1) & (jx <= n - 2))
          and np.all((iy >= 1) & (iy <= n - 2) & (jy >= 1) & (jy <= n - 1)))
    if not ok:
        raise ValueError("delta support reaches the level boundary")
