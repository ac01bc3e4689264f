"""Staggered-grid streamfunction-vorticity operators on one level (FP64, test oracle).

Layout (a reading: the paper defers the grid to Taira & Colonius / Colonius & Taira):

* A level has ``nx`` cells along x, ``ny`` along y (``n`` when square) and spacing ``h``.
  Vertex (i, j), i = 0..nx, j = 0..ny, sits at (x0 + i h, y0 + j h) and carries the
  streamfunction s and the circulation gamma = h^2 * vorticity.  Arrays are indexed
  ``[j, i]`` (row = y).  The unknowns are the (ny-1)(nx-1) interior vertices; the outer
  ring holds boundary values.  The operators below work on either shape.
* x-faces (vertical cell edges) carry the flux qx = u h at (x_i, y_{j+1/2}):
  ``qx[j, i] = s[j+1, i] - s[j, i]``, shape (n, n+1).
* y-faces carry qy = v h at (x_{i+1/2}, y_j): ``qy[j, i] = -(s[j, i+1] - s[j, i])``,
  shape (n+1, n).
* C is the curl s -> q above; C^T q is the circulation about each interior vertex, so
  C^T C is the positive 5-point Laplacian ``l5`` (Sec. 3.2.1: C^T C is the scalar
  Laplacian diagonalised by sine transforms).
* The vector Laplacian acting on divergence-free fluxes is L = -C C^T / (Re h^2), so
  A = I/dt - L/2 (Sec. 2.2) gives C^T A C = (1/dt) C^T C (I + alpha C^T C) with
  alpha = dt / (2 Re h^2) (Sec. 3.2.1, eq. (30)).
* Nonlinear term (the paper does not spell it out, Appendix A eq. (A.1)): rotational
  form u x omega.  In flux units, on an x-face it is the average over the two end
  vertices of (vbar * gamma) / h^2, on a y-face minus the average of
  (ubar * gamma) / h^2, with vbar / ubar the mean of the two y- / x-face fluxes
  meeting at the vertex.  It enters the right-hand side as + C^T N.
"""
import numpy as np


def l5(v):
    """4 v - (sum of the 4 neighbours) at the interior vertices of an (n+1, n+1) array."""
    return (4.0 * v[1:-1, 1:-1] - v[1:-1, 2:] - v[1:-1, :-2]
            - v[2:, 1:-1] - v[:-2, 1:-1])


def pad(interior, ring=None):
    """(ny+1, nx+1) array from (ny-1, nx-1) interior values and (optionally) a full
    array whose outer ring supplies the boundary values."""
    my, mx = interior.shape
    out = np.zeros((my + 2, mx + 2), dtype=interior.dtype) if ring is None else ring.copy()
    out[1:-1, 1:-1] = interior
    return out


def ring_only(full):
    """Copy of ``full`` with the interior zeroed."""
    out = full.copy()
    out[1:-1, 1:-1] = 0.0
    return out


def curl(s):
    """C s for a full (n+1, n+1) streamfunction: fluxes (qx, qy)."""
    qx = s[1:, :] - s[:-1, :]
    qy = -(s[:, 1:] - s[:, :-1])
    return qx, qy


def curl_t(qx, qy):
    """C^T q: circulation about every interior vertex (counter-clockwise)."""
    return qy[1:-1, 1:] - qy[1:-1, :-1] - qx[1:, 1:-1] + qx[:-1, 1:-1]


def nonlinear(qx, qy, g, h):
    """Rotational-form advection term N(q) on the faces needed by C^T N.

    ``g`` is the (n+1, n+1) circulation including the ring.  Returns
    ``nx[j, i-1]`` for x-faces i = 1..n-1, j = 0..n-1 and ``ny[j-1, i]`` for
    y-faces j = 1..n-1, i = 0..n-1.
    """
    vbar = 0.5 * (qy[:, :-1] + qy[:, 1:])      # vertex (i = 1..n-1, all j): [j, i-1]
    ubar = 0.5 * (qx[:-1, :] + qx[1:, :])      # vertex (all i, j = 1..n-1): [j-1, i]
    pv = vbar * g[:, 1:-1]
    pu = ubar * g[1:-1, :]
    nx = 0.5 * (pv[:-1, :] + pv[1:, :]) / (h * h)
    ny = -0.5 * (pu[:, :-1] + pu[:, 1:]) / (h * h)
    return nx, ny


def curl_t_nonlinear(nx, ny):
    """C^T N for the face arrays returned by ``nonlinear``."""
    return ny[:, 1:] - ny[:, :-1] - nx[1:, :] + nx[:-1, :]


def face_count(n):
    return n * (n + 1), (n + 1) * n


def flatten_faces(qx, qy):
    return np.concatenate([qx.ravel(), qy.ravel()])


def unflatten_faces(q, n):
    nqx, _ = face_count(n)
    return q[:nqx].reshape(n, n + 1), q[nqx:].reshape(n + 1, n)


def dense_curl(n):
    """Dense C mapping the (n-1)^2 interior unknowns (row-major [j, i]) to the
    flattened faces, with a zero ring.  For tiny grids only."""
    m = (n - 1) * (n - 1)
    cols = []
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        qx, qy = curl(pad(e.reshape(n - 1, n - 1)))
        cols.append(flatten_faces(qx, qy))
    return np.array(cols).T


class Level:
    """Geometry of nested level g (0 = finest): spacing h * 2^g about a common centre."""

    def __init__(self, flow, g):
        self.g = g
        self.nx, self.ny = flow.n, (getattr(flow, "ny", 0) or flow.n)
        self.n = self.nx  # the body operators use square levels
        self.h = flow.h * (2 ** g)
        self.dt = flow.dt
        self.re = flow.re
        self.alpha = flow.dt / (2.0 * flow.re * self.h * self.h)
        self.x0 = flow.cx - 0.5 * self.nx * self.h
        self.y0 = flow.cy - 0.5 * self.ny * self.h
        self.u_inf = tuple(flow.u_inf)

    def face_coords(self):
        """Coordinates of x-faces (xs, ys) and y-faces, as broadcastable 1-D arrays."""
        n, h = self.n, self.h
        xf_x = self.x0 + h * np.arange(n + 1)           # x-face columns
        xf_y = self.y0 + h * (np.arange(n) + 0.5)       # x-face rows
        yf_x = self.x0 + h * (np.arange(n) + 0.5)       # y-face columns
        yf_y = self.y0 + h * np.arange(n + 1)           # y-face rows
        return (xf_x, xf_y), (yf_x, yf_y)

    def flux(self, s):
        """Total flux C s + q_inf (the free stream in flux units u_inf * h)."""
        qx, qy = curl(s)
        return qx + self.u_inf[0] * self.h, qy + self.u_inf[1] * self.h
