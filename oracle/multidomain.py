"""Nested-level ("multi-domain") far-field treatment (FP64 oracle).

Sec. 5 uses a hierarchy of grids of increasing coarseness with zero vorticity at the
far boundary and refers to Colonius & Taira (2008) for the details, which the paper
does not give.  The reading adopted here:

1. Level g has the same nx x ny cells as level 0, spacing h 2^g, and all levels
   share one centre, so the coarse vertex (I, J) of level g+1 coincides with the fine
   vertex (2I - nx/2, 2J - ny/2) of level g (nx and ny divisible by 4).
2. The coarsest level has s = gamma = 0 on its boundary ring.
3. Levels are advanced coarse to fine.  The ring of level g at the new time is
   taken from level g+1's new streamfunction: coincident vertices are copied and the
   midpoints along the ring use the 4-point cubic (-1, 9, 9, -1)/16.  The ring
   circulation is interpolated the same way from the coarse circulation C^T C s
   and rescaled by (h_g / h_{g+1})^2 = 1/4.  Both new rings are lifted into the
   right-hand side of the level's solve.
4. Coarsification on read: where a coarse interior vertex coincides with an interior
   vertex of the next finer level, the coarse right-hand side uses the finer level's
   circulation at the old time (times 4) instead of its own; the coarse velocity is
   left as is.  No extra solve is spent on coarse levels.
5. The body forcing acts on level 0 only; its corrector uses homogeneous boundary
   values on level 0 (the ring is fixed by level 1).
"""
import numpy as np

from . import grid


def ring_from_coarse(vc, n, ny=None):
    """Ring values of a fine level from the coarse full array ``vc`` (ny+1, nx+1), nx = n.

    Returns an (ny+1, nx+1) array holding only the fine ring.  Along the bottom and top
    edges the fine index i maps to the coarse (i + nx/2) / 2 on the coarse rows ny/4 and
    3 ny/4; along the left and right edges the fine j maps to (j + ny/2) / 2 on the coarse
    columns nx/4 and 3 nx/4.
    """
    nx, ny = n, (n if ny is None else ny)
    out = np.zeros((ny + 1, nx + 1), dtype=vc.dtype)

    def along(line, i, q):
        # value at fine index i along a coarse line; fine i <-> coarse (i + q) / 2
        if (i + q) % 2 == 0:
            return line[(i + q) // 2]
        c = (i + q - 1) // 2
        return (-line[c - 1] + 9.0 * line[c] + 9.0 * line[c + 1] - line[c + 2]) / 16.0

    qx, qy = nx // 2, ny // 2
    jb, jt = qy // 2, (ny + qy) // 2        # coarse rows of the fine bottom / top edges
    ib, it = qx // 2, (nx + qx) // 2        # coarse columns of the fine left / right edges
    for i in range(nx + 1):
        out[0, i] = along(vc[jb, :], i, qx)
        out[ny, i] = along(vc[jt, :], i, qx)
    for j in range(ny + 1):
        out[j, 0] = along(vc[:, ib], j, qy)
        out[j, nx] = along(vc[:, it], j, qy)
    return out


def coarse_circulation(s_coarse):
    """Full (ny+1, nx+1) circulation of a level from its own streamfunction (ring = 0;
    only interior vertices are used by ``ring_from_coarse``)."""
    return grid.pad(grid.l5(s_coarse))


def circulation_for_rhs(s, g_ring, s_finer):
    """Circulation used by a level's explicit right-hand side at the old time.

    Interior: C^T C s, except at vertices coinciding with an interior vertex of the
    next finer level, where 4 (C^T C s_finer) is used.  Ring: the stored ring
    values ``g_ring`` (an (ny+1, nx+1) array whose ring is used).
    """
    ny, nx = s.shape[0] - 1, s.shape[1] - 1
    g = grid.pad(grid.l5(s), g_ring)
    if s_finer is not None:
        gf = grid.l5(s_finer)              # fine interior, [j-1, i-1]
        qx, qy = nx // 2, ny // 2
        for J in range(ny // 4 + 1, 3 * ny // 4):
            for I in range(nx // 4 + 1, 3 * nx // 4):
                g[J, I] = 4.0 * gf[2 * J - qy - 1, 2 * I - qx - 1]
    return g
