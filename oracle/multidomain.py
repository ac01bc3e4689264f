"""Nested-level ("multi-domain") far-field treatment (FP64 oracle).

Sec. 5 uses a hierarchy of grids of increasing coarseness with zero vorticity at the
far boundary and refers to Colonius & Taira (2008) for the details, which the paper
does not give.  The reading adopted here:

1. Level g has the same n cells per side as level 0, spacing h 2^g, and all levels
   share one centre, so the coarse vertex (I, J) of level g+1 coincides with the fine
   vertex (2I - n/2, 2J - n/2) of level g (n divisible by 4).
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


def ring_from_coarse(vc, n):
    """Ring values of a fine level from the coarse full array ``vc`` (n+1, n+1).

    Returns an (n+1, n+1) array holding only the fine ring.
    """
    out = np.zeros((n + 1, n + 1), dtype=vc.dtype)
    q = n // 2

    def along(line, i):
        # value at fine index i along a coarse line; fine i <-> coarse (i + n/2) / 2
        if (i + q) % 2 == 0:
            return line[(i + q) // 2]
        c = (i + q - 1) // 2
        return (-line[c - 1] + 9.0 * line[c] + 9.0 * line[c + 1] - line[c + 2]) / 16.0

    jb, jt = q // 2, (n + q) // 2           # coarse rows of the fine bottom / top edges
    for i in range(n + 1):
        out[0, i] = along(vc[jb, :], i)
        out[n, i] = along(vc[jt, :], i)
    for j in range(n + 1):
        out[j, 0] = along(vc[:, jb], j)
        out[j, n] = along(vc[:, jt], j)
    return out


def coarse_circulation(s_coarse):
    """Full (n+1, n+1) circulation of a level from its own streamfunction (ring = 0;
    only interior vertices are used by ``ring_from_coarse``)."""
    return grid.pad(grid.l5(s_coarse))


def circulation_for_rhs(s, g_ring, s_finer):
    """Circulation used by a level's explicit right-hand side at the old time.

    Interior: C^T C s, except at vertices coinciding with an interior vertex of the
    next finer level, where 4 (C^T C s_finer) is used.  Ring: the stored ring
    values ``g_ring`` (an (n+1, n+1) array whose ring is used).
    """
    n = s.shape[0] - 1
    g = grid.pad(grid.l5(s), g_ring)
    if s_finer is not None:
        gf = grid.l5(s_finer)              # fine interior, [j-1, i-1]
        q = n // 2
        for J in range(n // 4 + 1, 3 * n // 4):
            for I in range(n // 4 + 1, 3 * n // 4):
                g[J, I] = 4.0 * gf[2 * J - q - 1, 2 * I - q - 1]
    return g
