"""One time step of the strongly coupled IB method (FP64 oracle).

Follows the block-LU factored form (eqs. (16)-(20)) and its sub-domain version
(eqs. (36)-(40), Algorithms 1 and 2), re-derived from the un-factored discrete
system (eqs. (8)-(15), Appendix A eq. (A.17)) in this code's scaling:

predictor  (I + alpha L) L s* = dt r^f + lifted ring terms, per level, coarse to
           fine, with dt r^f = (I - alpha L) gamma_n + dt (3/2 C^T N_n - 1/2 C^T N_{n-1})
           (Appendix A, definition of r^f; L = C^T C).
stress     [ (dt/h^2) G diag(ds) + sum_t (2 ds/dt) S_t^T J^{-1} S_t
             + sum_d (2 ds/dt) T J_d^{-1} T^T ] f = b,
           G = E C K C^T E^T (exact) or P B' P^T (sub-domain), K = [L (I + alpha L)]^{-1},
           b = (1/h) E (C s* + q_inf) - u_rigid - S_t^T ((2/dt) J^{-1} r_phi - r_theta)
               - T ((2/dt)(chi^k + J_d^{-1} res^k) - r_chi)          (eq. (17) / (37))
update     theta^{k+1} = J^{-1} (r_phi + ds S_t f)                  (eq. (18))
           chi^{k+1} = chi^k + J_d^{-1} (res^k + ds T^T f)          (eq. (19))
corrector  s_{n+1} = s* - dt K C^T E^T (ds/h) f on level 0           (eq. (20) / (40))

Signs: f is the stress the fluid exerts on the body (this makes eqs. (A.3), (9) and
(11) consistent); the paper's S = [0, -QR ds, 0] carries one ds too many against
eq. (A.17)'s second row, and the reading here is S_t = Q R.

Rigid bodies in prescribed motion (Sec. 2.1, eq. (5); the driven plate of Sec. 5.1): their
points sit at the pose of the new time level t_{n+1}, (x, y) + R(angle) xy_ref, and carry
the prescribed velocity (vx, vy) + omega e_z x (R xy_ref) into b; in sub-domain mode they are
interpolated through P like the other moving points (not appended to B').  A torsional body
mounted on such a driver (Sec. 5.1's passive plate; structure.MountedState) takes its hinge
and reference angle from the driver at t_{n+1}, its points carry the driver's velocity at
their positions into b on top of the deflection rate, and its g is the pseudo-moment of the
hinge's acceleration at the current iterate.

FSI iteration (Algorithm 2): start from the old structure state, stop when
max |delta theta|, |delta chi| <= tol (both tests of Sec. 5 and Algorithm 2), at most
``newton_max`` iterations, or run exactly ``fixed_iters`` iterations (parity mode).
The corrector uses the interpolation operator of the last solve; the structure takes
the last update.  AB2 starts with N_{-1} := N_0.

Precision: float64 by default.  ``dtype=numpy.longdouble`` runs the flow part (problems
without bodies) in extended precision, as a reference finer than double rounding: the
double-precision oracle re-differences its streamfunction (C^T C s) for the circulation it
hands between levels, which amplifies the rounding of s by up to (n/pi)^2 / 2, so at
n >= 96 with nested levels its own s and vorticity carry errors of 1e-12 .. 1e-10.
"""
import numpy as np

import workloads as W

from . import delta, dst, grid, multidomain as md, structure, subdomain


TORS = ("torsional", "mounted")


class NotConverged(RuntimeError):
    pass


def moving_positions(b, t):
    """Points of a rigid body in prescribed motion at time t: (x, y) + R(angle) xy_ref."""
    x, y, ang, _, _, _ = b.pose(t)
    rot = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
    return b.xy_ref @ rot.T + np.array([x, y])


def moving_velocities(b, t):
    """Their velocities: (vx, vy) + omega e_z x (R(angle) xy_ref)."""
    x, y, ang, vx, vy, om = b.pose(t)
    rot = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
    r = b.xy_ref @ rot.T
    return np.stack([vx - om * r[:, 1], vy + om * r[:, 0]], axis=1)


class Oracle:
    def __init__(self, problem, newton_tol=1e-7, newton_max=20, fixed_iters=0,
                 drop_tol=0.007, subdomain_mode=None, dtype=np.float64):
        self.p = problem
        flow = problem.flow
        nx, ny = flow.nx_ny
        assert nx % 4 == 0 and ny % 4 == 0
        self.dtype = np.dtype(dtype)
        if self.dtype != np.float64 and problem.bodies:
            raise ValueError("extended precision covers the flow of problems without bodies")
        if nx != ny and problem.bodies:
            raise ValueError("bodies need square levels")
        self.levels = [grid.Level(flow, g) for g in range(flow.levels)]
        self.kernel = getattr(flow, "delta", "roma3")
        n = flow.n
        self.n = n
        self.nx, self.ny = nx, ny
        self.dt = flow.dt
        self.s = [self._zeros((ny + 1, nx + 1)) for _ in self.levels]
        self.hist = [None for _ in self.levels]
        self.gring = [self._zeros((ny + 1, nx + 1)) for _ in self.levels]
        self.newton_tol = newton_tol
        self.newton_max = newton_max
        self.fixed_iters = fixed_iters
        self.drop_tol = drop_tol
        self.step_count = 0
        self.last_iters = 0
        self.last_delta = 0.0
        self.f = None
        self.bodies = []
        for b in problem.bodies:
            if isinstance(b, W.Rigid):
                self.bodies.append(("rigid", b))
            elif isinstance(b, W.MovingRigid):
                self.bodies.append(("moving", b))
            elif isinstance(b, W.Torsional):
                self.bodies.append(("torsional", structure.TorsionalState(b, flow.dt)))
            elif isinstance(b, W.MountedTorsional):
                driver = problem.bodies[b.driver]
                if not isinstance(driver, W.MovingRigid):
                    raise TypeError("a mounted torsional body needs a MovingRigid driver")
                self.bodies.append(("mounted", structure.MountedState(b, driver, flow.dt)))
            elif isinstance(b, W.Deformable):
                self.bodies.append(("deformable", structure.BeamState(b, flow.dt)))
            else:
                raise TypeError(b)
        self.use_subdomain = (problem.subdomain is not None) if subdomain_mode is None else subdomain_mode
        if problem.vorticity0 is not None:
            self.set_vorticity(problem.vorticity0)
        self.prepared = False

    def _zeros(self, shape):
        return np.zeros(shape, dtype=self.dtype)

    # ------------------------------------------------------------------ setup
    def set_vorticity(self, omegas):
        """Streamfunction on every level from interior vorticity, coarse to fine."""
        nl = len(self.levels)
        for g in reversed(range(nl)):
            lv = self.levels[g]
            nx, ny = self.nx, self.ny
            if g == nl - 1:
                ring_s = self._zeros((ny + 1, nx + 1))
                ring_g = self._zeros((ny + 1, nx + 1))
            else:
                ring_s = md.ring_from_coarse(self.s[g + 1], nx, ny)
                ring_g = 0.25 * md.ring_from_coarse(md.coarse_circulation(self.s[g + 1]), nx, ny)
            om = (omegas[g] if g < len(omegas) and omegas[g] is not None
                  else self._zeros((ny - 1, nx - 1)))
            gam = lv.h * lv.h * np.asarray(om, dtype=self.dtype)
            bs = -grid.l5(grid.ring_only(ring_s))
            self.s[g] = grid.pad(dst.solve_poisson(gam + bs), ring_s)
            self.gring[g] = ring_g

    @staticmethod
    def _count(kind, b):
        if kind == "rigid":
            return b.xy.shape[0]
        if kind == "moving":
            return b.xy_ref.shape[0]
        return b.npts

    def npts_per_body(self):
        return [self._count(kind, b) for kind, b in self.bodies]

    def ds_vector(self):
        v = []
        for kind, b in self.bodies:
            v.append(np.full(2 * self._count(kind, b), b.ds))
        return np.concatenate(v) if v else np.zeros(0)

    def t_new(self):
        """Time level t_{n+1} of the step being taken (the constraint holds there)."""
        return (self.step_count + 1) * self.dt

    def prepare(self):
        """Offline stage: stationary exact Schur block, or B' (Algorithm 1)."""
        lv = self.levels[0]
        if not self.bodies:
            self.prepared = True
            return
        if self.use_subdomain:
            appended = [b.xy for kind, b in self.bodies if kind == "rigid"]
            app = np.concatenate(appended) if appended else None
            self.sd_boxes = subdomain.boxes_of(self.p.subdomain)
            self.sd_offsets, self.sd_ngrid = subdomain.box_offsets(lv, self.sd_boxes)
            # each moving body's rectangle: the first that holds all its points at the start
            # (torsional and deformable bodies); rigid bodies in prescribed motion and plates
            # mounted on them use the first rectangle
            self.sd_body_box = [None if kind == "rigid" else
                                (0 if kind in ("moving", "mounted") else
                                 subdomain.box_containing(lv, self.sd_boxes, self.positions(kind, b)))
                                for kind, b in self.bodies]
            self.sd_pts = subdomain.point_set(lv, self.sd_boxes, app)
            self.sd_total = self.sd_pts.shape[0]
            self.e0 = subdomain.sub_e0(lv, self.sd_pts, self.kernel)
            delta.check_support(lv, self.e0)
            self.b_full = subdomain.build_b(lv, self.e0)
            self.b_filtered = subdomain.filter_b(self.b_full, self.drop_tol)
        else:
            self.g_static = None
            if all(kind == "rigid" for kind, _ in self.bodies):
                eh = self.interp_operator()
                self.g_static = self.flow_block(eh)
        self.prepared = True

    # -------------------------------------------------------------- operators
    def positions(self, kind, b, it=None):
        if kind == "rigid":
            return b.xy
        if kind == "moving":
            return moving_positions(b, self.t_new())
        if kind in TORS:
            return b.positions(b.theta_k)
        return b.positions(b.chi_k)

    def interp_operator(self):
        """E (exact) or P E0 (sub-domain) at the current iterate; rows per body
        (x block, y block)."""
        lv = self.levels[0]
        blocks = []
        if not self.use_subdomain:
            for kind, b in self.bodies:
                e = delta.interpolation_matrix(lv, self.positions(kind, b), self.kernel)
                delta.check_support(lv, e)
                blocks.append(e.toarray())
            return np.vstack(blocks)
        return self.p_matrix() @ self.e0.toarray()

    def p_matrix(self):
        lv = self.levels[0]
        rows = []
        app_start = 0
        for (kind, b), bx in zip(self.bodies, self.sd_body_box):
            pos = self.positions(kind, b)
            m = pos.shape[0]
            app_idx = None
            box, off = self.sd_boxes[0], 0
            if kind == "rigid":
                app_idx = np.arange(app_start, app_start + m)
                app_start += m
            else:
                box, off = self.sd_boxes[bx], self.sd_offsets[bx]
            rows.append(subdomain.hat_rows(lv, box, self.sd_ngrid, self.sd_total, pos, 0, app_idx,
                                           off))
            rows.append(subdomain.hat_rows(lv, box, self.sd_ngrid, self.sd_total, pos,
                                           self.sd_total, app_idx, off))
        return np.vstack(rows)

    def flow_block(self, eh):
        """G = E C K C^T E^T by columns (the embedded large solve of eq. (17))."""
        lv = self.levels[0]
        n = lv.n
        cols = []
        for a in range(eh.shape[0]):
            qx, qy = grid.unflatten_faces(eh[a], n)
            s = grid.pad(dst.solve_cac(grid.curl_t(qx, qy), lv.alpha))
            cols.append(eh @ grid.flatten_faces(*grid.curl(s)))
        return np.array(cols).T

    # ------------------------------------------------------------------- step
    def step(self):
        if not self.prepared:
            self.prepare()
        nl = len(self.levels)
        n, nx, ny = self.n, self.nx, self.ny
        new_s = [None] * nl
        new_h = [None] * nl
        new_ring = [None] * nl
        for g in reversed(range(nl)):
            lv = self.levels[g]
            if g == nl - 1:
                ring_s = self._zeros((ny + 1, nx + 1))
                ring_g = self._zeros((ny + 1, nx + 1))
            else:
                ring_s = md.ring_from_coarse(new_s[g + 1], nx, ny)
                ring_g = 0.25 * md.ring_from_coarse(md.coarse_circulation(new_s[g + 1]), nx, ny)
            gam = md.circulation_for_rhs(self.s[g], self.gring[g], self.s[g - 1] if g > 0 else None)
            qx, qy = lv.flux(self.s[g])
            ctn = grid.curl_t_nonlinear(*grid.nonlinear(qx, qy, gam, lv.h))
            hprev = ctn if self.hist[g] is None else self.hist[g]
            r = gam[1:-1, 1:-1] - lv.alpha * grid.l5(gam) + lv.dt * (1.5 * ctn - 0.5 * hprev)
            bs = -grid.l5(grid.ring_only(ring_s))
            bg = -grid.l5(grid.ring_only(ring_g))
            r = r + lv.alpha * bg + bs + lv.alpha * grid.l5(grid.pad(bs))
            new_s[g] = grid.pad(dst.solve_cac(r, lv.alpha), ring_s)
            new_h[g] = ctn
            new_ring[g] = ring_g
        self.s_star = new_s[0].copy()
        if self.bodies:
            f, eh = self.fsi(new_s[0])
            lv = self.levels[0]
            lam = self.ds_vector() / lv.h * f
            qx, qy = grid.unflatten_faces(eh.T @ lam, n)
            corr = dst.solve_cac(grid.curl_t(qx, qy), lv.alpha)
            new_s[0][1:-1, 1:-1] -= lv.dt * corr
            self.f = f
            self.eh_last = eh
        self.s, self.hist, self.gring = new_s, new_h, new_ring
        self.step_count += 1

    def fsi(self, s_star):
        lv = self.levels[0]
        h, dt = lv.h, lv.dt
        q = grid.flatten_faces(*lv.flux(s_star))
        ds = self.ds_vector()
        counts = self.npts_per_body()
        for kind, b in self.bodies:
            if kind == "mounted":
                b.set_time(self.t_new())
            if kind in TORS:
                b.theta_k = b.theta
            elif kind == "deformable":
                b.chi_k = b.chi.copy()
        k = 0
        while True:
            eh = self.interp_operator()
            ustar = eh @ q / h
            if self.use_subdomain:
                p = self.p_matrix()
                gmat = p @ self.b_filtered @ p.T
            elif self.g_static is not None:
                gmat = self.g_static
            else:
                gmat = self.flow_block(eh)
            mat = (dt / h ** 2) * gmat * ds[None, :]
            rhs = ustar.copy()
            off = 0
            updates = []
            for (kind, b), m in zip(self.bodies, counts):
                blk = slice(off, off + 2 * m)
                if kind == "rigid":
                    if b.u_b is not None:
                        rhs[blk] -= np.concatenate([b.u_b[:, 0], b.u_b[:, 1]])
                elif kind == "moving":
                    ub = moving_velocities(b, self.t_new())
                    rhs[blk] -= np.concatenate([ub[:, 0], ub[:, 1]])
                elif kind in TORS:
                    jt = b.jac()
                    srow = b.s_row(b.theta_k)
                    mat[blk, blk] += (2.0 * b.ds / dt) * np.outer(srow, srow) / jt
                    rhs[blk] -= srow * ((2.0 / dt) * b.r_phi() / jt - b.r_theta())
                    if kind == "mounted":
                        uv = b.mount_velocity(b.theta_k)
                        rhs[blk] -= np.concatenate([uv[:, 0], uv[:, 1]])
                    updates.append((kind, b, blk, jt, srow))
                else:
                    jd, res = b.jacobian(b.chi_k)
                    t = b.t_matrix()
                    y = np.linalg.solve(jd, t.T)
                    mat[blk, blk] += (2.0 * b.ds / dt) * (t @ y)
                    free = b.free
                    chi_pred = b.chi_k[free] + np.linalg.solve(jd, res)
                    rhs[blk] -= t @ ((2.0 / dt) * chi_pred - b.r_chi()[free])
                    updates.append((kind, b, blk, jd, (t, res)))
                off += 2 * m
            f = np.linalg.solve(mat, rhs)
            delta_max = 0.0
            for kind, b, blk, jmat, extra in updates:
                if kind in TORS:
                    th_new = (b.r_phi() + b.ds * extra @ f[blk]) / jmat
                    delta_max = max(delta_max, abs(th_new - b.theta_k))
                    b.theta_new = th_new
                else:
                    t, res = extra
                    dchi = np.linalg.solve(jmat, res + b.ds * (t.T @ f[blk]))
                    delta_max = max(delta_max, float(np.max(np.abs(dchi))))
                    b.chi_new = b.chi_k.copy()
                    b.chi_new[b.free] += dchi
            k += 1
            done = (k >= self.fixed_iters) if self.fixed_iters > 0 else (delta_max <= self.newton_tol)
            if not updates:
                done = True
            if done or (self.fixed_iters == 0 and k >= self.newton_max):
                self.last_iters = k
                self.last_delta = delta_max
                self.eh_used = eh
                for kind, b, blk, jmat, extra in updates:
                    if kind in TORS:
                        b.theta_used = b.theta_k
                        b.finish(b.theta_new)
                        b.theta_k = b.theta
                    else:
                        b.finish(b.chi_new)
                        b.chi_k = b.chi.copy()
                if not done:
                    raise NotConverged(f"FSI iteration did not converge ({delta_max:g})")
                return f, eh
            for kind, b, blk, jmat, extra in updates:
                if kind in TORS:
                    b.theta_k = b.theta_new
                else:
                    b.chi_k = b.chi_new

    # ---------------------------------------------------------------- outputs
    def vorticity(self, g):
        lv = self.levels[g]
        return grid.l5(self.s[g]) / (lv.h * lv.h)

    def forces(self):
        out = []
        off = 0
        for (kind, b), m in zip(self.bodies, self.npts_per_body()):
            fx = self.f[off:off + m].sum() * b.ds
            fy = self.f[off + m:off + 2 * m].sum() * b.ds
            out.append((fx, fy))
            off += 2 * m
        return out

    def noslip_residual(self):
        """max |(1/h) E (C s_{n+1} + q_inf) - U_b| with the operator of the last solve
        (call after step(); moving bodies at the time level just reached)."""
        lv = self.levels[0]
        q = grid.flatten_faces(*lv.flux(self.s[0]))
        u = self.eh_used @ q / lv.h
        ub = np.zeros_like(u)
        off = 0
        for (kind, b), m in zip(self.bodies, self.npts_per_body()):
            if kind == "rigid" and b.u_b is not None:
                ub[off:off + m] = b.u_b[:, 0]
                ub[off + m:off + 2 * m] = b.u_b[:, 1]
            elif kind == "moving":
                v = moving_velocities(b, self.step_count * self.dt)
                ub[off:off + m] = v[:, 0]
                ub[off + m:off + 2 * m] = v[:, 1]
            elif kind == "torsional":
                ang = b.b.theta0 + b.theta_used
                j = np.arange(m) * b.ds
                ub[off:off + m] = -j * np.sin(ang) * b.phi
                ub[off + m:off + 2 * m] = j * np.cos(ang) * b.phi
            elif kind == "mounted":
                ang = b.ang0 + b.theta_used
                j = np.arange(m) * b.ds
                uv = b.mount_velocity(b.theta_used)
                ub[off:off + m] = uv[:, 0] - j * np.sin(ang) * b.phi
                ub[off + m:off + 2 * m] = uv[:, 1] + j * np.cos(ang) * b.phi
            elif kind == "deformable":
                ub[off:off + m] = b.zeta[0::3]
                ub[off + m:off + 2 * m] = b.zeta[1::3]
            off += 2 * m
        return float(np.max(np.abs(u - ub))) if u.size else 0.0
