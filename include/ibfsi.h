/* ibfsi: strongly coupled immersed-boundary flow step on MI355X (gfx950).
 *
 * One solver instance advances the 2-D incompressible flow around rigid,
 * torsionally hinged and deformable bodies with the block-LU factored, strongly
 * coupled immersed-boundary method of Nair & Goza ("A strongly coupled immersed
 * boundary method for fluid-structure interaction that mimics the efficiency of
 * stationary body methods"):
 *
 *   predictor   s* = (C^T A C)^{-1} r^f                     (Sec. 2.3, eq. (16))
 *   FSI loop    Schur system for the body stresses f,       (eqs. (17)-(19); with the
 *               structural Newton update, until              sub-domain operator:
 *               max |delta theta|, |delta chi| <= tol        eqs. (37)-(39), Alg. 2)
 *   corrector   s_{n+1} = s* - (C^T A C)^{-1} C^T E^T f      (eq. (20) / (40))
 *
 * on a staggered streamfunction-vorticity grid (Sec. 2.2) with nested levels that
 * double in extent about a common centre (far field, Sec. 5).  Moving bodies use the
 * precomputed, drop-tolerance filtered sub-domain operator B' (Sec. 3, Algorithm 1).
 *
 * Conventions
 *   - All host buffers are owned by the caller; the library copies what it needs.
 *   - Device state is owned by the solver and allocated through the optional
 *     allocator callbacks (e.g. PyTorch's caching allocator), else hipMalloc.
 *   - Work is enqueued on the HIP stream given at creation (NULL = default stream);
 *     ib_step returns once the work is enqueued unless a host decision is needed
 *     (FSI convergence test), ib_sync waits for it.
 *   - A solver handle is not thread-safe; distinct handles are independent.
 *   - Grid arrays are row-major with the y index outer: value (i, j) of an interior
 *     array of ny-1 rows of nx-1 values (nx = n; ny = n unless set) is at
 *     [(j-1) * (nx-1) + (i-1)].
 *   - Stresses of a body of m points are 2m values: the m x-components, then the m
 *     y-components (Sec. 4.2).  f is the stress the fluid exerts on the body (force
 *     per unit length), so the body's force is sum(f) * ds.
 *   - Every function returns IB_OK (0) or a negative ib_status; no exception
 *     crosses the ABI.  After a failed ib_step the handle stays readable but further
 *     steps return IB_ERR_STATE.
 */
#ifndef IBFSI_H
#define IBFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ib_status;
#define IB_OK 0
#define IB_ERR_ARG (-1)               /* invalid argument (null pointer, bad size, unsupported n) */
#define IB_ERR_STATE (-2)             /* wrong call order, or stepping after a failure */
#define IB_ERR_OOM (-3)               /* device allocation failed */
#define IB_ERR_HIP (-4)               /* HIP runtime error */
#define IB_ERR_NOT_CONVERGED (-5)     /* FSI iteration hit newton_max_iter */
#define IB_ERR_OUT_OF_SUBDOMAIN (-6)  /* a body point left the sub-domain rectangle */
#define IB_ERR_NEAR_BOUNDARY (-7)     /* delta support reaches the finest level's edge */
#define IB_ERR_NONFINITE (-8)         /* NaN or Inf in the state */
#define IB_ERR_CAPACITY (-9)          /* caller's output buffer is too small */
#define IB_ERR_BUDGET (-10)           /* the request's device-memory estimate exceeds the budget
                                         it is admitted against */
#define IB_ERR_SCRATCH (-11)          /* the call needs more than the fixed device scratch of an
                                         allocation-free entry point */

/* precision */
#define IB_FP64 0        /* everything in double precision */
#define IB_FP32_FLOW 1   /* stencils, sine transforms, spreading in float; Schur, LU and
                            structure in double */
#define IB_FP32_FLOW_BF16_DST 2  /* IB_FP32_FLOW with the predictor's sine transforms done as
                            dense products with the sine matrix on the BF16 matrix cores, each
                            operand split in two BF16 parts (three products, FP32
                            accumulation; about 16 significant bits per transform) */

/* discrete delta kernel of the interpolation E and regularisation E^T (Sec. 3.1, eq. (24):
 * the paper does not name its kernel) */
#define IB_DELTA_ROMA3 0    /* 3-point kernel of Roma, Peskin & Berger (1999), support 1.5 h */
#define IB_DELTA_PESKIN4 1  /* Peskin's 4-point kernel (2002), support 2 h; with the exact
                               operator only: in sub-domain mode the hat-combined E0 rows of
                               this kernel do not fit the 4 x 4 face window of a stress row
                               (ib_prepare returns IB_ERR_ARG) */

/* Schur operator */
#define IB_SCHUR_AUTO 0       /* sub-domain if a sub-domain is set, else exact */
#define IB_SCHUR_EXACT 1      /* E C (C^T A C)^{-1} C^T E^T with the true E (eq. (17));
                                 precomputed once when every body is rigid */
#define IB_SCHUR_SUBDOMAIN 2  /* P B' P^T (eqs. (23), (37)) */

typedef struct ib_solver ib_solver;

typedef struct {
  int32_t n;          /* cells along x of every level (and along y unless ny is set); one of
                         16, 20, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 384, 512,
                         640, 768, 1024, 1280 (2^a 3^b 5^c: the sine transforms' FFT
                         lengths), a multiple of 4 */
  int32_t levels;     /* nested levels (>= 1); level 0 is the finest */
  double h;           /* finest grid spacing */
  double cx, cy;      /* common centre of all levels */
  double re;          /* Reynolds number */
  double dt;          /* time step */
  double u_inf[2];    /* free stream */
  int32_t precision;  /* IB_FP64, IB_FP32_FLOW or IB_FP32_FLOW_BF16_DST */
  int32_t schur_mode; /* IB_SCHUR_* */
  double newton_tol;  /* FSI tolerance on max |delta theta|, |delta chi| (1e-7, Sec. 5) */
  int32_t newton_max_iter;   /* give up after this many FSI iterations (e.g. 20) */
  int32_t newton_fixed_iter; /* > 0: run exactly this many FSI iterations, no test */
  double drop_tol;    /* B' drop tolerance epsilon (0.007, Sec. 3.2.2) */
  int32_t delta;      /* IB_DELTA_ROMA3 (0, the default) or IB_DELTA_PESKIN4 */
  int32_t ny;         /* cells along y of every level (Sec. 5.3 runs on 2:1 levels); 0: ny = n.
                         From the same list as n, a multiple of 4.  Rectangular levels
                         (ny != n) carry flows without bodies (ib_prepare returns IB_ERR_ARG
                         when bodies were added), in IB_FP64 or IB_FP32_FLOW (not
                         IB_FP32_FLOW_BF16_DST) with the default transform configurations
                         (ib_set_flow_variants refuses others), and are not batch members.
                         Vorticity arrays are then (ny-1) rows of nx-1, streamfunction arrays
                         (ny+1) rows of nx+1. */
} ib_config;

typedef struct {
  void* (*alloc)(size_t bytes, void* ctx); /* returns device memory or NULL */
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} ib_allocator;

typedef struct {
  int64_t step;              /* completed steps */
  int32_t newton_iters;      /* FSI iterations of the last step */
  int32_t newton_iters_max;  /* largest count so far */
  double newton_delta;       /* last max |delta| */
  int64_t subdomain_points;  /* 2 n_sd (rows of B'), 0 when not used */
  int64_t subdomain_nnz;     /* stored entries of B' */
  double prepare_seconds;    /* wall time of the offline stage */
  int32_t refine_iters;      /* Schur refinement sweeps in the last FSI iteration */
  int32_t inverse_rebuilds;  /* fresh Schur inverses (LU) made so far */
  double refine_residual;    /* relative residual of the last Schur solve (max norms; when the
                                refinement stopped on a predicted residual, that prediction) */
  int32_t operator_source;   /* offline operator: 0 built, 1 from the cache, 2 imported,
                                -1 none (no bodies) */
  int64_t graph_launches;    /* steps replayed from a recorded graph (IB_OPT_GRAPHS) */
  int64_t graph_captures;    /* graphs recorded */
  int64_t fsi_resumes;       /* steps whose FSI iterations launched ahead did not suffice
                                and were continued on the host (IB_OPT_FSI_AHEAD) */
  int32_t converged;         /* 1 when the last step's final max |delta| <= newton_tol (also
                                without bodies or steps); 0 after a fixed iteration count that
                                stopped above it */
  double noslip_resid;       /* no-slip residual of the last step (Sec. 2.3, the constraint at
                                t_{n+1}): max over stress rows of |(1/h) W (C s_{n+1} + q_inf)
                                - U_b|, W the row's interpolation of the last FSI iterate (E,
                                or P E0 in sub-domain mode), U_b the body velocity at t_{n+1};
                                round-off with the exact operator, the sub-domain operator's
                                approximation error otherwise */
  double force[2];           /* total force of the fluid on all bodies, sum of f ds (x, y); per
                                body: ib_read_force */
  int64_t solve_fallbacks;   /* steps whose stress solves were redone by LU because the
                                refinement's device-wide barrier timed out */
  int32_t solve_by_lu;       /* 1 when every stress solve is an LU factorisation: the
                                refinement's workgroups cannot all be resident on this device */
} ib_stats;

/* Create a solver for the problem set-up of Algorithm 1 (grid hierarchy of Sec. 5, time step,
 * Reynolds number, free stream; the bodies and the sub-domain are added next).  `alloc` may be
 * NULL (hipMalloc); `hip_stream` is a hipStream_t or NULL.  The configuration is copied; the
 * handle owns nothing on the device until ib_prepare.  Errors: IB_ERR_ARG for unsupported
 * sizes (n or ny not in the list, not a multiple of 4, 4000 in IB_FP64, levels outside
 * 1..12) or non-positive h / dt / re. */
ib_status ib_create(const ib_config* cfg, const ib_allocator* alloc, void* hip_stream,
                    ib_solver** out);

/* Stationary or prescribed-velocity rigid body: m points xy[2m] (x0, y0, x1, y1, ...),
 * arc length per point ds, optional velocity u_b[2m] (NULL = at rest).  Eq. (5). */
ib_status ib_add_rigid(ib_solver* s, int32_t m, const double* xy, double ds,
                       const double* u_b, int32_t* body_id);

/* Pose of a rigid body's frame at time t and its rates: pose[0..5] = x, y, angle, vx, vy,
 * omega; optionally its accelerations pose[6..8] = ax, ay, alpha_dd (they arrive set to NaN
 * and are needed only when a mounted torsional body rides on the body).  Called on the
 * thread that calls ib_prepare / ib_step. */
typedef void (*ib_motion_fn)(double t, double* pose, void* ctx);

/* Rigid body in prescribed motion (Sec. 2.1, eq. (5): a rigid body moves with a prescribed
 * velocity; the driven plate of Sec. 5.1): m points xy_ref[2m] in the body frame, arc length
 * per point ds.  Before each step the library calls motion(t_{n+1}, pose, ctx) and enforces
 * no-slip at the points (x, y) + R(angle) xy_ref with velocity (vx, vy) + omega e_z x
 * (R(angle) xy_ref).  In sub-domain mode the points are interpolated through P like the
 * other moving points and must stay inside the sub-domain.  ib_read_deflection returns
 * the point positions (2m, as xy) at the last step's time level.  Errors: IB_ERR_ARG for
 * m < 1, ds <= 0 or no callback; IB_ERR_NONFINITE if a returned pose is not finite. */
ib_status ib_add_moving_rigid(ib_solver* s, int32_t m, const double* xy_ref, double ds,
                              ib_motion_fn motion, void* ctx, int32_t* body_id);

/* Torsionally hinged flat plate of m points at hinge + j ds (cos, sin)(theta0 + theta),
 * j = 0 .. m-1, ds = length / (m - 1); moment of inertia, spring stiffness and
 * damping about the hinge; initial deflection theta and rate phi.  Eqs. (3), (6),
 * (A.2)-(A.4). */
ib_status ib_add_torsional(ib_solver* s, int32_t m, double hinge_x, double hinge_y,
                           double length, double theta0, double inertia, double stiffness,
                           double damping, double theta, double phi, int32_t* body_id);

/* Torsional plate whose hinge rides on a rigid body in prescribed motion (Sec. 5.1: the
 * passive plate hinged to the driven plate).  driver: the body id of an ib_add_moving_rigid
 * body added earlier, whose callback must give accelerations.  The hinge sits at
 * (hinge_bx, hinge_by) in the driver's frame; the m points are at hinge + j ds (cos, sin)
 * (driver angle + theta_rel + theta), ds = length / (m - 1).  inertia, stiffness and
 * damping are about the hinge; mass and cg (hinge to centre of mass, along the plate) give
 * the pseudo-moment of the hinge's motion, g = -I_H alpha_dd - m r_G x a_H (r_G = cg along
 * the plate, a_H the hinge acceleration, alpha_dd the driver's angular acceleration), which
 * for Sec. 5.1's two plates is its equation of motion's right-hand side beyond the fluid
 * moment.  theta: deflection relative to the driver, with rate phi, at t = 0.  The points
 * carry the driver's velocity at their positions plus the deflection rate.
 * ib_read_deflection returns theta, phi, phi_dot as for ib_add_torsional.  Errors:
 * IB_ERR_ARG (m < 2, length or inertia <= 0, mass < 0, driver not a moving rigid body);
 * IB_ERR_NONFINITE at ib_prepare / ib_step when the driver gives no accelerations. */
ib_status ib_add_mounted_torsional(ib_solver* s, int32_t m, int32_t driver, double hinge_bx,
                                   double hinge_by, double theta_rel, double length,
                                   double inertia, double stiffness, double damping,
                                   double mass, double cg, double theta, double phi,
                                   int32_t* body_id);

/* Deformable beam clamped at its first node: stress-free straight reference xy_ref[2m],
 * mass per unit length, bending (ei) and stretching (ea) stiffness, initial node
 * positions xy0[2m] and rotations rot0[m] (relative to the reference), at rest.
 * Eqs. (4), (7), (A.5).  Finite elements: corotational Euler-Bernoulli beam. */
ib_status ib_add_deformable(ib_solver* s, int32_t m, const double* xy_ref, double mass,
                            double ei, double ea, const double* xy0, const double* rot0,
                            int32_t* body_id);

/* Sub-domain rectangle (Sec. 3.1.1); it is snapped outwards to finest-level vertices.  Each
 * call adds one rectangle (at most 8), for bodies that lie far apart: the sub-domain points
 * are the rectangles' vertex grids one after another (B' couples them all), and each
 * torsional or deformable body is interpolated on the first rectangle that holds all its
 * points at the start (rigid bodies in prescribed motion and plates mounted on them: on the
 * first rectangle).  Errors: IB_ERR_ARG (empty rectangle, a ninth one); at ib_prepare
 * IB_ERR_OUT_OF_SUBDOMAIN when a body lies in no rectangle. */
ib_status ib_set_subdomain(ib_solver* s, double x0, double x1, double y0, double y1);

/* Initial vorticity of one level: omega[(ny-1) (nx-1)] at interior vertices (host). */
ib_status ib_set_vorticity(ib_solver* s, int32_t level, const double* omega);

/* Offline stage: initial streamfunction from the vorticity, then the stationary
 * Schur inverse (exact mode, rigid bodies only) or B' (Algorithm 1). */
ib_status ib_prepare(ib_solver* s);

/* Online stage: advance nsteps time steps (Algorithm 2). */
ib_status ib_step(ib_solver* s, int32_t nsteps);

/* Wait until the work ib_step enqueued on the solver's stream is done (the state of
 * Algorithm 2's last step is then readable).  Errors: IB_ERR_ARG, IB_ERR_HIP. */
ib_status ib_sync(ib_solver* s);

/* Stresses f_{n+1} of a body after the last step (eq. (17) / (37)): 2m doubles, x block then
 * y block (Sec. 4.2), into the caller's host buffer of cap doubles.  Errors: IB_ERR_ARG (bad
 * id), IB_ERR_STATE (not prepared), IB_ERR_CAPACITY (cap < 2m). */
ib_status ib_read_stresses(ib_solver* s, int32_t body_id, double* f, int64_t cap);

/* Force of the fluid on a body after the last step (Sec. 5: forces and lift coefficients),
 * out[0..1] = (F_x, F_y) = ds * sum of the body's stresses, summed on the device.  With unit
 * free stream and chord, c_d = 2 F_x and c_l = 2 F_y.  (0, 0) before the first step; still
 * readable after ib_release.  Errors: IB_ERR_ARG, IB_ERR_STATE (not prepared),
 * IB_ERR_CAPACITY (cap < 2). */
ib_status ib_read_force(ib_solver* s, int32_t body_id, double* out, int64_t cap);

/* Structure state of a body after the last step (eqs. (18)-(19), Appendix A): torsional ->
 * (theta, phi, phidot); deformable -> 3m doubles (x, y, rotation per node); rigid -> its 2m
 * point coordinates.  Host buffer of cap doubles.  Errors: IB_ERR_ARG, IB_ERR_STATE,
 * IB_ERR_CAPACITY. */
ib_status ib_read_deflection(ib_solver* s, int32_t body_id, double* out, int64_t cap);

/* Vorticity of a level at interior vertices (Sec. 2.2: omega = C^T C s / h^2), (ny-1) (nx-1)
 * doubles: the level's circulation state gamma (= C^T C s, carried alongside s) divided by h^2.
 * Host buffer of cap doubles; level 0 stays readable after ib_release.  Errors: IB_ERR_ARG,
 * IB_ERR_STATE (nothing on the device), IB_ERR_CAPACITY. */
ib_status ib_read_vorticity(ib_solver* s, int32_t level, double* out, int64_t cap);

/* Streamfunction s of a level including its boundary ring (Sec. 2.2), (ny+1) (nx+1) doubles
 * into a host buffer of cap doubles.  Errors: IB_ERR_ARG, IB_ERR_STATE, IB_ERR_CAPACITY. */
ib_status ib_read_streamfunction(ib_solver* s, int32_t level, double* out, int64_t cap);

/* Statistics of the solver (ib_stats: Newton iterations and last update of Algorithm 2's
 * loop, sub-domain size and B' entries of Algorithm 1, outputs of the last step); still
 * readable after ib_release.  Errors: IB_ERR_ARG. */
ib_status ib_get_stats(ib_solver* s, ib_stats* out);

/* Kernel timing for measurement: while enabled, every launch of the classes below is
 * bracketed by HIP events on the solver's stream (adds a few microseconds per launch);
 * column-solve launches (IB_K_COL_SOLVE) record their events at the kernel's own start and
 * end (hipExtLaunchKernelGGL), so that class's time excludes the dispatch.
 * ib_get_kernel_timing synchronises and returns the launches and the summed kernel
 * time (milliseconds) of one class since timing was last enabled. */
#define IB_K_RHS_ROWDST 0   /* explicit right-hand side + row sine transform */
#define IB_K_COL_SOLVE 1    /* column transform, spectral solve, inverse (s and gamma) */
#define IB_K_ROW_IDST 2     /* inverse row transform into the level state */
#define IB_K_FSI 3          /* one FSI iteration (operator, Schur, LU, update) */
#define IB_K_CORRECT 4      /* corrector source + its row transform */
#define IB_K_RING 5         /* nested-level boundary rings */
#define IB_K_CLASSES 6
ib_status ib_set_kernel_timing(ib_solver* s, int32_t enable);
ib_status ib_get_kernel_timing(ib_solver* s, int32_t kernel_class, int64_t* launches,
                               double* total_ms);

/* Free the solver and everything it holds (device memory first, as ib_release).  The handle is
 * invalid afterwards.  Errors: IB_ERR_ARG (null). */
ib_status ib_destroy(ib_solver* s);

/* ---- execution options ----
 * IB_OPT_FSI_AHEAD (default 1): launch a step's FSI iterations ahead of their convergence
 *   tests (as many as the last step needed), each followed by a device-side test that stops
 *   the remaining ones; the host synchronises once per step and continues on its own only
 *   when they did not suffice.  0: the host tests after every iteration (Algorithm 2 as
 *   written).  Both give the same results.
 * IB_OPT_GRAPHS (default 0): with IB_OPT_FSI_AHEAD, record a step's launches once as a HIP
 *   graph (per alternation of the ring buffers and count of iterations launched ahead) and
 *   replay it for later steps (a non-null stream is needed).  Measured on the flag workload,
 *   replay neither shortens a step nor raises the throughput of concurrent solvers, hence
 *   the default.
 * IB_OPT_REFRESH_EVERY_ITER (default 2): when the approximate Schur inverse X is refreshed
 *   by one Newton-Schulz step X <- X (2I - M X) before a stress solve.  1: at every FSI
 *   iteration (the refined solve then needs fewer sweeps); 0: at the first iteration of
 *   every step; 2: at every iteration for up to 256 stress unknowns, above that only at the
 *   first iteration of a step whose previous solve needed more than 6 sweeps (the two
 *   n^3 products then cost more than the sweeps they save).  The solution is the same to
 *   round-off in every mode.
 * IB_OPT_TOP_AHEAD (default 2): within one ib_step call, with three or more levels, start
 *   the next step's coarse levels early, with spectral scratch of their own.  1: the
 *   coarsest level, on the solver's stream while the host waits for this step's
 *   convergence tests.  2: every level >= 2, on a second stream (default priority) of the
 *   solver as soon as this step's level 1 is done, concurrently with this step's level 0,
 *   FSI part and corrector.  0: off.  Those levels need only states that are final once
 *   this step's level 1 is (level 1 is never corrected), so the results are the same bit
 *   for bit.  Used only while no other solver of the process is inside ib_step (several
 *   solvers stepping at once fill the GPU without it), and not with IB_OPT_GRAPHS,
 *   IB_FP32_FLOW_BF16_DST or kernel timing.
 * Errors: IB_ERR_ARG for an unknown option or value. */
#define IB_OPT_FSI_AHEAD 1
#define IB_OPT_GRAPHS 2
#define IB_OPT_REFRESH_EVERY_ITER 3
#define IB_OPT_TOP_AHEAD 4
/* IB_OPT_BARRIER_SPIN (default 0 = the built-in bound, 2^22): the bound on the spins of the
 * stress refinement's device-wide barrier, up to 2^40.  The refinement keeps rows of the Schur
 * matrix and of its approximate inverse in the LDS of co-resident workgroups and meets at one
 * barrier per sweep; when a wait reaches the bound (the workgroups were not all resident,
 * e.g. beside other solvers' kernels) every workgroup leaves, and the host redoes that step's
 * FSI iterations with LU solves of the Schur matrix (ib_stats.solve_fallbacks).
 * IB_OPT_BARRIER_FORCE_TIMEOUT (default 0; 1 for tests of that path): every barrier waits for
 * one arrival more than the launch has workgroups, so every wait ends at the spin bound. */
#define IB_OPT_BARRIER_SPIN 5
#define IB_OPT_BARRIER_FORCE_TIMEOUT 6
ib_status ib_set_option(ib_solver* s, int32_t option, int64_t value);

/* ---- measured kernel configurations of the sine transforms ----
 * For single-precision flow and n in {256, 384, 512, 768, 1024}, ib_prepare times the
 * configurations of each of three kernels (right-hand side + row transform, column solve,
 * inverse row transform) on scratch buffers of one level's shape and keeps the fastest; the
 * choice is remembered per n for the process.  Row kernels have 8 configurations (0 .. 7)
 * and the column solve 9 (0 .. 8).  Configurations 0 .. 7 fix the rows (or columns) per
 * workgroup, the threads per workgroup and the largest FFT radix (16, 8 or 4) of the LDS
 * Stockham stages (Sec. 3.2.1 transforms).  Column configuration 8 exists for n = 1024: each
 * column's transform of length 1024 = 32 x 32 runs in registers on 32 lanes of one wave,
 * with one LDS transpose per transform and no workgroup barrier between its stages
 * (ib_flow_variant_info reports it as 4 columns, 128 threads, radix 32).  All
 * configurations compute the same transforms; they differ in rounding order only. */
#define IB_FLOW_VARIANTS 9
typedef struct {
  int32_t n;             /* grid size the choice was made for (0: none, defaults used) */
  int32_t rhs_variant;   /* chosen configurations, 0 .. IB_FLOW_VARIANTS-1 */
  int32_t col_variant;
  int32_t idst_variant;
  double rhs_us[IB_FLOW_VARIANTS];  /* measured average launch time (microseconds; */
  double col_us[IB_FLOW_VARIANTS];  /*   0 where not measured or not available for n) */
  double idst_us[IB_FLOW_VARIANTS];
} ib_flow_tuning;
ib_status ib_get_flow_tuning(ib_solver* s, ib_flow_tuning* out);

/* Fix the configurations instead of measuring (before or after ib_prepare).  Nonzero
 * variants need single precision and one of the measured sizes, column configuration 8
 * n = 1024 (IB_ERR_ARG otherwise); -1 keeps one as is. */
ib_status ib_set_flow_variants(ib_solver* s, int32_t rhs, int32_t col, int32_t idst);

/* Configuration `variant` of kind 0 (row kernels: rows per workgroup) or 1 (column solve:
 * columns per workgroup): width, threads per workgroup, largest radix. */
ib_status ib_flow_variant_info(int32_t kind, int32_t variant, int32_t* width, int32_t* threads,
                               int32_t* max_radix);

/* ---- device memory and streams (for schedulers running many solvers) ----
 * ib_create allocates no device memory; ib_prepare allocates all of it. */

/* Move the solver to another HIP stream (waits for the work on the current one). */
ib_status ib_set_stream(ib_solver* s, void* hip_stream);

/* Give all device memory back after copying the results to the host: afterwards
 * ib_read_stresses, ib_read_deflection and ib_read_vorticity (level 0 only) still work,
 * ib_step returns IB_ERR_STATE.  Safe to call on an unprepared solver. */
ib_status ib_release(ib_solver* s);

/* Device memory the solver will hold after ib_prepare (resident) and at most during
 * it (peak, including the offline stage's batch buffers), from its configuration and
 * bodies.  An estimate for admission control; B' is counted at 800 stored entries
 * per row at the drop tolerance 0.007. */
ib_status ib_estimate_bytes(const ib_solver* s, int64_t* resident, int64_t* peak);

/* ---- offline operator reuse (Sec. 3.2.2: the offline stage depends only on the grid,
 * dt, Re and the sub-domain, so it can serve many problems) ----
 * ib_prepare keeps every operator it builds (B' for moving bodies, the unscaled Schur
 * matrix for stationary ones) in a process-wide host cache keyed by exactly the numbers
 * it depends on (grid, dt, Re, drop tolerance, sub-domain, stationary points), and takes
 * it from there when a later solver has the same key. */

/* Cache capacity in bytes (default 8 GiB; 0 disables caching and empties the cache). */
ib_status ib_set_operator_cache(int64_t limit_bytes);

/* Serialise the operator the prepared solver uses into buf (cap bytes); *used receives the
 * size needed (IB_ERR_CAPACITY, with *used set, when buf is NULL or too small). */
ib_status ib_export_operator(ib_solver* s, void* buf, int64_t cap, int64_t* used);

/* Give an unprepared solver an operator exported earlier; ib_prepare checks that its key
 * matches the solver's problem (IB_ERR_ARG otherwise) and skips the offline stage. */
ib_status ib_import_operator(ib_solver* s, const void* buf, int64_t size);

/* ---- continuous-batching scheduler ----
 * A server runs submitted solvers (created, bodies added, not prepared) to completion
 * on max_active concurrent slots, each a host thread with its own non-blocking stream.
 * A request is admitted once its arrival time has passed, a slot is free and its peak
 * memory estimate fits in what the running requests leave of hbm_budget_bytes; in the
 * slot it is prepared, stepped (chunk_steps per call), synchronised and released
 * (results stay readable through the solver handle, which the caller destroys).  The
 * clock starts when ib_server_run is called; times are in seconds on that clock. */
typedef struct ib_server ib_server;

typedef struct {
  int64_t ticket;
  int32_t status;      /* 1 waiting, 2 running, 0 done, < 0 the solver's error */
  int32_t steps_done;
  double arrival;      /* as submitted */
  double admitted;     /* slot and memory granted */
  double started;      /* prepare finished, stepping begins */
  double finished;     /* results on the host */
  int64_t bytes;       /* admission estimate (peak) */
} ib_request_info;

ib_status ib_server_create(int32_t max_active, int64_t hbm_budget_bytes, int32_t chunk_steps,
                           ib_server** out);
/* Errors: IB_ERR_BUDGET when the request's peak estimate exceeds the whole budget (it could
 * never be admitted). */
ib_status ib_server_submit(ib_server* sv, ib_solver* s, int32_t nsteps, double arrival,
                           int64_t* ticket);
/* Run until every submitted request has finished or failed (blocking). */
ib_status ib_server_run(ib_server* sv);
ib_status ib_server_info(ib_server* sv, int64_t ticket, ib_request_info* out);
/* Destroys the server and its streams, not the solvers. */
ib_status ib_server_destroy(ib_server* sv);

/* ---- batches: many solvers per launch ----
 * A batch steps many independent solvers together (each is its own instance of
 * Algorithm 2).  Every kernel launch of a batched step covers all members that need it:
 * one launch per grid size (and transform configuration) for each flow kernel of the
 * predictor (Sec. 2.3 eq. (16), Sec. 3.2.1), the corrector (eq. (20)) and the level
 * coupling, and one launch over all members for each kernel of the FSI iterations (body
 * operators, Schur assembly eqs. (17), (37), its refreshed inverse and stress solve, the
 * structure update and convergence test), so a step costs a few dozen launches however many
 * members there are.  Members' FSI iterations run on the device with their own convergence
 * tests; a member that needs more than the iterations launched continues on the host.
 * Each member's results equal those of the same solver stepped alone.
 * A member's step runs alone (as ib_step would run it) when it is its first step, when its
 * Schur inverse must be rebuilt, or when it uses IB_FP32_FLOW_BF16_DST, the exact operator
 * for moving bodies, kernel timing or IB_OPT_FSI_AHEAD = 0.
 * members: `count` distinct prepared solvers of one precision class (IB_FP64, or the FP32
 * flow forms), owned by the caller, who must keep them alive and not step them elsewhere
 * while the batch exists.  From ib_batch_create on, every member's work runs on hip_stream
 * (the solvers' stream is set to it; NULL = the null stream).
 * Errors: IB_ERR_ARG (count < 1, a null or repeated member, mixed precision),
 * IB_ERR_STATE (a member not prepared, failed or released); ib_batch_step returns the
 * first failing member's error, marks that member failed, and ib_batch_last_error says
 * what happened. */
typedef struct ib_batch ib_batch;

typedef struct {
  int64_t steps;                 /* batched steps taken (ib_batch_step's nsteps summed) */
  int64_t member_steps_batched;  /* member steps that ran in batched launches */
  int64_t member_steps_alone;    /* member steps that ran alone */
  int64_t launches;              /* batched launches issued (tables copy excluded) */
  int64_t fsi_resumes;           /* members whose FSI part continued on the host */
} ib_batch_stats;

ib_status ib_batch_create(ib_solver* const* members, int32_t count, void* hip_stream,
                          ib_batch** out);
/* nsteps steps of every member; returns after the last step's convergence tests (the
 * members' control blocks are read right after their FSI iterations, so the last step's
 * corrector and final transforms, or with no moving bodies its flow, may still run on
 * hip_stream; the members' read calls wait for them). */
ib_status ib_batch_step(ib_batch* b, int32_t nsteps);
ib_status ib_batch_get_stats(const ib_batch* b, ib_batch_stats* out);
const char* ib_batch_last_error(const ib_batch* b);
/* Waits for the batch's work and frees the batch, not its members. */
ib_status ib_batch_destroy(ib_batch* b);

const char* ib_status_str(ib_status st);

/* What the last failing call on this solver reported (empty if none); valid until the
 * next call on the solver. */
const char* ib_last_error(const ib_solver* s);

/* ---- operator-level entry points (device pointers, enqueued on hip_stream) ---- */

/* out = [L (I + alpha L)]^{-1} in, L = C^T C with zero boundary values (the solve of
 * eqs. (16) and (20) without its dt factor; Sec. 3.2.1).  in/out: (n-1) x (n-1) arrays
 * of float (precision = IB_FP32_FLOW) or double (IB_FP64) with row pitch `pitch`
 * elements; in == out is allowed. */
ib_status ib_op_solve(int32_t n, int32_t precision, double alpha, const void* in, void* out,
                      int32_t pitch, void* hip_stream);

/* ib_op_solve for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same operation, arguments,
 * kernels and results, with no hipMalloc, hipFree or other allocating call.  The transform
 * tables that ib_op_solve allocates per call (twiddles exp(-i pi m/n), m < 2n, and the
 * eigenvalues 4 sin^2(pi k/2n)) are written into a fixed 64 KiB device array that the library
 * holds on each GPU it runs on until the process ends; the tables of every supported n fit
 * (at most 51,200 bytes, n = 1280 in double).  Every call overwrites the tables it uses, so
 * nothing needs clearing, but all calls on one GPU share the array: calls that overlap on one
 * GPU (other host threads, other streams) race.  Returns once the solve is complete, like
 * ib_op_solve.  Errors: IB_ERR_ARG as for ib_op_solve; IB_ERR_SCRATCH if the tables would not
 * fit; IB_ERR_HIP if the array's device address cannot be obtained or a launch fails. */
ib_status ib_op_solve_noalloc(int32_t n, int32_t precision, double alpha, const void* in,
                              void* out, int32_t pitch, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* IBFSI_H */
