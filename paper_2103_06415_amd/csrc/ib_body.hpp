// Device-side body description and the FSI-loop kernels' interface.
#pragma once

#include "ib_common.hpp"

namespace ib {

enum { BODY_RIGID = 0, BODY_TORSIONAL = 1, BODY_DEFORMABLE = 2, BODY_MOVING = 3 };

// Per-body data in device memory (double precision throughout).
// Rectangles of the sub-domain (Sec. 3.1.1; several when bodies lie far apart): vertex origin
// (i0, j0) and extent (npx x npy) of each, and its first sub-domain point `off` (the
// rectangles' vertex grids follow one another, row-major each).
constexpr int SD_MAX_BOXES = 8;
struct SdBoxes {
  int n;
  int i0[SD_MAX_BOXES], j0[SD_MAX_BOXES], npx[SD_MAX_BOXES], npy[SD_MAX_BOXES],
      off[SD_MAX_BOXES];
};

struct BodyDev {
  int kind;
  int npts;   // m
  int pt0;    // first point in the solver-wide point list; its rows start at 2 * pt0
  int app0;   // sub-domain mode: first appended sub-domain point of a rigid body
  int tors;   // index into the torsional state array; BODY_MOVING: index of its pose
  int dof0;   // deformable: offset of node 0's DOFs in the DOF arrays (3 per node)
  int has_ub; // rigid: prescribed velocity present
  int64_t yoff; // deformable: offset of its J_d^{-1} T^T workspace
  int moff;     // torsional on a driver: offset of its frame in FsiArgs::poses, else -1
  int sdbox;    // sub-domain mode, moving bodies: the rectangle its points are interpolated on
  double ds;
  double hx, hy, theta0, inertia, stiffness, damping;  // torsional (inertia about the hinge)
  double mass, ei, ea;                                 // deformable; mass also of a mounted body
  double cg;                                           // mounted: hinge to centre of mass
};

// Frame of a torsional body mounted on a rigid body in prescribed motion, at t_{n+1}
// (MOUNT_W doubles in FsiArgs::poses after the 6 per moving body): hinge (x, y), reference
// angle (driver angle + relative angle), hinge velocity (x, y), driver angular velocity,
// hinge acceleration (x, y), driver angular acceleration, unused.
constexpr int MOUNT_W = 10;
enum { MF_HX = 0, MF_HY, MF_ANG, MF_VX, MF_VY, MF_OM, MF_AX, MF_AY, MF_AL };

// Torsional state slots.
enum { TS_THETA = 0, TS_PHI, TS_PHIDOT, TS_NEW, TS_G, TS_COUNT };

// Everything the FSI kernels need.  Pointers are device pointers.
// flags[0] codes (the largest wins): 1 point outside the sub-domain, 2 delta support at
// the level-0 boundary, 3 singular or non-finite Schur matrix, 4 a device-wide barrier
// timed out.
constexpr int FLAG_BARRIER = 4;

// The solver's control block (device, 64 bytes), in int units: flags[2] (error code,
// refinement failure), the last max |delta| (double), the refinement report (3 doubles:
// relative residual, sweeps, 0), gate[2] and the next FSI iteration index.
struct FsiCtl {
  static constexpr int FLAGS = 0;   // ints 0, 1
  static constexpr int DELTA = 2;   // ints 2, 3 (double)
  static constexpr int ROUT = 4;    // ints 4 .. 9 (3 doubles)
  static constexpr int GATE = 10;   // ints 10, 11
  static constexpr int NEXT = 12;   // int 12
  static constexpr int UDONE = 13;  // int 13: workgroups of k_update finished (then reset)
  static constexpr int INTS = 14;   // ints cleared at the start of a step
  static constexpr int BYTES = 64;
};

struct FsiArgs {
  const BodyDev* bodies;
  int nbodies, npts, nf, ntors, ndef;
  int iter;            // FSI iteration (0 = start from the old structure state)
  // level 0 geometry
  int n, ps;
  double h, x0, y0, ux, uy, dt;
  int delta_kind;      // 0: 3-point kernel (Roma et al.), 1: 4-point kernel (Peskin); the
                       // latter with the true E only
  const void* sstar;   // predictor streamfunction, float or double per fp64
  int fp64;
  // sub-domain
  int use_sd, sd_ngrid, sd_total;
  SdBoxes sdb;
  const double* app_xy;     // appended exact points (2 per point)
  const int64_t* bp_ptr;    // B' CSR (rows = 2 sd_total)
  const int32_t* bp_col;
  const double* bp_val;
  // rigid geometry and prescribed velocities (2 per point, per body at pt0)
  const double* rigid_xy;   // BODY_MOVING: body-frame coordinates
  const double* rigid_ub;
  const double* poses;      // BODY_MOVING: x, y, angle, vx, vy, omega at t_{n+1}, 6 per body;
                            // then the frames of mounted torsional bodies (MOUNT_W each)
  // per-row operator: window base (i0, j0) and 4 x 4 weights; P (4 entries)
  int* st_base;
  double* st_w;
  int* p_idx;
  double* p_w;
  const double* gx;    // exact mode with moving bodies: E C K C^T E^T of this iterate (pitch pm)
  int* act;            // per B' row: a slot e (= 4 row + corner) of P that uses it
  double* pos;         // current point positions (2 per point)
  // FSI vectors and matrix
  double* ustar;       // (1/h) E (C s* + q_inf)
  double* rhs;
  double* f;
  double* M;
  int pm;
  const double* Minv;  // stationary inverse (exact, rigid only) or null
  // structure
  double* tors;        // [ntors][TS_COUNT]
  double* chi;         // deformable DOFs at time n
  double* zeta;
  double* zetadot;
  double* chi_new;     // latest iterate
  const double* dmass; // lumped mass per DOF
  const double* l0;    // per element (indexed like DOFs / 3)
  const double* beta0;
  double* ywork;       // J_d^{-1} T^T, per deformable body: (3m) x (2m)
  int* flags;          // [0] error code, [1] refinement failure
  // Device-side control of FSI iterations launched ahead of their convergence test (null:
  // the host decides).  gate[0] = 1 once this step's iterations have converged,
  // gate[1] = 1 when they must stop for the host (error, refinement failure, or the
  // launched iterations ran out).  Iteration kernels return at once when either is set;
  // the kernels after convergence (finish, corrector) run only when gate[0] = 1 and
  // gate[1] = 0.
  const int* gate;
  double* delta;       // [0] max |delta| of the last update
};

// Per-instance entries of the FSI launches that take many instances at once (ib_batch_*).
struct BeamJob {
  FsiArgs a;
  int bi, m;  // deformable body index and its point count
};
struct UpdateJob {
  FsiArgs a;
  double tol;
  int fixed;
  int nb;  // workgroups of this instance (update_blocks)
};
template <typename T>
struct SpreadJob {
  FsiArgs a;
  int jlo, jhi, ilo, ihi;
  T* out;
  int po;
};
struct MatvecJob {
  const double* A;
  int pa;
  const double* x;
  double* y;
  int n;
};
struct GemmJob {
  const double* A;
  const double* B;
  double* C;
  int n, p, two_minus;
  const int* gate;
};
struct RefineJob {
  const double* M;
  const double* X;
  int pm;
  const double* b;
  double* f;
  int n, rw, tpr, maxit, guess;
  double* ws;
  double* out;
  int* flags;
  const int* gate;
  double* xcopy;
  int nb;
  long spin;  // bound on the barrier's spins (0: the default)
};
// Launch shape of one refinement (as launch_refine chooses it); false if n is too large.
struct RefineShape {
  int nb, rw, tpr;
  bool cache;
  size_t lds;
  bool two;  // more than 32 workgroups: the shares are summed in slices (two barriers a sweep)
};
bool refine_shape(int n, RefineShape* out);
// Workgroups of k_update for nf stress unknowns.
int update_blocks(int nf);
// Dynamic LDS of the sub-domain Schur assembly (0 if it does not fit).
size_t schur_lds_bytes(const FsiArgs& a);
size_t beam_lds(int m);
constexpr int SPREAD_TILE_X = 64, SPREAD_TILE_Y = 4, SPREAD_ROWS_MAX = 4096;

template <typename T>
hipError_t launch_body_ops_multi(const FsiArgs* tab, int count, int max_npts, int it,
                                 hipStream_t st);
hipError_t launch_schur_sd_multi(const FsiArgs* tab, int count, int max_nf, size_t lds, int it,
                                 hipStream_t st);
// launch_body_ops_multi and launch_beam_multi (nbeam >= 1 jobs) in one launch.
template <typename T>
hipError_t launch_ops_beam_multi(const FsiArgs* fa, int ni, int max_npts, const BeamJob* beams,
                                 int nbeam, int max_m, size_t lds, int it, hipStream_t st);
hipError_t launch_beam_multi(const BeamJob* tab, int count, int max_m, size_t lds, int it,
                             hipStream_t st);
hipError_t launch_update_multi(const UpdateJob* tab, int count, int max_nb, int it, int K,
                               hipStream_t st);
hipError_t launch_finish_multi(const FsiArgs* tab, int count, hipStream_t st);
template <typename T>
hipError_t launch_spread_multi(const SpreadJob<T>* tab, int count, int max_gx, int max_gy,
                               int max_nf, hipStream_t st);
hipError_t launch_matvec_multi(const MatvecJob* tab, int count, int max_n, hipStream_t st);
// Waves per workgroup of the FP64 product, each taking an equal share of the k range.
constexpr int GEMM_KS = 8;
// k steps (of 4) per chunk of a wave such that n <= GEMM_ONE_N takes one chunk per wave.
constexpr int GEMM_KC = (52 + GEMM_KS - 1) / GEMM_KS;
constexpr int GEMM_ONE_N = 4 * GEMM_KC * GEMM_KS;
// kc52: every entry has n <= GEMM_ONE_N (the k range of each wave in one chunk); otherwise none has
hipError_t launch_gemm64_multi(const GemmJob* tab, int count, int max_n, int kc52,
                               hipStream_t st);
// cache: 0 uncached rows, 1 LDS-cached rows, 2 cached rows summed in slices (RefineShape::two)
hipError_t launch_refine_multi(const RefineJob* tab, int count, int max_nb, size_t lds, int cache,
                               hipStream_t st);
hipError_t launch_step_reset_multi(int* const* ctls, int count, hipStream_t st);
// out[FsiCtl::BYTES / 4 * b + i] = ctls[b][i]
hipError_t launch_gather_ctl(int* const* ctls, int count, int* out, hipStream_t st);

// Rows of the offline stage: body rows (from the operator arrays) or sub-domain points.
struct OffRows {
  int kind;  // 0: body rows from st arrays, 1: sub-domain points
  const int* st_base;
  const double* st_w;
  int sd_ngrid, sd_total;
  SdBoxes sdb;
  const double* app_xy;
  int n;
  double h, x0, y0;
};

template <typename T>
hipError_t launch_body_ops(const FsiArgs& a, hipStream_t st);
// No-slip residual of the last step and the force of every body (see k_outputs): out holds
// 1 + 2 nbodies doubles; s0 is level 0's streamfunction (ring included, pitch ps).
template <typename T>
hipError_t launch_outputs(const FsiArgs& a, const T* s0, int ps, double* out, hipStream_t st);
// LDS of the sub-domain Schur assembly per body row (acc, pw, cid, pidx) and its cap
constexpr size_t SCHUR_LDS_PER_ROW = 4 * (8 + 8 + 4 + 4);
constexpr size_t SCHUR_LDS_PER_ROW_ALL4 = 4 * (4 * 8 + 8 + 4 + 4);  // four hat points at once
constexpr size_t SCHUR_LDS_MAX = 150 * 1024;
// The four B' rows of a Schur row are scanned at once up to this much LDS per workgroup (one
// round of dependent loads instead of four); larger systems scan them one after another in a
// quarter of the LDS, so that several workgroups share a CU (the rows of M are the same)
constexpr size_t SCHUR_LDS_ALL4_MAX = 40 * 1024;
hipError_t launch_schur_sd(const FsiArgs& a, hipStream_t st);
// G[t][c0 + b] = vals[b][t] for the ns point-source columns of one offline batch
hipError_t launch_cols_to_matrix(const double* vals, int nf, int ns, int c0, double* G, int pm,
                                 hipStream_t st);
hipError_t launch_lu_solve(double* M, int pm, double* B, int pb, int n, int nrhs, int* flags,
                           hipStream_t st);
hipError_t launch_matvec(const double* A, int pa, const double* x, double* y, int n, hipStream_t st);
// Structure update; with a.gate set the last workgroup also runs the convergence test of
// iteration `it` of K launched ahead (tolerance tol, or a fixed count).
hipError_t launch_update(const FsiArgs& a, int it, int K, double tol, int fixed, hipStream_t st);
hipError_t launch_beam(const FsiArgs& a, int bi, int m, hipStream_t st);
// k_body_ops and k_beam (deformable body bi, m points) in one launch.
template <typename T>
hipError_t launch_ops_beam(const FsiArgs& a, int bi, int m, hipStream_t st);
hipError_t launch_finish(const FsiArgs& a, hipStream_t st);
// finish: one more workgroup runs k_finish's structure update (the spread reads none of the
// structure state that it writes, and both run only after converged iterations)
template <typename T>
hipError_t launch_spread(const FsiArgs& a, int jlo, int jhi, int ilo, int ihi, T* out, int po,
                         hipStream_t st, bool finish = false);
hipError_t launch_point_source_rowdst(const OffRows& o, int col0, int ncols, int nslots,
                                      const void* tw, double* out, int po, size_t bso,
                                      int* rows_first, hipStream_t st);
hipError_t launch_sample(const OffRows& o, int ntarget, const double* sl, int ps, size_t bss,
                         double* vals, int nslots, hipStream_t st);
hipError_t launch_filter_compact(const double* vals, int ntarget, int col0, int ncols, int nslots,
                                 double eps, int* out_col, double* out_val, int* counts,
                                 hipStream_t st);
hipError_t launch_gather_batch(const int* cols, const double* vals, int ntarget, const int* counts,
                               int nslots, int* out_col, double* out_val, hipStream_t st);
hipError_t launch_beam_init(const FsiArgs& a, hipStream_t st);
// f = M^{-1} b by refinement with the approximate inverse X, starting from X b or, with
// guess != 0, from the f passed in; ws holds refine_ws_doubles(n, maxit) doubles;
// out[0] = final relative residual, out[1] = sweeps, out[2] = 1 when `partial` is set and
// the maxit sweeps ran out before convergence (the caller continues with guess = 1);
// otherwise flags[1] is raised when the residual stays above 1e-9
// With ua set, the same launch then runs the structure update of FSI iteration uit of uK
// (launch_update's work, tolerance utol, fixed iteration count ufixed) with the new f.
hipError_t launch_refine(const double* M, int pm, const double* X, const double* b, double* f,
                         int n, int maxit, int guess, double* ws, double* out, int* flags,
                         const int* gate, double* xcopy, long spin, hipStream_t st,
                         const FsiArgs* ua = nullptr, int uit = 0, int uK = 0, double utol = 0.0,
                         int ufixed = 0);
// Whether a refinement of n unknowns fits on the device at once (all its workgroups resident,
// which its device-wide barrier needs); have / need: resident capacity and workgroups.
bool refine_coresident(int n, int* have, int* need);
size_t refine_ws_doubles(int n, int maxit);
hipError_t launch_identity(double* X, int p, int n, hipStream_t st);
// *out (zeroed by the caller) folds in max |W - I| over the n x n matrix (+Inf if not finite)
hipError_t launch_eye_resid(const double* W, int p, int n, double* out, hipStream_t st);
hipError_t launch_gemm64(const double* A, const double* B, double* C, int n, int p, int two_minus,
                         hipStream_t st, const int* gate = nullptr);
// Device-side FSI control (FsiCtl): clear it at the start of a step.
hipError_t launch_step_reset(int* ctl, hipStream_t st);

}  // namespace ib
