// Kernels of the FSI loop and of the offline stage.
//
// Body operator (Sec. 3.1): every stress row a (one component of one body point) is
// a window of 4 x 4 faces with weights.  Exact mode uses the true interpolation E
// (eq. (24), 3-point kernel of Roma et al.); sub-domain mode uses P E0 (eqs. (22),
// (26)-(29)): the hat interpolation over the 4 surrounding sub-domain vertices of
// their E0 rows, or weight 1 on an appended exact point.
//
// FSI iteration (eqs. (17)-(19) / (37)-(39)): body operator and u* = (1/h) E (C s* +
// q_inf), flow block of the Schur matrix (stationary inverse, or P B' P^T from the
// CSR of B'), structural blocks and right-hand side, LU solve for f, structure
// update and the convergence measure.  The host reads the measure and decides.
#include <math.h>

#include "ib_body.hpp"
#include "ib_internal.hpp"
#include "ib_fft.hpp"

namespace ib {

// FSI iteration kernels: skip when the step's iterations have converged or were stopped.
__device__ __forceinline__ bool iter_gated(const int* gate) {
  return gate != nullptr && (gate[0] != 0 || gate[1] != 0);
}
// Kernels after convergence: run only when the iterations converged and were not stopped.
__device__ __forceinline__ bool post_gated(const int* gate) {
  return gate != nullptr && (gate[0] != 1 || gate[1] != 0);
}


// Rectangle k of a sub-domain (origin, points per side, first point), read with constant
// indices only: the boxes sit in kernel arguments, and an index known only at run time would
// make every field a memory load of its own.
struct SdBox {
  int i0, j0, npx, npy, off;
};
__device__ __forceinline__ SdBox sd_box(const SdBoxes& s, int k) {
  int i0 = s.i0[0], j0 = s.j0[0], npx = s.npx[0], npy = s.npy[0], off = s.off[0];
#pragma unroll
  for (int q = 1; q < SD_MAX_BOXES; ++q) {
    const bool m = k == q;
    i0 = m ? s.i0[q] : i0;
    j0 = m ? s.j0[q] : j0;
    npx = m ? s.npx[q] : npx;
    npy = m ? s.npy[q] : npy;
    off = m ? s.off[q] : off;
  }
  return SdBox{i0, j0, npx, npy, off};
}

__device__ __forceinline__ double roma3(double r) {
  const double a = fabs(r);
  if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
  if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(fmax(0.0, 1.0 - 3.0 * (1.0 - a) * (1.0 - a)))) / 6.0;
  return 0.0;
}

__device__ __forceinline__ double peskin4(double r) {
  const double a = fabs(r);
  if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(fmax(0.0, -7.0 + 12.0 * a - 4.0 * a * a))) / 8.0;
  return 0.0;
}

// True-E window of a point for one component (0: x-faces, 1: y-faces).  kind 0: the 3-point
// kernel, 3 x 3 faces about the nearest face; kind 1: the 4-point kernel, the 4 x 4 faces
// within two cells (from floor(r) - 1 along each axis, r the point in face units).
__device__ void exact_window(double px, double py, int comp, double x0, double y0, double h,
                             int* base, double* w, int kind) {
  for (int e = 0; e < 16; ++e) w[e] = 0.0;
  if (kind == 1) {
    const double rx = comp == 0 ? (px - x0) / h : (px - x0) / h - 0.5;
    const double ry = comp == 0 ? (py - y0) / h - 0.5 : (py - y0) / h;
    base[0] = (int)floor(rx) - 1;
    base[1] = (int)floor(ry) - 1;
    for (int dj = 0; dj < 4; ++dj) {
      const int j = base[1] + dj;
      const double fy = comp == 0 ? y0 + h * (j + 0.5) : y0 + h * j;
      const double wy = peskin4((fy - py) / h);
      for (int di = 0; di < 4; ++di) {
        const int i = base[0] + di;
        const double fx = comp == 0 ? x0 + h * i : x0 + h * (i + 0.5);
        w[dj * 4 + di] = wy * peskin4((fx - px) / h);
      }
    }
    return;
  }
  int ic, jc;
  if (comp == 0) {
    ic = (int)rint((px - x0) / h);
    jc = (int)rint((py - y0) / h - 0.5);
  } else {
    ic = (int)rint((px - x0) / h - 0.5);
    jc = (int)rint((py - y0) / h);
  }
  base[0] = ic - 1;
  base[1] = jc - 1;
  for (int dj = 0; dj < 3; ++dj) {
    const int j = jc - 1 + dj;
    const double fy = comp == 0 ? y0 + h * (j + 0.5) : y0 + h * j;
    const double wy = roma3((fy - py) / h);
    for (int di = 0; di < 3; ++di) {
      const int i = ic - 1 + di;
      const double fx = comp == 0 ? x0 + h * i : x0 + h * (i + 0.5);
      w[dj * 4 + di] = wy * roma3((fx - px) / h);
    }
  }
}

// E0 row of sub-domain grid vertex (p, q) added with weight c into the window at base.
__device__ void add_e0_vertex(int p, int q, int comp, double c, double x0, double y0, double h,
                              const int* base, double* w) {
  const double px = x0 + p * h, py = y0 + q * h;
  for (int dj = 0; dj < 4; ++dj) {
    const int j = base[1] + dj;
    const double fy = comp == 0 ? y0 + h * (j + 0.5) : y0 + h * j;
    const double wy = roma3((fy - py) / h);
    if (wy == 0.0) continue;
    for (int di = 0; di < 4; ++di) {
      const int i = base[0] + di;
      const double fx = comp == 0 ? x0 + h * i : x0 + h * (i + 0.5);
      w[dj * 4 + di] += c * (wy * roma3((fx - px) / h));
    }
  }
}

// The faces touched with nonzero weight must have both end vertices interior.
__device__ bool window_ok(const int* base, const double* w, int comp, int n) {
  for (int dj = 0; dj < 4; ++dj)
    for (int di = 0; di < 4; ++di) {
      if (w[dj * 4 + di] == 0.0) continue;
      const int i = base[0] + di, j = base[1] + dj;
      if (comp == 0) {
        if (i < 1 || i > n - 1 || j < 1 || j > n - 2) return false;
      } else {
        if (i < 1 || i > n - 2 || j < 1 || j > n - 1) return false;
      }
    }
  return true;
}

template <typename T>
__device__ __forceinline__ double face_flux(const T* s, int ps, int comp, int i, int j, double ux,
                                            double uy) {
  if (comp == 0) return ((double)s[(size_t)(j + 1) * ps + i] - (double)s[(size_t)j * ps + i]) + ux;
  return -((double)s[(size_t)j * ps + i + 1] - (double)s[(size_t)j * ps + i]) + uy;
}

// Hinge and reference angle of a torsional body at t_{n+1}: its own, or those of its mount
// (Sec. 5.1's passive plate rides on the driven plate).
__device__ __forceinline__ void tors_frame(const FsiArgs& a, const BodyDev& b, double* hx,
                                           double* hy, double* ang0) {
  if (b.moff < 0) {
    *hx = b.hx;
    *hy = b.hy;
    *ang0 = b.theta0;
    return;
  }
  const double* q = a.poses + b.moff;
  *hx = q[MF_HX];
  *hy = q[MF_HY];
  *ang0 = q[MF_ANG];
}

// g of the torsional equation (Sec. 2.1 eq. (4); Appendix A r_phi) at deflection th: the
// body's constant, or for a mounted body the pseudo-moment of its moving hinge,
// -I_H alpha_dd - m r_G x a_H with r_G = cg (cos, sin)(angle), evaluated at t_{n+1} and the
// current iterate (for Sec. 5.1's two plates this is the right-hand side of its equation
// of motion beyond the fluid moment).
__device__ __forceinline__ double tors_g(const FsiArgs& a, const BodyDev& b, const double* ts,
                                         double th) {
  if (b.moff < 0) return ts[TS_G];
  const double* q = a.poses + b.moff;
  const double ph = q[MF_ANG] + th;
  return -b.inertia * q[MF_AL] - b.mass * b.cg * (cos(ph) * q[MF_AY] - sin(ph) * q[MF_AX]);
}

__device__ void point_position(const FsiArgs& a, const BodyDev& b, int local, double* px,
                               double* py) {
  if (b.kind == BODY_RIGID) {
    *px = a.rigid_xy[2 * (b.pt0 + local)];
    *py = a.rigid_xy[2 * (b.pt0 + local) + 1];
  } else if (b.kind == BODY_MOVING) {
    const double* q = a.poses + 6 * b.tors;
    const double rx = a.rigid_xy[2 * (b.pt0 + local)], ry = a.rigid_xy[2 * (b.pt0 + local) + 1];
    const double c = cos(q[2]), sn = sin(q[2]);
    *px = q[0] + c * rx - sn * ry;
    *py = q[1] + sn * rx + c * ry;
  } else if (b.kind == BODY_TORSIONAL) {
    const double* ts = a.tors + b.tors * TS_COUNT;
    const double th = a.iter == 0 ? ts[TS_THETA] : ts[TS_NEW];
    double hx, hy, ang0;
    tors_frame(a, b, &hx, &hy, &ang0);
    const double ang = ang0 + th;
    const double r = local * b.ds;
    *px = hx + r * cos(ang);
    *py = hy + r * sin(ang);
  } else {
    const double* c = a.iter == 0 ? a.chi : a.chi_new;
    *px = c[b.dof0 + 3 * local];
    *py = c[b.dof0 + 3 * local + 1];
  }
}

// The structural part subtracted from row (comp, local) of the Schur right-hand side:
//   rigid       the prescribed velocity u_b (if any)
//   moving      (vx, vy) + omega e_z x (R(angle) xy_ref) at t_{n+1}
//   torsional   S ((2/dt) r_phi / J - r_theta), plus on a mount the driver's velocity at the
//               point, v_H + omega e_z x (p - H)
//   deformable  0 here; k_schur_sd subtracts T ((2/dt)(chi^k + J_d^{-1} res) - r_chi)
__device__ double rhs_body_term(const FsiArgs& a, const BodyDev& b, int local, int comp) {
  const int m = b.npts;
  if (b.kind == BODY_RIGID) {
    return b.has_ub ? a.rigid_ub[2 * (b.pt0 + local) + comp] : 0.0;
  } else if (b.kind == BODY_MOVING) {
    const double* q = a.poses + 6 * b.tors;
    const double c = cos(q[2]), sn = sin(q[2]);
    const double rx = a.rigid_xy[2 * (b.pt0 + local)], ry = a.rigid_xy[2 * (b.pt0 + local) + 1];
    const double wx = c * rx - sn * ry, wy = sn * rx + c * ry;
    return comp == 0 ? q[3] - q[5] * wy : q[4] + q[5] * wx;
  } else if (b.kind == BODY_TORSIONAL) {
    const double dt = a.dt;
    const double* ts = a.tors + b.tors * TS_COUNT;
    const double th = a.iter == 0 ? ts[TS_THETA] : ts[TS_NEW];
    double hx, hy, ang0;
    tors_frame(a, b, &hx, &hy, &ang0);
    const double ang = ang0 + th;
    const double sn = sin(ang), cs = cos(ang);
    const double jt = 4.0 * b.inertia / (dt * dt) + 2.0 * b.damping / dt + b.stiffness;
    const double rphi = b.inertia * (4.0 * ts[TS_THETA] / (dt * dt) + 4.0 * ts[TS_PHI] / dt + ts[TS_PHIDOT]) +
                        b.damping * (2.0 * ts[TS_THETA] / dt + ts[TS_PHI]) + tors_g(a, b, ts, th);
    const double rth = ts[TS_PHI] + 2.0 * ts[TS_THETA] / dt;
    const double rc = (2.0 / dt) * rphi / jt - rth;
    const double r = local * b.ds;
    const double su = (comp == 0 ? -sn : cs) * r;
    (void)m;
    double v = su * rc;
    if (b.moff >= 0) {
      const double* q = a.poses + b.moff;
      v += comp == 0 ? q[MF_VX] - q[MF_OM] * r * sn : q[MF_VY] + q[MF_OM] * r * cs;
    }
    return v;
  }
  return 0.0;
}

// Body operator rows, u* and the Schur right-hand side for every point and velocity
// component (one thread each, the two of a point adjacent); point 0 also clears the
// convergence maximum that k_update folds into.  Launches take 2 npts threads.  Every global
// load comes before the first global store: the memory counter a wait uses also counts
// stores, so a load after a store would wait for that store's acknowledgement as well.
template <typename T>
__device__ __forceinline__ void body_ops_body(const FsiArgs& a, int bx) {
  if (iter_gated(a.gate)) return;
  const int t = bx * blockDim.x + threadIdx.x;
  const int p = t >> 1, comp = t & 1;
  if (p >= a.npts) return;
  int bi = 0;
  while (bi + 1 < a.nbodies && a.bodies[bi + 1].pt0 <= p) ++bi;
  const BodyDev b = a.bodies[bi];
  const int local = p - b.pt0;
  double px, py;
  point_position(a, b, local, &px, &py);
  const T* s = static_cast<const T*>(a.sstar);
  const int row = 2 * b.pt0 + comp * b.npts + local;
  int base[2];
  double w[16];
  // the P row of a sub-domain point (slots and hat weights) and the slots it names (act)
  int pidx[4] = {0, 0, 0, 0};
  double pw[4] = {0.0, 0.0, 0.0, 0.0};
  int nact = 0;  // act entries to set: pidx[e] for e < nact with pw[e] != 0 (rigid: e = 0)
  int flag = 0;  // error code for flags[0]
  if (!a.use_sd) {
    exact_window(px, py, comp, a.x0, a.y0, a.h, base, w, a.delta_kind);
  } else if (b.kind == BODY_RIGID) {
    const int app = a.sd_ngrid + b.app0 + local;
    exact_window(px, py, comp, a.x0, a.y0, a.h, base, w, a.delta_kind);
    for (int e = 0; e < 4; ++e) {
      pidx[e] = comp * a.sd_total + app;
      pw[e] = e == 0 ? 1.0 : 0.0;
    }
    nact = 1;
  } else {
    // the body's rectangle of the sub-domain
    const SdBox bb = sd_box(a.sdb, b.sdbox);
    const int bi0 = bb.i0, bj0 = bb.j0, npx = bb.npx, npy = bb.npy;
    const double xs0 = a.x0 + bi0 * a.h, ys0 = a.y0 + bj0 * a.h;
    const double rx = (px - xs0) / a.h, ry = (py - ys0) / a.h;
    const double tol = 1e-9;
    if (!(rx >= -tol && ry >= -tol && rx <= npx - 1 + tol && ry <= npy - 1 + tol)) {
      flag = 1;  // out of sub-domain (or non-finite position)
      for (int e = 0; e < 16; ++e) w[e] = 0.0;
      base[0] = base[1] = 2;
    } else {
      int ix = (int)floor(rx), iy = (int)floor(ry);
      ix = ix < 0 ? 0 : (ix > npx - 2 ? npx - 2 : ix);
      iy = iy < 0 ? 0 : (iy > npy - 2 ? npy - 2 : iy);
      const double fx = rx - ix, fy = ry - iy;
      const int gp = bi0 + ix, gq = bj0 + iy;
      base[0] = gp - 1;
      base[1] = gq - 1;
      for (int e = 0; e < 16; ++e) w[e] = 0.0;
      const double hw[4] = {(1.0 - fx) * (1.0 - fy), fx * (1.0 - fy), (1.0 - fx) * fy, fx * fy};
      const int dx[4] = {0, 1, 0, 1}, dy[4] = {0, 0, 1, 1};
      // E0 row of a vertex: the kernel at offsets (-1, 0, 1) across the component's
      // faces and (-1/2, 1/2) along them (the same pattern at every vertex)
      const double k0 = roma3(0.0), k1 = roma3(1.0), kh = roma3(0.5);
      const double across[3] = {k1, k0, k1};
      for (int e = 0; e < 4; ++e) {
        pidx[e] = comp * a.sd_total + bb.off + (iy + dy[e]) * npx + (ix + dx[e]);
        pw[e] = hw[e];
        for (int u = 0; u < 3; ++u)
          for (int v = 0; v < 2; ++v) {
            const double c = hw[e] * (across[u] * kh);
            if (comp == 0) w[(dy[e] + v) * 4 + dx[e] + u] += c;
            else w[(dy[e] + u) * 4 + dx[e] + v] += c;
          }
      }
      nact = 4;
    }
  }
  if (!window_ok(base, w, comp, a.n)) {
    flag = 2;  // near the boundary: keep every later access in bounds
    for (int e = 0; e < 16; ++e) w[e] = 0.0;
    base[0] = base[1] = 2;
  }
  // all 16 face fluxes of the window are loaded at once, then summed in window order;
  // indices are clamped to [0, n-1] (every access stays inside the (n+1)-row array):
  // that changes none of the nonzero-weight faces (window_ok), and the others carry
  // weight 0 on a finite value
  double fl[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int fi = min(max(base[0] + (e & 3), 0), a.n - 1);
    const int fj = min(max(base[1] + (e >> 2), 0), a.n - 1);
    fl[e] = face_flux(s, a.ps, comp, fi, fj, a.ux, a.uy);
  }
  const double term = rhs_body_term(a, b, local, comp);
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc += w[e] * fl[e];
  const double us = acc / a.h;
  // the stores
  if (p == 0 && comp == 0) a.delta[0] = 0.0;
  if (comp == 0) {
    a.pos[2 * p] = px;
    a.pos[2 * p + 1] = py;
  }
  if (flag == 1) atomicMax(&a.flags[0], 1);
  if (flag == 2) atomicMax(&a.flags[0], 2);
  if (a.use_sd) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a.p_idx[4 * row + e] = pidx[e];
      a.p_w[4 * row + e] = pw[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e < nact && (nact == 1 || pw[e] != 0.0))
        a.act[pidx[e]] = 4 * row + e;  // any writer of a shared row wins
  }
  a.st_base[3 * row] = base[0];
  a.st_base[3 * row + 1] = base[1];
  a.st_base[3 * row + 2] = comp;
#pragma unroll
  for (int e = 0; e < 16; ++e) a.st_w[16 * row + e] = w[e];
  a.ustar[row] = us;
  a.rhs[row] = us - term;
}

template <typename T>
__global__ void k_body_ops(FsiArgs a) {
  body_ops_body<T>(a, blockIdx.x);
}

// Many instances per launch (ib_batch_*): instance blockIdx.y's arguments from tab, at FSI
// iteration `it`.
template <typename T>
__global__ void k_body_ops_multi(const FsiArgs* __restrict__ tab, int it) {
  FsiArgs a = tab[blockIdx.y];
  a.iter = it;
  body_ops_body<T>(a, blockIdx.x);
}

__device__ __forceinline__ double row_ds(const FsiArgs& a, int row) {
  // rows of body bi are 2 pt0 .. 2 pt0 + 2m - 1
  int bi = 0;
  while (bi + 1 < a.nbodies && 2 * a.bodies[bi + 1].pt0 <= row) ++bi;
  return a.bodies[bi].ds;
}

__device__ __forceinline__ int row_body(const FsiArgs& a, int row) {
  int bi = 0;
  while (bi + 1 < a.nbodies && 2 * a.bodies[bi + 1].pt0 <= row) ++bi;
  return bi;
}

// Schur matrix in sub-domain mode, one workgroup per row a:
//   M_ab = (dt/h^2) (P B' P^T)_ab ds_b + structural block of the body owning a and b:
//   torsional (2 ds/dt) S_a S_b / J,  deformable (2 ds/dt) (T J_d^{-1} T^T)_ab, the latter
//   from the columns J_d^{-1} T^T that k_beam left in ywork (so it runs first).
// For each of the (up to 4) B' rows that P uses in row a, the CSR row is scanned once
// and the entries in columns that P uses anywhere are scattered into an LDS vector
// indexed by the P slot that names the column (act, set by k_body_ops: one slot per used
// B' row; each slot's canonical id is the act entry of its row); row a of P B' P^T is then
// a gather from that vector.  With all4 (when the LDS allows) the four CSR rows are
// scanned together into four vectors.
// Dynamic LDS: acc, pw (4 nf doubles each), cid, pidx (4 nf ints each).
constexpr int SCHUR_NT = 256;
constexpr int SCHUR_CPT = 8;  // columns per thread: nf <= 2048
__device__ __forceinline__ void schur_sd_body(const FsiArgs& a, int all4, int bx) {
  if (iter_gated(a.gate)) return;
  extern __shared__ double ssm[];
  const int nf = a.nf, ns = 4 * nf, r = bx, tid = threadIdx.x;
  double m[SCHUR_CPT];
  if (a.gx == nullptr && all4) {
    // the CSR rows of all four hat points of row r are scanned together into four LDS
    // vectors (one round of dependent loads instead of four)
    double* acc = ssm;  // 4 x ns
    double* pw = acc + 4 * ns;
    int* cid = reinterpret_cast<int*>(pw + ns);
    int* pidx = cid + ns;
    for (int e = tid; e < ns; e += SCHUR_NT) {
      const double w = a.p_w[e];
      const int pi = a.p_idx[e];
      pw[e] = w;
      pidx[e] = pi;
      cid[e] = w != 0.0 ? a.act[pi] : -1;  // the slot that names this B' row (act)
    }
    for (int e = tid; e < 4 * ns; e += SCHUR_NT) acc[e] = 0.0;
    __syncthreads();
    double wu[4];
    int64_t lo[4], off[5];
    off[0] = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      wu[u] = pw[4 * r + u];
      const int cu = pidx[4 * r + u];
      lo[u] = wu[u] != 0.0 ? a.bp_ptr[cu] : 0;
      const int64_t hi = wu[u] != 0.0 ? a.bp_ptr[cu + 1] : 0;
      off[u + 1] = off[u] + (hi - lo[u]);
    }
    constexpr int Q = 8;
    for (int64_t e0 = 0; e0 < off[4]; e0 += (int64_t)Q * SCHUR_NT) {
      int j[Q], id[Q], uq[Q];
      double v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t e = e0 + tid + (int64_t)q * SCHUR_NT;
        const int u = e < off[1] ? 0 : (e < off[2] ? 1 : (e < off[3] ? 2 : 3));
        const int64_t src = lo[u] + (e - off[u]);
        uq[q] = u;
        j[q] = e < off[4] ? a.bp_col[src] : -1;
        v[q] = e < off[4] ? a.bp_val[src] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) id[q] = j[q] >= 0 ? a.act[j[q]] : -1;
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (id[q] >= 0 && id[q] < ns && pw[id[q]] != 0.0 && pidx[id[q]] == j[q])
          acc[uq[q] * ns + id[q]] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCHUR_CPT; ++k) {
      m[k] = 0.0;
      const int c = tid + k * SCHUR_NT;
      if (c >= nf) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (wu[u] == 0.0) continue;
        double inner = 0.0;
        for (int w = 0; w < 4; ++w) {
          const double wv = pw[4 * c + w];
          if (wv != 0.0) inner += wv * acc[u * ns + cid[4 * c + w]];
        }
        m[k] += wu[u] * inner;
      }
    }
  } else if (a.gx != nullptr) {
    // exact operator of this iterate (moving bodies without a sub-domain)
#pragma unroll
    for (int k = 0; k < SCHUR_CPT; ++k) {
      const int c = tid + k * SCHUR_NT;
      m[k] = c < nf ? a.gx[(size_t)r * a.pm + c] : 0.0;
    }
  } else {
    double* acc = ssm;
    double* pw = acc + ns;
    int* cid = reinterpret_cast<int*>(pw + ns);
    int* pidx = cid + ns;
    for (int e = tid; e < ns; e += SCHUR_NT) {
      const double w = a.p_w[e];
      const int pi = a.p_idx[e];
      pw[e] = w;
      pidx[e] = pi;
      cid[e] = w != 0.0 ? a.act[pi] : -1;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCHUR_CPT; ++k) m[k] = 0.0;
    for (int u = 0; u < 4; ++u) {
      const double wu = pw[4 * r + u];
      if (wu == 0.0) continue;  // uniform over the workgroup
      const int cu = pidx[4 * r + u];
      for (int e = tid; e < ns; e += SCHUR_NT) acc[e] = 0.0;
      __syncthreads();
      const int64_t lo = a.bp_ptr[cu], hi = a.bp_ptr[cu + 1];
      constexpr int Q = 4;
      for (int64_t e0 = lo; e0 < hi; e0 += (int64_t)Q * SCHUR_NT) {
        int j[Q], id[Q];
        double v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int64_t e = e0 + tid + (int64_t)q * SCHUR_NT;
          j[q] = e < hi ? a.bp_col[e] : -1;
          v[q] = e < hi ? a.bp_val[e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) id[q] = j[q] >= 0 ? a.act[j[q]] : -1;
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (id[q] >= 0 && id[q] < ns && pw[id[q]] != 0.0 && pidx[id[q]] == j[q]) acc[id[q]] = v[q];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < SCHUR_CPT; ++k) {
        const int c = tid + k * SCHUR_NT;
        if (c < nf) {
          double inner = 0.0;
          for (int v = 0; v < 4; ++v) {
            const double wv = pw[4 * c + v];
            if (wv != 0.0) inner += wv * acc[cid[4 * c + v]];
          }
          m[k] += wu * inner;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < SCHUR_CPT; ++k) {
    const int c = tid + k * SCHUR_NT;
    if (c >= nf) continue;
    const int bc = row_body(a, c);
    const BodyDev b = a.bodies[bc];
    double mv = (a.dt / (a.h * a.h)) * m[k] * b.ds;
    const int r0 = 2 * b.pt0, mpts = b.npts;
    if (r >= r0 && r < r0 + 2 * mpts && (b.kind == BODY_TORSIONAL || b.kind == BODY_DEFORMABLE)) {
      const int u = r - r0, v = c - r0;
      const double coef = 2.0 * b.ds / a.dt;
      if (b.kind == BODY_TORSIONAL) {
        const double* ts = a.tors + b.tors * TS_COUNT;
        const double th = a.iter == 0 ? ts[TS_THETA] : ts[TS_NEW];
        const double ang = (b.moff < 0 ? b.theta0 : a.poses[b.moff + MF_ANG]) + th;
        const double sn = sin(ang), cs = cos(ang);
        const double dt = a.dt;
        const double jt = 4.0 * b.inertia / (dt * dt) + 2.0 * b.damping / dt + b.stiffness;
        const double su = (u < mpts ? -sn : cs) * (u % mpts) * b.ds;
        const double sv = (v < mpts ? -sn : cs) * (v % mpts) * b.ds;
        mv += (coef / jt) * su * sv;
      } else {
        const int node = u % mpts, cmp = u / mpts;
        if (node > 0) {
          const int du = 3 * node + cmp - 3;
          mv += coef * a.ywork[b.yoff + (size_t)du * (2 * mpts + 1) + v];
        }
      }
    }
    a.M[(size_t)r * a.pm + c] = mv;
  }
  // a deformable body's row: the right-hand side loses T ((2/dt)(chi^k + J_d^{-1} res) -
  // r_chi) (eqs. (17) and (37)), with the solve J_d^{-1} res that k_beam left in column 2m
  // of ywork
  if (tid == 0) {
    const BodyDev b = a.bodies[row_body(a, r)];
    if (b.kind == BODY_DEFORMABLE) {
      const int m = b.npts, u = r - 2 * b.pt0, node = u % m, cmp = u / m;
      if (node > 0) {
        const int g = 3 * node + cmp, ncol = 2 * m + 1;
        const double* ck = (a.iter == 0 ? a.chi : a.chi_new) + b.dof0;
        const double pred = ck[g] + a.ywork[b.yoff + (size_t)(g - 3) * ncol + 2 * m];
        const double rchi = a.zeta[b.dof0 + g] + 2.0 * a.chi[b.dof0 + g] / a.dt;
        a.rhs[r] -= (2.0 / a.dt) * pred - rchi;
      }
    }
  }
}

__global__ __launch_bounds__(SCHUR_NT) void k_schur_sd(FsiArgs a, int all4) {
  schur_sd_body(a, all4, blockIdx.x);
}

__device__ __forceinline__ int schur_all4(const FsiArgs& a) {
  return a.gx == nullptr && (size_t)a.nf * SCHUR_LDS_PER_ROW_ALL4 <= SCHUR_LDS_ALL4_MAX;
}

__global__ __launch_bounds__(SCHUR_NT) void k_schur_sd_multi(const FsiArgs* __restrict__ tab,
                                                             int it) {
  FsiArgs a = tab[blockIdx.y];
  a.iter = it;
  if ((int)blockIdx.x >= a.nf) return;
  schur_sd_body(a, schur_all4(a), blockIdx.x);
}

// -------------------------------------------------------- corotational beam
// Element internal force fe[6] and tangent ke[36] (Crisfield's 2-D corotational
// Euler-Bernoulli element; rotations relative to the straight reference).
__device__ void beam_element(const double* x, double l0, double beta0, double ea, double ei,
                             double* fe, double* ke) {
  const double dx = x[3] - x[0], dy = x[4] - x[1];
  const double len = sqrt(dx * dx + dy * dy);
  const double c = dx / len, s = dy / len;
  double al = atan2(dy, dx) - beta0;
  al = al - 2.0 * M_PI * floor((al + M_PI) / (2.0 * M_PI));
  double t1 = x[2] - al, t2 = x[5] - al;
  t1 = t1 - 2.0 * M_PI * floor((t1 + M_PI) / (2.0 * M_PI));
  t2 = t2 - 2.0 * M_PI * floor((t2 + M_PI) / (2.0 * M_PI));
  const double nax = ea * (len - l0) / l0;
  const double m1 = 2.0 * ei / l0 * (2.0 * t1 + t2);
  const double m2 = 2.0 * ei / l0 * (t1 + 2.0 * t2);
  const double r[6] = {-c, -s, 0.0, c, s, 0.0};
  const double z[6] = {s, -c, 0.0, -s, c, 0.0};
  double bm[3][6];
  for (int k = 0; k < 6; ++k) {
    bm[0][k] = r[k];
    bm[1][k] = (k == 2 ? 1.0 : 0.0) - z[k] / len;
    bm[2][k] = (k == 5 ? 1.0 : 0.0) - z[k] / len;
  }
  const double d[3][3] = {{ea / l0, 0.0, 0.0},
                          {0.0, 4.0 * ei / l0, 2.0 * ei / l0},
                          {0.0, 2.0 * ei / l0, 4.0 * ei / l0}};
  const double fl[3] = {nax, m1, m2};
  for (int k = 0; k < 6; ++k) fe[k] = bm[0][k] * fl[0] + bm[1][k] * fl[1] + bm[2][k] * fl[2];
  for (int p = 0; p < 6; ++p)
    for (int q = 0; q < 6; ++q) {
      double v = 0.0;
      for (int u = 0; u < 3; ++u) {
        double t = 0.0;
        for (int w = 0; w < 3; ++w) t += d[u][w] * bm[w][q];
        v += bm[u][p] * t;
      }
      v += (nax / len) * z[p] * z[q] + ((m1 + m2) / (len * len)) * (r[p] * z[q] + z[p] * r[q]);
      ke[p * 6 + q] = v;
    }
}

constexpr int MAX_BEAM_DOF = 600;  // free DOFs of one deformable body (<= 201 nodes)

constexpr int STRUCT_NT = 256;

// ------------------------------------------------ beam Jacobian: cyclic reduction
// J_d = 4 M/dt^2 + K(chi^k) over the free nodes is block tridiagonal with 3 x 3 blocks
// (node k+1 is block k): A_k on the diagonal, U_k = J(k, k+1), L_k = J(k, k-1).  It is
// factored by block cyclic reduction: at the level of stride s the blocks j with
// (j+1) mod 2s = s are eliminated into their neighbours j -+ s, which stay; every level
// is data parallel, so the sequential depth is log2(K) instead of K.  J_d is symmetric
// positive definite, so no pivoting is needed.  Each workgroup factors the same matrix
// (redundantly, no inter-workgroup traffic) and solves `nc` of the right-hand sides
// [T^T columns (2m, node 0's are zero), res].  Results go to ywork[u][2m+1].

// row-major 3 x 3 inverse entry (r, c) = cofactor(c, r) / det
__device__ inline double inv3_entry(const double* a, int r, int c) {
  auto cof = [&](int i, int j) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    return a[3 * i1 + j1] * a[3 * i2 + j2] - a[3 * i1 + j2] * a[3 * i2 + j1];
  };
  const double det = a[0] * cof(0, 0) + a[1] * cof(0, 1) + a[2] * cof(0, 2);
  return cof(c, r) / det;
}

constexpr int BEAM_NT = 512;
constexpr int BEAM_NC = 8;  // right-hand sides per workgroup
__device__ __forceinline__ void beam_body(const FsiArgs& a, int bi, int bx) {
  if (iter_gated(a.gate)) return;
  constexpr int NC = BEAM_NC;
  extern __shared__ double bsm[];
  const BodyDev b = a.bodies[bi];
  const int m = b.npts, K = m - 1, nd = 3 * K, ncol = 2 * m + 1;
  const int tid = threadIdx.x;
  const double dt = a.dt;
  double* A = bsm;           // 9K each: A, L, U contiguous
  double* Lb = A + 9 * K;
  double* Ub = Lb + 9 * K;
  double* Ai = Ub + 9 * K;   // inverse of A_j at the level that eliminates j
  double* P = Ai + 9 * K;    // per kept block and level: L_i A_{i-s}^{-1}, U_i A_{i+s}^{-1}
  double* rhs = P + 18 * K;  // [nd][NC]
  double* sres = rhs + nd * NC;
  double* ek = Ai;           // element forces and tangents [m-1][42], before Ai is used
  const double* ck = (a.iter == 0 ? a.chi : a.chi_new) + b.dof0;
  const double* xn = a.chi + b.dof0;
  const double* zn = a.zeta + b.dof0;
  const double* an = a.zetadot + b.dof0;
  const double* ms = a.dmass + b.dof0;
  double* sms = sres + nd;   // masses of the free DOFs
  // the free DOFs' masses and states are read first, so that their latency overlaps the
  // element phase (their loads would otherwise follow its barrier)
  constexpr int UPT = (MAX_BEAM_DOF + BEAM_NT - 1) / BEAM_NT;
  double pmass[UPT], px[UPT], pz[UPT], pa[UPT], pc[UPT];
#pragma unroll
  for (int q = 0; q < UPT; ++q) {
    const int u = tid + q * BEAM_NT, g = u + 3;
    pmass[q] = px[q] = pz[q] = pa[q] = pc[q] = 0.0;
    if (u < nd) {
      pmass[q] = ms[g];
      px[q] = xn[g];
      pz[q] = zn[g];
      pa[q] = an[g];
      pc[q] = ck[g];
    }
  }

  // element internal forces and tangents, one element per thread
  for (int el = tid; el < m - 1; el += BEAM_NT)
    beam_element(ck + 3 * el, a.l0[b.dof0 / 3 + el], a.beta0[b.dof0 / 3 + el], b.ea, b.ei,
                 ek + 42 * el, ek + 42 * el + 6);
#pragma unroll
  for (int q = 0; q < UPT; ++q)
    if (tid + q * BEAM_NT < nd) sms[tid + q * BEAM_NT] = pmass[q];
  __syncthreads();
  // blocks of node k+1: A_k from elements k (second node) and k+1 (first node),
  // U_k = J(k, k+1) from element k+1, L_k = J(k, k-1) from element k (node 0 is clamped)
  for (int e = tid; e < 27 * K; e += BEAM_NT) {
    const int blk = e / 9, w = e % 9, r = w / 3, c = w % 3;
    const int which = blk / K, k = blk % K;  // 0: A, 1: L, 2: U
    double v = 0.0;
    if (which == 0) {
      v = ek[42 * k + 6 + (r + 3) * 6 + c + 3];
      if (k + 1 <= m - 2) v += ek[42 * (k + 1) + 6 + r * 6 + c];
      if (r == c) v += 4.0 * sms[3 * k + c] / (dt * dt);  // ms[3 (k + 1) + c]
    } else if (which == 1) {
      if (k >= 1) v = ek[42 * k + 6 + (r + 3) * 6 + c];
    } else {
      if (k + 1 <= m - 2) v = ek[42 * (k + 1) + 6 + r * 6 + c + 3];
    }
    bsm[e] = v;
  }
#pragma unroll
  for (int q = 0; q < UPT; ++q) {
    const int u = tid + q * BEAM_NT;
    if (u >= nd) continue;
    const int g = u + 3, node = g / 3, c = g % 3;
    double rint = ek[42 * (node - 1) + 3 + c];
    if (node <= m - 2) rint += ek[42 * node + c];
    const double rz = pmass[q] * (4.0 * px[q] / (dt * dt) + 4.0 * pz[q] / dt + pa[q]);
    sres[u] = rz - 4.0 * pmass[q] * pc[q] / (dt * dt) - rint;
  }
  __syncthreads();

  // factorisation
  int po = 0, top = 0;
  for (int s = 1, lev = 0; s <= K; s *= 2, ++lev) {
    top = lev;
    const int ne = (K - s) / (2 * s) + 1;  // eliminated: j = s - 1 + 2 s q
    for (int t = tid; t < 9 * ne; t += BEAM_NT) {
      const int j = s - 1 + 2 * s * (t / 9), e = t % 9;
      Ai[9 * j + e] = inv3_entry(A + 9 * j, e / 3, e % 3);
    }
    __syncthreads();
    const int nk = K >> (lev + 1);  // kept: i = 2 s (q + 1) - 1
    for (int t = tid; t < 9 * nk; t += BEAM_NT) {
      const int q = t / 9, e = t % 9, r = e / 3, c = e % 3;
      const int i = 2 * s * (q + 1) - 1, j1 = i - s, j2 = i + s;
      double pl = 0.0, pu = 0.0;
      for (int k = 0; k < 3; ++k) pl += Lb[9 * i + 3 * r + k] * Ai[9 * j1 + 3 * k + c];
      if (j2 < K)
        for (int k = 0; k < 3; ++k) pu += Ub[9 * i + 3 * r + k] * Ai[9 * j2 + 3 * k + c];
      P[18 * (po + q) + e] = pl;
      P[18 * (po + q) + 9 + e] = pu;
    }
    __syncthreads();
    for (int t = tid; t < 9 * nk; t += BEAM_NT) {
      const int q = t / 9, e = t % 9, r = e / 3, c = e % 3;
      const int i = 2 * s * (q + 1) - 1, j1 = i - s, j2 = i + s;
      const double* pl = P + 18 * (po + q);
      const double* pu = pl + 9;
      double av = A[9 * i + e], lv = 0.0, uv = 0.0;
      for (int k = 0; k < 3; ++k) {
        av -= pl[3 * r + k] * Ub[9 * j1 + 3 * k + c];
        lv -= pl[3 * r + k] * Lb[9 * j1 + 3 * k + c];
      }
      if (j2 < K)
        for (int k = 0; k < 3; ++k) {
          av -= pu[3 * r + k] * Lb[9 * j2 + 3 * k + c];
          uv -= pu[3 * r + k] * Ub[9 * j2 + 3 * k + c];
        }
      A[9 * i + e] = av;
      Lb[9 * i + e] = lv;
      Ub[9 * i + e] = uv;
    }
    __syncthreads();
    po += nk;
  }

  // right-hand sides of this workgroup: columns c0 .. c0 + NC - 1
  const int c0 = bx * NC;
  for (int t = tid; t < nd * NC; t += BEAM_NT) {
    const int u = t / NC, col = c0 + t % NC;
    double v = 0.0;
    if (col < 2 * m) {
      const int node = col % m, cmp = col / m;
      v = (node > 0 && u == 3 * node + cmp - 3) ? 1.0 : 0.0;
    } else if (col == 2 * m) {
      v = sres[u];
    }
    rhs[t] = v;
  }
  __syncthreads();
  po = 0;
  for (int s = 1, lev = 0; s <= K; s *= 2, ++lev) {
    const int nk = K >> (lev + 1);
    for (int t = tid; t < nk * NC; t += BEAM_NT) {
      const int q = t / NC, cl = t % NC;
      const int i = 2 * s * (q + 1) - 1, j1 = i - s, j2 = i + s;
      const double* pl = P + 18 * (po + q);
      const double* pu = pl + 9;
      double bj1[3], bj2[3] = {0.0, 0.0, 0.0}, v[3];
      for (int k = 0; k < 3; ++k) bj1[k] = rhs[(3 * j1 + k) * NC + cl];
      if (j2 < K)
        for (int k = 0; k < 3; ++k) bj2[k] = rhs[(3 * j2 + k) * NC + cl];
      for (int r = 0; r < 3; ++r) {
        double x = rhs[(3 * i + r) * NC + cl];
        for (int k = 0; k < 3; ++k) x -= pl[3 * r + k] * bj1[k] + pu[3 * r + k] * bj2[k];
        v[r] = x;
      }
      for (int r = 0; r < 3; ++r) rhs[(3 * i + r) * NC + cl] = v[r];
    }
    __syncthreads();
    po += nk;
  }
  for (int lev = top; lev >= 0; --lev) {
    const int s = 1 << lev;
    const int ne = (K - s) / (2 * s) + 1;
    for (int t = tid; t < ne * NC; t += BEAM_NT) {
      const int j = s - 1 + 2 * s * (t / NC), cl = t % NC;
      double w[3];
      for (int r = 0; r < 3; ++r) w[r] = rhs[(3 * j + r) * NC + cl];
      if (j - s >= 0)
        for (int k = 0; k < 3; ++k) {
          const double x = rhs[(3 * (j - s) + k) * NC + cl];
          for (int r = 0; r < 3; ++r) w[r] -= Lb[9 * j + 3 * r + k] * x;
        }
      if (j + s < K)
        for (int k = 0; k < 3; ++k) {
          const double x = rhs[(3 * (j + s) + k) * NC + cl];
          for (int r = 0; r < 3; ++r) w[r] -= Ub[9 * j + 3 * r + k] * x;
        }
      for (int r = 0; r < 3; ++r)
        rhs[(3 * j + r) * NC + cl] =
            Ai[9 * j + 3 * r] * w[0] + Ai[9 * j + 3 * r + 1] * w[1] + Ai[9 * j + 3 * r + 2] * w[2];
    }
    __syncthreads();
  }
  double* y = a.ywork + b.yoff;
  for (int t = tid; t < nd * NC; t += BEAM_NT) {
    const int u = t / NC, col = c0 + t % NC;
    if (col < ncol) y[(size_t)u * ncol + col] = rhs[t];
  }
}

__global__ __launch_bounds__(BEAM_NT) void k_beam(FsiArgs a, int bi) {
  beam_body(a, bi, blockIdx.x);
}

__global__ __launch_bounds__(BEAM_NT) void k_beam_multi(const BeamJob* __restrict__ tab, int it) {
  const BeamJob& j = tab[blockIdx.y];
  FsiArgs a = j.a;
  a.iter = it;
  const int bi = j.bi, ncol = 2 * j.m + 1;
  if ((int)blockIdx.x >= (ncol + BEAM_NC - 1) / BEAM_NC) return;
  beam_body(a, bi, blockIdx.x);
}

// k_body_ops and k_beam of one deformable body in one launch: workgroups below nbeam solve
// the beam's right-hand sides, the others take BEAM_NT / 2 body points each (the two share no
// data: the beam's part of the Schur right-hand side is applied by k_schur_sd).
template <typename T>
__global__ __launch_bounds__(BEAM_NT) void k_ops_beam(FsiArgs a, int bi, int nbeam) {
  if ((int)blockIdx.x < nbeam) beam_body(a, bi, blockIdx.x);
  else body_ops_body<T>(a, blockIdx.x - nbeam);
}

// Many instances (ib_batch_*): rows y < nbeam of the grid solve beam job y's right-hand
// sides, the others take BEAM_NT / 2 body points each of instance y - nbeam (k_ops_beam's split).
template <typename T>
__global__ __launch_bounds__(BEAM_NT) void k_ops_beam_multi(const FsiArgs* __restrict__ fa, int ni,
                                                            const BeamJob* __restrict__ beams,
                                                            int nbeam, int it) {
  (void)ni;
  if ((int)blockIdx.y < nbeam) {
    const BeamJob& j = beams[blockIdx.y];
    if ((int)blockIdx.x >= (2 * j.m + 1 + BEAM_NC - 1) / BEAM_NC) return;
    FsiArgs a = j.a;
    a.iter = it;
    beam_body(a, j.bi, blockIdx.x);
  } else {
    FsiArgs a = fa[blockIdx.y - nbeam];
    a.iter = it;
    body_ops_body<T>(a, blockIdx.x);
  }
}

// LDS of k_beam: A, L, U, A^{-1} (9K each), P (18K), rhs (3K NC), residual (3K), masses
// (3K); the element scratch (42 (m-1)) overlays A^{-1} .. rhs, which is large enough for
// NC >= 5
size_t beam_lds_bytes(int m) {
  const size_t K = m - 1;
  return (size_t)(54 * K + 3 * K * BEAM_NC + 6 * K) * 8;
}

constexpr int LU_NT = 1024;

// Solve M X = B in place (partial pivoting, one workgroup).  M: n x n (pitch pm),
// B: n x nrhs (pitch pb).  M is overwritten.
__global__ __launch_bounds__(LU_NT) void k_lu_solve(double* M, int pm, double* B, int pb, int n,
                                                    int nrhs, int* flags) {
  __shared__ double sv[LU_NT / 64];
  __shared__ int si[LU_NT / 64];
  __shared__ int piv_s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += LU_NT) {
      const double v = fabs(M[(size_t)i * pm + k]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(best, off);
      const int oi = __shfl_down(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      sv[wv] = best;
      si[wv] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b2 = sv[0];
      int i2 = si[0];
      for (int w = 1; w < LU_NT / 64; ++w)
        if (sv[w] > b2 || (sv[w] == b2 && si[w] < i2)) {
          b2 = sv[w];
          i2 = si[w];
        }
      piv_s = i2;
      if (!(b2 > 0.0)) flags[0] = flags[0] > 3 ? flags[0] : 3;  // singular / non-finite
    }
    __syncthreads();
    const int p = piv_s;
    if (p != k) {
      for (int j = k + tid; j < n; j += LU_NT) {
        const double t = M[(size_t)k * pm + j];
        M[(size_t)k * pm + j] = M[(size_t)p * pm + j];
        M[(size_t)p * pm + j] = t;
      }
      for (int j = tid; j < nrhs; j += LU_NT) {
        const double t = B[(size_t)k * pb + j];
        B[(size_t)k * pb + j] = B[(size_t)p * pb + j];
        B[(size_t)p * pb + j] = t;
      }
    }
    __syncthreads();
    const double pivot = M[(size_t)k * pm + k];
    const int rows = n - k - 1;
    const int wcols = (n - k - 1) + nrhs;
    for (int e = tid; e < rows * wcols; e += LU_NT) {
      const int i = k + 1 + e / wcols, c = e % wcols;
      const double l = M[(size_t)i * pm + k] / pivot;
      if (c < n - k - 1) {
        const int j = k + 1 + c;
        M[(size_t)i * pm + j] -= l * M[(size_t)k * pm + j];
      } else {
        const int j = c - (n - k - 1);
        B[(size_t)i * pb + j] -= l * B[(size_t)k * pb + j];
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double d = M[(size_t)k * pm + k];
    for (int j = tid; j < nrhs; j += LU_NT) B[(size_t)k * pb + j] /= d;
    __syncthreads();
    for (int e = tid; e < k * nrhs; e += LU_NT) {
      const int i = e / nrhs, j = e % nrhs;
      B[(size_t)i * pb + j] -= M[(size_t)i * pm + k] * B[(size_t)k * pb + j];
    }
    __syncthreads();
  }
}

// f = Minv rhs (stationary bodies).
__device__ __forceinline__ void matvec_body(const double* A, int pa, const double* x, double* y,
                                            int n, int r) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) acc += A[(size_t)r * pa + c] * x[c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) y[r] = red[0];
}

__global__ void k_matvec(const double* A, int pa, const double* x, double* y, int n) {
  matvec_body(A, pa, x, y, n, blockIdx.x);
}

__global__ void k_matvec_multi(const MatvecJob* __restrict__ tab) {
  const MatvecJob j = tab[blockIdx.y];
  if ((int)blockIdx.x >= j.n) return;
  matvec_body(j.A, j.pa, j.x, j.y, j.n, blockIdx.x);
}

// Convergence test after FSI iteration `it` of K launched ahead (Algorithm 2's test on
// max |delta|, or a fixed count): sets gate[0] and the iteration count on convergence;
// stops the iterations (gate[1]) on an error or refinement flag, a non-finite update, or
// when iteration K - 1 has not converged, recording where the host should go on.
__device__ void convergence_test(int* ctl, double d, int it, int K, double tol, int fixed) {
  int* gate = ctl + FsiCtl::GATE;
  if (gate[0] != 0 || gate[1] != 0) return;
  if (ctl[FsiCtl::FLAGS] != 0 || ctl[FsiCtl::FLAGS + 1] != 0 || !(d == d) || d > 1e308) {
    ctl[FsiCtl::NEXT] = it;  // the host handles it (a refinement failure redoes iteration it)
    gate[1] = 1;
    return;
  }
  if (fixed > 0 ? it + 1 >= fixed : d <= tol) {
    ctl[FsiCtl::NEXT] = it + 1;
    gate[0] = 1;
    return;
  }
  if (it + 1 >= K) {
    ctl[FsiCtl::NEXT] = it + 1;
    gate[1] = 1;
  }
}

// Structure update from the new stresses and the convergence measure max |delta|,
// folded into delta[0] (zeroed by k_body_ops) with atomicMax on the bit pattern of the
// non-negative maxima; a non-finite update reports +Inf.  Many workgroups: one wave per
// group of 4 beam rows.
__device__ __forceinline__ void update_body(const FsiArgs& a, int it, int K, double tol, int fixed,
                                            int bx, int gx, const double* fs) {
  if (iter_gated(a.gate)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NW = STRUCT_NT / 64;
  const int gw = bx * NW + w, nwaves = gx * NW;
  double my = 0.0;
  bool bad = false;
  auto fold = [&](double d) {
    if (!(d == d) || d > 1e308) bad = true;
    else my = fmax(my, d);
  };
  for (int bi = 0; bi < a.nbodies; ++bi) {
    const BodyDev b = a.bodies[bi];
    const int m = b.npts, r0 = 2 * b.pt0;
    if (b.kind == BODY_TORSIONAL) {
      if (gw == 0) {
        double* ts = a.tors + b.tors * TS_COUNT;
        const double dt = a.dt;
        const double th = a.iter == 0 ? ts[TS_THETA] : ts[TS_NEW];
        const double ang = (b.moff < 0 ? b.theta0 : a.poses[b.moff + MF_ANG]) + th;
        const double sn = sin(ang), cs = cos(ang);
        const double jt = 4.0 * b.inertia / (dt * dt) + 2.0 * b.damping / dt + b.stiffness;
        const double rphi = b.inertia * (4.0 * ts[TS_THETA] / (dt * dt) + 4.0 * ts[TS_PHI] / dt + ts[TS_PHIDOT]) +
                            b.damping * (2.0 * ts[TS_THETA] / dt + ts[TS_PHI]) + tors_g(a, b, ts, th);
        double sf = 0.0;
        for (int u = lane; u < 2 * m; u += 64) sf += (u < m ? -sn : cs) * (u % m) * b.ds * fs[r0 + u];
        for (int off = 32; off > 0; off >>= 1) sf += __shfl_xor(sf, off);
        if (lane == 0) {
          const double thn = (rphi + b.ds * sf) / jt;
          fold(fabs(thn - th));
          ts[TS_NEW] = thn;
        }
      }
    } else if (b.kind == BODY_DEFORMABLE) {
      // delta chi = J_d^{-1} (res + ds T^T f) = y_res + ds Y f with Y = J_d^{-1} T^T; lanes
      // across the columns, every load of a group of rows in flight at once
      const int nd = 3 * m - 3, ncol = 2 * m + 1;
      const double* y = a.ywork + b.yoff;
      const double* ck = (a.iter == 0 ? a.chi : a.chi_new) + b.dof0;
      double* cn = a.chi_new + b.dof0;
      constexpr int CQ = 7;  // 2m <= 448 columns
      for (int u0 = 4 * gw; u0 < nd; u0 += 4 * nwaves) {
        // every load of the group (rows of Y, the residual column, chi^k) before its stores
        double v[4][CQ], yr[4], fc[CQ], cv[4];
#pragma unroll
        for (int k = 0; k < CQ; ++k) {
          const int c = lane + 64 * k;
          fc[k] = c < 2 * m ? fs[r0 + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = u0 + q;
          yr[q] = u < nd ? y[(size_t)u * ncol + 2 * m] : 0.0;
          cv[q] = (lane == 0 && u < nd) ? ck[u + 3] : 0.0;
#pragma unroll
          for (int k = 0; k < CQ; ++k) {
            const int c = lane + 64 * k;
            v[q][k] = (u < nd && c < 2 * m) ? y[(size_t)u * ncol + c] : 0.0;
          }
        }
        double dxq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < CQ; ++k) acc += v[q][k] * fc[k];
          for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
          dxq[q] = yr[q] + b.ds * acc;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = u0 + q;
          if (lane == 0 && u < nd) {
            fold(fabs(dxq[q]));
            cn[u + 3] = cv[q] + dxq[q];  // ck may alias cn: this lane read it above
          }
        }
      }
      if (gw == 0 && lane == 0) {
        cn[0] = ck[0];
        cn[1] = ck[1];
        cn[2] = ck[2];
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) my = fmax(my, __shfl_xor(my, off));
  const bool anybad = __any(bad);
  if (lane == 0) {
    const double v = anybad ? INFINITY : my;
    atomicMax(reinterpret_cast<unsigned long long*>(a.delta), (unsigned long long)__double_as_longlong(v));
  }
  if (a.gate == nullptr) return;  // the host tests convergence
  // iterations launched ahead: the last workgroup to finish runs the convergence test
  __syncthreads();
  if (threadIdx.x == 0) {
    int* ctl = a.flags;
    __threadfence();
    if (atomicAdd(&ctl[FsiCtl::UDONE], 1) == gx - 1) {
      __threadfence();
      const unsigned long long bits = __hip_atomic_load(
          reinterpret_cast<unsigned long long*>(a.delta), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      convergence_test(ctl, __longlong_as_double((long long)bits), it, K, tol, fixed);
      atomicExch(&ctl[FsiCtl::UDONE], 0);
    }
  }
}

__global__ __launch_bounds__(STRUCT_NT) void k_update(FsiArgs a, int it, int K, double tol,
                                                     int fixed) {
  update_body(a, it, K, tol, fixed, blockIdx.x, gridDim.x, a.f);
}

__global__ __launch_bounds__(STRUCT_NT) void k_update_multi(const UpdateJob* __restrict__ tab,
                                                           int it, int K) {
  const UpdateJob& j = tab[blockIdx.y];
  FsiArgs a = j.a;
  a.iter = it;
  const int nb = j.nb;
  if ((int)blockIdx.x >= nb) return;
  update_body(a, it, K, j.tol, j.fixed, blockIdx.x, nb, a.f);
}

// Newmark completion of the step with the accepted iterate.
__device__ __forceinline__ void finish_body(const FsiArgs& a) {
  if (post_gated(a.gate)) return;
  const int tid = threadIdx.x;
  const double dt = a.dt;
  for (int bi = 0; bi < a.nbodies; ++bi) {
    const BodyDev b = a.bodies[bi];
    if (b.kind == BODY_TORSIONAL) {
      if (tid == 0) {
        double* ts = a.tors + b.tors * TS_COUNT;
        const double thn = ts[TS_NEW];
        const double rth = ts[TS_PHI] + 2.0 * ts[TS_THETA] / dt;
        const double phin = 2.0 * thn / dt - rth;
        const double phidn = 4.0 * (thn - ts[TS_THETA]) / (dt * dt) - 4.0 * ts[TS_PHI] / dt - ts[TS_PHIDOT];
        ts[TS_THETA] = thn;
        ts[TS_PHI] = phin;
        ts[TS_PHIDOT] = phidn;
      }
    } else if (b.kind == BODY_DEFORMABLE) {
      for (int u = tid; u < 3 * b.npts; u += STRUCT_NT) {
        const int g = b.dof0 + u;
        if (u < 3) {
          a.zeta[g] = 0.0;
          a.zetadot[g] = 0.0;
          continue;
        }
        const double xnew = a.chi_new[g];
        const double rchi = a.zeta[g] + 2.0 * a.chi[g] / dt;
        const double zn = 2.0 * xnew / dt - rchi;
        const double an = 4.0 * (xnew - a.chi[g]) / (dt * dt) - 4.0 * a.zeta[g] / dt - a.zetadot[g];
        a.chi[g] = xnew;
        a.zeta[g] = zn;
        a.zetadot[g] = an;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(STRUCT_NT) void k_finish(FsiArgs a) { finish_body(a); }

__global__ __launch_bounds__(STRUCT_NT) void k_finish_multi(const FsiArgs* __restrict__ tab) {
  const FsiArgs a = tab[blockIdx.y];
  finish_body(a);
}

// Corrector source C^T E^T lambda at interior vertices of rows [jlo, jhi]; entries
// outside columns [ilo, ihi] are zero.  lambda_a = (ds_a / h) f_a.  Each workgroup
// covers a 64 x 4 tile of vertices.  It first lists (in row order, by wave ballots) the
// operator rows whose window reaches the tile, stages their windows and coefficients
// in LDS (SPREAD_STAGE rows at a time), and then every vertex sums those rows in that
// fixed order, so the result is deterministic.  Dynamic LDS (spread_lds_bytes): the list
// (nf ints), then the staged rows; small enough that every workgroup of a launch is
// resident at once.
constexpr int SPREAD_TX = SPREAD_TILE_X, SPREAD_TY = SPREAD_TILE_Y, SPREAD_NT = SPREAD_TX * SPREAD_TY;
constexpr int SPREAD_MAXROWS = SPREAD_ROWS_MAX;
constexpr int SPREAD_STAGE = 64;

size_t spread_lds_bytes(int nf) {
  return (size_t)SPREAD_STAGE * (16 * 8 + 8 + 4 * 4) + (size_t)(nf + 1) / 2 * 8;
}

template <typename T>
__device__ __forceinline__ void spread_body(const FsiArgs& a, int jlo, int jhi, int ilo, int ihi,
                                            T* out, int po, int bx, int by) {
  constexpr int NW = SPREAD_NT / 64;
  extern __shared__ double spl[];
  double (*sw)[16] = reinterpret_cast<double (*)[16]>(spl);  // [SPREAD_STAGE][16]
  double* sc = spl + SPREAD_STAGE * 16;                        // [SPREAD_STAGE]
  int4* sb = reinterpret_cast<int4*>(sc + SPREAD_STAGE);       // [SPREAD_STAGE]: base, comp
  int* list = reinterpret_cast<int*>(sb + SPREAD_STAGE);       // [nf]
  __shared__ int wcount[NW];
  if (post_gated(a.gate)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int tx = tid % SPREAD_TX, ty = tid / SPREAD_TX;
  const int ti0 = 1 + bx * SPREAD_TX, tj0 = jlo + by * SPREAD_TY;
  const int i = ti0 + tx, j = tj0 + ty;
  const bool tile_hit = !(ti0 + SPREAD_TX - 1 < ilo || ti0 > ihi);
  int cnt = 0;
  if (tile_hit) {
    for (int r0 = 0; r0 < a.nf; r0 += SPREAD_NT) {
      const int r = r0 + tid;
      bool hit = false;
      if (r < a.nf) {
        const int i0 = a.st_base[3 * r], j0 = a.st_base[3 * r + 1];
        // vertices touched by the window's faces: columns i0 .. i0+4, rows j0 .. j0+4
        hit = !(i0 + 4 < ti0 || i0 > ti0 + SPREAD_TX - 1 || j0 + 4 < tj0 || j0 > tj0 + SPREAD_TY - 1);
      }
      const unsigned long long bal = __ballot(hit);
      const int below = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[wv] = __popcll(bal);
      __syncthreads();
      int off = cnt;
      for (int w = 0; w < wv; ++w) off += wcount[w];
      if (hit) list[off + below] = r;
      for (int w = 0; w < NW; ++w) cnt += wcount[w];
      __syncthreads();
    }
  }
  double src = 0.0;
  for (int q0 = 0; q0 < cnt; q0 += SPREAD_STAGE) {
    const int nq = min(SPREAD_STAGE, cnt - q0);
    if (tid < nq) {
      const int r = list[q0 + tid];
      int bb[3];
      double ww[16];
      for (int k = 0; k < 3; ++k) bb[k] = a.st_base[3 * r + k];
      for (int k = 0; k < 16; ++k) ww[k] = a.st_w[16 * r + k];
      const double coef = (row_ds(a, r) / a.h) * a.f[r];
      sb[tid] = make_int4(bb[0], bb[1], bb[2], 0);
      for (int k = 0; k < 16; ++k) sw[tid][k] = ww[k];
      sc[tid] = coef;
    }
    __syncthreads();
    if (i >= ilo && i <= ihi && i <= a.n - 1 && j <= jhi) {
      // first the staged rows whose window reaches this vertex, as a bit mask (no branch per
      // row, so the LDS reads of many rows are in flight together), then those rows in
      // staging order
      unsigned long long hit = 0;
#pragma unroll 16
      for (int q = 0; q < nq; ++q) {
        const int4 bq = sb[q];
        const unsigned di = (unsigned)(i - bq.x), dj = (unsigned)(j - bq.y);
        hit |= (unsigned long long)(di <= 4u && dj <= 4u) << q;
      }
      while (hit != 0) {
        const int q = __builtin_ctzll(hit);
        hit &= hit - 1;
        const int4 bq = sb[q];
        const int di = i - bq.x, dj = j - bq.y;
        const double* w = sw[q];
        double c = 0.0;
        if (bq.z == 0) {
          // x-faces [j][i] (-) and [j-1][i] (+)
          if (di < 4 && dj < 4) c -= w[dj * 4 + di];
          if (di < 4 && dj >= 1) c += w[(dj - 1) * 4 + di];
        } else {
          // y-faces [j][i] (+) and [j][i-1] (-)
          if (di < 4 && dj < 4) c += w[dj * 4 + di];
          if (di >= 1 && dj < 4) c -= w[dj * 4 + di - 1];
        }
        if (c != 0.0) src += c * sc[q];
      }
    }
    __syncthreads();
  }
  if (i > a.n - 1 || j > jhi) return;
  out[(size_t)(j - 1) * po + (i - 1)] = (T)src;
}

template <typename T>
__global__ __launch_bounds__(SPREAD_NT) void k_spread(FsiArgs a, int jlo, int jhi, int ilo, int ihi,
                                                      T* out, int po, int fin_bx) {
  // the workgroups of the column fin_bx (launched only with the structure finish): block
  // (fin_bx, 0) runs it, the others have nothing to do
  if ((int)blockIdx.x == fin_bx) {
    if (blockIdx.y == 0) finish_body(a);
    return;
  }
  spread_body<T>(a, jlo, jhi, ilo, ihi, out, po, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(SPREAD_NT) void k_spread_multi(const SpreadJob<T>* __restrict__ tab) {
  const SpreadJob<T>& j = tab[blockIdx.z];
  const FsiArgs a = j.a;
  const int jlo = j.jlo, jhi = j.jhi;
  if ((int)blockIdx.x >= (a.n - 1 + SPREAD_TX - 1) / SPREAD_TX ||
      (int)blockIdx.y >= (jhi - jlo + 1 + SPREAD_TY - 1) / SPREAD_TY)
    return;
  spread_body<T>(a, jlo, jhi, j.ilo, j.ihi, j.out, j.po, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------ offline stage

__device__ void off_window(const OffRows& o, int row, int* base, int* comp, double* w) {
  if (o.kind == 0) {
    base[0] = o.st_base[3 * row];
    base[1] = o.st_base[3 * row + 1];
    *comp = o.st_base[3 * row + 2];
    for (int e = 0; e < 16; ++e) w[e] = o.st_w[16 * row + e];
    return;
  }
  *comp = row >= o.sd_total ? 1 : 0;
  const int pt = row - (*comp) * o.sd_total;
  if (pt < o.sd_ngrid) {
    int k = 0;  // the rectangle holding sub-domain point pt
#pragma unroll
    for (int q = 1; q < SD_MAX_BOXES; ++q)
      if (q < o.sdb.n && o.sdb.off[q] <= pt) k = q;
    const SdBox bb = sd_box(o.sdb, k);
    const int loc = pt - bb.off;
    const int p = bb.i0 + loc % bb.npx, q = bb.j0 + loc / bb.npx;
    base[0] = p - 1;
    base[1] = q - 1;
    for (int e = 0; e < 16; ++e) w[e] = 0.0;
    add_e0_vertex(p, q, *comp, 1.0, o.x0, o.y0, o.h, base, w);
  } else {
    const int ap = pt - o.sd_ngrid;
    // appended exact points exist in sub-domain mode only, which uses the 3-point kernel
    exact_window(o.app_xy[2 * ap], o.app_xy[2 * ap + 1], *comp, o.x0, o.y0, o.h, base, w, 0);
  }
}

// Row-transformed point sources: slot b holds C^T E^T e_{col0 + b} after the row DST,
// as 6 consecutive rows starting at rows_first[b] (1-based).
template <typename T>
__global__ void k_point_source_rowdst(OffRows o, int col0, int ncols, const c2<T>* __restrict__ tw,
                                      T* out, int po, size_t bso, int* rows_first) {
  const int b = blockIdx.y;
  if (col0 + b >= ncols) return;
  int base[2], comp;
  double w[16];
  off_window(o, col0 + b, base, &comp, w);
  // vertex source on a 6 x 6 patch of vertices starting at (base[0], base[1])
  double v[6][6];
  for (int q = 0; q < 6; ++q)
    for (int p = 0; p < 6; ++p) v[q][p] = 0.0;
  for (int dj = 0; dj < 4; ++dj)
    for (int di = 0; di < 4; ++di) {
      const double ww = w[dj * 4 + di];
      if (ww == 0.0) continue;
      if (comp == 0) {  // x-face [j][i]: vertex (i, j) -w, vertex (i, j+1) +w
        v[dj][di] -= ww;
        v[dj + 1][di] += ww;
      } else {          // y-face [j][i]: vertex (i, j) +w, vertex (i+1, j) -w
        v[dj][di] += ww;
        v[dj][di + 1] -= ww;
      }
    }
  const int n = o.n;
  if (threadIdx.x == 0 && blockIdx.x == 0) rows_first[b] = base[1];
  T* ob = out + (size_t)b * bso;
  // row DST: X_k = sum_i v_i sin(pi i k / n); sin(pi m / n) = -Im tw[m mod 2n]
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 6 * (n - 1); e += gridDim.x * blockDim.x) {
    const int rq = e / (n - 1), k = 1 + e % (n - 1);
    const int j = base[1] + rq;
    double acc = 0.0;
    if (j >= 1 && j <= n - 1) {
      for (int p = 0; p < 6; ++p) {
        const int i = base[0] + p;
        if (v[rq][p] == 0.0 || i < 1 || i > n - 1) continue;
        acc += v[rq][p] * (-(double)tw[(i * k) % (2 * n)].y);
      }
    }
    ob[(size_t)rq * po + (k - 1)] = (T)acc;
  }
}

// Sample E C s of every target row for each slot: vals[b * ntarget + t].
template <typename T>
__global__ void k_sample(OffRows o, int ntarget, const T* sl, int ps, size_t bss, double* vals,
                         int nslots) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (t >= ntarget || b >= nslots) return;
  int base[2], comp;
  double w[16];
  off_window(o, t, base, &comp, w);
  const T* s = sl + (size_t)b * bss;
  double acc = 0.0;
  for (int dj = 0; dj < 4; ++dj)
    for (int di = 0; di < 4; ++di) {
      const double ww = w[dj * 4 + di];
      if (ww != 0.0) acc += ww * face_flux(s, ps, comp, base[0] + di, base[1] + dj, 0.0, 0.0);
    }
  vals[(size_t)b * ntarget + t] = acc;
}

// Drop filter of column col0 + b (eq. (34), kept iff |b_tc| > eps |b_cc|) and
// compaction in target order: cols/vals at b * ntarget, count in counts[b].
constexpr int CMP_NT = 1024;
__global__ __launch_bounds__(CMP_NT) void k_filter_compact(const double* vals, int ntarget, int col0,
                                                           int ncols, double eps, int* out_col,
                                                           double* out_val, int* counts) {
  const int b = blockIdx.x;
  if (col0 + b >= ncols) return;
  __shared__ int scan[CMP_NT];
  __shared__ int base_s;
  const double* v = vals + (size_t)b * ntarget;
  const double thr = eps * fabs(v[col0 + b]);
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  for (int t0 = 0; t0 < ntarget; t0 += CMP_NT) {
    const int t = t0 + threadIdx.x;
    const int keep = (t < ntarget && fabs(v[t]) > thr) ? 1 : 0;
    scan[threadIdx.x] = keep;
    __syncthreads();
    for (int off = 1; off < CMP_NT; off <<= 1) {
      const int add = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += add;
      __syncthreads();
    }
    if (keep) {
      const int pos = base_s + scan[threadIdx.x] - 1;
      out_col[(size_t)b * ntarget + pos] = t;
      out_val[(size_t)b * ntarget + pos] = v[t];
    }
    __syncthreads();
    if (threadIdx.x == 0) base_s += scan[CMP_NT - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[b] = base_s;
}

// ------------------------------------------------- Schur solve by refinement
// The Schur matrix changes little between FSI iterations and between steps, so the
// solve keeps X ~ M^{-1}: refreshed once per step by one Newton-Schulz iteration
// X <- X (2I - M X) (two GEMMs), then f = X b corrected by iterative refinement
// f <- f + X (b - M f) to working accuracy.  A fresh inverse (LU) is made at the
// first use and whenever the refinement stops contracting.
//
// The refinement is one launch of nb co-resident workgroups.  Workgroup w owns rows R_w of
// M and columns R_w of X (held in LDS when they fit).  Each sweep it forms r = b - M f on R_w,
// its share X[:, R_w] r_{R_w} of the update and max |r| over R_w, and publishes both; after
// one grid barrier every workgroup reads all shares and maxima and adds the shares in
// workgroup order, so all hold the same f and take the same decision.  Sweeps stop when the
// relative residual |r|/|b| (max norms) is at most 1e-16 n or no longer halves, after at most
// maxit sweeps; f then keeps the value whose residual was tested.  They also stop right after
// an update when the residual it leaves, predicted from the last contraction (|r_k|^2 /
// |r_{k-1}|), is below 1/100 of that target: the sweep that would only confirm it is not run,
// and the reported residual is that prediction.  With no guess, f starts at 0, so the first
// sweep gives f = X b.  Workspace `ws` (doubles): [0] relative residual,
// [1] sweeps, [2] barrier arrivals, [3] exits (32-bit counters), then two buffers of nb rows
// of n + 1 values (the share, then the maximum); alternate sweeps use alternate buffers, so a
// row is never overwritten while another workgroup may still read it.  The last workgroup to
// leave zeroes the counters for the next launch.  Large systems (TWO) take more workgroups, so
// that their rows of M and columns of X still fit in LDS; then summing all shares in every
// workgroup would cost nb n loads each, so workgroup w sums only its slice of the columns (in
// workgroup order) into a reduced vector (two more buffers of n + 1 after the shares), and
// after a second barrier every workgroup reads that vector.
constexpr int REF_HDR = 4;
constexpr int REF_NB_ONE = 32;   // workgroups up to which every workgroup sums all shares
constexpr int REF_NB_MAX = 128;
constexpr size_t REF_LDS_CACHE = 48 * 1024;
constexpr size_t REF_LDS_BIG = 120 * 1024;
constexpr int REF_LOADS = 12;     // loads of a thread per matrix in flight while LDS fills
constexpr double REF_PREDICT = 0.01;  // margin of the predicted stop (see refine_body)
size_t refine_ws_doubles(int n, int) {
  return (size_t)REF_HDR + (size_t)2 * REF_NB_MAX * (n + 1) + (size_t)2 * (n + 1);
}

__device__ inline unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ inline double bitsd(unsigned long long v) { return __longlong_as_double((long long)v); }

// Barrier over the workgroups of one launch, which must all be resident.  Arrivals count up
// in `cnt` (the k-th barrier waits for k * gridDim.x).  Data that crosses it is written and
// read only with agent-scope atomic stores and loads, which are coherent across the chip's
// L2 caches, so readers need no cache invalidation; every thread's agent-scope release fence
// before the workgroup barrier makes its stores complete before the arrival.  The wait is bounded:
// on time-out it records FLAG_BARRIER in flags[0] and returns false, and every other
// waiting workgroup then leaves its wait at once.  `limit` > 0 replaces the default bound
// on the spins; `limit` < 0 is a test hook of the host: the wait then needs one arrival more
// than the launch has workgroups, which never comes, so every wait ends at the bound -limit
// and the kernel's time-out path runs (every workgroup still leaves normally).
constexpr long BARRIER_SPIN_LIMIT = 1L << 22;
__device__ bool grid_barrier(unsigned* cnt, unsigned target, int* flags, long limit) {
  const long lim = limit > 0 ? limit : (limit < 0 ? -limit : BARRIER_SPIN_LIMIT);
  const unsigned want = limit < 0 ? target + 1u : target;
  __shared__ int ok_s;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > lim ||
          ((spins & 255) == 0 &&
           __hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == FLAG_BARRIER)) {
        atomicMax(&flags[0], FLAG_BARRIER);
        ok = 0;
        break;
      }
    }
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

__device__ inline void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double nanmax(double m, double v) { return (v > m || v != v) ? v : m; }

// A double moved between lanes by a DPP control (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over aligned groups of g lanes (g a power of two <= 64), the same value in every lane
// of a group: within quads by quad permutations, then half rows and rows by mirrors (each
// step adds two partial sums, the same two in both lanes of a pair, so every lane ends with
// the same bits), then across rows by shuffles.  Every lane of the wave must be active.
__device__ __forceinline__ double lane_group_sum(double v, int g) {
  if (g >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  if (g >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  if (g >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
  if (g >= 16) v += dpp_move<0x140>(v); // row_mirror
  if (g >= 32) v += __shfl_xor(v, 16);
  if (g >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Returns whether the solve completed (its f is then in the first n doubles of the dynamic
// LDS, the same in every workgroup).
template <bool CACHE, bool TWO>
__device__ __forceinline__ bool refine_body(const double* __restrict__ M,
                                            const double* __restrict__ X, int pm,
                                            const double* __restrict__ b, double* f, int n,
                                            int rw, int tpr, int maxit, int guess, double* ws,
                                            double* out, int* flags, const int* gate,
                                            double* xcopy, long spin, int bx, int gx) {
  if (iter_gated(gate)) return false;  // the same for every workgroup: none enters a barrier
  extern __shared__ double lds[];
  double* sf = lds;           // f (n)
  double* sd = sf + n;        // the update of this sweep (n)
  double* sr = sd + n;        // r on the own rows (rw)
  double* sb = sr + rw;       // b on the own rows (rw)
  double* sred = sb + rw;     // 4 partial maxima
  double* sm = sred + 4;      // rows R_w of M (rw x n) when CACHE
  double* sx = sm + (size_t)rw * n;  // columns R_w of X (n x rw) when CACHE
  double* sp = CACHE ? sx + (size_t)rw * n : sm;    // TWO: this slice of every share (nb x cs)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = gx, w = bx, ns = n + 1;
  const int r0 = w * rw, r1 = min(n, r0 + rw), nr = max(0, r1 - r0);
  unsigned* cnt = reinterpret_cast<unsigned*>(ws + 2);
  unsigned* ext = reinterpret_cast<unsigned*>(ws + 3);
  double* shares = ws + REF_HDR;
  // Every global value of the set-up is requested before any is used, so that one round trip
  // covers b, f, and (CACHE) the first REF_LOADS elements per thread of rows R_w of M and of
  // columns R_w of X (both just written elsewhere on the chip, so each round trip is long).
  constexpr int BF = 2;  // elements of b and f per thread held in registers; more are looped
  double bv[BF], fv[BF];
#pragma unroll
  for (int q = 0; q < BF; ++q) {
    const int i = tid + 256 * q;
    bv[q] = i < n ? b[i] : 0.0;
    fv[q] = (guess && i < n) ? f[i] : 0.0;
  }
  const double bown = tid < nr ? b[r0 + tid] : 0.0;
  const int tot = nr * n;
  double vm[REF_LOADS], vx[REF_LOADS];
  if (CACHE) {
#pragma unroll
    for (int u = 0; u < REF_LOADS; ++u) {
      const int e = min(tid + u * 256, tot - 1);
      vm[u] = M[(size_t)(r0 + e / n) * pm + e % n];
      vx[u] = X[(size_t)(e / nr) * pm + r0 + e % nr];
    }
  }
  // |b| and the starting f (the same in every workgroup)
  double mb = 0.0;
#pragma unroll
  for (int q = 0; q < BF; ++q) {
    const int i = tid + 256 * q;
    if (i < n) {
      mb = nanmax(mb, fabs(bv[q]));
      sf[i] = fv[q];
    }
  }
  for (int i = tid + 256 * BF; i < n; i += 256) {
    mb = nanmax(mb, fabs(b[i]));
    sf[i] = guess ? f[i] : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) mb = nanmax(mb, __shfl_xor(mb, off));
  if (lane == 0) sred[wv] = mb;
  if (tid < nr) sb[tid] = bown;
  for (int k = tid + 256; k < nr; k += 256) sb[k] = b[r0 + k];
  if (CACHE) {
    // rows R_w of M and columns R_w of X into LDS: the first round is in flight already, the
    // rest follow REF_LOADS loads of a thread at a time
    for (int e0 = tid; e0 < tot; e0 += 256 * REF_LOADS) {
      if (e0 != tid) {
#pragma unroll
        for (int u = 0; u < REF_LOADS; ++u) {
          const int e = min(e0 + u * 256, tot - 1);
          vm[u] = M[(size_t)(r0 + e / n) * pm + e % n];
          vx[u] = X[(size_t)(e / nr) * pm + r0 + e % nr];
        }
      }
#pragma unroll
      for (int u = 0; u < REF_LOADS; ++u) {
        const int e = e0 + u * 256;
        if (e >= tot) continue;
        sm[e] = vm[u];
        const int j = e / nr, k = e % nr;
        sx[(size_t)j * rw + k] = vx[u];
        if (xcopy) xcopy[(size_t)j * pm + r0 + k] = vx[u];
      }
    }
  } else if (xcopy) {
    for (int e = tid; e < nr * n; e += 256) {
      const int j = e / nr, k = e % nr;
      xcopy[(size_t)j * pm + r0 + k] = X[(size_t)j * pm + r0 + k];
    }
  }
  __syncthreads();
  const double nbv = nanmax(nanmax(sred[0], sred[1]), nanmax(sred[2], sred[3]));
  double prev = 1e300, rel = 0.0;
  int sweeps = maxit;
  bool ok = true;
  unsigned target = 0;
  const int rk = tid / tpr, rp = tid % tpr;  // row and part of this thread in r = b - M f
  if constexpr (CACHE && !TWO) {
    // Rows and columns in LDS.  r on the own rows with tpr lanes per row summed across the
    // lanes (DPP); then thread e forms element e of the share X[:, R_w] r_{R_w}, and the thread
    // of element n the maximum |r| on R_w.
    for (int it = 0; it < maxit; ++it) {
      double acc = 0.0;
      if (rk < nr) {
        const double* mr = sm + (size_t)rk * n;
#pragma unroll 4
        for (int j = rp; j < n; j += tpr) acc = fma(mr[j], sf[j], acc);
      }
      acc = lane_group_sum(acc, tpr);
      if (rk < nr && rp == 0) sr[rk] = sb[rk] - acc;
      __syncthreads();
      double* sh = shares + (size_t)(it & 1) * REF_NB_MAX * ns + (size_t)w * ns;
      for (int e = tid; e <= n; e += 256) {
        double v = 0.0;
        if (e < n) {
          const double* xr = sx + (size_t)e * rw;
          for (int k = 0; k < nr; ++k) v = fma(xr[k], sr[k], v);
        } else {
          for (int k = 0; k < nr; ++k) v = nanmax(v, fabs(sr[k]));
        }
        st_agent(&sh[e], v);
      }
      target += (unsigned)nb;
      if (!grid_barrier(cnt, target, flags, spin)) {
        ok = false;
        break;
      }
      // all shares and maxima, loads in flight together; shares added in workgroup order
      const double* all = shares + (size_t)(it & 1) * REF_NB_MAX * ns;
      for (int e = tid; e <= n; e += 256) {
        double a = 0.0;
        for (int q0 = 0; q0 < nb; q0 += 16) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = ld_agent(&all[(size_t)min(q0 + u, nb - 1) * ns + e]);
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (q0 + u < nb) a = e < n ? a + v[u] : nanmax(a, v[u]);
        }
        if (e < n) sd[e] = a;
        else sred[0] = a;
      }
      __syncthreads();
      const double nrm = sred[0];
      rel = nbv > 0.0 ? nrm / nbv : 0.0;
      if (!(rel > 1e-16 * n) || !(nrm < 0.5 * prev)) {
        sweeps = it;
        break;
      }
      const double pred = it > 0 ? nrm * (nrm / prev) : INFINITY;
      prev = nrm;
      for (int j = tid; j < n; j += 256) sf[j] += sd[j];
      __syncthreads();
      if (pred <= REF_PREDICT * 1e-16 * n * nbv) {
        sweeps = it + 1;
        rel = pred / nbv;
        break;
      }
    }
  } else {
  for (int it = 0; it < maxit; ++it) {
    // r = b - M f on the own rows: tpr threads per row
    {
      double acc = 0.0;
      if (rk < nr) {
        const double* mr = CACHE ? sm + (size_t)rk * n : M + (size_t)(r0 + rk) * pm;
        for (int j0 = rp; j0 < n; j0 += 8 * tpr) {
          double mv[8], fv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = min(j0 + u * tpr, n - 1);
            mv[u] = mr[j];
            fv[u] = j0 + u * tpr < n ? sf[j] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += mv[u] * fv[u];
        }
      }
      for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (rk < nr && rp == 0) sr[rk] = sb[rk] - acc;
    }
    __syncthreads();
    double* sh = shares + (size_t)(it & 1) * REF_NB_MAX * ns + (size_t)w * ns;
    if (wv == 0) {
      double m = 0.0;
      for (int k = lane; k < nr; k += 64) m = nanmax(m, fabs(sr[k]));
      for (int off = 32; off > 0; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
      if (lane == 0) st_agent(&sh[n], m);
    }
    // this workgroup's share of X r
    for (int j = tid; j < n; j += 256) {
      double acc = 0.0;
      for (int k0 = 0; k0 < nr; k0 += 8) {
        double xv[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = min(k0 + u, nr - 1);
          xv[u] = CACHE ? sx[(size_t)j * rw + k] : X[(size_t)j * pm + r0 + k];
          rv[u] = k0 + u < nr ? sr[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += xv[u] * rv[u];
      }
      st_agent(&sh[j], acc);
    }
    target += (unsigned)nb;
    if (!grid_barrier(cnt, target, flags, spin)) {
      ok = false;
      break;
    }
    // all maxima and shares, loads in flight together; shares summed in workgroup order
    const double* all = shares + (size_t)(it & 1) * REF_NB_MAX * ns;
    double nrm = 0.0;
    if constexpr (TWO) {
      const int cs = (n + nb - 1) / nb, c0 = w * cs, c1 = min(n, c0 + cs), nc = max(0, c1 - c0);
      double* red = shares + (size_t)2 * REF_NB_MAX * ns + (size_t)(it & 1) * ns;
      for (int e = tid; e < nc * nb; e += 256)
        sp[e] = ld_agent(&all[(size_t)(e / nc) * ns + c0 + e % nc]);
      for (int q = tid; q < nb; q += 256) nrm = nanmax(nrm, ld_agent(&all[(size_t)q * ns + n]));
      __syncthreads();
      if (tid < nc) {
        double acc = 0.0;
        for (int q = 0; q < nb; ++q) acc += sp[q * nc + tid];
        st_agent(&red[c0 + tid], acc);
      }
      target += (unsigned)nb;
      if (!grid_barrier(cnt, target, flags, spin)) {
        ok = false;
        break;
      }
      for (int j = tid; j < n; j += 256) sd[j] = ld_agent(&red[j]);
      // every thread needs the maximum over all workgroups
      for (int off = 32; off > 0; off >>= 1) nrm = nanmax(nrm, __shfl_xor(nrm, off));
      if (lane == 0) sred[wv] = nrm;
      __syncthreads();
      nrm = nanmax(nanmax(sred[0], sred[1]), nanmax(sred[2], sred[3]));
    } else {
    for (int j0 = 0; j0 < n; j0 += 256) {
      const int j = j0 + tid, jc = min(j, n - 1);
      double acc = 0.0;
      for (int q0 = 0; q0 < nb; q0 += 16) {
        double v[16], u[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = ld_agent(&all[(size_t)min(q0 + q, nb - 1) * ns + jc]);
        if (j0 == 0) {
#pragma unroll
          for (int q = 0; q < 16; ++q) u[q] = ld_agent(&all[(size_t)min(q0 + q, nb - 1) * ns + n]);
#pragma unroll
          for (int q = 0; q < 16; ++q) nrm = nanmax(nrm, u[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += q0 + q < nb ? v[q] : 0.0;
      }
      if (j < n) sd[j] = acc;
    }
    }
    rel = nbv > 0.0 ? nrm / nbv : 0.0;
    if (!(rel > 1e-16 * n) || !(nrm < 0.5 * prev)) {
      sweeps = it;
      break;
    }
    // the residual after this update if it contracts as the last one did
    const double pred = it > 0 ? nrm * (nrm / prev) : INFINITY;
    prev = nrm;
    for (int j = tid; j < n; j += 256) sf[j] += sd[j];
    __syncthreads();
    if (pred <= REF_PREDICT * 1e-16 * n * nbv) {
      // below the target with a wide margin: the sweep that would only confirm it is skipped
      sweeps = it + 1;
      rel = pred / nbv;
      break;
    }
  }
  }
  if (ok) {
    for (int i = r0 + tid; i < r1; i += 256) f[i] = sf[i];
    if (w == 0 && tid == 0) {
      ws[0] = rel;
      ws[1] = sweeps;
      out[0] = rel;
      out[1] = sweeps;
      out[2] = 0.0;
      if (!(rel < 1e-9)) atomicMax(&flags[1], 1);  // the inverse is stale
    }
  }
  if (tid == 0) {
    if (__hip_atomic_fetch_add(ext, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        (unsigned)nb - 1) {
      __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ext, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return ok;
}

template <bool CACHE, bool TWO>
__global__ __launch_bounds__(256) void k_refine(const double* __restrict__ M,
                                                const double* __restrict__ X, int pm,
                                                const double* __restrict__ b, double* f, int n,
                                                int rw, int tpr, int maxit, int guess, double* ws,
                                                double* out, int* flags, const int* gate,
                                                double* xcopy, long spin) {
  refine_body<CACHE, TWO>(M, X, pm, b, f, n, rw, tpr, maxit, guess, ws, out, flags, gate, xcopy,
                          spin, blockIdx.x, gridDim.x);
}

// The refinement followed by the structure update of the same FSI iteration (k_update's
// work) on the same workgroups, which all hold the new f in LDS: one launch fewer per
// iteration.  When the refinement gave up, the update reads f from memory, as k_update would.
template <bool CACHE, bool TWO>
__global__ __launch_bounds__(256) void k_refine_update(const double* __restrict__ M,
                                                       const double* __restrict__ X, int pm,
                                                       const double* __restrict__ b, double* f,
                                                       int n, int rw, int tpr, int maxit,
                                                       int guess, double* ws, double* out,
                                                       int* flags, const int* gate, double* xcopy,
                                                       long spin, FsiArgs ua, int uit, int uK,
                                                       double utol, int ufixed) {
  const bool ok = refine_body<CACHE, TWO>(M, X, pm, b, f, n, rw, tpr, maxit, guess, ws, out,
                                          flags, gate, xcopy, spin, blockIdx.x, gridDim.x);
  extern __shared__ double lds[];
  __syncthreads();
  update_body(ua, uit, uK, utol, ufixed, blockIdx.x, gridDim.x, ok ? lds : ua.f);
}

// Many instances per launch: instance blockIdx.y's nb workgroups are its own barrier group
// (counters in its own workspace); the workgroups of one instance are consecutive in the
// dispatch order.
template <bool CACHE, bool TWO>
__global__ __launch_bounds__(256) void k_refine_multi(const RefineJob* __restrict__ tab) {
  const RefineJob j = tab[blockIdx.y];
  if ((int)blockIdx.x >= j.nb) return;
  refine_body<CACHE, TWO>(j.M, j.X, j.pm, j.b, j.f, j.n, j.rw, j.tpr, j.maxit, j.guess, j.ws, j.out,
                     j.flags, j.gate, j.xcopy, j.spin, blockIdx.x, j.nb);
}

// C = A B for n x n FP64 matrices (pitch p), optionally C = 2 I - A B, on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64; A fragment: lane l holds A[i0 + l % 16][k + l / 16], B
// fragment B[k + l / 16][j0 + l % 16], result item v of lane l is C[i0 + l / 16 + 4 v]
// [j0 + l % 16]).  One 16 x 16 tile of C per workgroup of GEMM_KS waves: wave w takes the
// w-th of GEMM_KS equal k ranges (multiples of 4), so the dependent MFMA chain of a wave is
// 1/GEMM_KS of the k extent (at n = 202: 7 products of 64 cycles each at this chip's FP64
// matrix rate, instead of 52 for a wave that owns its tile's whole k range).
typedef double v4d __attribute__((ext_vector_type(4)));
// KC k steps (of 4) per chunk, loaded before any is used; when a wave's k range fits one
// chunk (n <= GEMM_ONE_N with KC = GEMM_KC) each wave waits for memory once.  Two
// accumulators alternate over k; the partial tiles are added in wave order through LDS
// (deterministic).
template <int KC>
__device__ __forceinline__ void gemm64_body(const double* A, const double* B, double* C, int n,
                                            int p, int two_minus, const int* gate, int bx, int by) {
  __shared__ v4d part[GEMM_KS - 1][64];
  if (iter_gated(gate)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = by * 16, j0 = bx * 16;
  const int li = lane & 15, lk = lane >> 4;
  const int ai = i0 + li, bj = j0 + li;
  const int per = ((n + 3) / 4 + GEMM_KS - 1) / GEMM_KS;  // k steps of 4 per wave
  const int kbeg = 4 * per * w, kend = min(n, 4 * per * (w + 1));
  v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = kbeg; k0 < kend; k0 += 4 * KC) {
    double av[KC], bv[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int k = k0 + 4 * c + lk;
      av[c] = (ai < n && k < kend) ? A[(size_t)ai * p + k] : 0.0;
      bv[c] = (bj < n && k < kend) ? B[(size_t)k * p + bj] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < KC; c += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c], bv[c], acc0, 0, 0, 0);
      if (c + 1 < KC) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c + 1], bv[c + 1], acc1, 0, 0, 0);
    }
  }
  acc0 += acc1;
  if (w > 0) part[w - 1][lane] = acc0;
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int q = 0; q < GEMM_KS - 1; ++q) acc0 += part[q][lane];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + lk + 4 * v, j = j0 + li;
    if (i < n && j < n) {
      double val = acc0[v];
      if (two_minus) val = (i == j ? 2.0 : 0.0) - val;
      C[(size_t)i * p + j] = val;
    }
  }
}

template <int KC>
__global__ __launch_bounds__(64 * GEMM_KS) void k_gemm64(const double* A, const double* B, double* C, int n,
                                                int p, int two_minus, const int* gate) {
  gemm64_body<KC>(A, B, C, n, p, two_minus, gate, blockIdx.x, blockIdx.y);
}

template <int KC>
__global__ __launch_bounds__(64 * GEMM_KS) void k_gemm64_multi(const GemmJob* __restrict__ tab) {
  const GemmJob j = tab[blockIdx.z];
  const int nb = (j.n + 15) / 16;
  if ((int)blockIdx.x >= nb || (int)blockIdx.y >= nb) return;
  gemm64_body<KC>(j.A, j.B, j.C, j.n, j.p, j.two_minus, j.gate, blockIdx.x, blockIdx.y);
}

// out (bits of a non-negative double, atomicMax) = max |W_ij - delta_ij| over n x n.
__global__ __launch_bounds__(256) void k_eye_resid(const double* W, int p, int n, double* out) {
  double m = 0.0;
  bool bad = false;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < (size_t)n * n;
       e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double d = fabs(W[(size_t)i * p + j] - (i == j ? 1.0 : 0.0));
    if (!(d == d)) bad = true;
    else m = fmax(m, d);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  const bool anybad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    const double v = anybad ? INFINITY : m;
    atomicMax(reinterpret_cast<unsigned long long*>(out), (unsigned long long)__double_as_longlong(v));
  }
}

hipError_t launch_eye_resid(const double* W, int p, int n, double* out, hipStream_t st) {
  const size_t tot = (size_t)n * n;
  const int nb = (int)std::min<size_t>(1024, (tot + 255) / 256);
  hipLaunchKernelGGL(k_eye_resid, dim3(nb), dim3(256), 0, st, W, p, n, out);
  return hipGetLastError();
}

// Start of a step's FSI control: clears the error and refinement flags, the gates and the
// iteration count (ctl layout in FsiCtl).
__global__ void k_step_reset(int* ctl) {
  if (threadIdx.x < FsiCtl::INTS) ctl[threadIdx.x] = 0;
}

__global__ void k_step_reset_multi(int* const* __restrict__ ctls) {
  int* ctl = ctls[blockIdx.x];
  if (threadIdx.x < FsiCtl::INTS) ctl[threadIdx.x] = 0;
}

// Copies the control blocks of many instances into one array (FsiCtl::BYTES each), so
// that one transfer brings them all to the host.
__global__ void k_gather_ctl(int* const* __restrict__ ctls, int* out) {
  constexpr int W = FsiCtl::BYTES / 4;
  const int* ctl = ctls[blockIdx.x];
  if (threadIdx.x < W) out[blockIdx.x * W + threadIdx.x] = ctl[threadIdx.x];
}

hipError_t launch_step_reset(int* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(64), 0, st, ctl);
  return hipGetLastError();
}

__global__ void k_identity(double* X, int p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) X[(size_t)i * p + i] = 1.0;
}

// ----------------------------------------------------------------- launchers
hipError_t launch_identity(double* X, int p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_identity, dim3((n + 255) / 256), dim3(256), 0, st, X, p, n);
  return hipGetLastError();
}
bool refine_shape(int n, RefineShape* out) {
  if (n < 1) return false;
  int nb = std::min(16, (n + 7) / 8);
  int rw = (n + nb - 1) / nb;
  if ((size_t)2 * rw * n * 8 > REF_LDS_CACHE) {
    nb = std::min(REF_NB_ONE, (n + 7) / 8);
    rw = (n + nb - 1) / nb;
  }
  bool cache = (size_t)2 * rw * n * 8 <= REF_LDS_CACHE;
  if (!cache) {
    // the fewest workgroups whose rows of M and columns of X fit REF_LDS_BIG
    const int rwmax = (int)(REF_LDS_BIG / ((size_t)16 * n));
    if (rwmax >= 1 && (n + rwmax - 1) / rwmax <= REF_NB_MAX) {
      rw = rwmax;
      cache = true;
    }
  }
  nb = (n + rw - 1) / rw;  // no workgroup without rows
  const bool two = nb > REF_NB_ONE;
  int tpr = 64;            // threads per row of r = b - M f: a power of two, tpr * rw <= 256
  while (tpr > 1 && tpr * rw > 256) tpr >>= 1;
  if (tpr * rw > 256) return false;
  const size_t lds = ((size_t)2 * n + 2 * rw + 4 + (cache ? (size_t)2 * rw * n : 0) +
                      (two ? (size_t)n + nb : 0)) * 8;
  if (lds > 150 * 1024) return false;
  *out = RefineShape{nb, rw, tpr, cache, lds, two};
  return true;
}

hipError_t launch_refine(const double* M, int pm, const double* X, const double* b, double* f,
                         int n, int maxit, int guess, double* ws, double* out, int* flags,
                         const int* gate, double* xcopy, long spin, hipStream_t st,
                         const FsiArgs* ua, int uit, int uK, double utol, int ufixed) {
  RefineShape r;
  if (maxit < 1 || !refine_shape(n, &r)) return hipErrorInvalidValue;
  if (ua != nullptr) {
    if (r.two)
      hipLaunchKernelGGL((k_refine_update<true, true>), dim3(r.nb), dim3(256), r.lds, st, M, X, pm,
                         b, f, n, r.rw, r.tpr, maxit, guess, ws, out, flags, gate, xcopy, spin,
                         *ua, uit, uK, utol, ufixed);
    else if (r.cache)
      hipLaunchKernelGGL((k_refine_update<true, false>), dim3(r.nb), dim3(256), r.lds, st, M, X,
                         pm, b, f, n, r.rw, r.tpr, maxit, guess, ws, out, flags, gate, xcopy, spin,
                         *ua, uit, uK, utol, ufixed);
    else
      hipLaunchKernelGGL((k_refine_update<false, false>), dim3(r.nb), dim3(256), r.lds, st, M, X,
                         pm, b, f, n, r.rw, r.tpr, maxit, guess, ws, out, flags, gate, xcopy, spin,
                         *ua, uit, uK, utol, ufixed);
    return hipGetLastError();
  }
  if (r.two)
    hipLaunchKernelGGL((k_refine<true, true>), dim3(r.nb), dim3(256), r.lds, st, M, X, pm, b, f, n,
                       r.rw, r.tpr, maxit, guess, ws, out, flags, gate, xcopy, spin);
  else if (r.cache)
    hipLaunchKernelGGL((k_refine<true, false>), dim3(r.nb), dim3(256), r.lds, st, M, X, pm, b, f,
                       n, r.rw, r.tpr, maxit, guess, ws, out, flags, gate, xcopy, spin);
  else
    hipLaunchKernelGGL((k_refine<false, false>), dim3(r.nb), dim3(256), r.lds, st, M, X, pm, b, f,
                       n, r.rw, r.tpr, maxit, guess, ws, out, flags, gate, xcopy, spin);
  return hipGetLastError();
}

// Whether the nb workgroups of one refinement of n unknowns can all be resident at once on
// this device (the device-wide barrier needs that): the kernel's occupancy per compute unit,
// for its threads and LDS, times the compute units.
bool refine_coresident(int n, int* have, int* need) {
  RefineShape r;
  *have = *need = 0;
  if (!refine_shape(n, &r)) return false;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  hipError_t e;
  if (r.two)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_refine<true, true>, 256, r.lds);
  else if (r.cache)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_refine<true, false>, 256, r.lds);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_refine<false, false>, 256, r.lds);
  if (e != hipSuccess) return false;
  *have = per * cus;
  *need = r.nb;
  return *have >= *need;
}
hipError_t launch_gemm64(const double* A, const double* B, double* C, int n, int p, int two_minus,
                         hipStream_t st, const int* gate) {
  const int nb = (n + 15) / 16;
  if (n <= GEMM_ONE_N)
    hipLaunchKernelGGL(k_gemm64<GEMM_KC>, dim3(nb, nb), dim3(64 * GEMM_KS), 0, st, A, B, C, n, p,
                       two_minus, gate);
  else
    hipLaunchKernelGGL(k_gemm64<16>, dim3(nb, nb), dim3(64 * GEMM_KS), 0, st, A, B, C, n, p,
                       two_minus, gate);
  return hipGetLastError();
}


template <typename T>
hipError_t launch_body_ops(const FsiArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_body_ops<T>), dim3((2 * a.npts + 63) / 64), dim3(64), 0, st, a);
  return hipGetLastError();
}
__global__ void k_cols_to_matrix(const double* vals, int nf, int ns, int c0, double* G, int pm) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nf * ns) return;
  const int t = e % nf, b = e / nf;
  G[(size_t)t * pm + c0 + b] = vals[(size_t)b * nf + t];
}

hipError_t launch_cols_to_matrix(const double* vals, int nf, int ns, int c0, double* G, int pm,
                                 hipStream_t st) {
  const int tot = nf * ns;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cols_to_matrix, dim3((tot + 255) / 256), dim3(256), 0, st, vals, nf, ns,
                     c0, G, pm);
  return hipGetLastError();
}

size_t schur_lds_bytes(const FsiArgs& a) {
  size_t lds = a.gx != nullptr ? 8 : (size_t)a.nf * SCHUR_LDS_PER_ROW;
  if (lds > SCHUR_LDS_MAX || a.nf > SCHUR_CPT * SCHUR_NT) return 0;
  const int all4 = a.gx == nullptr && (size_t)a.nf * SCHUR_LDS_PER_ROW_ALL4 <= SCHUR_LDS_ALL4_MAX;
  if (all4) lds = (size_t)a.nf * SCHUR_LDS_PER_ROW_ALL4;
  return lds;
}

hipError_t launch_schur_sd(const FsiArgs& a, hipStream_t st) {
  const size_t lds = schur_lds_bytes(a);
  if (lds == 0) return hipErrorInvalidValue;
  const int all4 = a.gx == nullptr && (size_t)a.nf * SCHUR_LDS_PER_ROW_ALL4 <= SCHUR_LDS_ALL4_MAX;
  hipLaunchKernelGGL(k_schur_sd, dim3(a.nf), dim3(SCHUR_NT), lds, st, a, all4);
  return hipGetLastError();
}
hipError_t launch_lu_solve(double* M, int pm, double* B, int pb, int n, int nrhs, int* flags,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(LU_NT), 0, st, M, pm, B, pb, n, nrhs, flags);
  return hipGetLastError();
}
hipError_t launch_matvec(const double* A, int pa, const double* x, double* y, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_matvec, dim3(n), dim3(256), 0, st, A, pa, x, y, n);
  return hipGetLastError();
}
hipError_t launch_beam(const FsiArgs& a, int bi, int m, hipStream_t st) {
  const int ncol = 2 * m + 1;
  // BEAM_NC right-hand sides per workgroup; every workgroup repeats the factorisation,
  // which costs no extra latency and spreads the solves over more CUs
  const size_t lds = beam_lds_bytes(m);
  if (m < 2 || lds > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_beam, dim3((ncol + BEAM_NC - 1) / BEAM_NC), dim3(BEAM_NT), lds, st, a, bi);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_ops_beam(const FsiArgs& a, int bi, int m, hipStream_t st) {
  const size_t lds = beam_lds_bytes(m);
  if (m < 2 || lds > 150 * 1024) return hipErrorInvalidValue;
  const int nbeam = (2 * m + 1 + BEAM_NC - 1) / BEAM_NC;
  const int nops = (2 * a.npts + BEAM_NT - 1) / BEAM_NT;
  hipLaunchKernelGGL((k_ops_beam<T>), dim3(nbeam + nops), dim3(BEAM_NT), lds, st, a, bi, nbeam);
  return hipGetLastError();
}
template hipError_t launch_ops_beam<float>(const FsiArgs&, int, int, hipStream_t);
template hipError_t launch_ops_beam<double>(const FsiArgs&, int, int, hipStream_t);

int update_blocks(int nf) {
  // enough waves for one group of 4 rows of the largest beam (3m - 3 <= 1.5 nf rows)
  const int groups = (3 * nf / 2 + 3) / 4;
  return std::max(1, (groups + STRUCT_NT / 64 - 1) / (STRUCT_NT / 64));
}

hipError_t launch_update(const FsiArgs& a, int it, int K, double tol, int fixed, hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3(update_blocks(a.nf)), dim3(STRUCT_NT), 0, st, a, it, K, tol,
                     fixed);
  return hipGetLastError();
}
hipError_t launch_finish(const FsiArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(STRUCT_NT), 0, st, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_spread(const FsiArgs& a, int jlo, int jhi, int ilo, int ihi, T* out, int po,
                         hipStream_t st, bool finish) {
  if (a.nf > SPREAD_MAXROWS) return hipErrorInvalidValue;
  static_assert(SPREAD_NT == STRUCT_NT, "the structure finish runs in a spread workgroup");
  const int gx = (a.n - 1 + SPREAD_TX - 1) / SPREAD_TX;
  dim3 g(gx + (finish ? 1 : 0), (jhi - jlo + 1 + SPREAD_TY - 1) / SPREAD_TY);
  hipLaunchKernelGGL((k_spread<T>), g, dim3(SPREAD_NT), spread_lds_bytes(a.nf), st, a, jlo, jhi,
                     ilo, ihi, out, po, finish ? gx : -1);
  return hipGetLastError();
}
hipError_t launch_point_source_rowdst(const OffRows& o, int col0, int ncols, int nslots,
                                      const void* tw, double* out, int po, size_t bso,
                                      int* rows_first, hipStream_t st) {
  hipLaunchKernelGGL((k_point_source_rowdst<double>), dim3(4, nslots), dim3(256), 0, st, o, col0,
                     ncols, static_cast<const c2<double>*>(tw), out, po, bso, rows_first);
  return hipGetLastError();
}
hipError_t launch_sample(const OffRows& o, int ntarget, const double* sl, int ps, size_t bss,
                         double* vals, int nslots, hipStream_t st) {
  hipLaunchKernelGGL((k_sample<double>), dim3((ntarget + 255) / 256, nslots), dim3(256), 0, st, o,
                     ntarget, sl, ps, bss, vals, nslots);
  return hipGetLastError();
}
hipError_t launch_filter_compact(const double* vals, int ntarget, int col0, int ncols, int nslots,
                                 double eps, int* out_col, double* out_val, int* counts,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_filter_compact, dim3(nslots), dim3(CMP_NT), 0, st, vals, ntarget, col0,
                     ncols, eps, out_col, out_val, counts);
  return hipGetLastError();
}

// Concatenate the compacted entries of every slot (in slot order).
__global__ void k_gather_batch(const int* cols, const double* vals, int ntarget, const int* counts,
                               int* out_col, double* out_val) {
  const int b = blockIdx.x;
  int off = 0;
  for (int q = 0; q < b; ++q) off += counts[q];
  const int c = counts[b];
  for (int e = threadIdx.x; e < c; e += blockDim.x) {
    out_col[off + e] = cols[(size_t)b * ntarget + e];
    out_val[off + e] = vals[(size_t)b * ntarget + e];
  }
}

// M[:, c] *= s * colscale[c]

// Initial acceleration of the deformable bodies at rest: zetadot = -R(chi) / m.
__global__ __launch_bounds__(STRUCT_NT) void k_beam_init(FsiArgs a) {
  const int tid = threadIdx.x;
  for (int bi = 0; bi < a.nbodies; ++bi) {
    const BodyDev b = a.bodies[bi];
    if (b.kind != BODY_DEFORMABLE) continue;
    const int m = b.npts;
    __shared__ double rint[MAX_BEAM_DOF + 3];
    for (int e = tid; e < 3 * m; e += STRUCT_NT) rint[e] = 0.0;
    __syncthreads();
    for (int parity = 0; parity < 2; ++parity) {
      for (int el = 2 * tid + parity; el < m - 1; el += 2 * STRUCT_NT) {
        double fe[6], ke[36];
        beam_element(a.chi + b.dof0 + 3 * el, a.l0[b.dof0 / 3 + el], a.beta0[b.dof0 / 3 + el],
                     b.ea, b.ei, fe, ke);
        for (int p = 0; p < 6; ++p) rint[3 * el + p] += fe[p];
      }
      __syncthreads();
    }
    for (int e = tid; e < 3 * m; e += STRUCT_NT) {
      const int g = b.dof0 + e;
      a.zeta[g] = 0.0;
      a.zetadot[g] = e < 3 ? 0.0 : -rint[e] / a.dmass[g];
    }
    __syncthreads();
  }
}

hipError_t launch_gather_batch(const int* cols, const double* vals, int ntarget, const int* counts,
                               int nslots, int* out_col, double* out_val, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_batch, dim3(nslots), dim3(256), 0, st, cols, vals, ntarget, counts,
                     out_col, out_val);
  return hipGetLastError();
}
hipError_t launch_beam_init(const FsiArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_beam_init, dim3(1), dim3(STRUCT_NT), 0, st, a);
  return hipGetLastError();
}

size_t beam_lds(int m) { return beam_lds_bytes(m); }

// ------------------------------------------------------- many instances per launch
template <typename T>
hipError_t launch_body_ops_multi(const FsiArgs* tab, int count, int max_npts, int it,
                                 hipStream_t st) {
  if (count <= 0 || max_npts <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_body_ops_multi<T>), dim3((2 * max_npts + 63) / 64, count), dim3(64), 0, st,
                     tab, it);
  return hipGetLastError();
}
hipError_t launch_schur_sd_multi(const FsiArgs* tab, int count, int max_nf, size_t lds, int it,
                                 hipStream_t st) {
  if (count <= 0 || max_nf <= 0) return hipSuccess;
  if (lds == 0 || lds > SCHUR_LDS_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_schur_sd_multi, dim3(max_nf, count), dim3(SCHUR_NT), lds, st, tab, it);
  return hipGetLastError();
}
hipError_t launch_beam_multi(const BeamJob* tab, int count, int max_m, size_t lds, int it,
                             hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (max_m < 2 || lds > 150 * 1024) return hipErrorInvalidValue;
  const int ncol = 2 * max_m + 1;
  hipLaunchKernelGGL(k_beam_multi, dim3((ncol + BEAM_NC - 1) / BEAM_NC, count), dim3(BEAM_NT), lds,
                     st, tab, it);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_ops_beam_multi(const FsiArgs* fa, int ni, int max_npts, const BeamJob* beams,
                                 int nbeam, int max_m, size_t lds, int it, hipStream_t st) {
  if (ni <= 0) return hipSuccess;
  if (max_m < 2 || lds > 150 * 1024) return hipErrorInvalidValue;
  const int gx =
      std::max((2 * max_m + 1 + BEAM_NC - 1) / BEAM_NC, (2 * max_npts + BEAM_NT - 1) / BEAM_NT);
  hipLaunchKernelGGL((k_ops_beam_multi<T>), dim3(gx, nbeam + ni), dim3(BEAM_NT), lds, st, fa, ni,
                     beams, nbeam, it);
  return hipGetLastError();
}
template hipError_t launch_ops_beam_multi<float>(const FsiArgs*, int, int, const BeamJob*, int, int,
                                                 size_t, int, hipStream_t);
template hipError_t launch_ops_beam_multi<double>(const FsiArgs*, int, int, const BeamJob*, int, int,
                                                  size_t, int, hipStream_t);
hipError_t launch_update_multi(const UpdateJob* tab, int count, int max_nb, int it, int K,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_multi, dim3(max_nb, count), dim3(STRUCT_NT), 0, st, tab, it, K);
  return hipGetLastError();
}
hipError_t launch_finish_multi(const FsiArgs* tab, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finish_multi, dim3(1, count), dim3(STRUCT_NT), 0, st, tab);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_spread_multi(const SpreadJob<T>* tab, int count, int max_gx, int max_gy,
                               int max_nf, hipStream_t st) {
  if (count <= 0 || max_gx <= 0 || max_gy <= 0) return hipSuccess;
  if (max_nf > SPREAD_MAXROWS) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_spread_multi<T>), dim3(max_gx, max_gy, count), dim3(SPREAD_NT),
                     spread_lds_bytes(max_nf), st, tab);
  return hipGetLastError();
}
hipError_t launch_matvec_multi(const MatvecJob* tab, int count, int max_n, hipStream_t st) {
  if (count <= 0 || max_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_matvec_multi, dim3(max_n, count), dim3(256), 0, st, tab);
  return hipGetLastError();
}
hipError_t launch_gemm64_multi(const GemmJob* tab, int count, int max_n, int kc52,
                               hipStream_t st) {
  if (count <= 0 || max_n <= 0) return hipSuccess;
  const int nb = (max_n + 15) / 16;
  if (kc52)
    hipLaunchKernelGGL(k_gemm64_multi<GEMM_KC>, dim3(nb, nb, count), dim3(64 * GEMM_KS), 0, st, tab);
  else
    hipLaunchKernelGGL(k_gemm64_multi<16>, dim3(nb, nb, count), dim3(64 * GEMM_KS), 0, st, tab);
  return hipGetLastError();
}
hipError_t launch_refine_multi(const RefineJob* tab, int count, int max_nb, size_t lds, int cache,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (lds > 150 * 1024 || max_nb < 1 || max_nb > REF_NB_MAX) return hipErrorInvalidValue;
  if (cache == 2)
    hipLaunchKernelGGL((k_refine_multi<true, true>), dim3(max_nb, count), dim3(256), lds, st, tab);
  else if (cache == 1)
    hipLaunchKernelGGL((k_refine_multi<true, false>), dim3(max_nb, count), dim3(256), lds, st, tab);
  else
    hipLaunchKernelGGL((k_refine_multi<false, false>), dim3(max_nb, count), dim3(256), lds, st, tab);
  return hipGetLastError();
}
hipError_t launch_step_reset_multi(int* const* ctls, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step_reset_multi, dim3(count), dim3(64), 0, st, ctls);
  return hipGetLastError();
}
hipError_t launch_gather_ctl(int* const* ctls, int count, int* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_ctl, dim3(count), dim3(64), 0, st, ctls, out);
  return hipGetLastError();
}

template hipError_t launch_body_ops_multi<float>(const FsiArgs*, int, int, int, hipStream_t);
template hipError_t launch_body_ops_multi<double>(const FsiArgs*, int, int, int, hipStream_t);
template hipError_t launch_spread_multi<float>(const SpreadJob<float>*, int, int, int, int,
                                                 hipStream_t);
template hipError_t launch_spread_multi<double>(const SpreadJob<double>*, int, int, int, int,
                                                 hipStream_t);
// Outputs of the last step (Sec. 5: forces and lift; Sec. 2.3: the no-slip constraint at
// t_{n+1}), one workgroup:
//   out[0]           max over stress rows of |(1/h) W (C s_{n+1} + q_inf) - U_b|, with W the
//                    row's operator of the last FSI iterate (E, or P E0 in sub-domain mode)
//                    and U_b the body velocity at t_{n+1}: the prescribed one (rigid,
//                    moving), phi_{n+1} e_z x (p - hinge) at the last iterate's points
//                    (torsional; plus the driver's velocity on a mount), zeta_{n+1} at the
//                    node (deformable);
//   out[1 + 2b + c]  force of body b in direction c, ds * sum of its stresses (tree sum in a
//                    fixed order).
constexpr int OUT_NT = 256;
template <typename T>
__global__ __launch_bounds__(OUT_NT) void k_outputs(FsiArgs a, const T* __restrict__ s0, int ps,
                                                    double* out) {
  __shared__ double red[OUT_NT];
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int row = tid; row < a.nf; row += OUT_NT) {
    const BodyDev b = a.bodies[row_body(a, row)];
    const int rel = row - 2 * b.pt0;
    const int comp = a.st_base[3 * row + 2];
    const int local = rel - comp * b.npts;
    const int p = b.pt0 + local;
    const int bx = a.st_base[3 * row], by = a.st_base[3 * row + 1];
    double acc = 0.0;
    for (int e = 0; e < 16; ++e) {
      const double w = a.st_w[16 * row + e];
      if (w != 0.0) acc += w * face_flux(s0, ps, comp, bx + (e & 3), by + (e >> 2), a.ux, a.uy);
    }
    double tgt = 0.0;
    if (b.kind == BODY_RIGID || b.kind == BODY_MOVING) {
      tgt = rhs_body_term(a, b, local, comp);
    } else if (b.kind == BODY_TORSIONAL) {
      const double* ts = a.tors + b.tors * TS_COUNT;
      double hx, hy, ang0;
      tors_frame(a, b, &hx, &hy, &ang0);
      const double dx = a.pos[2 * p] - hx, dy = a.pos[2 * p + 1] - hy;
      tgt = comp == 0 ? -ts[TS_PHI] * dy : ts[TS_PHI] * dx;
      if (b.moff >= 0) {
        const double* q = a.poses + b.moff;
        tgt += comp == 0 ? q[MF_VX] - q[MF_OM] * dy : q[MF_VY] + q[MF_OM] * dx;
      }
    } else {
      tgt = a.zeta[b.dof0 + 3 * local + comp];
    }
    mx = fmax(mx, fabs(acc / a.h - tgt));
  }
  red[tid] = mx;
  __syncthreads();
  for (int w = OUT_NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) out[0] = red[0];
  __syncthreads();
  for (int bi = 0; bi < a.nbodies; ++bi) {
    const BodyDev b = a.bodies[bi];
    for (int c = 0; c < 2; ++c) {
      double sum = 0.0;
      for (int k = tid; k < b.npts; k += OUT_NT) sum += a.f[2 * b.pt0 + c * b.npts + k];
      red[tid] = sum;
      __syncthreads();
      for (int w = OUT_NT / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
      }
      if (tid == 0) out[1 + 2 * bi + c] = red[0] * b.ds;
      __syncthreads();
    }
  }
}

template <typename T>
hipError_t launch_outputs(const FsiArgs& a, const T* s0, int ps, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_outputs<T>), dim3(1), dim3(OUT_NT), 0, st, a, s0, ps, out);
  return hipGetLastError();
}
template hipError_t launch_outputs<float>(const FsiArgs&, const float*, int, double*, hipStream_t);
template hipError_t launch_outputs<double>(const FsiArgs&, const double*, int, double*, hipStream_t);

template hipError_t launch_body_ops<float>(const FsiArgs&, hipStream_t);
template hipError_t launch_body_ops<double>(const FsiArgs&, hipStream_t);
template hipError_t launch_spread<float>(const FsiArgs&, int, int, int, int, float*, int, hipStream_t,
                                         bool);
template hipError_t launch_spread<double>(const FsiArgs&, int, int, int, int, double*, int,
                                          hipStream_t, bool);

}  // namespace ib
