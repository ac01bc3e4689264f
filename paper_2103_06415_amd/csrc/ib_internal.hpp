// Internal interfaces between the kernel files and the host engine.
#pragma once

#include <shared_mutex>

#include "ib_common.hpp"

namespace ib {

// Explicit right-hand side of one level (see ib_flow.hip).
template <typename T>
struct RhsArgs {
  const T* s;          // streamfunction at time n, (n+1) rows x ps, ring included
  const T* g;          // circulation gamma = C^T C s at time n, interior, (n-1) rows x pg
  const T* gf;         // finer level's circulation at time n (coarsification on read), or null
  const T* gring;      // ring circulation at time n, [4][n+1]
  const T* gring_new;  // new circulation ring [4][n+1], or null (zero ring)
  const T* hist_in;    // C^T N_{n-1}, (n-1) rows x ph, or null on the first step
  T* hist_out;         // C^T N_n (may alias hist_in)
  T* out;              // row-transformed right-hand side, (n-1) rows x po
  int n, ps, pg, pgf, ph, po;  // n: cells along x (the row transform's length)
  T alpha, dt, ux, uy, cn;  // cn = -1 / (2 h^2); ux, uy = free-stream flux u_inf h
  int var;             // kernel configuration (ROW_VARIANTS; 0 = default)
  int ny;              // cells along y; 0: ny = n (square level)
};

// Row-wise transform of rows [r0, r1] (1-based interior rows).
template <typename T>
struct RowArgs {
  const T* in;
  T* out;
  int pi, po;
  int r0, r1;
  size_t bsi, bso;  // batch strides (elements)
  int interior_out; // inverse transform: write an (n-1)-row interior array instead of a
                    // full (n+1)-row array with its ring
  const T* in2;     // inverse transform: a second array transformed alongside `in`
  T* out2;          //   into the interior array out2 (pitch po); batch 1 only
  int var;          // inverse transform with in2: kernel configuration (ROW_VARIANTS)
  const int* gate;  // if set: run only when gate[0] = 1 and gate[1] = 0 (FsiArgs::gate)
  int ny;           // inverse transform with its ring: cells along y; 0: the row length
  int* reset;       // inverse transform: if set, its first workgroup also clears `nreset`
  int nreset;       //   ints there (a control block that only later launches read)
};

// Column transform + spectral scale + inverse column transform.
template <typename T>
struct ColArgs {
  const T* in;
  T* out;
  int pi, po;
  int r0, r1;        // nonzero input rows (1-based interior rows)
  T alpha, scale;    // multiplier scale / (lam (1 + alpha lam)) for `out` and
  T* out2;           //   scale / (1 + alpha lam) for `out2` (if set; pitch po, stride bso)
  const T* lift;     // if set: 1-D DSTs of the new streamfunction ring's four edges,
                     //   [4][n-1]; `out` then solves L s = gamma + B(s_ring) instead
  int accumulate;    // out += result instead of out = result
  size_t bsi, bso;
  const int* rfirst; // if set: slot b's input holds rows rfirst[b] .. rfirst[b] + rcount - 1
  int rcount;        //   compactly (row rfirst[b] at input row 0)
  int w0, w1;        // output rows written (1-based); others untouched
  int var;           // kernel configuration (COL_VARIANTS; 0 = default)
  const int* gate;   // if set: run only when gate[0] = 1 and gate[1] = 0 (FsiArgs::gate)
  hipEvent_t ev0, ev1;  // host side, if set (kernel timing): recorded at the kernel's start and
                        //   end by the launch itself (hipExtLaunchKernelGGL), without its dispatch
  // rectangular levels (the column transform runs along y, of length ny): the nx - 1 columns,
  // the x eigenvalues lam_x[k - 1] and sin(pi k / nx), k <= nx; 0 / null: square level
  int ncols;
  const T* lamx;
  const T* sinx;
};

// Per-instance entries of the flow launches that take many instances of one grid size
// (ib_batch_*): the inverse row transform with its ring, and a new ring from the next coarser
// level with the edge transforms of its streamfunction part.
template <typename T>
struct IdstJob {
  RowArgs<T> a;
  const T* ring;
  int ring_rows;
};
template <typename T>
struct RingJob {
  const T* sc;  // coarser level's streamfunction, pitch psc
  int psc;
  const T* gc;  // coarser level's circulation (interior vertices), pitch pgc
  int pgc;
  T* sring;
  T* gring;
  T* lift;
  int nx, ny;   // cells of the fine level
};

// Kernel configurations of the row and column sine-transform kernels, selected per grid
// size by measurement (single precision, n >= FLOW_TUNE_MIN_N; otherwise entry 0).
// Rows: rows per workgroup, threads, largest radix; columns: columns per workgroup,
// threads, largest radix.
struct FlowVariant {
  int width, nt, maxr;
};
// Row kernels have ROW_VARIANT_COUNT configurations, the column solve COL_VARIANT_COUNT;
// FLOW_VARIANTS is the larger (the size of the measurement tables).  Column configuration
// COL_REG_VARIANT is the register-resident form (ib_flow_reg.hpp: columns per workgroup,
// threads, FFT split P = 32), available where n = P^2 (n = 1024).
constexpr int ROW_VARIANT_COUNT = 8;
constexpr int COL_VARIANT_COUNT = 9;
constexpr int FLOW_VARIANTS = 9;
constexpr int COL_REG_VARIANT = 8;
constexpr int FLOW_TUNE_MIN_N = 256;
constexpr FlowVariant ROW_VARIANTS[ROW_VARIANT_COUNT] = {
    {2, 256, 16}, {2, 256, 8}, {2, 512, 16}, {2, 512, 8},
    {2, 512, 4},  {4, 512, 8}, {4, 1024, 8}, {4, 1024, 16}};
constexpr FlowVariant COL_VARIANTS[COL_VARIANT_COUNT] = {
    {4, 256, 16}, {4, 256, 8}, {2, 256, 4},  {4, 512, 16},
    {4, 512, 8},  {4, 1024, 16}, {8, 512, 16}, {8, 1024, 16}, {4, 128, 32}};
bool flow_variant_available(int n, int fp64);
// Whether configuration v of kind 0 (row kernels) or 1 (column solve) exists for n.
bool flow_kind_variant_available(int kind, int v, int n, int fp64);
// Shared side of the lock between graph recording and the library's other HIP calls.
std::shared_lock<std::shared_mutex> hip_shared_lock();
// Single-precision launches of configuration var (1 .. FLOW_VARIANTS-1), n >= FLOW_TUNE_MIN_N.
hipError_t launch_rhs_rowdst_var(const RhsArgs<float>& a, const void* tw, hipStream_t st);
hipError_t launch_col_solve_var(const ColArgs<float>& a, int n, int batch, const void* tw,
                                const void* lam, hipStream_t st);
hipError_t launch_row_idst_var(const RowArgs<float>& a, int n, int batch, const void* tw,
                               const float* ring, int ring_rows, hipStream_t st);

// Sine transform as a BF16-split matrix product (ib_gemm.hip): C = S X (mode 0) or
// C = X S (mode 1), S = shi + slo the (kpad x kpad, zero padded) DST-I matrix of size nv,
// X FP32 (nv x nv valid, pitch px).  With lam set (mode 0 only) the output is the spectral
// solve of the column pass: c = (y / (1 + alpha L) + lift) scale / L and
// c2 = y / (1 + alpha L) scale, L = lam[row] + lam[col], lift from the ring edge transforms
// (as in k_col_solve) with sinv[k] = sin(pi k / n).
struct GemmArgs {
  const __bf16* shi;
  const __bf16* slo;
  int ps;
  const float* x;
  int px;
  float* c;
  int pc;
  float* c2;
  int pc2;
  int nv, kpad;
  const float* lam;
  float alpha, scale;
  const float* lift;
  const float* sinv;
  int tn;  // stage depth in k of the products (64 or 128); 0: chosen by size
};
hipError_t launch_dst_gemm(const GemmArgs& g, int mode, hipStream_t st);

bool supported_n(int n);
// Transform lengths that run in double precision (every supported one below 4000).
bool supported_n_fp64(int n);

// transform = 0: only the explicit right-hand side, written to a.out row by row
template <typename T>
hipError_t launch_rhs_rowdst(const RhsArgs<T>& a, const void* tw, hipStream_t st, int transform = 1);
template <typename T>
hipError_t launch_rowdst(const RowArgs<T>& a, int n, int batch, const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_col_solve(const ColArgs<T>& a, int n, int batch, const void* tw, const void* lam,
                            hipStream_t st);
template <typename T>
hipError_t launch_row_idst(const RowArgs<T>& a, int n, int batch, const void* tw, const T* ring,
                           int ring_rows, hipStream_t st);
// Rings of an nx x ny level (ring_off layout) from the next coarser level; twx / twy are the
// transform tables of lengths nx and ny (the same on a square level).
template <typename T>
hipError_t launch_ring(const T* sc, int psc, const T* gc, int pgc, int nx, int ny, T* sring,
                       T* gring, hipStream_t st);
template <typename T>
hipError_t launch_ring_edge_dst(const T* sring, int nx, int ny, const void* twx, const void* twy,
                                T* lift, hipStream_t st);
// launch_ring and launch_ring_edge_dst in one launch per edge length (the same results).
template <typename T>
hipError_t launch_ring_dst(const T* sc, int psc, const T* gc, int pgc, int nx, int ny, T* sring,
                           T* gring, const void* twx, const void* twy, T* lift, hipStream_t st);

// The same launches for `count` instances of grid size n at once, their arguments in device
// tables (entry b for blockIdx.y = b); var as above, the same for all instances.  maxrows:
// the largest r1 - r0 + 1 over the entries.  launch_ring_multi makes the new rings and
// then their edge transforms.
template <typename T>
hipError_t launch_rhs_rowdst_multi(const RhsArgs<T>* tab, int count, int n, int var,
                                   const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_col_solve_multi(const ColArgs<T>* tab, int count, int n, int var, const void* tw,
                                  const void* lam, hipStream_t st);
template <typename T>
hipError_t launch_row_idst_multi(const IdstJob<T>* tab, int count, int n, int maxrows, int dual,
                                 int var, const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_rowdst_multi(const RowArgs<T>* tab, int count, int n, int maxrows,
                               const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_ring_multi(const RingJob<T>* tab, int count, int n, const void* tw,
                             hipStream_t st);
hipError_t launch_rhs_rowdst_multi_var(const RhsArgs<float>* tab, int count, int n, int var,
                                       const void* tw, hipStream_t st);
hipError_t launch_col_solve_multi_var(const ColArgs<float>* tab, int count, int n, int var,
                                      const void* tw, const void* lam, hipStream_t st);
hipError_t launch_row_idst_multi_var(const IdstJob<float>* tab, int count, int n, int maxrows,
                                     int var, const void* tw, hipStream_t st);

}  // namespace ib
