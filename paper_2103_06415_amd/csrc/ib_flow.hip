// Launchers of the flow kernels (templates in ib_flow_kernels.hpp) in their default
// configuration; a nonzero `var` in the arguments selects a measured alternative
// (ib_flow_tuned.hip) for single precision.
#include "ib_flow_kernels.hpp"

namespace ib {

// ---------------------------------------------------------------- launchers

// Default configuration of transform length N: rows (or columns) per workgroup and threads.
// From N = 2000 on, one row per workgroup and two columns (one in double precision or at 4000)
// keep the staged rows, the transform buffers and the twiddle table inside the 160 KB of LDS.
template <typename T, int N>
struct Cfg {
  static constexpr bool BIG = N >= 2000;
  static constexpr int ROWS = BIG ? 1 : 2;
  static constexpr int NTR = 256;
  static constexpr int CW = BIG ? ((sizeof(T) == 8 || N >= 4000) ? 1 : 2) : 4;
  static constexpr int NTC = 256;
};
// Transform lengths whose kernels fit the LDS in this precision: 4000 in single precision only
// (its double-precision row staging alone would take 192 KB).
template <typename T, int N>
constexpr bool fits_lds() {
  return !(sizeof(T) == 8 && N >= 4000);
}

#define IB_DISPATCH_N(n, MACRO)                                \
  switch (n) {                                                 \
    case 16: MACRO(16); break;                                 \
    case 20: MACRO(20); break;                                 \
    case 32: MACRO(32); break;                                 \
    case 40: MACRO(40); break;                                 \
    case 48: MACRO(48); break;                                 \
    case 64: MACRO(64); break;                                 \
    case 80: MACRO(80); break;                                 \
    case 96: MACRO(96); break;                                 \
    case 128: MACRO(128); break;                               \
    case 160: MACRO(160); break;                               \
    case 192: MACRO(192); break;                               \
    case 256: MACRO(256); break;                               \
    case 320: MACRO(320); break;                               \
    case 384: MACRO(384); break;                               \
    case 512: MACRO(512); break;                               \
    case 640: MACRO(640); break;                               \
    case 768: MACRO(768); break;                               \
    case 1024: MACRO(1024); break;                             \
    case 1280: MACRO(1280); break;                             \
    case 2000: MACRO(2000); break;                             \
    case 4000: MACRO(4000); break;                             \
    default: return hipErrorInvalidValue;                      \
  }

bool supported_n(int n) {
  switch (n) {
    case 16: case 20: case 32: case 40: case 48: case 64: case 80: case 96: case 128:
    case 160: case 192: case 256: case 320: case 384: case 512: case 640: case 768:
    case 1024: case 1280: case 2000: case 4000:
      return true;
    default:
      return false;
  }
}

bool supported_n_fp64(int n) { return supported_n(n) && n < 4000; }

// sizes with measured alternative configurations (ib_flow_tuned.hip, ib_flow_multi_tuned.hip)
bool flow_variant_available(int n, int fp64) {
  return !fp64 && (n == 256 || n == 384 || n == 512 || n == 768 || n == 1024);
}

bool flow_kind_variant_available(int kind, int v, int n, int fp64) {
  if (v == 0) return true;
  if (v < 0 || !flow_variant_available(n, fp64)) return false;
  if (kind == 0) return v < ROW_VARIANT_COUNT;
  if (v == COL_REG_VARIANT) return n == 1024;
  return v < COL_VARIANT_COUNT;
}

template <typename T>
hipError_t launch_rhs_rowdst(const RhsArgs<T>& a, const void* tw, hipStream_t st, int transform) {
  if constexpr (sizeof(T) == 4) {
    if (a.var != 0) {
      if (!transform || !flow_kind_variant_available(0, a.var, a.n, 0))
        return hipErrorInvalidValue;
      return launch_rhs_rowdst_var(a, tw, st);
    }
  }
  const int rows = (a.ny > 0 ? a.ny : a.n) - 1;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN)                                                                                   \
  {                                                                                              \
    if constexpr (fits_lds<T, NN>()) {                                                           \
      constexpr int R = Cfg<T, NN>::ROWS, NT = Cfg<T, NN>::NTR;                                  \
      const int nb = (rows + R - 1) / R;                                                         \
      if (transform) hipLaunchKernelGGL((k_rhs_rowdst<T, NN, R, NT, 1>), dim3(xcd_grid(nb)), dim3(NT), 0, st, a, t, nb); \
      else hipLaunchKernelGGL((k_rhs_rowdst<T, NN, R, NT, 0>), dim3(xcd_grid(nb)), dim3(NT), 0, st, a, t, nb); \
    } else {                                                                                     \
      return hipErrorInvalidValue;                                                               \
    }                                                                                            \
  }
  IB_DISPATCH_N(a.n, L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rowdst(const RowArgs<T>& a, int n, int batch, const void* tw, hipStream_t st) {
  if (a.r1 < a.r0) return hipSuccess;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN)                                                                                   \
  {                                                                                              \
    if constexpr (fits_lds<T, NN>()) {                                                           \
      constexpr int R = Cfg<T, NN>::ROWS, NT = Cfg<T, NN>::NTR;                                  \
      const int nb = (a.r1 - a.r0 + 1 + R - 1) / R;                                              \
      hipLaunchKernelGGL((k_rowdst<T, NN, R, NT>), dim3(xcd_grid(nb), batch), dim3(NT), 0, st, a, t, nb); \
    } else {                                                                                     \
      return hipErrorInvalidValue;                                                               \
    }                                                                                            \
  }
  IB_DISPATCH_N(n, L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_solve(const ColArgs<T>& a, int n, int batch, const void* tw, const void* lam,
                            hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (a.var != 0) {
      if (!flow_kind_variant_available(1, a.var, n, 0)) return hipErrorInvalidValue;
      return launch_col_solve_var(a, n, batch, tw, lam, st);
    }
  }
  const int cols = a.ncols > 0 ? a.ncols : n - 1;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
  const T* l = static_cast<const T*>(lam);
#define L_(NN)                                                                                     \
  {                                                                                                \
    if constexpr (fits_lds<T, NN>()) {                                                             \
      constexpr int CW = Cfg<T, NN>::CW, NT = Cfg<T, NN>::NTC;                                     \
      const int nb = (cols + CW - 1) / CW;                                                         \
      if (a.ev0)                                                                                   \
        hipExtLaunchKernelGGL((k_col_solve<T, NN, CW, NT>), dim3(xcd_grid(nb), batch), dim3(NT), 0, st, \
                              a.ev0, a.ev1, 0, a, t, l, nb);                                       \
      else                                                                                         \
        hipLaunchKernelGGL((k_col_solve<T, NN, CW, NT>), dim3(xcd_grid(nb), batch), dim3(NT), 0, st, a, \
                           t, l, nb);                                                              \
    } else {                                                                                       \
      return hipErrorInvalidValue;                                                                 \
    }                                                                                              \
  }
  IB_DISPATCH_N(n, L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row_idst(const RowArgs<T>& a, int n, int batch, const void* tw, const T* ring,
                           int ring_rows, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (a.var != 0 && a.in2 != nullptr) {
      if (!flow_kind_variant_available(0, a.var, n, 0)) return hipErrorInvalidValue;
      return launch_row_idst_var(a, n, batch, tw, ring, ring_rows, st);
    }
  }
  if (a.r1 < a.r0) return hipSuccess;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN)                                                                                   \
  {                                                                                              \
    if constexpr (fits_lds<T, NN>()) {                                                           \
      constexpr int R = Cfg<T, NN>::ROWS, NT = Cfg<T, NN>::NTR;                                  \
      const int nb = (a.r1 - a.r0 + 1 + R - 1) / R;                                              \
      if (a.in2) hipLaunchKernelGGL((k_row_idst<T, NN, R, NT, 1>), dim3(xcd_grid(nb), batch), dim3(NT), 0, st, a, t, ring, ring_rows, nb); \
      else hipLaunchKernelGGL((k_row_idst<T, NN, R, NT, 0>), dim3(xcd_grid(nb), batch), dim3(NT), 0, st, a, t, ring, ring_rows, nb); \
    } else {                                                                                     \
      return hipErrorInvalidValue;                                                               \
    }                                                                                            \
  }
  IB_DISPATCH_N(n, L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ring(const T* sc, int psc, const T* gc, int pgc, int nx, int ny, T* sring,
                       T* gring, hipStream_t st) {
  const int tot = ring_len(nx, ny);
  hipLaunchKernelGGL((k_ring<T>), dim3((tot + 255) / 256), dim3(256), 0, st, sc, psc, gc, pgc, nx,
                     ny, sring, gring);
  return hipGetLastError();
}

// Edge transforms of a ring: all four edges in one workgroup on a square level; on a
// rectangular one the bottom and top edges (length nx, tables twx) and the left and right
// edges (length ny, tables twy) in one workgroup each.  From length 2000 on, one workgroup
// per edge (the LDS holds one sequence of that length).
template <typename T>
hipError_t launch_ring_edge_dst(const T* sring, int nx, int ny, const void* twx, const void* twy,
                                T* lift, hipStream_t st) {
  for (int pass = 0; pass < (nx == ny ? 1 : 2); ++pass) {
    const int n = pass == 0 ? nx : ny, e0 = pass == 0 ? 0 : 2, ne = nx == ny ? 4 : 2;
    const c2<T>* t = static_cast<const c2<T>*>(pass == 0 ? twx : twy);
#define L_(NN)                                                                                   \
  {                                                                                              \
    if constexpr (!fits_lds<T, NN>()) {                                                          \
      return hipErrorInvalidValue;                                                               \
    } else if constexpr (NN >= 2000) {                                                           \
      hipLaunchKernelGGL((k_ring_edge_dst<T, NN, 256, 1>), dim3(ne), dim3(256), 0, st, sring, t, lift, e0, ne, nx, ny); \
    } else {                                                                                     \
      hipLaunchKernelGGL((k_ring_edge_dst<T, NN, 256, 4>), dim3(1), dim3(256), 0, st, sring, t, lift, e0, ne, nx, ny); \
    }                                                                                            \
  }
    IB_DISPATCH_N(n, L_)
#undef L_
  }
  return hipGetLastError();
}

// New rings and their edge transforms, one workgroup per edge (two launches on a rectangular
// level: the bottom and top edges with the x tables, the left and right with the y tables).
template <typename T>
hipError_t launch_ring_dst(const T* sc, int psc, const T* gc, int pgc, int nx, int ny, T* sring,
                           T* gring, const void* twx, const void* twy, T* lift, hipStream_t st) {
  for (int pass = 0; pass < (nx == ny ? 1 : 2); ++pass) {
    const int n = pass == 0 ? nx : ny, e0 = pass == 0 ? 0 : 2, ne = nx == ny ? 4 : 2;
    const c2<T>* t = static_cast<const c2<T>*>(pass == 0 ? twx : twy);
#define L_(NN)                                                                                   \
  {                                                                                              \
    if constexpr (fits_lds<T, NN>()) {                                                           \
      hipLaunchKernelGGL((k_ring_dst<T, NN, 256>), dim3(ne), dim3(256), 0, st, sc, psc, gc, pgc, sring, gring, t, lift, e0, nx, ny); \
    } else {                                                                                     \
      return hipErrorInvalidValue;                                                               \
    }                                                                                            \
  }
    IB_DISPATCH_N(n, L_)
#undef L_
  }
  return hipGetLastError();
}

#define IB_INST(T)                                                                              \
  template hipError_t launch_rhs_rowdst<T>(const RhsArgs<T>&, const void*, hipStream_t, int); \
  template hipError_t launch_rowdst<T>(const RowArgs<T>&, int, int, const void*, hipStream_t); \
  template hipError_t launch_col_solve<T>(const ColArgs<T>&, int, int, const void*, const void*, \
                                          hipStream_t);                                        \
  template hipError_t launch_row_idst<T>(const RowArgs<T>&, int, int, const void*, const T*, int, \
                                         hipStream_t);                                         \
  template hipError_t launch_ring<T>(const T*, int, const T*, int, int, int, T*, T*, hipStream_t); \
  template hipError_t launch_ring_edge_dst<T>(const T*, int, int, const void*, const void*, T*,  \
                                              hipStream_t);                                     \
  template hipError_t launch_ring_dst<T>(const T*, int, const T*, int, int, int, T*, T*,         \
                                         const void*, const void*, T*, hipStream_t);
IB_INST(float)
IB_INST(double)
#undef IB_INST

}  // namespace ib
