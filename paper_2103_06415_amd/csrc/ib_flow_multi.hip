// Launchers of the flow kernels for many instances of one grid size per launch (ib_batch_*),
// in the default configuration of each kernel; a nonzero `var` selects a measured alternative
// (ib_flow_multi_tuned.hip) for single precision, as for one instance.
#include "ib_flow_kernels.hpp"

namespace ib {

#define IB_MULTI_N(n, MACRO)                                   \
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
    default: return hipErrorInvalidValue;                      \
  }

template <typename T>
hipError_t launch_rhs_rowdst_multi(const RhsArgs<T>* tab, int count, int n, int var,
                                   const void* tw, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (var != 0) {
      if (!flow_kind_variant_available(0, var, n, 0)) return hipErrorInvalidValue;
      return launch_rhs_rowdst_multi_var(tab, count, n, var, tw, st);
    }
  }
  constexpr int R = ROW_VARIANTS[0].width, NT = ROW_VARIANTS[0].nt;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN) return launch_rhs_multi_cfg<T, NN, R, NT, 1, 16>(tab, count, t, st)
  IB_MULTI_N(n, L_)
#undef L_
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_col_solve_multi(const ColArgs<T>* tab, int count, int n, int var, const void* tw,
                                  const void* lam, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (var != 0) {
      if (!flow_kind_variant_available(1, var, n, 0)) return hipErrorInvalidValue;
      return launch_col_solve_multi_var(tab, count, n, var, tw, lam, st);
    }
  }
  constexpr int CW = COL_VARIANTS[0].width, NT = COL_VARIANTS[0].nt;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
  const T* l = static_cast<const T*>(lam);
#define L_(NN) return launch_col_multi_cfg<T, NN, CW, NT, 16>(tab, count, t, l, st)
  IB_MULTI_N(n, L_)
#undef L_
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_row_idst_multi(const IdstJob<T>* tab, int count, int n, int maxrows, int dual,
                                 int var, const void* tw, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (var != 0 && dual) {
      if (!flow_kind_variant_available(0, var, n, 0)) return hipErrorInvalidValue;
      return launch_row_idst_multi_var(tab, count, n, maxrows, var, tw, st);
    }
  }
  constexpr int R = ROW_VARIANTS[0].width, NT = ROW_VARIANTS[0].nt;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN)                                                                          \
  return dual ? launch_idst_multi_cfg<T, NN, R, NT, 1, 16>(tab, count, maxrows, t, st) \
              : launch_idst_multi_cfg<T, NN, R, NT, 0, 16>(tab, count, maxrows, t, st)
  IB_MULTI_N(n, L_)
#undef L_
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_rowdst_multi(const RowArgs<T>* tab, int count, int n, int maxrows,
                               const void* tw, hipStream_t st) {
  constexpr int R = ROW_VARIANTS[0].width, NT = ROW_VARIANTS[0].nt;
  const int nb = (maxrows + R - 1) / R;
  if (count <= 0 || nb <= 0) return hipSuccess;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN)                                                                              \
  hipLaunchKernelGGL((k_rowdst_multi<T, NN, R, NT>), dim3(xcd_grid(nb), count), dim3(NT), 0, \
                     st, tab, t)
  IB_MULTI_N(n, L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ring_multi(const RingJob<T>* tab, int count, int n, const void* tw,
                             hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const c2<T>* t = static_cast<const c2<T>*>(tw);
#define L_(NN) \
  hipLaunchKernelGGL((k_ring_dst_multi<T, NN, 256>), dim3(4, count), dim3(256), 0, st, tab, t)
  IB_MULTI_N(n, L_)
#undef L_
  return hipGetLastError();
}

#define IB_INST(T)                                                                             \
  template hipError_t launch_rhs_rowdst_multi<T>(const RhsArgs<T>*, int, int, int, const void*, \
                                                 hipStream_t);                                 \
  template hipError_t launch_col_solve_multi<T>(const ColArgs<T>*, int, int, int, const void*,  \
                                                const void*, hipStream_t);                     \
  template hipError_t launch_row_idst_multi<T>(const IdstJob<T>*, int, int, int, int, int,      \
                                               const void*, hipStream_t);                      \
  template hipError_t launch_rowdst_multi<T>(const RowArgs<T>*, int, int, int, const void*,     \
                                             hipStream_t);                                     \
  template hipError_t launch_ring_multi<T>(const RingJob<T>*, int, int, const void*, hipStream_t);
IB_INST(float)
IB_INST(double)
#undef IB_INST

}  // namespace ib
