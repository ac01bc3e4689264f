// Alternative configurations of the single-precision row and column transform kernels
// (ROW_VARIANTS, COL_VARIANTS): rows or columns per workgroup, threads per workgroup and the
// largest FFT radix.  The engine measures them per grid size and launches the fastest.
#include "ib_flow_kernels.hpp"
#include "ib_flow_reg.hpp"

namespace ib {

namespace {

template <int V>
constexpr FlowVariant RV = ROW_VARIANTS[V];
template <int V>
constexpr FlowVariant CV = COL_VARIANTS[V];

template <int N, int V>
hipError_t rhs_v(const RhsArgs<float>& a, const c2<float>* t, hipStream_t st) {
  if constexpr (V >= ROW_VARIANT_COUNT) {
    return hipErrorInvalidValue;
  } else {
    if (a.var != V) return rhs_v<N, V + 1>(a, t, st);
    return launch_rhs_cfg<float, N, RV<V>.width, RV<V>.nt, 1, RV<V>.maxr>(a, t, st);
  }
}

template <int N, int V>
hipError_t col_v(const ColArgs<float>& a, int n, int batch, const c2<float>* t, const float* l,
                 hipStream_t st) {
  if constexpr (V >= COL_VARIANT_COUNT) {
    return hipErrorInvalidValue;
  } else {
    if (a.var != V) return col_v<N, V + 1>(a, n, batch, t, l, st);
    if constexpr (V == COL_REG_VARIANT) {
      if constexpr (N == 1024) return launch_col_reg<float, 32, CV<V>.nt / 64>(a, batch, t, l, st);
      else return hipErrorInvalidValue;
    } else {
      return launch_col_cfg<float, N, CV<V>.width, CV<V>.nt, CV<V>.maxr>(a, n, batch, t, l, st);
    }
  }
}

template <int N, int V>
hipError_t idst_v(const RowArgs<float>& a, int batch, const c2<float>* t, const float* ring,
                  int ring_rows, hipStream_t st) {
  if constexpr (V >= ROW_VARIANT_COUNT) {
    return hipErrorInvalidValue;
  } else {
    if (a.var != V) return idst_v<N, V + 1>(a, batch, t, ring, ring_rows, st);
    return launch_idst_cfg<float, N, RV<V>.width, RV<V>.nt, 1, RV<V>.maxr>(a, batch, t, ring,
                                                                          ring_rows, st);
  }
}

}  // namespace

#define IB_TUNED_N(n, MACRO)          \
  switch (n) {                        \
    case 256: return MACRO(256);      \
    case 384: return MACRO(384);      \
    case 512: return MACRO(512);      \
    case 768: return MACRO(768);      \
    case 1024: return MACRO(1024);    \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_rhs_rowdst_var(const RhsArgs<float>& a, const void* tw, hipStream_t st) {
  const c2<float>* t = static_cast<const c2<float>*>(tw);
#define M_(NN) rhs_v<NN, 1>(a, t, st)
  IB_TUNED_N(a.n, M_)
#undef M_
}

hipError_t launch_col_solve_var(const ColArgs<float>& a, int n, int batch, const void* tw,
                                const void* lam, hipStream_t st) {
  const c2<float>* t = static_cast<const c2<float>*>(tw);
  const float* l = static_cast<const float*>(lam);
#define M_(NN) col_v<NN, 1>(a, n, batch, t, l, st)
  IB_TUNED_N(n, M_)
#undef M_
}

hipError_t launch_row_idst_var(const RowArgs<float>& a, int n, int batch, const void* tw,
                               const float* ring, int ring_rows, hipStream_t st) {
  const c2<float>* t = static_cast<const c2<float>*>(tw);
#define M_(NN) idst_v<NN, 1>(a, batch, t, ring, ring_rows, st)
  IB_TUNED_N(n, M_)
#undef M_
}

}  // namespace ib
