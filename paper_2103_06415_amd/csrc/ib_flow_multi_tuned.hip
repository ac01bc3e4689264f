// The measured alternative configurations (ROW_VARIANTS, COL_VARIANTS) of the single-precision
// flow kernels for many instances of one grid size per launch.
#include "ib_flow_kernels.hpp"
#include "ib_flow_reg.hpp"

namespace ib {

namespace {

template <int V>
constexpr FlowVariant RV = ROW_VARIANTS[V];
template <int V>
constexpr FlowVariant CV = COL_VARIANTS[V];

template <int N, int V>
hipError_t rhs_mv(const RhsArgs<float>* tab, int count, int var, const c2<float>* t,
                  hipStream_t st) {
  if constexpr (V >= ROW_VARIANT_COUNT) {
    return hipErrorInvalidValue;
  } else {
    if (var != V) return rhs_mv<N, V + 1>(tab, count, var, t, st);
    return launch_rhs_multi_cfg<float, N, RV<V>.width, RV<V>.nt, 1, RV<V>.maxr>(tab, count, t, st);
  }
}

template <int N, int V>
hipError_t col_mv(const ColArgs<float>* tab, int count, int var, const c2<float>* t,
                  const float* l, hipStream_t st) {
  if constexpr (V >= COL_VARIANT_COUNT) {
    return hipErrorInvalidValue;
  } else {
    if (var != V) return col_mv<N, V + 1>(tab, count, var, t, l, st);
    if constexpr (V == COL_REG_VARIANT) {
      if constexpr (N == 1024) return launch_col_reg_multi<float, 32, CV<V>.nt / 64>(tab, count, t, l, st);
      else return hipErrorInvalidValue;
    } else {
      return launch_col_multi_cfg<float, N, CV<V>.width, CV<V>.nt, CV<V>.maxr>(tab, count, t, l, st);
    }
  }
}

template <int N, int V>
hipError_t idst_mv(const IdstJob<float>* tab, int count, int maxrows, int var,
                   const c2<float>* t, hipStream_t st) {
  if constexpr (V >= ROW_VARIANT_COUNT) {
    return hipErrorInvalidValue;
  } else {
    if (var != V) return idst_mv<N, V + 1>(tab, count, maxrows, var, t, st);
    return launch_idst_multi_cfg<float, N, RV<V>.width, RV<V>.nt, 1, RV<V>.maxr>(tab, count,
                                                                               maxrows, t, st);
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

hipError_t launch_rhs_rowdst_multi_var(const RhsArgs<float>* tab, int count, int n, int var,
                                       const void* tw, hipStream_t st) {
  const c2<float>* t = static_cast<const c2<float>*>(tw);
#define M_(NN) rhs_mv<NN, 1>(tab, count, var, t, st)
  IB_TUNED_N(n, M_)
#undef M_
}

hipError_t launch_col_solve_multi_var(const ColArgs<float>* tab, int count, int n, int var,
                                      const void* tw, const void* lam, hipStream_t st) {
  const c2<float>* t = static_cast<const c2<float>*>(tw);
  const float* l = static_cast<const float*>(lam);
#define M_(NN) col_mv<NN, 1>(tab, count, var, t, l, st)
  IB_TUNED_N(n, M_)
#undef M_
}

hipError_t launch_row_idst_multi_var(const IdstJob<float>* tab, int count, int n, int maxrows,
                                     int var, const void* tw, hipStream_t st) {
  const c2<float>* t = static_cast<const c2<float>*>(tw);
#define M_(NN) idst_mv<NN, 1>(tab, count, maxrows, var, t, st)
  IB_TUNED_N(n, M_)
#undef M_
}

}  // namespace ib
