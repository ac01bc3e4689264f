// Column solve with register-resident transforms (grid size n = P^2 cells, P = 32 or 16).
//
// The same operation as col_solve_body (ib_flow_kernels.hpp): for every column of the
// row-transformed array, the DST-I of length n - 1 down the column, the spectral divide
// scale / (lam (1 + alpha lam)) (and scale / (1 + alpha lam) for the circulation), the ring's
// split lift, and the inverse DST-I (Sec. 3.2.1, eqs. (30)-(31)).
//
// Each DST-I is one complex FFT of length n of the packed odd extension
// w_m = z_{2m} + i z_{2m+1} (as in ib_fft.hpp), computed here by the four-step split
// n = P x P with P lanes per column, all inside one wave:
//   lane t holds w_{t + P q}, q = 0 .. P-1, in registers and transforms over q (DFT-P);
//   multiplies by exp(-2 pi i t k2 / n);
//   one LDS transpose within the column's lanes;
//   lane k2 transforms over t (DFT-P) and then holds W_{k2 + P k1}, k1 = 0 .. P-1.
// The DST unpacking pairs W_k with W_{n-k}, held by lane (P - k2) mod P, through a lane
// shuffle; the spectrum is re-packed for the inverse through LDS.  Every exchange stays
// within the column's wave, so the only workgroup barrier follows the load of the twiddle
// and eigenvalue tables into LDS.  64 / P columns share a wave; WPB waves per workgroup.
#pragma once

#include "ib_flow_kernels.hpp"

namespace ib {

// In-order completion of this wave's LDS writes before its later LDS reads of other lanes'
// data (a wave's LDS instructions execute in order; the fences keep the compiler from
// moving the accesses across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place DFT of 32 values in natural order, X_k = sum_q v_q e^{-2 pi i q k / 32}: two
// DFT-16 over the even and odd entries, then the twiddles e^{-i pi k / 16}.
template <typename T>
__device__ __forceinline__ void dft32(c2<T>* v) {
  constexpr double C[16] = {1.0,
                            0.98078528040323044912618223613424,
                            0.92387953251128675612818318939679,
                            0.83146961230254523707878837761791,
                            0.70710678118654752440084436210485,
                            0.55557023301960222474283081394853,
                            0.38268343236508977172845998403040,
                            0.19509032201612826784828486847702,
                            0.0,
                            -0.19509032201612826784828486847702,
                            -0.38268343236508977172845998403040,
                            -0.55557023301960222474283081394853,
                            -0.70710678118654752440084436210485,
                            -0.83146961230254523707878837761791,
                            -0.92387953251128675612818318939679,
                            -0.98078528040323044912618223613424};
  c2<T> e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft_small<T, 16>(e);
  dft_small<T, 16>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    // e^{-i pi k / 16} = (cos, -sin), sin(pi k / 16) = cos(pi (8 - k) / 16)
    const T c = T(C[k]), sn = T(k <= 8 ? C[8 - k] : C[k - 8]);
    const c2<T> w = o[k];
    const c2<T> tw = c2<T>{w.x * c + w.y * sn, w.y * c - w.x * sn};
    v[k] = cadd(e[k], tw);
    v[k + 16] = csub(e[k], tw);
  }
}

template <typename T, int P>
__device__ __forceinline__ void dft_p(c2<T>* v) {
  if constexpr (P == 32) dft32<T>(v);
  else dft_small<T, P>(v);
}

template <typename T>
__device__ __forceinline__ c2<T> shfl_c2(c2<T> v, int src) {
  return c2<T>{__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// Forward complex FFT of length P^2 of one column's values, four-step as described at the
// top: on entry lane t holds v[q] = w_{t + P q}; on exit it holds v[k1] = W_{t + P k1}.
// buf: the column's LDS buffer (P rows of P + 1); stw: e^{-i pi m / n}, m < 2n, in LDS.
template <typename T, int P>
__device__ __forceinline__ void fft_reg(c2<T>* v, c2<T>* buf, const c2<T>* stw, int t) {
  constexpr int TP = P + 1;
  dft_p<T, P>(v);
#pragma unroll
  for (int k2 = 0; k2 < P; ++k2) {
    // e^{-2 pi i t k2 / n} = stw[2 t k2] (t k2 < n)
    v[k2] = cmul(v[k2], stw[2 * t * k2]);
    buf[k2 * TP + t] = v[k2];
  }
  wave_lds_sync();
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = buf[t * TP + s];
  wave_lds_sync();  // the buffer is written again only after every lane has read it
  dft_p<T, P>(v);
}

// DST-I outputs X_k, k = t + P k1, from W (lane t holds W_{t + P k1} in v[k1]); the partner
// W_{n-k} sits in lane (P - t) mod P at slot P - 1 - k1 (t > 0) or in lane 0 at slot
// (P - k1) mod P (t = 0).  grp0: the first lane of this column within the wave.
template <typename T, int P>
__device__ __forceinline__ void dst_unpack_reg(const c2<T>* v, const c2<T>* stw, int t, int grp0,
                                               T* x) {
  const int src = grp0 + ((P - t) & (P - 1));
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) {
    c2<T> b = shfl_c2(v[P - 1 - k1], src);
    if (t == 0) b = v[(P - k1) & (P - 1)];
    const c2<T> a = v[k1];
    const int k = t + P * k1;
    const T e_im = T(0.5) * (a.y - b.y);
    const c2<T> d = c2<T>{a.x - b.x, a.y + b.y};
    const c2<T> o = c2<T>{T(0.5) * d.y, -T(0.5) * d.x};
    const c2<T> p = cmul(stw[k], o);
    x[k1] = -T(0.5) * (e_im + p.y);
  }
}

template <typename T, int P, int WPB>
__device__ __forceinline__ void col_solve_reg_body(const ColArgs<T>& a, const c2<T>* __restrict__ tw,
                                                   const T* __restrict__ lam, int nblocks, int bx,
                                                   int by) {
  constexpr int N = P * P;
  constexpr int CPW = 64 / P;         // columns per wave
  constexpr int CW = CPW * WPB;       // columns per workgroup
  constexpr int NT = 64 * WPB;
  constexpr int TP = P + 1;
  __shared__ c2<T> stw[2 * N];        // e^{-i pi m / n}, m < 2n
  __shared__ T slam[N];               // lam_k at k - 1
  __shared__ c2<T> sbuf[CW * P * TP]; // per column: transpose and re-packing buffer
  static_assert(sizeof(stw) + sizeof(slam) + sizeof(sbuf) <= 160 * 1024, "LDS");
  static_assert(P * TP * 2 >= N + 1, "re-packing fits the transpose buffer");
  const int blk = xcd_block(bx, nblocks);
  if (blk < 0 || flow_gated(a.gate)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int grp = lane / P, t = lane % P, grp0 = grp * P;
  const int cl = wv * CPW + grp;
  const int col = blk * CW + cl;
  const bool live = col < N - 1;
  const int colc = live ? col : N - 2;  // loads of an idle column stay in bounds
  c2<T>* buf = sbuf + cl * P * TP;
  T* ybuf = reinterpret_cast<T*>(buf);
  const T* in = a.in + (size_t)by * a.bsi;
  const int rf = a.rfirst != nullptr ? a.rfirst[by] : 0;
  // ---- loads, all in flight together: the column's packed odd extension
  //   w_m = z_{2m} + i z_{2m+1}, m = t + P q; z_j = x_j (0 < j < n), 0 at 0 and n,
  //   -x_{2n-j} (n < j < 2n); x_j is row j of the input (0 outside the nonzero rows)
  T ld0[P], ld1[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int m = t + P * q;
    const bool lo = q < P / 2;
    const int j0 = lo ? 2 * m : 2 * N - 2 * m;
    const int j1 = lo ? 2 * m + 1 : 2 * N - 2 * m - 1;
    T r[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = u == 0 ? j0 : j1;
      bool ok = j >= 1 && j <= N - 1;
      long idx;
      if (a.rfirst != nullptr) {
        const int qq = j - rf;
        ok = ok && qq >= 0 && qq < a.rcount;
        idx = (long)qq * a.pi + colc;
      } else {
        ok = ok && j >= a.r0 && j <= a.r1;
        idx = (long)(j - 1) * a.pi + colc;
      }
      r[u] = ok ? in[idx] : T(0);
    }
    ld0[q] = r[0];
    ld1[q] = r[1];
  }
  {
    constexpr int PT = (2 * N + NT - 1) / NT, PL = (N + NT - 1) / NT;
    c2<T> tv[PT];
    T lv[PL];
#pragma unroll
    for (int b = 0; b < PT; ++b) tv[b] = tw[min(tid + b * NT, 2 * N - 1)];
#pragma unroll
    for (int b = 0; b < PL; ++b) lv[b] = tid + b * NT < N - 1 ? lam[tid + b * NT] : T(1);
#pragma unroll
    for (int b = 0; b < PT; ++b)
      if (tid + b * NT < 2 * N) stw[tid + b * NT] = tv[b];
#pragma unroll
    for (int b = 0; b < PL; ++b)
      if (tid + b * NT < N) slam[tid + b * NT] = lv[b];
  }
  __syncthreads();
  c2<T> v[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const T sg = q < P / 2 ? T(1) : T(-1);
    v[q] = c2<T>{sg * ld0[q], sg * ld1[q]};
  }
  fft_reg<T, P>(v, buf, stw, t);
  T x[P];
  dst_unpack_reg<T, P>(v, stw, t, grp0, x);
  // ---- spectral divide, split lift; the two spectra for s (ys) and gamma (yg)
  const T lk = slam[colc];
  const int kx = colc + 1;
  const T sk = -stw[kx].y;                      // sin(pi kx / n)
  const T pk = (kx & 1) ? T(1) : T(-1);         // (-1)^(kx+1)
  const bool lift = a.lift != nullptr;
  const T eb = lift ? a.lift[colc] : T(0);      // bottom and top edge transforms at kx
  const T et = lift ? a.lift[(N - 1) + colc] : T(0);
  T ys[P], yg[P];
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) {
    const int l = t + P * k1;
    const int lc = l > 0 ? l : 1;
    const T l1 = lk + slam[lc - 1];
    const T ga = x[k1] / (T(1) + a.alpha * l1);
    T fa = T(0);
    if (lift) {
      const T sl = -stw[lc].y;                  // sin(pi l / n)
      const T pl = (lc & 1) ? T(1) : T(-1);
      fa = eb * sl + et * sl * pl + sk * a.lift[2 * (N - 1) + lc - 1] +
           sk * pk * a.lift[3 * (N - 1) + lc - 1];
    }
    ys[k1] = l > 0 ? (ga + fa) * (a.scale / l1) : T(0);
    yg[k1] = l > 0 ? ga * a.scale : T(0);
  }
  // ---- inverse transforms, one per output
  const int nout = a.out2 != nullptr ? 2 : 1;
  for (int o = 0; o < nout; ++o) {
    T* dst = (o == 0 ? a.out : a.out2) + (size_t)by * a.bso;
    const T* y = o == 0 ? ys : yg;
    // previous values of an accumulated output, fetched while the transform runs
    T prev[P];
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      const int j = t + P * k1;
      const bool ok = a.accumulate && live && j >= 1 && j >= a.w0 && j <= a.w1;
      prev[k1] = ok ? dst[(size_t)(j - 1) * a.po + col] : T(0);
    }
    // re-pack: Y_l at ybuf[l] (Y_0 = Y_n = 0), then lane t reads the odd extension pairs
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) ybuf[t + P * k1] = y[k1];
    if (t == 0) ybuf[N] = T(0);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int m = t + P * q;
      const bool lo = q < P / 2;
      const int j0 = lo ? 2 * m : 2 * N - 2 * m;
      const int j1 = lo ? 2 * m + 1 : 2 * N - 2 * m - 1;
      const T sg = lo ? T(1) : T(-1);
      v[q] = c2<T>{sg * ybuf[j0], sg * ybuf[j1]};
    }
    wave_lds_sync();
    fft_reg<T, P>(v, buf, stw, t);
    T r[P];
    dst_unpack_reg<T, P>(v, stw, t, grp0, r);
    if (live) {
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) {
        const int j = t + P * k1;
        if (j >= 1 && j >= a.w0 && j <= a.w1) dst[(size_t)(j - 1) * a.po + col] = prev[k1] + r[k1];
      }
    }
  }
}

template <typename T, int P, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_col_solve_reg(ColArgs<T> a, const c2<T>* __restrict__ tw,
                                                            const T* __restrict__ lam, int nblocks) {
  col_solve_reg_body<T, P, WPB>(a, tw, lam, nblocks, blockIdx.x, blockIdx.y);
}

template <typename T, int P, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_col_solve_reg_multi(const ColArgs<T>* __restrict__ tab,
                                                                  const c2<T>* __restrict__ tw,
                                                                  const T* __restrict__ lam) {
  const ColArgs<T> a = tab[blockIdx.y];
  constexpr int nb = (P * P - 1 + (64 / P) * WPB - 1) / ((64 / P) * WPB);
  if ((int)blockIdx.x >= xcd_grid(nb)) return;
  col_solve_reg_body<T, P, WPB>(a, tw, lam, nb, blockIdx.x, 0);
}

template <typename T, int P, int WPB>
hipError_t launch_col_reg(const ColArgs<T>& a, int batch, const c2<T>* t, const T* l,
                          hipStream_t st) {
  constexpr int CW = (64 / P) * WPB;
  const int nb = (P * P - 1 + CW - 1) / CW;
  if (a.ev0)
    hipExtLaunchKernelGGL((k_col_solve_reg<T, P, WPB>), dim3(xcd_grid(nb), batch), dim3(64 * WPB), 0,
                          st, a.ev0, a.ev1, 0, a, t, l, nb);
  else
    hipLaunchKernelGGL((k_col_solve_reg<T, P, WPB>), dim3(xcd_grid(nb), batch), dim3(64 * WPB), 0,
                       st, a, t, l, nb);
  return hipGetLastError();
}

template <typename T, int P, int WPB>
hipError_t launch_col_reg_multi(const ColArgs<T>* tab, int count, const c2<T>* t, const T* l,
                                hipStream_t st) {
  constexpr int CW = (64 / P) * WPB;
  constexpr int nb = (P * P - 1 + CW - 1) / CW;
  hipLaunchKernelGGL((k_col_solve_reg_multi<T, P, WPB>), dim3(xcd_grid(nb), count), dim3(64 * WPB),
                     0, st, tab, t, l);
  return hipGetLastError();
}

}  // namespace ib
