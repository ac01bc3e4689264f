#pragma once
// Flow kernels of one level (templates; instantiated by ib_flow.hip and ib_flow_tuned.hip): explicit right-hand side fused with the row sine
// transform, the column transform + spectral solve, the inverse row transform, the
// nested-level boundary rings, and a plain row transform for sparse sources.
//
// Per level g the predictor solves (Sec. 2.3 eq. (16), Appendix A r^f)
//   (I + a L) L s_{n+1} = gamma_n - a L gamma_n + dt (3/2 C^T N_n - 1/2 C^T N_{n-1})
//                         + a B(gamma_ring_{n+1}) + (I + a L) B(s_ring_{n+1}),
// L = C^T C (5-point), a = dt / (2 Re h_g^2), B(.) = ring values adjacent to an
// interior vertex.  (I + a L) L is diagonal in the 2-D DST-I basis (Sec. 3.2.1), so
// the solve is row DST -> column DST, scale, inverse column DST -> inverse row DST.
// It is split into its two factors, both formed from one spectral right-hand side:
//   gamma_{n+1} = (I + a L)^{-1} [rhs without the s ring]           (gamma^ = r^/(1 + a lam))
//   s_{n+1}     = L^{-1} [gamma_{n+1} + B(s_ring_{n+1})]            (s^ = (gamma^ + B^)/lam)
// so the circulation state never passes through the large streamfunction values
// (differencing s would lose about log10((n/pi)^2) digits in single precision), and
// B(s_ring)^ is a sum of four outer products of 1-D edge transforms.
#include <hip/hip_ext.h>

#include "ib_internal.hpp"
#include "ib_fft.hpp"

namespace ib {

// Kernels after the FSI iterations of a step (corrector, final inverse transform) run
// only when those converged: gate[0] = 1 and gate[1] = 0 (null: always).
__device__ __forceinline__ bool flow_gated(const int* gate) {
  return gate != nullptr && (gate[0] != 1 || gate[1] != 0);
}

template <typename T>
__device__ __forceinline__ T ld(const T* p, int pitch, int j, int i) {
  return p[(size_t)j * pitch + i];
}

// Where the circulation seen by the stencil at vertex (i, j), 0 <= i, j <= n, lives:
// boundary ring, coarsification on read (the finer level's circulation at the
// coincident vertex, scaled by (h_coarse / h_fine)^2 = 4) or the level's own interior.
// Returned as pointer, index and scale (selects only), so that the caller can issue all
// of its loads before it uses any of them.
template <typename T>
__device__ __forceinline__ const T* gamma_src(const RhsArgs<T>& a, int i, int j, int& idx, T& sc) {
  const int nx = a.n, ny = a.ny > 0 ? a.ny : a.n;
  const T* p = a.g;
  idx = (j - 1) * a.pg + (i - 1);
  sc = T(1);
  if (a.gf != nullptr && i > nx / 4 && i < 3 * nx / 4 && j > ny / 4 && j < 3 * ny / 4) {
    p = a.gf;
    idx = (2 * j - ny / 2 - 1) * a.pgf + (2 * i - nx / 2 - 1);
    sc = T(4);
  }
  if (i == nx) { p = a.gring; idx = ring_off(RING_R, nx, ny) + j; sc = T(1); }
  if (i == 0) { p = a.gring; idx = ring_off(RING_L, nx, ny) + j; sc = T(1); }
  if (j == ny) { p = a.gring; idx = ring_off(RING_T, nx, ny) + i; sc = T(1); }
  if (j == 0) { p = a.gring; idx = ring_off(RING_B, nx, ny) + i; sc = T(1); }
  return p;
}

// Build the LDS twiddle table (layout TwLayout<N, MAXR>) from the global table
// exp(-i pi m / N), m < 2N; all loads of a thread in flight at once.
template <typename T, int N, int NT, int MAXR = 16>
__device__ __forceinline__ void load_table(c2<T>* stw, const c2<T>* __restrict__ tw, int tid) {
  constexpr int TOT = TwLayout<N, MAXR>::total;
  constexpr int PER = (TOT + NT - 1) / NT;
  c2<T> v[PER];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int e = min(tid + b * NT, TOT - 1);  // clamped: every lane loads, no branch
    v[b] = tw[e < TwLayout<N, MAXR>::U ? e : tw_source<N, MAXR>(e)];
  }
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int e = tid + b * NT;
    if (e < TOT) stw[e] = v[b];
  }
}

// Sum of the new boundary-ring values adjacent to interior vertex (i, j).
template <typename T>
__device__ __forceinline__ T ring_adj(const T* ring, int n, int i, int j) {
  T v = T(0);
  if (i == 1) v += ring[RING_L * (n + 1) + j];
  if (i == n - 1) v += ring[RING_R * (n + 1) + j];
  if (j == 1) v += ring[RING_B * (n + 1) + i];
  if (j == n - 1) v += ring[RING_T * (n + 1) + i];
  return v;
}

// Right-hand side at interior vertex (i, j) from staged rows: ss / sg hold s and gamma
// of rows j-1, j, j+1 (each W wide, column index = i); hprev_in is C^T N_{n-1} (unused
// on the first step, which takes the new value); ring_term the adjacent new ring
// circulation; writes C^T N_n to the history.
template <typename T, int W>
__device__ __forceinline__ T rhs_staged(const RhsArgs<T>& a, const T* ss, const T* sg, int i, int j,
                                        T hprev_in, bool has_prev, T ring_term) {
  const T* sm = ss;          // row j-1
  const T* sp = ss + 2 * W;  // row j+1
  const T* gm = sg;
  const T* g0r = sg + W;
  const T* gp = sg + 2 * W;
  const T g0 = g0r[i];
  const T gE = g0r[i + 1], gW = g0r[i - 1];
  const T gN = gp[i], gS = gm[i];
  // vertex-averaged fluxes (total flux, free stream included)
  const T uE = T(0.5) * (sp[i + 1] - sm[i + 1]) + a.ux;
  const T uW = T(0.5) * (sp[i - 1] - sm[i - 1]) + a.ux;
  const T vN = T(0.5) * (sp[i - 1] - sp[i + 1]) + a.uy;
  const T vS = T(0.5) * (sm[i - 1] - sm[i + 1]) + a.uy;
  // C^T N with N = (vbar gamma, -ubar gamma) / h^2 averaged onto the faces
  const T ctn = a.cn * ((uE * gE - uW * gW) + (vN * gN - vS * gS));
  a.hist_out[(size_t)(j - 1) * a.ph + (i - 1)] = ctn;
  const T hprev = has_prev ? hprev_in : ctn;
  const T lap = T(4) * g0 - gE - gW - gN - gS;
  return g0 - a.alpha * lap + a.dt * (T(1.5) * ctn - T(0.5) * hprev) + a.alpha * ring_term;
}

// Explicit right-hand side of ROWS interior rows fused with their row DST.  The rows
// j-1 .. j+ROWS of s and gamma are staged in LDS (every load of a thread in flight at
// once); the staging area is then reused as the transform buffer.
template <typename T, int N, int ROWS, int NT, int DST, int MAXR>
__device__ __forceinline__ void rhs_rowdst_body(const RhsArgs<T>& a, const c2<T>* __restrict__ tw,
                                                int nblocks, int bx) {
  constexpr int W = N + 1;           // staged row width, ring columns included
  constexpr int SR = ROWS + 2;       // staged rows j0-1 .. j0+ROWS
  constexpr int STG = 2 * SR * W;    // s and gamma, in T units
  constexpr int BUFT = 2 * ROWS * fft_pad_len<N>(); // transform buffer, in T units
  constexpr int UNI = (STG > BUFT ? STG : BUFT) / 2 + 1;
  __shared__ c2<T> uni[UNI];
  __shared__ c2<T> stw[TwLayout<N, MAXR>::total];
  // new circulation ring: the bottom and top rows (staged below length 2000; above, the first
  // and last row blocks read them from memory) and the left and right entries at this block's
  // rows
  constexpr bool STAGE_BT = N < 2000;
  __shared__ T sbt[2][STAGE_BT ? W : 1];
  __shared__ T slr[2][ROWS];
  static_assert(sizeof(uni) + sizeof(stw) + sizeof(sbt) + sizeof(slr) <= 160 * 1024, "LDS");
  const int blk = xcd_block(bx, nblocks);
  if (blk < 0) return;
  const int tid = threadIdx.x;
  const int ny = a.ny > 0 ? a.ny : N;  // rows of the level (the row length is N)
  const int j0 = 1 + blk * ROWS;
  T* ss = reinterpret_cast<T*>(uni);
  T* sg = ss + SR * W;
  constexpr int NPT = ROWS * (N - 1);
  constexpr int PP = (NPT + NT - 1) / NT;
  T hp[PP];
  {
    // every load of this thread is issued before any is used; indices are clamped to
    // valid memory and the unused values are dropped afterwards
    constexpr int CNT = SR * W;
    constexpr int PER = (CNT + NT - 1) / NT;
    T vs[PER], vg[PER], gsc[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      const int r = e / W, i = e % W;
      const int j = min(j0 - 1 + r, ny);
      int gi;
      const T* gp = gamma_src(a, i, j, gi, gsc[b]);
      vs[b] = a.s[j * a.ps + i];  // indices fit in 32 bits (n <= 1024)
      vg[b] = gp[gi];
    }
#pragma unroll
    for (int b = 0; b < PP; ++b) {
      const int e = tid + b * NT;
      const int t = e / (N - 1), i = 1 + e % (N - 1), j = min(j0 + t, ny - 1);
      hp[b] = a.hist_in != nullptr ? a.hist_in[(j - 1) * a.ph + (i - 1)] : T(0);
    }
    // the ring entries this block uses: the bottom and top rows, the left and right entries
    // of rows j0 .. j0 + ROWS - 1 (clamped to the ring)
    constexpr int BW = STAGE_BT ? 2 * W : 0;
    constexpr int RC = BW + 2 * ROWS;
    constexpr int PR = (RC + NT - 1) / NT;
    T rv0[PR];
    if (a.gring_new != nullptr) {
#pragma unroll
      for (int b = 0; b < PR; ++b) {
        const int e = min(tid + b * NT, RC - 1);
        const int idx = e < BW ? ring_off(e / W, N, ny) + e % W
                               : ring_off(RING_L + (e - BW) / ROWS, N, ny) +
                                     min(j0 + (e - BW) % ROWS, ny);
        rv0[b] = a.gring_new[idx];
      }
    }
    load_table<T, N, NT, MAXR>(stw, tw, tid);
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e < CNT) {
        const bool ok = j0 - 1 + e / W <= ny;
        ss[e] = ok ? vs[b] : T(0);
        sg[e] = ok ? gsc[b] * vg[b] : T(0);
      }
    }
    if (a.gring_new != nullptr) {
#pragma unroll
      for (int b = 0; b < PR; ++b) {
        const int e = tid + b * NT;
        if (e < BW) (&sbt[0][0])[e] = rv0[b];
        else if (e < RC) (&slr[0][0])[e - BW] = rv0[b];
      }
    }
  }
  __syncthreads();
  T rv[PP];
#pragma unroll
  for (int b = 0; b < PP; ++b) {
    const int e = tid + b * NT;
    const int t = e / (N - 1), i = 1 + e % (N - 1), j = j0 + t;
    rv[b] = T(0);
    if (e < NPT && j <= ny - 1) {
      T ring = T(0);
      if (a.gring_new != nullptr) {
        if (i == 1) ring += slr[0][t];
        if (i == N - 1) ring += slr[1][t];
        if constexpr (STAGE_BT) {
          if (j == 1) ring += sbt[RING_B][i];
          if (j == ny - 1) ring += sbt[RING_T][i];
        } else {
          if (j == 1) ring += a.gring_new[ring_off(RING_B, N, ny) + i];
          if (j == ny - 1) ring += a.gring_new[ring_off(RING_T, N, ny) + i];
        }
      }
      rv[b] = rhs_staged<T, W>(a, ss + t * W, sg + t * W, i, j, hp[b], a.hist_in != nullptr, ring);
    }
  }
  if constexpr (DST == 0) {
    // right-hand side only (the transforms run elsewhere)
#pragma unroll
    for (int b = 0; b < PP; ++b) {
      const int e = tid + b * NT;
      const int j = j0 + e / (N - 1);
      if (e < NPT && j <= ny - 1) a.out[(size_t)(j - 1) * a.po + e % (N - 1)] = rv[b];
    }
    return;
  }
  __syncthreads();  // the staging area becomes the transform buffer
  c2<T>* buf = uni;
#pragma unroll
  for (int b = 0; b < PP; ++b) {
    const int e = tid + b * NT;
    if (e < NPT) dst_pack<T, N>(buf + (e / (N - 1)) * fft_pad_len<N>(), 1 + e % (N - 1), rv[b]);
  }
  for (int t = tid; t < ROWS; t += NT) dst_pack_zeros<T, N>(buf + t * fft_pad_len<N>());
  __syncthreads();
  fft_lds<T, N, ROWS, NT, MAXR>(buf, stw, tid);
  for (int e = tid; e < ROWS * (N / 2); e += NT) {
    const int t = e / (N / 2), k = 1 + e % (N / 2);
    const int j = j0 + t;
    if (j > ny - 1) continue;
    T xk, xnk;
    dst_unpack<T, N>(buf + t * fft_pad_len<N>(), stw, k, xk, xnk);
    T* o = a.out + (size_t)(j - 1) * a.po;
    o[k - 1] = xk;
    if (k != N / 2) o[N - k - 1] = xnk;
  }
}

template <typename T, int N, int ROWS, int NT, int DST, int MAXR = 16>
__global__ __launch_bounds__(NT) void k_rhs_rowdst(RhsArgs<T> a, const c2<T>* __restrict__ tw,
                                                   int nblocks) {
  rhs_rowdst_body<T, N, ROWS, NT, DST, MAXR>(a, tw, nblocks, blockIdx.x);
}

// Many instances of one grid size in one launch: instance blockIdx.y takes its arguments
// from tab[blockIdx.y]; workgroups beyond its own row blocks leave at once.
template <typename T, int N, int ROWS, int NT, int DST, int MAXR = 16>
__global__ __launch_bounds__(NT) void k_rhs_rowdst_multi(const RhsArgs<T>* __restrict__ tab,
                                                         const c2<T>* __restrict__ tw) {
  const RhsArgs<T> a = tab[blockIdx.y];
  const int nb = ((a.ny > 0 ? a.ny : a.n) - 1 + ROWS - 1) / ROWS;
  if ((int)blockIdx.x >= xcd_grid(nb)) return;
  rhs_rowdst_body<T, N, ROWS, NT, DST, MAXR>(a, tw, nb, blockIdx.x);
}

// Plain row DST of rows [r0, r1] (1-based interior rows) of a real array; batched
// over `by` (blockIdx.y) with the given strides.
template <typename T, int N, int ROWS, int NT>
__device__ __forceinline__ void rowdst_body(const RowArgs<T>& a, const c2<T>* __restrict__ tw,
                                            int nblocks, int bx, int by) {
  __shared__ c2<T> buf[ROWS * fft_pad_len<N>()];
  __shared__ c2<T> stw[TwLayout<N>::total];
  const int blk = xcd_block(bx, nblocks);
  if (blk < 0 || flow_gated(a.gate)) return;
  const int tid = threadIdx.x;
  const T* in = a.in + (size_t)by * a.bsi;
  T* out = a.out + (size_t)by * a.bso;
  const int j0 = a.r0 + blk * ROWS;
  {
    constexpr int CNT = ROWS * (N - 1);
    constexpr int PER = (CNT + NT - 1) / NT;
    T v[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      const int t = e / (N - 1), i = 1 + e % (N - 1), j = j0 + t;
      v[b] = (e < CNT && j <= a.r1) ? in[(size_t)(j - 1) * a.pi + (i - 1)] : T(0);
    }
    load_table<T, N, NT>(stw, tw, tid);
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e < CNT) dst_pack<T, N>(buf + (e / (N - 1)) * fft_pad_len<N>(), 1 + e % (N - 1), v[b]);
    }
  }
  for (int t = tid; t < ROWS; t += NT) dst_pack_zeros<T, N>(buf + t * fft_pad_len<N>());
  __syncthreads();
  fft_lds<T, N, ROWS, NT>(buf, stw, tid);
  for (int e = tid; e < ROWS * (N / 2); e += NT) {
    const int t = e / (N / 2), k = 1 + e % (N / 2);
    const int j = j0 + t;
    if (j > a.r1) continue;
    T xk, xnk;
    dst_unpack<T, N>(buf + t * fft_pad_len<N>(), stw, k, xk, xnk);
    T* o = out + (size_t)(j - 1) * a.po;
    o[k - 1] = xk;
    if (k != N / 2) o[N - k - 1] = xnk;
  }
}

template <typename T, int N, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_rowdst(RowArgs<T> a, const c2<T>* __restrict__ tw,
                                               int nblocks) {
  rowdst_body<T, N, ROWS, NT>(a, tw, nblocks, blockIdx.x, blockIdx.y);
}

template <typename T, int N, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_rowdst_multi(const RowArgs<T>* __restrict__ tab,
                                                     const c2<T>* __restrict__ tw) {
  const RowArgs<T> a = tab[blockIdx.y];
  const int nb = (a.r1 - a.r0 + 1 + ROWS - 1) / ROWS;
  if (nb <= 0 || (int)blockIdx.x >= xcd_grid(nb)) return;
  rowdst_body<T, N, ROWS, NT>(a, tw, nb, blockIdx.x, 0);
}

// Column DST, spectral scale scale / (lam (1 + alpha lam)), inverse column DST.
// Reads input rows [r0, r1] (others are zero) and writes
//   out = (accumulate ? out : 0) + result
// for every row; input and output may alias when accumulate == 0.
// 1 / x: the hardware reciprocal in single precision (within 1 ulp), a division in double.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename T, int N, int CW, int NT, int MAXR>
__device__ __forceinline__ void col_solve_body(const ColArgs<T>& a, const c2<T>* __restrict__ tw,
                                               const T* __restrict__ lam, int nblocks, int bx,
                                               int by) {
  // With room for 2 CW transforms, the two inverse column transforms (s and gamma) run as one
  // pass over 2 CW sequences: half the dependent stages, twice the butterflies per stage.
  constexpr size_t REST = sizeof(c2<T>) * TwLayout<N, MAXR>::total + sizeof(T) * (3 * N + 2 * CW);
  constexpr bool MERGE = REST + sizeof(c2<T>) * 2 * CW * fft_pad_len<N>() <= 160 * 1024;
  __shared__ c2<T> buf[(MERGE ? 2 : 1) * CW * fft_pad_len<N>()];
  __shared__ c2<T> stw[TwLayout<N, MAXR>::total];
  __shared__ T slam[N];
  __shared__ T slift[2 * N];    // edge transforms of the left and right ring columns
  __shared__ T slift01[2 * CW]; // bottom and top edge transforms at this block's columns
  static_assert(sizeof(buf) + sizeof(stw) + sizeof(slam) + sizeof(slift) + sizeof(slift01) <=
                    160 * 1024, "LDS");
  const int blk = xcd_block(bx, nblocks);
  if (blk < 0 || flow_gated(a.gate)) return;
  const int tid = threadIdx.x;
  const int k0 = blk * CW;
  const int nc = a.ncols > 0 ? a.ncols : N - 1;  // columns (x); the transform runs along y (N)
  const T* in = a.in + (size_t)by * a.bsi;
  {
    constexpr int CNT = (N - 1) * CW;
    constexpr int PER = (CNT + NT - 1) / NT;
    T v[PER];
    const int rf = a.rfirst != nullptr ? a.rfirst[by] : 0;
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      const int r = e / CW, col = k0 + e % CW;
      bool ok = e < CNT && col < nc;
      long idx;
      if (a.rfirst != nullptr) {
        const int q = r + 1 - rf;
        ok = ok && q >= 0 && q < a.rcount;
        idx = (long)q * a.pi + col;
      } else {
        ok = ok && r + 1 >= a.r0 && r + 1 <= a.r1;
        idx = (long)r * a.pi + col;
      }
      v[b] = ok ? in[idx] : T(0);
    }
    load_table<T, N, NT, MAXR>(stw, tw, tid);
    constexpr int PL = (N - 1 + NT - 1) / NT;
    T lv[PL];
#pragma unroll
    for (int b = 0; b < PL; ++b) lv[b] = tid + b * NT < N - 1 ? lam[tid + b * NT] : T(1);
    constexpr int PF = (2 * (N - 1) + NT - 1) / NT;
    T fv[PF];
    T f01 = T(0);
    if (a.lift != nullptr) {
#pragma unroll
      for (int b = 0; b < PF; ++b) {
        const int e = tid + b * NT;
        fv[b] = e < 2 * (N - 1) ? a.lift[2 * nc + e] : T(0);
      }
      if (tid < 2 * CW) {
        const int col = k0 + tid % CW;
        f01 = col < nc ? a.lift[(tid / CW) * nc + col] : T(0);
      }
    }
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e < CNT) dst_pack<T, N>(buf + (e % CW) * fft_pad_len<N>(), e / CW + 1, v[b]);
    }
#pragma unroll
    for (int b = 0; b < PL; ++b)
      if (tid + b * NT < N) slam[tid + b * NT] = lv[b];
    if (a.lift != nullptr) {
#pragma unroll
      for (int b = 0; b < PF; ++b)
        if (tid + b * NT < 2 * (N - 1)) slift[tid + b * NT] = fv[b];
      if (tid < 2 * CW) slift01[tid] = f01;
    }
  }
  for (int c = tid; c < CW; c += NT) dst_pack_zeros<T, N>(buf + c * fft_pad_len<N>());
  __syncthreads();
  fft_lds<T, N, CW, NT, MAXR>(buf, stw, tid);
  constexpr int NP = CW * (N / 2);
  constexpr int PER = (NP + NT - 1) / NT;
  T xa[PER], xb[PER];   // forward column transform, raw
  T la[PER], lb[PER];   // lam of each pair
  T ea[PER], eb[PER];   // 1 + alpha lam
  T fa[PER], fb[PER];   // spectral B(s_ring) of each pair
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int e = tid + b * NT;
    if (e < NP) {
      const int c = e % CW, l = 1 + e / CW;
      const int col = k0 + c;
      dst_unpack<T, N>(buf + c * fft_pad_len<N>(), stw, l, xa[b], xb[b]);
      const T lk = (col < nc) ? (a.lamx != nullptr ? a.lamx[col] : slam[col]) : T(1);
      const T l1 = lk + slam[l - 1];
      const T l2 = lk + slam[N - l - 1];
      la[b] = l1;
      lb[b] = l2;
      ea[b] = T(1) + a.alpha * l1;
      eb[b] = T(1) + a.alpha * l2;
      fa[b] = T(0);
      fb[b] = T(0);
      if (a.lift != nullptr && col < nc) {
        // sum_{i,j} B(s_ring)_{ij} sin(pi i k / nx) sin(pi j l / ny) over the four edges
        const int k = col + 1;
        const T sk = a.sinx != nullptr ? a.sinx[k] : tw_sin<T, N>(stw, k);  // sin(pi k / nx)
        const T sl = tw_sin<T, N>(stw, l);                                  // sin(pi l / ny)
        const T pk = (k & 1) ? T(1) : T(-1);     // (-1)^(k+1)
        const T pl = (l & 1) ? T(1) : T(-1);     // (-1)^(l+1) = (-1)^(n-l+1)
        const T eb_k = slift01[c], et_k = slift01[CW + c];
        fa[b] = eb_k * sl + et_k * sl * pl + sk * slift[l - 1] + sk * pk * slift[(N - 1) + l - 1];
        fb[b] = eb_k * sl + et_k * sl * pl + sk * slift[N - l - 1] +
                sk * pk * slift[(N - 1) + N - l - 1];
      }
    }
  }
  const int nout = a.out2 != nullptr ? 2 : 1;
  if constexpr (MERGE) {
    if (nout == 2) {
      T* dsts[2] = {a.out + (size_t)by * a.bso, a.out2 + (size_t)by * a.bso};
      // previous values of the accumulated outputs, fetched while the transform runs
      T pa[2][PER], pb[2][PER];
#pragma unroll
      for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int b = 0; b < PER; ++b) {
          const int e = tid + b * NT;
          const int c = e % CW, j = 1 + e / CW, col = k0 + c, j2 = N - j;
          const bool ok = a.accumulate && e < NP && col < nc;
          pa[o][b] = (ok && j >= a.w0 && j <= a.w1) ? dsts[o][(size_t)(j - 1) * a.po + col] : T(0);
          pb[o][b] = (ok && j != N / 2 && j2 >= a.w0 && j2 <= a.w1)
                         ? dsts[o][(size_t)(j2 - 1) * a.po + col]
                         : T(0);
        }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < PER; ++b) {
        const int e = tid + b * NT;
        if (e < NP) {
          const int c = e % CW, l = 1 + e / CW;
          // s = (g + f) scale / L and gamma = g scale with g = x / (1 + alpha L), from one
          // reciprocal of L (1 + alpha L) per mode (single precision: the hardware reciprocal)
          const T sa = a.scale * recip(ea[b] * la[b]), sb = a.scale * recip(eb[b] * lb[b]);
          c2<T>* w0 = buf + c * fft_pad_len<N>();
          c2<T>* w1 = buf + (CW + c) * fft_pad_len<N>();
          dst_pack<T, N>(w0, l, (xa[b] + fa[b] * ea[b]) * sa);
          dst_pack<T, N>(w1, l, xa[b] * la[b] * sa);
          if (l != N / 2) {
            dst_pack<T, N>(w0, N - l, (xb[b] + fb[b] * eb[b]) * sb);
            dst_pack<T, N>(w1, N - l, xb[b] * lb[b] * sb);
          }
        }
      }
      for (int c = tid; c < 2 * CW; c += NT) dst_pack_zeros<T, N>(buf + c * fft_pad_len<N>());
      __syncthreads();
      fft_lds<T, N, 2 * CW, NT, MAXR>(buf, stw, tid);
#pragma unroll
      for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int b = 0; b < PER; ++b) {
          const int e = tid + b * NT;
          if (e >= NP) continue;
          const int c = e % CW, j = 1 + e / CW;
          const int col = k0 + c;
          if (col >= nc) continue;
          T yk, ynk;
          dst_unpack<T, N>(buf + (o * CW + c) * fft_pad_len<N>(), stw, j, yk, ynk);
          if (j >= a.w0 && j <= a.w1) dsts[o][(size_t)(j - 1) * a.po + col] = pa[o][b] + yk;
          const int j2 = N - j;
          if (j != N / 2 && j2 >= a.w0 && j2 <= a.w1)
            dsts[o][(size_t)(j2 - 1) * a.po + col] = pb[o][b] + ynk;
        }
      return;
    }
  }
  for (int o = 0; o < nout; ++o) {
    T* dst = (o == 0 ? a.out : a.out2) + (size_t)by * a.bso;
    // previous values of the accumulated outputs, fetched while the transform runs
    T pa[PER], pb[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      const int c = e % CW, j = 1 + e / CW, col = k0 + c, j2 = N - j;
      const bool ok = a.accumulate && e < NP && col < nc;
      pa[b] = (ok && j >= a.w0 && j <= a.w1) ? dst[(size_t)(j - 1) * a.po + col] : T(0);
      pb[b] = (ok && j != N / 2 && j2 >= a.w0 && j2 <= a.w1) ? dst[(size_t)(j2 - 1) * a.po + col]
                                                              : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e < NP) {
        const int c = e % CW, l = 1 + e / CW;
        const T ga = xa[b] / ea[b], gb = xb[b] / eb[b];
        const T va = o == 0 ? (ga + fa[b]) * (a.scale / la[b]) : ga * a.scale;
        const T vb = o == 0 ? (gb + fb[b]) * (a.scale / lb[b]) : gb * a.scale;
        dst_pack<T, N>(buf + c * fft_pad_len<N>(), l, va);
        if (l != N / 2) dst_pack<T, N>(buf + c * fft_pad_len<N>(), N - l, vb);
      }
    }
    for (int c = tid; c < CW; c += NT) dst_pack_zeros<T, N>(buf + c * fft_pad_len<N>());
    __syncthreads();
    fft_lds<T, N, CW, NT, MAXR>(buf, stw, tid);
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e >= NP) continue;
      const int c = e % CW, j = 1 + e / CW;
      const int col = k0 + c;
      if (col >= nc) continue;
      T yk, ynk;
      dst_unpack<T, N>(buf + c * fft_pad_len<N>(), stw, j, yk, ynk);
      if (j >= a.w0 && j <= a.w1) dst[(size_t)(j - 1) * a.po + col] = pa[b] + yk;
      const int j2 = N - j;
      if (j != N / 2 && j2 >= a.w0 && j2 <= a.w1) dst[(size_t)(j2 - 1) * a.po + col] = pb[b] + ynk;
    }
  }
}

template <typename T, int N, int CW, int NT, int MAXR = 16>
__global__ __launch_bounds__(NT) void k_col_solve(ColArgs<T> a, const c2<T>* __restrict__ tw,
                                                  const T* __restrict__ lam, int nblocks) {
  col_solve_body<T, N, CW, NT, MAXR>(a, tw, lam, nblocks, blockIdx.x, blockIdx.y);
}

template <typename T, int N, int CW, int NT, int MAXR = 16>
__global__ __launch_bounds__(NT) void k_col_solve_multi(const ColArgs<T>* __restrict__ tab,
                                                        const c2<T>* __restrict__ tw,
                                                        const T* __restrict__ lam) {
  const ColArgs<T> a = tab[blockIdx.y];
  constexpr int nb = (N - 1 + CW - 1) / CW;
  if ((int)blockIdx.x >= xcd_grid(nb)) return;
  col_solve_body<T, N, CW, NT, MAXR>(a, tw, lam, nb, blockIdx.x, 0);
}

// Inverse row DST of rows [r0, r1] into the interior of a full (ny+1)-row array (rows of N+1
// entries, ny = a.ny or N); the ring columns (and, when ring rows are requested, rows 0 and
// ny) come from `ring` (zero when null).  With interior_out the output is an (n-1)-row interior array.
// With in2/out2 set the same rows of a second array are transformed in the same
// workgroup into the interior array out2 (the level's circulation).
template <typename T, int N, int ROWS, int NT, int DUAL, int MAXR>
__device__ __forceinline__ void row_idst_body(const RowArgs<T>& a, const c2<T>* __restrict__ tw,
                                              const T* __restrict__ ring, int ring_rows,
                                              int nblocks, int bx, int by) {
  constexpr int NS = ROWS * (DUAL ? 2 : 1);
  __shared__ c2<T> buf[NS * fft_pad_len<N>()];
  __shared__ c2<T> stw[TwLayout<N, MAXR>::total];
  static_assert(sizeof(buf) + sizeof(stw) <= 160 * 1024, "LDS");
  if (a.reset != nullptr && bx == 0 && by == 0 && (int)threadIdx.x < a.nreset)
    a.reset[threadIdx.x] = 0;
  const int blk = xcd_block(bx, nblocks);
  if (blk < 0 || flow_gated(a.gate)) return;
  const int tid = threadIdx.x;
  const T* in = a.in + (size_t)by * a.bsi;
  T* out = a.out + (size_t)by * a.bso;
  const int j0 = a.r0 + blk * ROWS;
  {
    constexpr int CNT = NS * (N - 1);
    constexpr int PER = (CNT + NT - 1) / NT;
    T v[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      const int t = e / (N - 1), k = 1 + e % (N - 1), j = j0 + (t % ROWS);
      const T* src = t < ROWS ? in : a.in2;
      v[b] = (e < CNT && j <= a.r1) ? src[(size_t)(j - 1) * a.pi + (k - 1)] : T(0);
    }
    load_table<T, N, NT, MAXR>(stw, tw, tid);
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e < CNT) dst_pack<T, N>(buf + (e / (N - 1)) * fft_pad_len<N>(), 1 + e % (N - 1), v[b]);
    }
  }
  static_assert(ROWS <= NT, "one thread per ring row");
  // the ring values this workgroup writes last are read now: a load issued after the output
  // stores would wait for their acknowledgement too
  const int ny = a.ny > 0 ? a.ny : N;
  constexpr int RB = (N + 1 + NT - 1) / NT;
  T rlv = T(0), rrv = T(0), rbv[RB], rtv[RB];
  if (!a.interior_out && ring != nullptr) {
    if (tid < ROWS && j0 + tid <= a.r1) {
      rlv = ring[ring_off(RING_L, N, ny) + j0 + tid];
      rrv = ring[ring_off(RING_R, N, ny) + j0 + tid];
    }
    if (ring_rows && blk == 0) {
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int i = tid + q * NT;
        rbv[q] = i <= N ? ring[ring_off(RING_B, N, ny) + i] : T(0);
        rtv[q] = i <= N ? ring[ring_off(RING_T, N, ny) + i] : T(0);
      }
    }
  }
  for (int t = tid; t < NS; t += NT) dst_pack_zeros<T, N>(buf + t * fft_pad_len<N>());
  __syncthreads();
  fft_lds<T, N, NS, NT, MAXR>(buf, stw, tid);
  for (int e = tid; e < NS * (N / 2); e += NT) {
    const int t = e / (N / 2), k = 1 + e % (N / 2);
    const int j = j0 + (t % ROWS);
    if (j > a.r1) continue;
    T xk, xnk;
    dst_unpack<T, N>(buf + t * fft_pad_len<N>(), stw, k, xk, xnk);
    if (t >= ROWS) {
      T* o = a.out2 + (size_t)(j - 1) * a.po;
      o[k - 1] = xk;
      if (k != N / 2) o[N - k - 1] = xnk;
    } else if (a.interior_out) {
      T* o = out + (size_t)(j - 1) * a.po;
      o[k - 1] = xk;
      if (k != N / 2) o[N - k - 1] = xnk;
    } else {
      T* o = out + (size_t)j * a.po;
      o[k] = xk;
      if (k != N / 2) o[N - k] = xnk;
    }
  }
  if (a.interior_out) return;
  if (tid < ROWS && j0 + tid <= a.r1) {
    T* o = out + (size_t)(j0 + tid) * a.po;
    o[0] = rlv;
    o[N] = rrv;
  }
  if (ring_rows && blk == 0) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int i = tid + q * NT;
      if (i > N) continue;
      out[i] = ring != nullptr ? rbv[q] : T(0);
      out[(size_t)ny * a.po + i] = ring != nullptr ? rtv[q] : T(0);
    }
  }
}

template <typename T, int N, int ROWS, int NT, int DUAL, int MAXR = 16>
__global__ __launch_bounds__(NT) void k_row_idst(RowArgs<T> a, const c2<T>* __restrict__ tw,
                                                 const T* __restrict__ ring, int ring_rows,
                                                 int nblocks) {
  row_idst_body<T, N, ROWS, NT, DUAL, MAXR>(a, tw, ring, ring_rows, nblocks, blockIdx.x,
                                            blockIdx.y);
}

template <typename T, int N, int ROWS, int NT, int DUAL, int MAXR = 16>
__global__ __launch_bounds__(NT) void k_row_idst_multi(const IdstJob<T>* __restrict__ tab,
                                                       const c2<T>* __restrict__ tw) {
  const IdstJob<T> j = tab[blockIdx.y];
  const int nb = (j.a.r1 - j.a.r0 + 1 + ROWS - 1) / ROWS;
  if (nb <= 0 || (int)blockIdx.x >= xcd_grid(nb)) return;
  row_idst_body<T, N, ROWS, NT, DUAL, MAXR>(j.a, tw, j.ring, j.ring_rows, nb, blockIdx.x, 0);
}

// New boundary rings of a fine level from the next coarser level's new state: coincident
// vertices are copied, midpoints use the cubic (-1, 9, 9, -1)/16 along the edge.  The
// streamfunction ring interpolates the coarse s; the circulation ring interpolates the
// coarse level's circulation C^T C s, read from its carried state gc (interior vertex
// (i, j) at gc[(j - 1) pgc + i - 1]; the ring only reads coarse vertices n/4 - 1 .. 3n/4 + 1,
// all interior), scaled by 1/4 (gamma = h^2 omega and h halves).  Reading the carried
// circulation instead of differencing s keeps the ring at the circulation's own relative
// rounding (differencing amplifies the rounding of s by up to (n/pi)^2 / 2).
template <typename T>
__device__ __forceinline__ T coarse_s(const T* sc, int p, int edge, int line, int I) {
  const int j = (edge < 2) ? line : I;
  const int i = (edge < 2) ? I : line;
  return sc[(size_t)j * p + i];
}

template <typename T>
__device__ __forceinline__ T coarse_g(const T* gc, int p, int edge, int line, int I) {
  const int j = (edge < 2) ? line : I;
  const int i = (edge < 2) ? I : line;
  return gc[(size_t)(j - 1) * p + (i - 1)];
}

// Entry idx of ring edge `edge` of an nx x ny level: along the bottom and top edges the fine i
// sits at coarse (i + nx/2) / 2 on the coarse rows ny/4 and 3 ny/4; along the left and right
// edges the fine j sits at (j + ny/2) / 2 on the coarse columns nx/4 and 3 nx/4.
template <typename T>
__device__ __forceinline__ void ring_values(const T* __restrict__ sc, int psc,
                                            const T* __restrict__ gc, int pgc, int nx, int ny,
                                            int edge, int idx, T& sv, T& gv) {
  const int q = edge < 2 ? nx / 2 : ny / 2;
  const int line = edge == RING_B ? ny / 4 : edge == RING_T ? (3 * ny) / 4
                 : edge == RING_L ? nx / 4 : (3 * nx) / 4;
  if (((idx + q) & 1) == 0) {
    const int I = (idx + q) / 2;
    sv = coarse_s(sc, psc, edge, line, I);
    gv = coarse_g(gc, pgc, edge, line, I);
  } else {
    const int c = (idx + q - 1) / 2;
    sv = (-coarse_s(sc, psc, edge, line, c - 1) + T(9) * coarse_s(sc, psc, edge, line, c) +
          T(9) * coarse_s(sc, psc, edge, line, c + 1) - coarse_s(sc, psc, edge, line, c + 2)) /
         T(16);
    gv = (-coarse_g(gc, pgc, edge, line, c - 1) + T(9) * coarse_g(gc, pgc, edge, line, c) +
          T(9) * coarse_g(gc, pgc, edge, line, c + 1) - coarse_g(gc, pgc, edge, line, c + 2)) /
         T(16);
  }
  gv = T(0.25) * gv;
}

template <typename T>
__device__ __forceinline__ void ring_body(const T* __restrict__ sc, int psc,
                                          const T* __restrict__ gc, int pgc, int nx, int ny,
                                          T* sring, T* gring, int e) {
  if (e >= ring_len(nx, ny)) return;
  const int edge = e < 2 * (nx + 1) ? e / (nx + 1) : 2 + (e - 2 * (nx + 1)) / (ny + 1);
  const int idx = e - ring_off(edge, nx, ny);
  T sv, gv;
  ring_values(sc, psc, gc, pgc, nx, ny, edge, idx, sv, gv);
  sring[e] = sv;
  gring[e] = gv;
}

template <typename T>
__global__ void k_ring(const T* __restrict__ sc, int psc, const T* __restrict__ gc, int pgc, int nx,
                       int ny, T* sring, T* gring) {
  ring_body(sc, psc, gc, pgc, nx, ny, sring, gring, blockIdx.x * blockDim.x + threadIdx.x);
}


// Unnormalised 1-D DSTs of edges edge0 .. edge0 + nedge - 1 (nedge <= 4) of a streamfunction
// ring, as they appear in B(s_ring): bottom edge values s(i, 0) sit on interior row 1, top
// s(i, ny) on row ny-1, left s(0, j) on column 1, right s(nx, j) on column nx-1.  N is the
// length of those edges' transforms (nx for bottom and top, ny for left and right).  Each
// workgroup transforms NEB of the edges (workgroup b the edges edge0 + NEB b onwards).
template <typename T, int N, int NT, int NEB>
__device__ __forceinline__ void ring_edge_dst_body(const T* __restrict__ sring,
                                                   const c2<T>* __restrict__ tw, T* lift,
                                                   int edge0, int nedge, int nx, int ny, int bx) {
  __shared__ c2<T> buf[NEB * fft_pad_len<N>()];
  __shared__ c2<T> stw[TwLayout<N>::total];
  const int tid = threadIdx.x;
  edge0 += NEB * bx;
  nedge = min(NEB, nedge - NEB * bx);
  {
    constexpr int CNT = NEB * (N - 1);
    constexpr int PER = (CNT + NT - 1) / NT;
    T v[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT, q = e / (N - 1);
      v[b] = (e < CNT && q < nedge) ? sring[ring_off(edge0 + q, nx, ny) + 1 + e % (N - 1)] : T(0);
    }
    load_table<T, N, NT>(stw, tw, tid);
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int e = tid + b * NT;
      if (e < CNT) dst_pack<T, N>(buf + (e / (N - 1)) * fft_pad_len<N>(), 1 + e % (N - 1), v[b]);
    }
  }
  for (int q = tid; q < NEB; q += NT) dst_pack_zeros<T, N>(buf + q * fft_pad_len<N>());
  __syncthreads();
  fft_lds<T, N, NEB, NT>(buf, stw, tid);
  for (int e = tid; e < nedge * (N / 2); e += NT) {
    const int q = e / (N / 2), k = 1 + e % (N / 2);
    T xk, xnk;
    dst_unpack<T, N>(buf + q * fft_pad_len<N>(), stw, k, xk, xnk);
    T* lo = lift + lift_off(edge0 + q, nx, ny);
    lo[k - 1] = xk;
    if (k != N / 2) lo[N - k - 1] = xnk;
  }
}

template <typename T, int N, int NT, int NEB>
__global__ __launch_bounds__(NT) void k_ring_edge_dst(const T* __restrict__ sring,
                                                      const c2<T>* __restrict__ tw, T* lift,
                                                      int edge0, int nedge, int nx, int ny) {
  ring_edge_dst_body<T, N, NT, NEB>(sring, tw, lift, edge0, nedge, nx, ny, blockIdx.x);
}

// k_ring and k_ring_edge_dst in one launch: workgroup `edge` makes that edge's ring values
// (the same arithmetic as k_ring) and transforms its streamfunction part (the same
// arithmetic as k_ring_edge_dst, one sequence per workgroup).  N is the edge's transform
// length: nx for the bottom and top edges, ny for the left and right.
template <typename T, int N, int NT>
__device__ __forceinline__ void ring_dst_body(const T* __restrict__ sc, int psc,
                                              const T* __restrict__ gc, int pgc, T* sring, T* gring,
                                              const c2<T>* __restrict__ tw, T* lift, int edge,
                                              int nx, int ny) {
  __shared__ c2<T> buf[fft_pad_len<N>()];
  __shared__ c2<T> stw[TwLayout<N>::total];
  const int tid = threadIdx.x;
  load_table<T, N, NT>(stw, tw, tid);
  const int off = ring_off(edge, nx, ny);
  // every value is read before the first store (a load issued after a store waits for that
  // store's acknowledgement too)
  constexpr int PR = (N + 1 + NT - 1) / NT;
  T sv[PR], gv[PR];
#pragma unroll
  for (int q = 0; q < PR; ++q) {
    const int idx = tid + q * NT;
    sv[q] = gv[q] = T(0);
    if (idx <= N) ring_values(sc, psc, gc, pgc, nx, ny, edge, idx, sv[q], gv[q]);
  }
#pragma unroll
  for (int q = 0; q < PR; ++q) {
    const int idx = tid + q * NT;
    if (idx > N) continue;
    sring[off + idx] = sv[q];
    gring[off + idx] = gv[q];
    if (idx >= 1 && idx <= N - 1) dst_pack<T, N>(buf, idx, sv[q]);
  }
  if (tid == 0) dst_pack_zeros<T, N>(buf);
  __syncthreads();
  fft_lds<T, N, 1, NT>(buf, stw, tid);
  T* lo = lift + lift_off(edge, nx, ny);
  for (int k = 1 + tid; k <= N / 2; k += NT) {
    T xk, xnk;
    dst_unpack<T, N>(buf, stw, k, xk, xnk);
    lo[k - 1] = xk;
    if (k != N / 2) lo[N - k - 1] = xnk;
  }
}

template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_ring_dst(const T* __restrict__ sc, int psc,
                                                 const T* __restrict__ gc, int pgc, T* sring,
                                                 T* gring, const c2<T>* __restrict__ tw, T* lift,
                                                 int edge0, int nx, int ny) {
  ring_dst_body<T, N, NT>(sc, psc, gc, pgc, sring, gring, tw, lift, edge0 + (int)blockIdx.x, nx,
                          ny);
}

// Many instances of one (square) grid size: workgroup (edge, instance blockIdx.y).
template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_ring_dst_multi(const RingJob<T>* __restrict__ tab,
                                                       const c2<T>* __restrict__ tw) {
  const RingJob<T> j = tab[blockIdx.y];
  ring_dst_body<T, N, NT>(j.sc, j.psc, j.gc, j.pgc, j.sring, j.gring, tw, j.lift, blockIdx.x, N, N);
}

// ------------------------------------------------ launches of one kernel configuration

template <typename T, int N, int ROWS, int NT, int DST, int MAXR>
hipError_t launch_rhs_cfg(const RhsArgs<T>& a, const c2<T>* t, hipStream_t st) {
  const int nb = ((a.ny > 0 ? a.ny : a.n) - 1 + ROWS - 1) / ROWS;
  hipLaunchKernelGGL((k_rhs_rowdst<T, N, ROWS, NT, DST, MAXR>), dim3(xcd_grid(nb)), dim3(NT), 0, st,
                     a, t, nb);
  return hipGetLastError();
}

template <typename T, int N, int CW, int NT, int MAXR>
hipError_t launch_col_cfg(const ColArgs<T>& a, int n, int batch, const c2<T>* t, const T* l,
                          hipStream_t st) {
  const int nb = ((a.ncols > 0 ? a.ncols : n - 1) + CW - 1) / CW;
  if (a.ev0)
    hipExtLaunchKernelGGL((k_col_solve<T, N, CW, NT, MAXR>), dim3(xcd_grid(nb), batch), dim3(NT), 0,
                          st, a.ev0, a.ev1, 0, a, t, l, nb);
  else
    hipLaunchKernelGGL((k_col_solve<T, N, CW, NT, MAXR>), dim3(xcd_grid(nb), batch), dim3(NT), 0, st,
                       a, t, l, nb);
  return hipGetLastError();
}

template <typename T, int N, int ROWS, int NT, int DUAL, int MAXR>
hipError_t launch_idst_cfg(const RowArgs<T>& a, int batch, const c2<T>* t, const T* ring,
                           int ring_rows, hipStream_t st) {
  const int nb = (a.r1 - a.r0 + 1 + ROWS - 1) / ROWS;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_row_idst<T, N, ROWS, NT, DUAL, MAXR>), dim3(xcd_grid(nb), batch), dim3(NT),
                     0, st, a, t, ring, ring_rows, nb);
  return hipGetLastError();
}

// Many instances of grid size N per launch (tables in device memory, `count` entries);
// maxrows: the largest row count [r0, r1] over the instances (row kernels).
template <typename T, int N, int ROWS, int NT, int DST, int MAXR>
hipError_t launch_rhs_multi_cfg(const RhsArgs<T>* tab, int count, const c2<T>* t, hipStream_t st) {
  const int nb = (N - 1 + ROWS - 1) / ROWS;
  hipLaunchKernelGGL((k_rhs_rowdst_multi<T, N, ROWS, NT, DST, MAXR>), dim3(xcd_grid(nb), count),
                     dim3(NT), 0, st, tab, t);
  return hipGetLastError();
}

template <typename T, int N, int CW, int NT, int MAXR>
hipError_t launch_col_multi_cfg(const ColArgs<T>* tab, int count, const c2<T>* t, const T* l,
                                hipStream_t st) {
  const int nb = (N - 1 + CW - 1) / CW;
  hipLaunchKernelGGL((k_col_solve_multi<T, N, CW, NT, MAXR>), dim3(xcd_grid(nb), count), dim3(NT),
                     0, st, tab, t, l);
  return hipGetLastError();
}

template <typename T, int N, int ROWS, int NT, int DUAL, int MAXR>
hipError_t launch_idst_multi_cfg(const IdstJob<T>* tab, int count, int maxrows, const c2<T>* t,
                                 hipStream_t st) {
  const int nb = (maxrows + ROWS - 1) / ROWS;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_row_idst_multi<T, N, ROWS, NT, DUAL, MAXR>), dim3(xcd_grid(nb), count),
                     dim3(NT), 0, st, tab, t);
  return hipGetLastError();
}

}  // namespace ib
