// Sine transforms as dense matrix products on the BF16 matrix cores (DST-as-GEMM).
//
// The unnormalised DST-I of length n-1 is a product with the symmetric matrix
// S_jk = sin(pi (j+1)(k+1) / n), j, k < n-1 (Sec. 3.2.1: C^T C = S Lambda S up to the
// normalisation).  Here S is held split in two BF16 matrices, S = S_hi + S_lo, and the FP32
// operand x is split the same way when it is loaded (x_hi = bf16(x), x_lo = bf16(x - x_hi)),
// so that S x = S_hi x_hi + S_hi x_lo + S_lo x_hi up to the dropped S_lo x_lo term and the
// FP32 accumulation: three v_mfma_f32_32x32x16_bf16 per 32 x 32 x 16 block.  Lane layout of
// that instruction (checked on the device): lane l holds A[l % 32][8 (l / 32) + q] and
// B[8 (l / 32) + q][l % 32], q < 8, and result item v is C[8 (v / 4) + 4 (l / 32) + v % 4]
// [l % 32].  Each wave owns a 32 x 32 tile of C, four waves a 64 x 64 workgroup tile.
#include <hip/hip_runtime.h>

#include "ib_internal.hpp"

namespace ib {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split8(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const __bf16 h = (__bf16)v[q];
    hi[q] = h;
    lo[q] = (__bf16)(v[q] - (float)h);
  }
}

__device__ __forceinline__ bf16x8 load8(const __bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// MODE 0: C = S X (S is the left operand); MODE 1: C = X S.  EPI 1: spectral solve on the
// output (see GemmArgs).
template <int MODE, int EPI>
__global__ __launch_bounds__(256) void k_dst_gemm(GemmArgs g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = blockIdx.y * 64 + (w >> 1) * 32, j0 = blockIdx.x * 64 + (w & 1) * 32;
  const int lr = lane & 31, lq = (lane >> 5) * 8;
  const int nv = g.nv;
  f32x16 acc = {};
  for (int k0 = 0; k0 < g.kpad; k0 += 16) {
    const int kb = k0 + lq;  // this lane's 8 consecutive k
    bf16x8 ahi, alo, bhi, blo;
    float v[8];
    if constexpr (MODE == 0) {
      ahi = load8(g.shi + (size_t)(i0 + lr) * g.ps + kb);
      alo = load8(g.slo + (size_t)(i0 + lr) * g.ps + kb);
      const int j = j0 + lr;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (kb + q < nv && j < nv) ? g.x[(size_t)(kb + q) * g.px + j] : 0.0f;
      split8(v, bhi, blo);
    } else {
      const int i = i0 + lr;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (i < nv && kb + q < nv) ? g.x[(size_t)i * g.px + kb + q] : 0.0f;
      split8(v, ahi, alo);
      bhi = load8(g.shi + (size_t)(j0 + lr) * g.ps + kb);  // S is symmetric
      blo = load8(g.slo + (size_t)(j0 + lr) * g.ps + kb);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc, 0, 0, 0);
  }
  const int col = j0 + lr;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = i0 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
    if (row >= nv || col >= nv) continue;
    const float y = acc[v];
    if constexpr (EPI == 0) {
      g.c[(size_t)row * g.pc + col] = y;
    } else {
      // row = mode l - 1 (along j), col = mode k - 1 (along i)
      const float lsum = g.lam[col] + g.lam[row];
      const float gam = y / (1.0f + g.alpha * lsum);
      float lift = 0.0f;
      if (g.lift != nullptr) {
        const int k = col + 1, l = row + 1, n = nv + 1;
        const float sk = g.sinv[k], sl = g.sinv[l];
        const float pk = (k & 1) ? 1.0f : -1.0f, pl = (l & 1) ? 1.0f : -1.0f;
        lift = g.lift[k - 1] * sl + g.lift[(n - 1) + k - 1] * sl * pl +
               sk * g.lift[2 * (n - 1) + l - 1] + sk * pk * g.lift[3 * (n - 1) + l - 1];
      }
      g.c[(size_t)row * g.pc + col] = (gam + lift) * (g.scale / lsum);
      g.c2[(size_t)row * g.pc2 + col] = gam * g.scale;
    }
  }
}

hipError_t launch_dst_gemm(const GemmArgs& g, int mode, hipStream_t st) {
  const int nb = g.kpad / 64;
  const dim3 grid(nb, nb), blk(256);
  if (mode == 0 && g.lam == nullptr) hipLaunchKernelGGL((k_dst_gemm<0, 0>), grid, blk, 0, st, g);
  else if (mode == 0) hipLaunchKernelGGL((k_dst_gemm<0, 1>), grid, blk, 0, st, g);
  else hipLaunchKernelGGL((k_dst_gemm<1, 0>), grid, blk, 0, st, g);
  return hipGetLastError();
}

}  // namespace ib
