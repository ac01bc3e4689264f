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
// [l % 32].
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

// Workgroup tile 64 x 64 of C, four waves in a 2 x 2 arrangement, each wave one 32 x 32 MFMA
// tile.  The k range is walked in stages of BK: the S part (already split, BF16) and the X
// part (FP32, split as it is staged) of the next stage are loaded into registers while the
// matrix cores work on the current stage from LDS, then stored into the other of two LDS
// buffers; one barrier per stage.  A stage must carry enough products to cover the latency of
// its loads (which come from L2 or the last-level cache): with BK = 32 each of the 32 stages
// at n = 1024 waited for its loads, so the stages are 64 or 128 deep (measured choice).  In LDS
// both operands are held row by row with k contiguous -- the A tile as [row of C][k], the B
// tile as [column of C][k] -- so that every fragment is one 16-byte read: lane l reads row
// l % 32 at k offset 8 (l / 32).  Rows are padded by 8 BF16.  The k blocks of 16 are
// accumulated in increasing order with the three products of a block in the order hi.hi,
// hi.lo, lo.hi.
__device__ __forceinline__ void split_store(const float* v, __bf16* hi, __bf16* lo) {
  bf16x8 h, l;
  split8(v, h, l);
  *reinterpret_cast<bf16x8*>(hi) = h;
  *reinterpret_cast<bf16x8*>(lo) = l;
}

// Tile (ti, tj) of workgroup `bid`: consecutive workgroups, which the dispatcher spreads over
// the XCDs, are first renumbered so that each XCD holds a contiguous range (xcd_block), and
// the range is then walked in groups of 4 tile rows, so that the workgroups of one XCD share
// a few S and X panels in its L2.
__device__ __forceinline__ bool gemm_tile(int bid, int nbi, int nbj, int& ti, int& tj) {
  const int t = xcd_block(bid, nbi * nbj);
  if (t < 0) return false;
  constexpr int G = 4;
  const int per = G * nbj, grp = t / per, first = grp * G, rows = min(G, nbi - first);
  const int r = t % per;
  ti = first + r % rows;
  tj = r / rows;
  return true;
}

template <int BK>
constexpr size_t gemm_lds_bytes() {
  return (size_t)2 * 4 * 64 * (BK + 8) * sizeof(__bf16);  // 2 buffers x (A, B) x (hi, lo)
}

// MODE 0: C = S X (S is the left operand); MODE 1: C = X S.  EPI 1: spectral solve on the
// output (see GemmArgs).
template <int MODE, int EPI, int BK>
__global__ __launch_bounds__(256) void k_dst_gemm(GemmArgs g) {
  constexpr int LDK = BK + 8, TILE = 64 * LDK;  // one operand part of one buffer, in BF16
  constexpr int CPR = BK / 8;                   // 16-byte chunks per row of a stage
  constexpr int SCH = 64 * CPR / 256;           // S chunks per thread
  constexpr int XCH = BK / 32;                  // groups of 8 X values per thread
  extern __shared__ __bf16 lds[];
  // buffer b: A hi, A lo, B hi, B lo
  auto part = [&](int b, int q) { return lds + (size_t)(4 * b + q) * TILE; };
  const int nbi = g.kpad / 64, nbj = g.kpad / 64;
  int ti, tj;
  if (!gemm_tile(blockIdx.x, nbi, nbj, ti, tj)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = ti * 64, j0 = tj * 64;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lr = lane & 31, lq = (lane >> 5) * 8;
  const int nv = g.nv;

  bf16x8 s_hi[SCH], s_lo[SCH];
  float xv[XCH][8];
  auto load_stage = [&](int k0) {
    // S part: MODE 0 -> A rows i0 + row; MODE 1 -> B rows j0 + row
#pragma unroll
    for (int u = 0; u < SCH; ++u) {
      const int e = tid + 256 * u, row = e / CPR, ch = e % CPR;
      const int grow = (MODE == 0 ? i0 : j0) + row;
      s_hi[u] = load8(g.shi + (size_t)grow * g.ps + k0 + 8 * ch);
      s_lo[u] = load8(g.slo + (size_t)grow * g.ps + k0 + 8 * ch);
    }
    if constexpr (MODE == 0) {
      // B tile [column c][k] = X[k0 + k][j0 + c]: a lane takes one column and 8 k per group
      const int c = tid & 63, j = j0 + c;
#pragma unroll
      for (int u = 0; u < XCH; ++u) {
        const int kc = (tid >> 6) + 4 * u;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + 8 * kc + q;
          xv[u][q] = (k < nv && j < nv) ? g.x[(size_t)k * g.px + j] : 0.0f;
        }
      }
    } else {
      // A tile [row r][k] = X[i0 + r][k0 + k]: a lane takes 8 consecutive k of one row per group
#pragma unroll
      for (int u = 0; u < XCH; ++u) {
        const int e = tid + 256 * u, r = e / CPR, kc = e % CPR;
        const int i = i0 + r, kb = k0 + 8 * kc;
        if (i < nv) {
          const float4 a = *reinterpret_cast<const float4*>(g.x + (size_t)i * g.px + kb);
          const float4 b = *reinterpret_cast<const float4*>(g.x + (size_t)i * g.px + kb + 4);
          const float t8[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) xv[u][q] = kb + q < nv ? t8[q] : 0.0f;
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) xv[u][q] = 0.0f;
        }
      }
    }
  };
  auto store_stage = [&](int b) {
#pragma unroll
    for (int u = 0; u < SCH; ++u) {
      const int e = tid + 256 * u, row = e / CPR, ch = e % CPR;
      const int off = row * LDK + 8 * ch;
      *reinterpret_cast<bf16x8*>(part(b, MODE == 0 ? 0 : 2) + off) = s_hi[u];
      *reinterpret_cast<bf16x8*>(part(b, MODE == 0 ? 1 : 3) + off) = s_lo[u];
    }
    if constexpr (MODE == 0) {
      const int c = tid & 63;
#pragma unroll
      for (int u = 0; u < XCH; ++u) {
        const int kc = (tid >> 6) + 4 * u;
        split_store(xv[u], part(b, 2) + c * LDK + 8 * kc, part(b, 3) + c * LDK + 8 * kc);
      }
    } else {
#pragma unroll
      for (int u = 0; u < XCH; ++u) {
        const int e = tid + 256 * u, r = e / CPR, kc = e % CPR;
        split_store(xv[u], part(b, 0) + r * LDK + 8 * kc, part(b, 1) + r * LDK + 8 * kc);
      }
    }
  };

  f32x16 acc = {};
  const int nst = g.kpad / BK;
  load_stage(0);
  store_stage(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int b = st & 1;
    if (st + 1 < nst) load_stage((st + 1) * BK);
    const __bf16* ah = part(b, 0) + (wr + lr) * LDK + lq;
    const __bf16* al = part(b, 1) + (wr + lr) * LDK + lq;
    const __bf16* bh = part(b, 2) + (wc + lr) * LDK + lq;
    const __bf16* bl = part(b, 3) + (wc + lr) * LDK + lq;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(ah + ks);
      const bf16x8 alo = *reinterpret_cast<const bf16x8*>(al + ks);
      const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(bh + ks);
      const bf16x8 blo = *reinterpret_cast<const bf16x8*>(bl + ks);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc, 0, 0, 0);
    }
    if (st + 1 < nst) store_stage(b ^ 1);
    __syncthreads();
  }

  const int col = j0 + wc + lr;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = i0 + wr + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
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

// Stage depth 128 when the padded size is a multiple of it, else 64 (every padded size is a
// multiple of 64).
int gemm_bk(int kpad) { return kpad % 128 == 0 ? 128 : 64; }

template <int BK>
hipError_t launch_dst_gemm_bk(const GemmArgs& g, int mode, hipStream_t st) {
  const int tiles = (g.kpad / 64) * (g.kpad / 64);
  const size_t lds = gemm_lds_bytes<BK>();
  const dim3 grid(xcd_grid(tiles)), blk(256);
  if (mode == 0 && g.lam == nullptr) hipLaunchKernelGGL((k_dst_gemm<0, 0, BK>), grid, blk, lds, st, g);
  else if (mode == 0) hipLaunchKernelGGL((k_dst_gemm<0, 1, BK>), grid, blk, lds, st, g);
  else hipLaunchKernelGGL((k_dst_gemm<1, 0, BK>), grid, blk, lds, st, g);
  return hipGetLastError();
}

hipError_t launch_dst_gemm(const GemmArgs& g, int mode, hipStream_t st) {
  if (g.kpad <= 0 || g.kpad % 64 != 0 || g.nv > g.kpad) return hipErrorInvalidValue;
  const int bk = g.tn > 0 ? g.tn : gemm_bk(g.kpad);
  if (bk == 128 && g.kpad % 128 == 0) return launch_dst_gemm_bk<128>(g, mode, st);
  if (bk == 64) return launch_dst_gemm_bk<64>(g, mode, st);
  return hipErrorInvalidValue;
}

}  // namespace ib
