// Shared definitions for the immersed-boundary HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace ib {

template <typename T>
struct c2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return c2<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return c2<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return c2<T>{a.x - b.x, a.y - b.y}; }
// multiply by -i
template <typename T>
__device__ __forceinline__ c2<T> cmul_mi(c2<T> a) { return c2<T>{a.y, -a.x}; }

// Ring layout of a level's boundary values on an nx x ny level: the bottom (j = 0, index i)
// and top (j = ny, index i) edges of nx+1 entries, then the left (i = 0, index j) and right
// (i = nx, index j) edges of ny+1 entries (on a square level: 4 edges of n+1 each).  The 1-D
// edge transforms ("lift") of a ring keep the same order with the corner entries left out:
// nx-1, nx-1, ny-1, ny-1 values.
enum { RING_B = 0, RING_T = 1, RING_L = 2, RING_R = 3 };
__host__ __device__ __forceinline__ int ring_off(int edge, int nx, int ny) {
  return edge < 2 ? edge * (nx + 1) : 2 * (nx + 1) + (edge - 2) * (ny + 1);
}
__host__ __device__ __forceinline__ int ring_len(int nx, int ny) { return 2 * (nx + 1) + 2 * (ny + 1); }
__host__ __device__ __forceinline__ int lift_off(int edge, int nx, int ny) {
  return edge < 2 ? edge * (nx - 1) : 2 * (nx - 1) + (edge - 2) * (ny - 1);
}

// Workgroup -> row-block mapping that keeps consecutive row blocks on one XCD.
// Workgroups are dispatched round-robin over the 8 XCDs of MI355X; launching
// xcd_grid(nblocks) workgroups and mapping workgroup `bid` to block
// (bid % 8) * per + bid / 8 gives every XCD one contiguous band of rows, so the
// stencil halo rows shared by neighbouring blocks stay in that XCD's L2.  The map
// is a bijection onto [0, 8 per); blocks >= nblocks return -1 (idle workgroup).
// Correctness does not depend on the dispatch order.
__host__ __device__ __forceinline__ int xcd_grid(int nblocks) {
  return nblocks < 16 ? nblocks : 8 * ((nblocks + 7) / 8);
}
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  if (nblocks < 16) return bid;
  int per = (nblocks + 7) / 8;
  int b = (bid % 8) * per + bid / 8;
  return b < nblocks ? b : -1;
}

}  // namespace ib
