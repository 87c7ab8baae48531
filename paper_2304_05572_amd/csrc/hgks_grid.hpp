// Grid helpers shared by the kernels of every dimension: problem lookup of a block in a batched launch,
// XCD-aware block renumbering and the block-wide minimum of the CFL reduction.
#pragma once

#include <hip/hip_runtime.h>

namespace hk {

__device__ inline int find_prob(const int* __restrict__ off, int nprob, int b) {
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD receives a contiguous
// range of tiles and neighbouring tiles share its L2.
__device__ inline int xcd_swizzle(int b, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int x = b & 7, idx = b >> 3;
  return x * q + (x < r ? x : r) + idx;
}

__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide minimum (wavefront shuffles, then the waves' minima through LDS); thread 0 returns it.
__device__ inline double block_min(double q) {
  __shared__ double red[16];
  q = wave_min(q);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = q;
  __syncthreads();
  double m = red[0];
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 1; k < nw; ++k) m = fmin(m, red[k]);
  }
  return m;
}

}  // namespace hk
