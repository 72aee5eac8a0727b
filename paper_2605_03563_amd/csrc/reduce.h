// Device helpers shared by the kernels: XCD-aware block numbering and
// deterministic (fixed-order) wavefront / block reductions.
#pragma once

#include <hip/hip_runtime.h>

namespace psn {

constexpr long long kPartialCap = 1 << 16;  // partial-sum slots per reduction

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Renumber the blocks so that XCD x receives a contiguous
// run of logical blocks (a contiguous range of planes), keeping the plane
// neighbours of a stencil inside one L2.
__device__ inline void xcd_block(int& bx, int& by, int& bz) {
  const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const unsigned total = gx * gy * gz;
  unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if ((total & 7u) == 0u) {
    const unsigned per = total >> 3;
    lin = (lin & 7u) * per + (lin >> 3);
  }
  bx = (int)(lin % gx);
  const unsigned t = lin / gx;
  by = (int)(t % gy);
  bz = (int)(t / gy);
}

__device__ inline long long linear_block() {
  return blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block (blockDim multiple of 64, <= 1024) in a fixed order;
// result valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double red[16];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  v = wave_sum(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    for (int w = 0; w < (nthreads + 63) / 64; ++w) s += red[w];
  }
  return s;
}

}  // namespace psn
