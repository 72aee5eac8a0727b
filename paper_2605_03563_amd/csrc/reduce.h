// Device helpers shared by the kernels: XCD-aware block numbering and
// deterministic (fixed-order) wavefront / block reductions.
#pragma once

#include <hip/hip_runtime.h>

namespace psn {

constexpr long long kPartialCap = 1 << 16;  // partial-sum slots per reduction

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Renumber the blocks so that XCD x receives a contiguous
// run of logical blocks (a contiguous range of planes), keeping the plane
// neighbours of a stencil inside one L2.  With total = 8q + r blocks, XCD x
// holds q + (x < r) of them, and its runs start where the previous end.
__device__ inline void xcd_block(int& bx, int& by, int& bz) {
  const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const unsigned total = gx * gy * gz;
  unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned q = total >> 3, r = total & 7u, x = lin & 7u;
  lin = x * q + (x < r ? x : r) + (lin >> 3);
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

// Sum of p[0 .. nb) by one block in a fixed order: thread t takes the
// entries t, t + T, t + 2T, ... into four interleaved accumulators (four
// independent loads in flight per round), then the block reduces.  Result
// valid in thread 0.  Call from every thread of the block.
__device__ inline double sum_partials(const double* __restrict__ p, int nb) {
  const int T = blockDim.x * blockDim.y * blockDim.z;
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = tid;
  for (; i + 3 * T < nb; i += 4 * T) {
    a0 += p[i];
    a1 += p[i + T];
    a2 += p[i + 2 * T];
    a3 += p[i + 3 * T];
  }
  for (; i < nb; i += T) a0 += p[i];
  return block_sum((a0 + a1) + (a2 + a3));
}

// threads of the one-block kernels that finish a reduction
constexpr int kFinishThreads = 1024;

}  // namespace psn
