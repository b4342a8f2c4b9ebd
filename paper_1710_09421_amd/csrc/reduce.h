// Deterministic reductions for 64-wide wavefronts: butterfly within a wave,
// then the block's waves in a fixed order.  Partial sums land in
// partials[c * nblocks + block] and are summed by a single block later, so the
// result depends only on the launch shape, never on scheduling.
#pragma once

#include <hip/hip_runtime.h>

namespace ek {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A block of up to 1024 threads (a whole number of waves); four waves are
// added pairwise, other counts in wave order.
template <int NC>
__device__ inline void block_partials(const double (&v)[NC], double* partials, int bid,
                                      int nblocks) {
  __shared__ double sh[NC][16];
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int lane = tid & 63, wid = tid >> 6;
  const int nw = int(blockDim.x * blockDim.y) >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double s = wave_sum(v[c]);
    if (lane == 0) sh[c][wid] = s;
  }
  __syncthreads();
  if (tid < NC) {
    double s;
    if (nw == 4) {
      s = ((sh[tid][0] + sh[tid][1]) + (sh[tid][2] + sh[tid][3]));
    } else {
      s = sh[tid][0];
      for (int w = 1; w < nw; ++w) s += sh[tid][w];
    }
    partials[(size_t)tid * nblocks + bid] = s;
  }
}

// Sum of one component over nblocks partials by a block of 256 threads
// (strided sums, then a fixed tree).  Result valid in thread 0.
__device__ inline double block_sum_256(const double* part, int nblocks) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < nblocks; i += 256) s += part[i];
  sh[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Sums of NC components of nblocks partials (layout [c * nblocks + block]) by
// one block of 1024 threads: strided sums of every component first, then a
// fixed tree per component.  Results valid in thread 0.  A thread adds its
// partials in the order of i; the loads of U consecutive ones are issued
// before the first of them is added, so that they are in flight together
// (one load at a time would leave the sum of 65536 partials waiting on 64
// memory latencies in a row).
template <int NC>
__device__ inline void block_sums_1024(const double* part, int nblocks, double (&out)[NC]) {
  __shared__ double sh[NC][1024];
  constexpr int U = NC >= 32 ? 1 : 32 / NC;
  const int tid = threadIdx.x;
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0.0;
  int i = tid;
  for (; i + (U - 1) * 1024 < nblocks; i += U * 1024) {
    double v[U][NC];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) v[u][c] = part[(size_t)c * nblocks + i + u * 1024];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += v[u][c];
  }
  for (; i < nblocks; i += 1024) {
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] += part[(size_t)c * nblocks + i];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) sh[c][tid] = s[c];
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int c = 0; c < NC; ++c) sh[c][tid] += sh[c][tid + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = sh[c][0];
}

}  // namespace ek
