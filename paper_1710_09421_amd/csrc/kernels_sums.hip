// Final sums of the block partials the lattice step and the charge pass write
// (Sec. II: the species masses and momentum checked for conservation, and the
// mean charge the periodic Poisson problem removes).  Deterministic: a fixed
// partition and fixed trees, whatever the scheduling.
#include "ek_internal.h"

#include "reduce.h"

namespace ek {

namespace {

constexpr int FOLD_BLOCKS = 256;   // first-stage blocks of a two-stage sum
constexpr int FOLD_MIN = 8192;     // partials below this are summed by one block

// First stage: block b adds the partials of its contiguous share of the
// nblocks, component by component (strided over its threads, then a fixed
// tree), and writes out[c * gridDim.x + b].  One block of 1024 threads alone
// reads 65536 partials at the speed of one compute unit (80 us for seven
// components at 256x256x512); the chip's blocks share the reads.
template <int NC>
__global__ __launch_bounds__(256) void k_fold_partials(const double* __restrict__ part,
                                                       int nblocks, double* __restrict__ out) {
  __shared__ double sh[NC][256];
  const int tid = threadIdx.x, b = blockIdx.x, nb = gridDim.x;
  const int per = (nblocks + nb - 1) / nb;
  const int lo = b * per, hi = min(nblocks, lo + per);
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0.0;
  for (int i = lo + tid; i < hi; i += 256) {
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] += part[(size_t)c * nblocks + i];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) sh[c][tid] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int c = 0; c < NC; ++c) sh[c][tid] += sh[c][tid + w];
    }
    __syncthreads();
  }
  if (tid < NC) out[(size_t)tid * nb + b] = sh[tid][0];
}

// out[0..6] = sums of the seven components; out[7] += out[6] when `count`
// (sites updated by the timed launches).
__global__ __launch_bounds__(1024) void k_sum7(const double* __restrict__ partials, int nblocks,
                                               double* __restrict__ out, int count) {
  double t[7];
  block_sums_1024<7>(partials, nblocks, t);
  if (threadIdx.x == 0) {
    for (int c = 0; c < 7; ++c) out[c] = t[c];
    if (count) out[7] += t[6];
  }
}

__global__ __launch_bounds__(1024) void k_mean_shift(const double* __restrict__ partials,
                                                     int nblocks, double inv_n, double inv_eps,
                                                     PoissonScalars* ps) {
  double t[1];
  block_sums_1024<1>(partials, nblocks, t);
  if (threadIdx.x == 0) {
    ps->shift = t[0] * inv_n * inv_eps;
    ps->done = 0;
    ps->iters = 0;
    ps->zero_rhs = 0;
    ps->cycles = 0;
  }
}

// The partials to hand to the final single-block sum: `partials` itself, or
// their first-stage fold into `scratch` (when they are many and it has room
// for NC * FOLD_BLOCKS values); nblocks is updated.
template <int NC>
const double* fold(const double* partials, int& nblocks, double* scratch, long long room,
                   hipStream_t s) {
  if (!scratch || nblocks < FOLD_MIN || room < (long long)NC * FOLD_BLOCKS) return partials;
  hipLaunchKernelGGL(k_fold_partials<NC>, dim3(FOLD_BLOCKS), dim3(256), 0, s, partials, nblocks,
                     scratch);
  nblocks = FOLD_BLOCKS;
  return scratch;
}

}  // namespace

void launch_sum_partials(const double* partials, int nblocks, double* out, int count,
                         hipStream_t s, double* scratch, long long room) {
  const double* p = fold<7>(partials, nblocks, scratch, room, s);
  hipLaunchKernelGGL(k_sum7, dim3(1), dim3(1024), 0, s, p, nblocks, out, count);
}

void launch_mean_shift(const double* partials, int nblocks, double inv_n, double inv_eps,
                       PoissonScalars* ps, hipStream_t s, double* scratch, long long room) {
  const double* p = fold<1>(partials, nblocks, scratch, room, s);
  hipLaunchKernelGGL(k_mean_shift, dim3(1), dim3(1024), 0, s, p, nblocks, inv_n, inv_eps, ps);
}

}  // namespace ek
