// Pore observables on the lattice state (Sec. IV.B: the ionic current
// through the pore, from which the conductance follows): the particles of
// each species that the streaming which formed the current densities carried
// across a z link plane.
//
// The stored populations are the post-collision ones that the next pull
// streams; the densities reported for the current time are those pulled
// values.  So the populations crossing the plane between z and z + 1 are the
// stored ones at the pull sources of the sites on either side: a fluid site
// at z + 1 pulls its +z populations from plane z, a fluid site at z pulls its
// -z populations from plane z + 1, and a link whose source is solid (bit p of
// the site's link word) is bounced back and carries nothing across.
#include <cmath>

#include "ek_context.h"

using namespace ek;

namespace {

constexpr int FLUX_THREADS = 1024;   // one workgroup; a power of two for the tree

__device__ inline int wrap_axis(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// One workgroup over the nx * ny columns of the plane.  Each thread keeps
// float64 sums of its columns' crossing populations; the populations are
// stored as deviations from w_p nref, and over the open links of a plane the
// reference parts cancel (a link and its reverse are both open or both
// bounced, and have the same weight), so the deviations give the flux.  The
// per-thread sums are combined in a fixed tree (deterministic).
template <typename T>
__global__ __launch_bounds__(FLUX_THREADS) void k_plane_flux(const T* __restrict__ f,
                                                             const uint32_t* __restrict__ mask,
                                                             Dims d, int z, double v0, double v1,
                                                             double v2, double* __restrict__ out) {
  const int zu = z + 1 == d.nz ? 0 : z + 1;
  double acc[3] = {0.0, 0.0, 0.0};
  const int ncol = d.nx * d.ny;
  for (int t = threadIdx.x; t < ncol; t += blockDim.x) {
    const int x = t % d.nx, y = t / d.nx;
    // +z populations arriving at (x, y, z + 1) from plane z
    {
      const long long r = ((long long)zu * d.ny + y) * d.nx + x;
      const uint32_t m = mask[r];
      if (!(m & MASK_SOLID)) {
#pragma unroll
        for (int p = 1; p < Q; ++p) {
          if (CZ[p] != 1 || ((m >> p) & 1u)) continue;
          const long long src =
              ((long long)z * d.ny + wrap_axis(y - CY[p], d.ny)) * d.nx + wrap_axis(x - CX[p], d.nx);
#pragma unroll
          for (int s = 0; s < 3; ++s) acc[s] += double(f[(size_t)(s * Q + p) * d.n + src]);
        }
      }
    }
    // -z populations arriving at (x, y, z) from plane z + 1
    {
      const long long r = ((long long)z * d.ny + y) * d.nx + x;
      const uint32_t m = mask[r];
      if (!(m & MASK_SOLID)) {
#pragma unroll
        for (int p = 1; p < Q; ++p) {
          if (CZ[p] != -1 || ((m >> p) & 1u)) continue;
          const long long src =
              ((long long)zu * d.ny + wrap_axis(y - CY[p], d.ny)) * d.nx + wrap_axis(x - CX[p], d.nx);
#pragma unroll
          for (int s = 0; s < 3; ++s) acc[s] -= double(f[(size_t)(s * Q + p) * d.n + src]);
        }
      }
    }
  }
  __shared__ double red[3][FLUX_THREADS];
#pragma unroll
  for (int s = 0; s < 3; ++s) red[s][threadIdx.x] = acc[s];
  __syncthreads();
  for (int w = FLUX_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int s = 0; s < 3; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
    out[2] = red[2][0];
    out[3] = v0 * red[0][0] + v1 * red[1][0] + v2 * red[2][0];
  }
}

}  // namespace

extern "C" ek_status ek_plane_flux(ek_ctx* ctx, int32_t z, double* out) {
  if (!ctx) return EK_EINVAL;
  if (!out) return ctx->fail(EK_EINVAL, "out is NULL");
  if (z < 0 || z >= ctx->dims.nz) return ctx->fail(EK_EINVAL, "plane index outside [0, nz)");
  if (!ctx->have_geometry || !ctx->have_species[0] || !ctx->have_species[1] ||
      !ctx->have_species[2])
    return ctx->fail(EK_ESTATE, "set the geometry and all three species first");
  const LBParams lp = ctx->lb_params();
  double* dev = (double*)ctx->fnext();   // the free population buffer holds the 4 sums
  if (ctx->p.precision == EK_FP64)
    hipLaunchKernelGGL(k_plane_flux<double>, dim3(1), dim3(FLUX_THREADS), 0, ctx->stream,
                       (const double*)ctx->fcur(), ctx->mask, ctx->dims, (int)z, lp.valence[0],
                       lp.valence[1], lp.valence[2], dev);
  else
    hipLaunchKernelGGL(k_plane_flux<float>, dim3(1), dim3(FLUX_THREADS), 0, ctx->stream,
                       (const float*)ctx->fcur(), ctx->mask, ctx->dims, (int)z, lp.valence[0],
                       lp.valence[1], lp.valence[2], dev);
  if (hipMemcpyAsync(out, dev, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return ctx->fail(EK_EHIP, "copying the plane flux failed");
  return ctx->sync();
}
