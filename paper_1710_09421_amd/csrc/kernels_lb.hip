// Grid-wide lattice kernels (one thread per site): initial populations, the
// fused pull-stream + collide step and the moment read-out (the ion-density
// pass is in kernels_charge.hip).  The per-site bodies are in lb_site.h.
#include "ek_internal.h"
#include <hip/hip_ext.h>

#include "lb_site.h"
#include "md_chain.h"
#include "reduce.h"

namespace ek {

namespace {

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_init_species(T* __restrict__ f,
                                                        const uint32_t* __restrict__ mask,
                                                        const double* __restrict__ n0, int s,
                                                        double nref, Dims d) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.n) return;
  const int x = int(r % d.nx), y = int((r / d.nx) % d.ny), z = int(r / ((long long)d.nx * d.ny));
  const uint32_t m = mask[r];
  const Nbr nb = neighbours(x, y, z, d);
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    T v = T(0);
    if (!(m & MASK_SOLID)) {
      // post-collision value that streams into f_p(r + c_p) = w_p n(r + c_p),
      // or that bounces back into f_opp(p)(r) = w_p n(r) if r + c_p is solid
      const long long dst = nb.zo[1 + CZ[p]] + nb.yo[1 + CY[p]] + nb.xo[1 + CX[p]];
      const bool dst_solid = mask[dst] & MASK_SOLID;
      const double n = dst_solid ? n0[r] : n0[dst];
      v = T(weight(p) * (n - nref));
    }
    f[(size_t)(s * Q + p) * d.n + r] = v;
  }
}

// Fused step at every fluid site: pull + bounce-back, moments, field from the
// potential, closed-form implicit drag, BGK collision with the half-force
// (Guo) forcing term, aligned store; partial sums of species mass and total
// momentum of f(t) in float64, and the number of sites updated.  Sites with
// a `skip` bit are left to k_lb_tail.  Partials: [c * nblocks + block], the
// blocks of this launch first.
// Variants V of the fused step: bit 0 the thermal fluctuations, bit 1 the
// field of insulating walls.
template <typename T, typename I, int V>
__global__ __launch_bounds__(BLOCK) void k_lb_step(const T* __restrict__ fsrc,
                                                   T* __restrict__ fdst,
                                                   const uint32_t* __restrict__ mask,
                                                   const double* __restrict__ psi, LBParams lp,
                                                   BeadTableView bt,
                                                   double* __restrict__ partials, int nblocks,
                                                   uint32_t skip, Dims d, int zb, NoiseParams np,
                                                   WallView wv) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (x < d.nx && y < d.ny)
    for (int k = 0; k < zb; ++k)
      if (lb_site<T, I, 7, (V & 1) != 0, (V & 2) != 0>(fsrc, fdst, mask, psi, lp, bt, x, y,
                                                        blockIdx.z * zb + k, d, acc, skip, &np,
                                                        &wv))
        acc[6] += 1.0;
  block_partials<7>(acc, partials, bid, nblocks);
}

// The sites left by k_lb_step (MASK_DEFER: the nodes of the bead boxes),
// once the chain has spread its friction (component 6, the count of sites
// the fused kernel updated, gets nothing from here).  Item = (bead i, box node t); a
// node in several boxes is updated by the lowest bead whose box holds it
// (the boxes' origins are fixed for the step).  It leaves the flags set, so
// that it can run beside k_lb_step (which skips the flagged sites);
// k_defer_clear clears them once both have ended.  Needs every side of the
// box >= BOX (no box overlaps itself).
template <typename T, typename I, int V>
__global__ __launch_bounds__(BLOCK) void k_lb_tail(const T* __restrict__ fsrc,
                                                   T* __restrict__ fdst,
                                                   const uint32_t* __restrict__ mask,
                                                   const double* __restrict__ psi, LBParams lp,
                                                   BeadTableView bt,
                                                   const int* __restrict__ origin, int n_beads,
                                                   double* __restrict__ partials,
                                                   int first_block, int nblocks, Dims d,
                                                   NoiseParams np, WallView wv) {
  // origins of the beads up to this block's last one, staged in LDS for the
  // test against every lower bead
  extern __shared__ int so[];
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb_blk = min(n_beads, ((blockIdx.x + 1) * blockDim.x + BOX3 - 1) / BOX3);
  for (int k = threadIdx.x; k < 3 * nb_blk; k += blockDim.x) so[k] = origin[k];
  __syncthreads();
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (item < n_beads * BOX3) {
    const int i = item / BOX3, t = item % BOX3;
    const int gx = so[3 * i] + t % BOX, gy = so[3 * i + 1] + (t / BOX) % BOX,
              gz = so[3 * i + 2] + t / (BOX * BOX);
    bool first = true;
    for (int j = 0; j < i && first; ++j)
      if (wrap(gx - so[3 * j], d.nx) < BOX && wrap(gy - so[3 * j + 1], d.ny) < BOX &&
          wrap(gz - so[3 * j + 2], d.nz) < BOX)
        first = false;
    if (first) {
      const int x = wrap(gx, d.nx), y = wrap(gy, d.ny), z = wrap(gz, d.nz);
      lb_site<T, I, 7, (V & 1) != 0, (V & 2) != 0>(fsrc, fdst, mask, psi, lp, bt, x, y, z, d,
                                                    acc, 0u, &np, &wv);   // not counted in acc[6]
    }
  }
  block_partials<7>(acc, partials, first_block + blockIdx.x, nblocks);
}

// Clears MASK_DEFER on every node of the n_beads boxes (item = bead, node).
__global__ __launch_bounds__(BLOCK) void k_defer_clear(uint32_t* __restrict__ mask,
                                                       const int* __restrict__ origin,
                                                       int n_beads, Dims d) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= n_beads * BOX3) return;
  const int i = item / BOX3, t = item % BOX3;
  const int x = wrap(origin[3 * i] + t % BOX, d.nx), y = wrap(origin[3 * i + 1] + (t / BOX) % BOX, d.ny),
            z = wrap(origin[3 * i + 2] + t / (BOX * BOX), d.nz);
  atomicAnd(&mask[((long long)z * d.ny + y) * d.nx + x], ~MASK_DEFER);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_moments(const T* __restrict__ f,
                                                   const uint32_t* __restrict__ mask, int s,
                                                   double nref, double* __restrict__ n_out,
                                                   double* __restrict__ u_out, Dims d) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.n) return;
  const int x = int(r % d.nx), y = int((r / d.nx) % d.ny), z = int(r / ((long long)d.nx * d.ny));
  const uint32_t m = mask[r];
  double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  if (!(m & MASK_SOLID)) {
    const Nbr nb = neighbours(x, y, z, d);
    T g[Q];
    pull(f, s, r, m, nb, d.n, g);
    double dn = 0.0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      dn += double(g[p]);
      jx += CX[p] * double(g[p]);
      jy += CY[p] * double(g[p]);
      jz += CZ[p] * double(g[p]);
    }
    n = nref + dn;
    jx /= n; jy /= n; jz /= n;
  }
  if (n_out) n_out[r] = n;
  if (u_out) {
    u_out[r] = jx;
    u_out[d.n + r] = jy;
    u_out[2 * d.n + r] = jz;
  }
}

}  // namespace

SiteGrid site_grid(int nx, int ny, int nz, int bx_pref) {
  int bx = bx_pref;
  if (bx <= 0) {
    bx = 64;
    while (bx > 8 && nx % bx != 0) bx >>= 1;
    if (nx < bx) bx = nx;
  }
  int by = BLOCK / bx;
  SiteGrid g;
  g.block = dim3(bx, by, 1);
  g.grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nz);
  return g;
}

// Charge pass and fused step: blocks of whole x-rows where a power-of-two
// row length allows (256 or 128 sites), else the default shape.  Reading
// each population plane in runs of a whole row measured 14 % faster (fused
// step) and 15 % faster (charge pass) on a 256x256x512 box than blocks of
// 64 x 4 sites; multigrid keeps the default shape (whole rows were slower).
SiteGrid lattice_grid(int nx, int ny, int nz) {
  for (int bx = BLOCK; bx >= 128; bx >>= 1)
    if (nx % bx == 0) return site_grid(nx, ny, nz, bx);
  return site_grid(nx, ny, nz, 0);
}

SiteGrid colour_grid(int nx, int ny, int nz, int bx_pref) {
  return site_grid(nx / 2, ny, nz, bx_pref);
}

template <typename T>
void launch_init_species(T* f, const uint32_t* mask, const double* n_dev, int species,
                         double nref, Dims d, hipStream_t s) {
  const int blocks = int((d.n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_init_species<T>, dim3(blocks), dim3(BLOCK), 0, s, f, mask, n_dev, species,
                     nref, d);
}

// z-planes per block of the fused step: each block sums its sites' masses
// and momentum once, so two planes per block halve the block-reduction work;
// more planes per block measured slower (fewer blocks walking longer), and at
// least 1024 blocks remain.
int lb_planes_per_block(const SiteGrid& g, int nz) {
  int zb = 1;
  while (zb < 2 && nz % (2 * zb) == 0 && (long long)g.grid.x * g.grid.y * (nz / (2 * zb)) >= 1024)
    zb *= 2;
  return zb;
}

int lb_step_blocks(const SiteGrid& g, int nz) {
  return int(g.grid.x * g.grid.y * (nz / lb_planes_per_block(g, nz)));
}

int lb_tail_blocks(int n_beads) { return (n_beads * BOX3 + BLOCK - 1) / BLOCK; }

template <typename T>
int launch_lb_step(const T* fsrc, T* fdst, const uint32_t* mask, const double* psi,
                   const LBParams& lp, const BeadTableView& bt, double* partials, int nblocks,
                   uint32_t skip, Dims d, const SiteGrid& g, hipStream_t s, hipEvent_t start,
                   hipEvent_t stop, const NoiseParams* noise, const WallView* walls) {
  const int zb = lb_planes_per_block(g, d.nz);
  const dim3 grid(g.grid.x, g.grid.y, d.nz / zb);
  const NoiseParams np = noise ? *noise : NoiseParams{};
  const WallView wv = walls ? *walls : WallView{};
  // the events (when given) are stamped at the kernel's own start and end
  auto go = [&](auto kernel) {
    hipExtLaunchKernelGGL(kernel, grid, g.block, 0, s, start, stop, 0, fsrc, fdst, mask, psi, lp,
                          bt, partials, nblocks, skip, d, zb, np, wv);
  };
  const int v = (noise ? 1 : 0) | (walls ? 2 : 0);
  if (fits_idx32<T>(d.n)) {
    if (v == 0) go(k_lb_step<T, uint32_t, 0>);
    else if (v == 1) go(k_lb_step<T, uint32_t, 1>);
    else if (v == 2) go(k_lb_step<T, uint32_t, 2>);
    else go(k_lb_step<T, uint32_t, 3>);
  } else {
    if (v == 0) go(k_lb_step<T, long long, 0>);
    else if (v == 1) go(k_lb_step<T, long long, 1>);
    else if (v == 2) go(k_lb_step<T, long long, 2>);
    else go(k_lb_step<T, long long, 3>);
  }
  return int(grid.x * grid.y * grid.z);
}

template <typename T>
void launch_lb_tail(const T* fsrc, T* fdst, const uint32_t* mask, const double* psi,
                    const LBParams& lp, const BeadTableView& bt, const int* origin, int n_beads,
                    double* partials, int first_block, int nblocks, Dims d, hipStream_t s,
                    const NoiseParams* noise, const WallView* walls) {
  const int blocks = lb_tail_blocks(n_beads);
  const size_t lds = (size_t)3 * n_beads * sizeof(int);   // at most 12 KiB (MAX_BEADS = 1024)
  const NoiseParams np = noise ? *noise : NoiseParams{};
  const WallView wv = walls ? *walls : WallView{};
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(BLOCK), lds, s, fsrc, fdst, mask, psi, lp, bt,
                       origin, n_beads, partials, first_block, nblocks, d, np, wv);
  };
  const int v = (noise ? 1 : 0) | (walls ? 2 : 0);
  if (fits_idx32<T>(d.n)) {
    if (v == 0) go(k_lb_tail<T, uint32_t, 0>);
    else if (v == 1) go(k_lb_tail<T, uint32_t, 1>);
    else if (v == 2) go(k_lb_tail<T, uint32_t, 2>);
    else go(k_lb_tail<T, uint32_t, 3>);
  } else {
    if (v == 0) go(k_lb_tail<T, long long, 0>);
    else if (v == 1) go(k_lb_tail<T, long long, 1>);
    else if (v == 2) go(k_lb_tail<T, long long, 2>);
    else go(k_lb_tail<T, long long, 3>);
  }
}

template <typename T>
void launch_moments(const T* f, const uint32_t* mask, int species, double nref, double* n_out,
                    double* u_out, Dims d, hipStream_t s) {
  const int blocks = int((d.n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_moments<T>, dim3(blocks), dim3(BLOCK), 0, s, f, mask, species, nref,
                     n_out, u_out, d);
}

void launch_defer_clear(uint32_t* mask, const int* origin, int n_beads, Dims d, hipStream_t s) {
  const int blocks = lb_tail_blocks(n_beads);
  hipLaunchKernelGGL(k_defer_clear, dim3(blocks), dim3(BLOCK), 0, s, mask, origin, n_beads, d);
}

#define EK_INST(T)                                                                          \
  template void launch_init_species<T>(T*, const uint32_t*, const double*, int, double, Dims, \
                                       hipStream_t);                                         \
  template int launch_lb_step<T>(const T*, T*, const uint32_t*, const double*,               \
                                 const LBParams&, const BeadTableView&, double*, int,        \
                                 uint32_t, Dims, const SiteGrid&, hipStream_t, hipEvent_t,   \
                                 hipEvent_t, const NoiseParams*, const WallView*);           \
  template void launch_lb_tail<T>(const T*, T*, const uint32_t*, const double*, const LBParams&,\
                                  const BeadTableView&, const int*, int, double*, int, int,  \
                                  Dims, hipStream_t, const NoiseParams*, const WallView*);   \
  template void launch_moments<T>(const T*, const uint32_t*, int, double, double*, double*,  \
                                  Dims, hipStream_t);
EK_INST(float)
EK_INST(double)

}  // namespace ek
