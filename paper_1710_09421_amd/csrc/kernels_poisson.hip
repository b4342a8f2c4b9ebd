// Poisson solver kernels: red-black SOR half sweeps with the Chebyshev
// schedule, residual norms in float64 with deterministic reductions, and the
// gauge fix (mean of psi removed).
//
// The stored right-hand side is b_raw = -rho_e / eps; the solver adds the
// device scalar `shift` = mean(rho_e) / eps, so that the problem it solves is
// A psi = -(rho_e - mean rho_e) / eps on the periodic box.
//
// Every kernel first reads the converged flag and returns at once when it is
// set: the host enqueues iterations ahead of the convergence test and the
// iterations past convergence do no work.
#include "ek_internal.h"
#include "reduce.h"

namespace ek {

namespace {

__global__ __launch_bounds__(BLOCK) void k_sor_half(double* __restrict__ psi,
                                                    const double* __restrict__ b,
                                                    const PoissonScalars* __restrict__ ps,
                                                    int colour, double omega, Dims d) {
  if (ps->done) return;
  const int tx = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (tx >= d.nx / 2 || y >= d.ny) return;
  const int x = 2 * tx + ((colour + y + z) & 1);   // (x + y + z) % 2 == colour
  const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const long long nxy = (long long)d.nx * d.ny;
  const long long row = z * nxy + (long long)y * d.nx;
  const long long r = row + x;
  const double nbsum = psi[row + xm] + psi[row + xp] + psi[z * nxy + (long long)ym * d.nx + x] +
                       psi[z * nxy + (long long)yp * d.nx + x] + psi[zm * nxy + (long long)y * d.nx + x] +
                       psi[zp * nxy + (long long)y * d.nx + x];
  const double rhs = b[r] + ps->shift;
  const double old = psi[r];
  psi[r] = old + omega * ((nbsum - rhs) * (1.0 / 6.0) - old);
}

// z planes per block of the residual: a thread sums the sites of a short
// column (more loads in flight, the z neighbours shared through the cache,
// a quarter of the block reductions and partials)
constexpr int RESIDUAL_PLANES = 4;

// Partial sums of r^2, b^2 and psi with r = b - A psi (7-point operator).
__global__ __launch_bounds__(BLOCK) void k_residual(const double* __restrict__ psi,
                                                    const double* __restrict__ b,
                                                    const PoissonScalars* __restrict__ ps,
                                                    double* __restrict__ partials, Dims d) {
  if (ps->done) return;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int nblocks = gridDim.x * gridDim.y * gridDim.z;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < RESIDUAL_PLANES; ++k) {
  const int z = blockIdx.z * RESIDUAL_PLANES + k;
  if (x < d.nx && y < d.ny && z < d.nz) {
    const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
    const long long nxy = (long long)d.nx * d.ny;
    const long long row = z * nxy + (long long)y * d.nx;
    const long long r = row + x;
    const double c = psi[r];
    const double lap = psi[row + xm] + psi[row + xp] + psi[z * nxy + (long long)ym * d.nx + x] +
                       psi[z * nxy + (long long)yp * d.nx + x] +
                       psi[zm * nxy + (long long)y * d.nx + x] +
                       psi[zp * nxy + (long long)y * d.nx + x] - 6.0 * c;
    const double rhs = b[r] + ps->shift;
    const double res = rhs - lap;
    acc[0] += res * res;
    acc[1] += rhs * rhs;
    acc[2] += c;
  }
  }
  block_partials<3>(acc, partials, bid, nblocks);
}

// The same sums marching up z: a workgroup owns a RZ_TX x RZ_TY tile of zc
// planes and keeps three planes of the tile and a one-site ring in LDS (a
// fourth receives the plane after them), so psi and b are read once from
// memory (the rings and the planes either side of a chunk again by the
// neighbouring workgroups, mostly from the cache).  Each thread adds its
// sites' terms in plane order; block_partials combines the threads.  The
// loads are issued a step ahead and without branches (indexes past the end
// are clamped, their values never used), so the compiler waits only for the
// load in use.
constexpr int RZ_TX = 64, RZ_TY = 8, RZ_THREADS = 256;

template <int TX, int TY>
__global__ __launch_bounds__(RZ_THREADS) void k_residual_z(const double* __restrict__ psi,
                                                           const double* __restrict__ b,
                                                           const PoissonScalars* __restrict__ ps,
                                                           double* __restrict__ partials, Dims d,
                                                           int zc) {
  constexpr int RX = TX + 2, RY = TY + 2, REGION = RX * RY;
  constexpr int XPT = (REGION + RZ_THREADS - 1) / RZ_THREADS;
  constexpr int SPT = TX * TY / RZ_THREADS;
  static_assert((TX * TY) % RZ_THREADS == 0, "whole tiles per thread");
  struct Regs {
    double x[XPT];   // a psi plane (tile and ring), to be stored in LDS
    double b[SPT];   // b at this thread's tile sites of a plane
  };
  __shared__ double P[4][RY][RX];
  if (ps->done) return;
  const double shift = ps->shift;
  const int nx = d.nx, ny = d.ny, nz = d.nz, tid = threadIdx.x;
  // workgroup -> (tile, chunk), neighbouring tiles of a chunk on one XCD
  const int ntx = nx / TX, nty = ny / TY, nblk = gridDim.x;
  int bb = blockIdx.x;
  if ((nblk & 7) == 0) bb = (bb & 7) * (nblk >> 3) + (bb >> 3);
  const int tx_i = bb % ntx, rest = bb / ntx, ty_i = rest % nty, chunk = rest / nty;
  const int x0 = tx_i * TX, y0 = ty_i * TY, z0 = chunk * zc, z1 = z0 + zc;
  auto wrapi = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  auto plane_base = [&](int q) {
    int zq = q % nz;
    if (zq < 0) zq += nz;
    return (long long)zq * ny * nx;
  };
  auto slot = [&](int q) { return (q - z0 + 1) & 3; };
  auto gather_x = [&](int q, double (&r)[XPT]) {
    const long long base = plane_base(q);
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int t = min(tid + u * RZ_THREADS, REGION - 1);
      const int j = t / RX, i = t - j * RX;
      r[u] = psi[base + (long long)wrapi(y0 - 1 + j, ny) * nx + wrapi(x0 - 1 + i, nx)];
    }
  };
  auto store_x = [&](int sl, const double (&r)[XPT]) {
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int t = tid + u * RZ_THREADS;
      if (t < REGION) {
        const int j = t / RX, i = t - j * RX;
        P[sl][j][i] = r[u];
      }
    }
  };
  auto gather_b = [&](int k, double (&r)[SPT]) {
    const long long base = plane_base(k);
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int t = tid + u * RZ_THREADS;
      const int jj = t / TX, ii = t - jj * TX;
      r[u] = b[base + (long long)(y0 + jj) * nx + x0 + ii];
    }
  };
  double acc[3] = {0.0, 0.0, 0.0};
  // step k: the residual of plane k (planes k-1, k, k+1 in LDS, b of plane k
  // in cur); nxt receives plane k+3 (stored at the end of step k+1) and b of
  // plane k+1
  auto step = [&](int k, Regs& cur, Regs& nxt) {
    gather_x(min(k + 3, z1), nxt.x);
    gather_b(min(k + 1, z1 - 1), nxt.b);
    const int s0 = slot(k), sm = slot(k - 1), sp = slot(k + 1);
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int t = tid + u * RZ_THREADS;
      const int j = 1 + t / TX, i = 1 + t % TX;
      const double c = P[s0][j][i];
      const double lap = P[s0][j][i - 1] + P[s0][j][i + 1] + P[s0][j - 1][i] + P[s0][j + 1][i] +
                         P[sm][j][i] + P[sp][j][i] - 6.0 * c;
      const double rhs = cur.b[u] + shift;
      const double res = rhs - lap;
      acc[0] += res * res;
      acc[1] += rhs * rhs;
      acc[2] += c;
    }
    if (k + 2 <= z1) store_x(slot(k + 2), cur.x);
    __syncthreads();
  };
  Regs A, B;
  for (int q = z0 - 1; q <= z0 + 1; ++q) {
    gather_x(q, A.x);
    store_x(slot(q), A.x);
  }
  gather_x(min(z0 + 2, z1), A.x);
  gather_b(z0, A.b);
  __syncthreads();
  int k = z0;
  for (; k + 1 < z1; k += 2) {
    step(k, A, B);
    step(k + 1, B, A);
  }
  if (k < z1) step(k, A, B);
  block_partials<3>(acc, partials, blockIdx.x, gridDim.x);
}

// Chunk height of the z-marching residual, or 0 where its tile does not
// divide the lattice or it would give fewer than 512 workgroups.
int residual_zc(const Dims& d) {
  if (d.nx % RZ_TX || d.ny % RZ_TY) return 0;
  const long long tiles = (long long)(d.nx / RZ_TX) * (d.ny / RZ_TY);
  int zc = d.nz;
  while (zc % 2 == 0 && zc / 2 >= 8 && tiles * (d.nz / zc) < 1024) zc /= 2;
  return tiles * (d.nz / zc) >= 512 ? zc : 0;
}

__global__ __launch_bounds__(1024) void k_residual_final(const double* __restrict__ partials,
                                                         int nblocks, double tol, int iter,
                                                         int initial, PoissonScalars* ps) {
  if (ps->done) return;
  double t[3];
  block_sums_1024<3>(partials, nblocks, t);
  if (threadIdx.x == 0) {
    if (iter < 0) iter = ps->cycles;   // counted on the device (replayed launches)
    const double r2 = t[0], b2 = t[1];
    double rel;
    if (b2 > 0.0) rel = sqrt(r2 / b2);
    else rel = r2 == 0.0 ? 0.0 : INFINITY;
    ps->r2 = r2;
    ps->b2 = b2;
    ps->psum = t[2];
    ps->rel = rel;
    if (initial) ps->rel0 = rel;
    if (b2 == 0.0) {
      ps->zero_rhs = 1;
      ps->done = 1;
      ps->iters = iter;
    } else if (rel <= tol) {
      ps->done = 1;
      ps->iters = iter;
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_psi_shift(double* __restrict__ psi,
                                                     const PoissonScalars* __restrict__ ps,
                                                     double inv_n, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  psi[r] = mean_removed(psi[r], ps, inv_n);
}

__global__ __launch_bounds__(BLOCK) void k_fill(double* __restrict__ x, double v, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) x[r] = v;
}


__global__ __launch_bounds__(BLOCK) void k_rho_to_b(const double* __restrict__ rho,
                                                    double* __restrict__ b,
                                                    double* __restrict__ partials,
                                                    double inv_eps, Dims d) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int nblocks = gridDim.x * gridDim.y * gridDim.z;
  double acc[1] = {0.0};
  if (x < d.nx && y < d.ny) {
    const long long r = ((long long)z * d.ny + y) * d.nx + x;
    const double v = rho[r];
    b[r] = -v * inv_eps;
    acc[0] = v;
  }
  block_partials<1>(acc, partials, bid, nblocks);
}

// ---------------------------------------------------------------------------
// Insulating walls: the operator over the fluid sites only.  Bits 1..6 of the
// link word mark the solid face neighbours (bit p: the site r - c_p is
// solid): bit 1 the -x neighbour, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z.  The walls'
// surface charge is in b already (charge pass), so a solid face simply
// drops out of the sum; b + shift is the right-hand side at fluid sites.
// ---------------------------------------------------------------------------
struct FaceNbrs {
  long long xm, xp, ym, yp, zm, zp;
};

__device__ inline FaceNbrs face_nbrs(int x, int y, int z, const Dims& d) {
  const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const long long nxy = (long long)d.nx * d.ny;
  const long long row = z * nxy + (long long)y * d.nx;
  return FaceNbrs{row + xm, row + xp, z * nxy + (long long)ym * d.nx + x,
                  z * nxy + (long long)yp * d.nx + x, zm * nxy + (long long)y * d.nx + x,
                  zp * nxy + (long long)y * d.nx + x};
}

// Sum of psi over the fluid face neighbours and their number.
__device__ inline double open_sum(const double* __restrict__ psi, uint32_t m, const FaceNbrs& n,
                                  int& k) {
  double s = 0.0;
  k = 0;
  if (!(m & (1u << 1))) { s += psi[n.xm]; ++k; }
  if (!(m & (1u << 2))) { s += psi[n.xp]; ++k; }
  if (!(m & (1u << 3))) { s += psi[n.ym]; ++k; }
  if (!(m & (1u << 4))) { s += psi[n.yp]; ++k; }
  if (!(m & (1u << 5))) { s += psi[n.zm]; ++k; }
  if (!(m & (1u << 6))) { s += psi[n.zp]; ++k; }
  return s;
}

__global__ __launch_bounds__(BLOCK) void k_sor_half_neu(double* __restrict__ psi,
                                                        const double* __restrict__ b,
                                                        const uint32_t* __restrict__ mask,
                                                        const PoissonScalars* __restrict__ ps,
                                                        int colour, double omega, Dims d) {
  if (ps->done) return;
  const int tx = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (tx >= d.nx / 2 || y >= d.ny) return;
  const int x = 2 * tx + ((colour + y + z) & 1);
  const long long r = ((long long)z * d.ny + y) * d.nx + x;
  const uint32_t m = mask[r];
  if (m & MASK_SOLID) return;
  int k;
  const double nbsum = open_sum(psi, m, face_nbrs(x, y, z, d), k);
  const double rhs = b[r] + ps->shift;
  const double old = psi[r];
  psi[r] = old + omega * ((nbsum - rhs) / double(k) - old);
}

// Partial sums of r^2, b^2 and psi over the fluid sites, r = b - A_N psi.
__global__ __launch_bounds__(BLOCK) void k_residual_neu(const double* __restrict__ psi,
                                                        const double* __restrict__ b,
                                                        const uint32_t* __restrict__ mask,
                                                        const PoissonScalars* __restrict__ ps,
                                                        double* __restrict__ partials, Dims d) {
  if (ps->done) return;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int nblocks = gridDim.x * gridDim.y * gridDim.z;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int kz = 0; kz < RESIDUAL_PLANES; ++kz) {
    const int z = blockIdx.z * RESIDUAL_PLANES + kz;
    if (x < d.nx && y < d.ny && z < d.nz) {
      const long long r = ((long long)z * d.ny + y) * d.nx + x;
      const uint32_t m = mask[r];
      if (!(m & MASK_SOLID)) {
        int k;
        const double c = psi[r];
        const double lap = open_sum(psi, m, face_nbrs(x, y, z, d), k) - double(k) * c;
        const double rhs = b[r] + ps->shift;
        const double res = rhs - lap;
        acc[0] += res * res;
        acc[1] += rhs * rhs;
        acc[2] += c;
      }
    }
  }
  block_partials<3>(acc, partials, bid, nblocks);
}

// psi - (fluid mean of psi) at fluid sites, 0 at solid sites.
__global__ __launch_bounds__(BLOCK) void k_psi_shift_neu(double* __restrict__ psi,
                                                         const uint32_t* __restrict__ mask,
                                                         const PoissonScalars* __restrict__ ps,
                                                         double inv_nf, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  psi[r] = (ps->zero_rhs || (mask[r] & MASK_SOLID)) ? 0.0 : psi[r] - ps->psum * inv_nf;
}

}  // namespace

void launch_sor_half_neu(double* psi, const double* b, const uint32_t* mask,
                         const PoissonScalars* ps, int colour, double omega, Dims d,
                         const SiteGrid& g, hipStream_t s) {
  hipLaunchKernelGGL(k_sor_half_neu, g.grid, g.block, 0, s, psi, b, mask, ps, colour, omega, d);
}

int launch_residual_neu(const double* psi, const double* b, const uint32_t* mask,
                        PoissonScalars* ps, double* partials, Dims d, const SiteGrid& g,
                        hipStream_t s) {
  dim3 grid = g.grid;
  grid.z = (d.nz + RESIDUAL_PLANES - 1) / RESIDUAL_PLANES;
  hipLaunchKernelGGL(k_residual_neu, grid, g.block, 0, s, psi, b, mask, ps, partials, d);
  return int(grid.x * grid.y * grid.z);
}

void launch_psi_shift_neu(double* psi, const uint32_t* mask, const PoissonScalars* ps,
                          double inv_nf, Dims d, hipStream_t s) {
  const int blocks = int((d.n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_psi_shift_neu, dim3(blocks), dim3(BLOCK), 0, s, psi, mask, ps, inv_nf, d.n);
}

void launch_sor_half(double* psi, const double* b, const PoissonScalars* ps, int colour,
                     double omega, Dims d, const SiteGrid& g, hipStream_t s) {
  hipLaunchKernelGGL(k_sor_half, g.grid, g.block, 0, s, psi, b, ps, colour, omega, d);
}

int residual_blocks(const Dims& d, const SiteGrid& g) {
  if (const int zc = residual_zc(d)) return (d.nx / RZ_TX) * (d.ny / RZ_TY) * (d.nz / zc);
  return int(g.grid.x * g.grid.y * ((d.nz + RESIDUAL_PLANES - 1) / RESIDUAL_PLANES));
}

int launch_residual(const double* psi, const double* b, PoissonScalars* ps, double* partials,
                    Dims d, const SiteGrid& g, hipStream_t s) {
  const int nblocks = residual_blocks(d, g);
  if (const int zc = residual_zc(d)) {
    hipLaunchKernelGGL((k_residual_z<RZ_TX, RZ_TY>), dim3(nblocks), dim3(RZ_THREADS), 0, s, psi, b,
                       ps, partials, d, zc);
    return nblocks;
  }
  dim3 grid = g.grid;
  grid.z = (d.nz + RESIDUAL_PLANES - 1) / RESIDUAL_PLANES;
  hipLaunchKernelGGL(k_residual, grid, g.block, 0, s, psi, b, ps, partials, d);
  return nblocks;
}

void launch_residual_final(const double* partials, int nblocks, double tol, int iter,
                           int initial, PoissonScalars* ps, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(1024), 0, s, partials, nblocks, tol, iter,
                     initial, ps);
}

void launch_psi_shift(double* psi, const PoissonScalars* ps, double inv_n, Dims d,
                      hipStream_t s) {
  const int blocks = int((d.n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_psi_shift, dim3(blocks), dim3(BLOCK), 0, s, psi, ps, inv_n, d.n);
}

void launch_fill(double* x, double v, long long n, hipStream_t s) {
  const int blocks = int((n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(BLOCK), 0, s, x, v, n);
}

void launch_rho_to_b(const double* rho, double* b, double* partials, double inv_eps, Dims d,
                     const SiteGrid& g, hipStream_t s) {
  hipLaunchKernelGGL(k_rho_to_b, g.grid, g.block, 0, s, rho, b, partials, inv_eps, d);
}

}  // namespace ek

namespace ek {
namespace {
__global__ void k_ps_reset(PoissonScalars* ps, double shift) {
  if (threadIdx.x == 0) {
    ps->shift = shift;
    ps->r2 = ps->b2 = ps->psum = 0.0;
    ps->rel = ps->rel0 = 0.0;
    ps->done = 0;
    ps->iters = 0;
    ps->zero_rhs = 0;
    ps->cycles = 0;
  }
}
// Clears the convergence flags before the residual of another start is
// evaluated; the right-hand-side shift stays.
__global__ void k_ps_rearm(PoissonScalars* ps) {
  if (threadIdx.x == 0) {
    ps->done = 0;
    ps->iters = 0;
    ps->zero_rhs = 0;
    ps->cycles = 0;
  }
}

// out = b + shift: the right-hand side of the last solve with its mean removed
__global__ __launch_bounds__(BLOCK) void k_rhs_copy(const double* __restrict__ b,
                                                    const PoissonScalars* __restrict__ ps,
                                                    double* __restrict__ out, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = b[r] + ps->shift;
}
}  // namespace
void launch_ps_rearm(PoissonScalars* ps, hipStream_t s) {
  hipLaunchKernelGGL(k_ps_rearm, dim3(1), dim3(64), 0, s, ps);
}
void launch_rhs_copy(const double* b, const PoissonScalars* ps, double* out, long long n,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_copy, dim3(int((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, b, ps, out, n);
}
void launch_ps_reset(PoissonScalars* ps, double shift, hipStream_t s) {
  hipLaunchKernelGGL(k_ps_reset, dim3(1), dim3(64), 0, s, ps, shift);
}
}  // namespace ek
