// Red-black multigrid for the periodic Poisson problem A psi = b.
//
// Not a method of the paper (which uses SOR with Chebyshev acceleration): a
// solver for the same discrete problem, used to finish the solve faster on
// large boxes.  Cell-centred hierarchy on the periodic box, each level half
// the previous in every direction while all sides stay even:
//   level l, spacing h = 2^l:  (sum of 6 neighbours - 6 x) / h^2 = f_l
//   smoother   red-black Gauss-Seidel (x = (sum nb - h^2 f) / 6) over-relaxed
//              by MG_OMEGA (MG_OMEGA_FINEST in the z-marching sweeps of the
//              finest level), nu1 = NU1 = 1 and nu2 = NU2 = 2 (on the finest
//              level NU1_FUSED in the first cycle of a solve and
//              NU1_FUSED_NEXT in the later ones where its last
//              pre-smoothing sweep restricts, NU1_FINEST and
//              NU1_FINEST_NEXT where it has no z-marching sweeps;
//              NU2_COARSE = 1 on the levels of the one-workgroup coarse
//              kernel)
//   restriction  f_{l+1} = average of the 8 fine residuals (fused with the
//                residual, also zeroes the coarse iterate)
//   prolongation trilinear cell-centred interpolation (weights 3/4, 1/4 per
//                axis) added to the fine iterate
// A level is halved only while every side stays even (red-black colouring
// needs even periodic sides).  The coarsest levels whose iterates and
// right-hand sides fit in COARSE_LDS_BYTES of LDS run inside one workgroup
// (one launch for the whole coarse part of the cycle); a coarsest level of at
// most COARSEST_DIRECT_MAX sites is solved directly, a larger one gets
// red-black SOR sweeps at the optimal relaxation factor of that grid,
// enough of them to reduce its error by COARSEST_REDUCTION (a cycle reduces
// the residual by about 1e-2, so a coarsest solve to 1e-3 leaves the cycle's
// rate unchanged; a box that cannot be coarsened is solved by these sweeps
// alone, each "cycle" then reducing its error by 1e-10; a coarsest level
// too large for one workgroup's LDS gets those sweeps as grid-wide
// launches).  Level 0 is the context's psi and b (b
// plus the scalar shift that removes the mean charge).  The launches of one
// cycle are recorded once as a graph and replayed (see ek_ctx::MG).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ek_context.h"
#include "mg_site.h"
#include "reduce.h"

using namespace ek;

namespace {

constexpr size_t COARSE_LDS_BYTES = 40 * 1024;    // one-workgroup coarse cycle: levels of up to ~2k sites
constexpr int COARSEST_SWEEPS = 40;
constexpr double COARSEST_REDUCTION = 1e-3;
// A coarsest level of at most this many sites is solved directly (one
// matrix-vector product with a precomputed inverse, instead of SOR sweeps).
constexpr int COARSEST_DIRECT_MAX = 64;
// Levels of at most this many sites take the coarse-grid correction inside
// their first post-smoothing sweep; that sweep reads the coarse iterate about
// seven times per site, which pays while the level is launch-bound and costs
// more than the separate prolongation pass on large levels (measured: 2^18
// beat 2^21 and 2^23 on 64x64x128 and 256x256x512 boxes; fusing the
// 2^25-site level of the latter made its Poisson solve 13 % slower).
constexpr long long FUSED_CORRECTION_MAX_SITES = 1ll << 18;
// Post-smoothing sweeps on the levels inside the one-workgroup coarse kernel,
// whose barrier phases on a 1k-site level are bound by LDS bandwidth: one
// sweep there left the cycle counts of the pore systems from the
// extrapolated start unchanged (64x64x128 and 256x256x512) and took 2 % off
// the 64x64x128 pore's step; from the previous solution it needed about 3 %
// more cycles, which cancels the gain.
constexpr int NU2_COARSE = 1;
// Pre-smoothing sweeps on a finest level whose last pre-smoothing sweep also
// restricts (k_sweep_zr), in the first cycle of a solve and in the later
// ones: with the over-relaxed sweeps a V(1,2) cycle there reduces the
// residual about 45-fold, so the 1e-8 of the pore systems from the quadratic
// start (1e-5 to 1e-4) takes three such cycles; three pre-smoothing sweeps
// in every cycle made it two (256x256x512: 2.94 -> 2.00 cycles per step,
// 3.16 -> 3.00 ms of Poisson; two gave 2.31 cycles and the same time), and
// the later cycles, which start far closer, need only the one (2.18 cycles,
// 2.57 -> 2.37 ms; two there: 2.02 cycles, 2.41 ms; none, a plain
// restriction: 2.89 cycles, 2.72 ms; four or five in the first cycle:
// 2.47 / 2.64 ms).
constexpr int NU1_FUSED = 3;
constexpr int NU1_FUSED_NEXT = 1;
// Relaxation factor of the z-marching sweeps on the finest level (the other
// levels keep MG_OMEGA): with the cycle counts above the 256x256x512 pore
// takes 2.02 cycles and 2.22 ms of Poisson per step at 1.2, against 2.18
// cycles and 2.36 ms at 1.25, 2.21 / 2.25 ms at 1.18 / 1.22, 2.23 ms at 1.15
// and 2.66 ms at 1.1, 2.23 ms with level 1's z-marching sweeps at 1.2 too
// (400 steps; 1.25 in the first cycle and 1.2 in the later ones: 2.28 ms,
// the reverse splits 2.21 ms).  The box sweeps of a smaller finest level keep
// MG_OMEGA (the 64x64x128 pore: 0.264 against 0.261 ms at 1.2).
constexpr double MG_OMEGA_FINEST = 1.2;
// Pre-smoothing sweeps on a finest level too small for the z-marching sweeps
// (one launch per full sweep on BOX^3 tiles), in the first cycle of a solve
// and in the later ones: the 64x64x128 pore's solve from the cubic
// start took 3.17 cycles per step with two in every cycle, 2.64 with four,
// at 0.313 and 0.307 ms of Poisson per step; from the quadratic start four
// in the first cycle and two in the later ones took 2.66 cycles and 0.278
// against 0.290 ms (six and two: 0.276 ms; none in the later ones: 0.313;
// with the 512-thread box sweeps four, six and eight in the first cycle all
// take 0.260 ms at 2.66 / 2.47 / 2.31 cycles)
// (with half sweeps, from the quadratic start: 3.71 cycles with one, 3.02
// with two, 0.38 -> 0.34 ms).
constexpr int NU1_FINEST = 4;
constexpr int NU1_FINEST_NEXT = 2;
// A solve tests its residual from one cycle before the previous solve's count
// on, unless the previous solve was this far above the tolerance one cycle
// before its end (256x256x512 pore: 2.37 ms of Poisson per step at 4 and at
// 8, 2.41 at 2).
constexpr double EARLY_MARGIN = 4.0;

// --- grid-wide kernels for the fine levels (3-D launch: x, y from the block,
// z = blockIdx.z, so no index division) ------------------------------------
__global__ __launch_bounds__(256) void k_smooth(Lvl L, int colour, const PoissonScalars* ps,
                                                int level0, double omega) {
  if (ps->done) return;
  const int tx = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (tx >= L.nx / 2 || y >= L.ny) return;
  smooth_site(L, colour, tx, y, blockIdx.z, level0 ? ps->shift : 0.0, omega);
}

__global__ __launch_bounds__(256) void k_restrict(Lvl F, Lvl C, const PoissonScalars* ps,
                                                  int level0, double omega_red) {
  if (ps->done) return;
  const int X = blockIdx.x * blockDim.x + threadIdx.x;
  const int Y = blockIdx.y * blockDim.y + threadIdx.y;
  if (X >= C.nx || Y >= C.ny) return;
  restrict_site(F, C, X, Y, blockIdx.z, level0 ? ps->shift : 0.0, omega_red);
}

// Prolongation fused into the first post-smoothing sweep (colour 0, then 1).
__global__ __launch_bounds__(256) void k_corrected_smooth(Lvl L, Lvl C, int colour,
                                                          const PoissonScalars* ps, int level0,
                                                          double omega) {
  if (ps->done) return;
  const int tx = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (tx >= L.nx / 2 || y >= L.ny) return;
  corrected_smooth_site(L, C, colour, tx, y, blockIdx.z, level0 ? ps->shift : 0.0, omega);
}

// One thread per coarse cell (launched over the coarse level).
__global__ __launch_bounds__(256) void k_prolong(Lvl F, Lvl C, const PoissonScalars* ps) {
  if (ps->done) return;
  const int X = blockIdx.x * blockDim.x + threadIdx.x;
  const int Y = blockIdx.y * blockDim.y + threadIdx.y;
  if (X >= C.nx || Y >= C.ny) return;
  prolong_cell(F, C, X, Y, blockIdx.z);
}

// Out-of-place prolongation: dst = src + P e over the 8 children of a coarse
// cell (the finest level, whose pre-smoothed iterate is in the sweep buffer).
__global__ __launch_bounds__(256) void k_prolong_to(Lvl F, Lvl C, const double* src, double* dst,
                                                    const PoissonScalars* ps) {
  if (ps->done) return;
  const int X = blockIdx.x * blockDim.x + threadIdx.x;
  const int Y = blockIdx.y * blockDim.y + threadIdx.y;
  if (X >= C.nx || Y >= C.ny) return;
  prolong_cell(F, C, X, Y, blockIdx.z, src, dst);
}

// --- one full red-black sweep per launch on BOX^3 tiles (small levels) --------
// xout = (colour-0 half sweep, then colour-1 half sweep)(xin), out of place,
// for levels too small for the z-marching sweeps below, whose every launch
// costs about the same few microseconds whatever its size: one launch per
// sweep instead of two.  A workgroup loads its BOX^3 tile of xin with a
// two-site ring, and the right-hand side with a one-site ring, into LDS,
// relaxes the colour-0 sites of the tile and of a one-site ring around it
// (the ring's sites are relaxed again by the neighbouring workgroups, from
// the same old values in the same order), then the colour-1 sites of the
// tile, and writes the tile.  The formula and summation order are those of
// smooth_site.  With CORR the sweep is the first post-smoothing sweep of a
// cycle: every loaded iterate value first gets the trilinear coarse-grid
// correction of level C (prolong_value's weights and order, from a coarse
// window in LDS), so the launch is a prolongation followed by the sweep.
// With NIN it also takes the residual norms of its input (the start of a
// solve, in the first cycle's first sweep) at the tile's sites, from the
// windows before the sweep: block partials of r^2, (f + shift)^2 and xin as
// k_residual's.  BOX divides nx, ny and nz.
constexpr int BOX = 8;
constexpr int BOX_X = BOX + 4;        // iterate window side (two-site ring)
constexpr int BOX_F = BOX + 2;        // right-hand side window side
constexpr int BOX_C = BOX / 2 + 4;    // coarse window side
// 512 threads per workgroup (at most one or two sites per thread and
// phase): the 64x64x128 pore's solve takes 0.259 ms per step against 0.268
// with 256, 0.272 with 1024 and 0.309 with 128
constexpr int BOX_THREADS = 512;

__device__ inline int wrap_index(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Tile of workgroup b among n: workgroups are dispatched to the eight XCDs in
// turn, so with n a multiple of 8 XCD k takes the k-th eighth of the tiles
// (numbered x fastest, then y, then z: whole z-slabs), whose windows overlap
// in its own L2.
__device__ inline int box_tile(int b, int n) { return (n & 7) ? b : (b & 7) * (n >> 3) + (b >> 3); }

template <bool CORR, bool NIN = false>
__global__ __launch_bounds__(BOX_THREADS) void k_sweep_box(Lvl L, const double* __restrict__ xin,
                                                           double* __restrict__ xout,
                                                           const PoissonScalars* ps, int level0,
                                                           double omega, Lvl C,
                                                           double* __restrict__ partials) {
  static_assert(!(CORR && NIN), "the input norms belong to a pre-smoothing sweep");
  __shared__ double sx[BOX_X * BOX_X * BOX_X];
  __shared__ double sf[BOX_F * BOX_F * BOX_F];
  __shared__ double sc[CORR ? BOX_C * BOX_C * BOX_C : 1];
  const int tiles_x = L.nx / BOX, tiles_y = L.ny / BOX;
  const int b = box_tile(blockIdx.x, gridDim.x);
  const int bxy = b % (tiles_x * tiles_y);
  const int x0 = (bxy % tiles_x) * BOX, y0 = (bxy / tiles_x) * BOX;
  const int z0 = (b / (tiles_x * tiles_y)) * BOX;
  // window coordinate i of a side starts at x0 - 2 (iterate), x0 - 1
  // (right-hand side) and x0 / 2 - 2 (coarse).  Every load of the windows is
  // issued before the first of them is stored (branch-free: a thread past a
  // window's end reloads its last site and stores nothing), so the
  // workgroup waits for memory once; the test of a finished solve is taken
  // after the loads are on their way.
  constexpr int NX = BOX_X * BOX_X * BOX_X, NF = BOX_F * BOX_F * BOX_F;
  constexpr int NC = CORR ? BOX_C * BOX_C * BOX_C : 1;
  constexpr int PX = (NX + BOX_THREADS - 1) / BOX_THREADS, PF = (NF + BOX_THREADS - 1) / BOX_THREADS;
  constexpr int PC = (NC + BOX_THREADS - 1) / BOX_THREADS;
  double vx[PX], vf[PF], vc[PC];
#pragma unroll
  for (int q = 0; q < PX; ++q) {
    const int t = min((int)threadIdx.x + q * BOX_THREADS, NX - 1);
    const int i = t % BOX_X, j = (t / BOX_X) % BOX_X, k = t / (BOX_X * BOX_X);
    vx[q] = xin[idx3(wrap_index(x0 - 2 + i, L.nx), wrap_index(y0 - 2 + j, L.ny),
                     wrap_index(z0 - 2 + k, L.nz), L)];
  }
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const int t = min((int)threadIdx.x + q * BOX_THREADS, NF - 1);
    const int i = t % BOX_F, j = (t / BOX_F) % BOX_F, k = t / (BOX_F * BOX_F);
    vf[q] = L.f[idx3(wrap_index(x0 - 1 + i, L.nx), wrap_index(y0 - 1 + j, L.ny),
                     wrap_index(z0 - 1 + k, L.nz), L)];
  }
  if (CORR) {
    const int X0 = x0 / 2 - 2, Y0 = y0 / 2 - 2, Z0 = z0 / 2 - 2;
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const int t = min((int)threadIdx.x + q * BOX_THREADS, NC - 1);
      const int i = t % BOX_C, j = (t / BOX_C) % BOX_C, k = t / (BOX_C * BOX_C);
      vc[q] = C.x[idx3(wrap_index(X0 + i, C.nx), wrap_index(Y0 + j, C.ny),
                       wrap_index(Z0 + k, C.nz), C)];
    }
  }
  if (ps->done) return;
  const double shift = level0 ? ps->shift : 0.0;
#pragma unroll
  for (int q = 0; q < PX; ++q) {
    const int t = (int)threadIdx.x + q * BOX_THREADS;
    if (t < NX) sx[t] = vx[q];
  }
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const int t = (int)threadIdx.x + q * BOX_THREADS;
    if (t < NF) sf[t] = vf[q] + shift;
  }
  if (CORR) {
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const int t = (int)threadIdx.x + q * BOX_THREADS;
      if (t < NC) sc[t] = vc[q];
    }
  }
  __syncthreads();
  if (CORR) {
    // fine window site i lies at x0 - 2 + i (an even x0: the parity of i),
    // in coarse cell x0 / 2 - 1 + (i >> 1), window column 1 + (i >> 1); its
    // second cell is the next one for an odd site, the previous for an even
    constexpr int CS = BOX_C, CS2 = BOX_C * BOX_C;
    const double a = 0.75, bb = 0.25;
    for (int t = threadIdx.x; t < BOX_X * BOX_X * BOX_X; t += BOX_THREADS) {
      const int i = t % BOX_X, j = (t / BOX_X) % BOX_X, k = t / (BOX_X * BOX_X);
      const int X = 1 + (i >> 1), Y = 1 + (j >> 1), Z = 1 + (k >> 1);
      const int Xn = (i & 1) ? X + 1 : X - 1, Yn = (j & 1) ? Y + 1 : Y - 1;
      const int Zn = (k & 1) ? Z + 1 : Z - 1;
      const double e = a * a * a * sc[Z * CS2 + Y * CS + X] + bb * a * a * sc[Z * CS2 + Y * CS + Xn] +
                       a * bb * a * sc[Z * CS2 + Yn * CS + X] + a * a * bb * sc[Zn * CS2 + Y * CS + X] +
                       bb * bb * a * sc[Z * CS2 + Yn * CS + Xn] +
                       bb * a * bb * sc[Zn * CS2 + Y * CS + Xn] +
                       a * bb * bb * sc[Zn * CS2 + Yn * CS + X] +
                       bb * bb * bb * sc[Zn * CS2 + Yn * CS + Xn];
      sx[t] = sx[t] + e;
    }
    __syncthreads();
  }
  constexpr int SX = BOX_X, SX2 = BOX_X * BOX_X;
  const double h2 = L.h2;
  if constexpr (NIN) {
    const double ih2 = 1.0 / h2;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < BOX * BOX * BOX; t += BOX_THREADS) {
      const int i = 2 + t % BOX, j = 2 + (t / BOX) % BOX, k = 2 + t / (BOX * BOX);
      const int w = (k * SX + j) * SX + i;
      const double c = sx[w];
      const double nb = sx[w - 1] + sx[w + 1] + sx[w - SX] + sx[w + SX] + sx[w - SX2] + sx[w + SX2];
      const double rhs = sf[((k - 1) * BOX_F + (j - 1)) * BOX_F + (i - 1)];
      const double res = rhs - (nb - 6.0 * c) * ih2;
      acc[0] += res * res;
      acc[1] += rhs * rhs;
      acc[2] += c;
    }
    block_partials<3>(acc, partials, blockIdx.x, gridDim.x);   // its barrier orders the reads
  }
  // colour 0 ((x + y + z) even; x0, y0, z0 are even, so i + j + k even) on
  // the window's sites 1 .. BOX + 2 of every side: BOX / 2 + 1 per row
  constexpr int RROW = BOX / 2 + 1, RSIDE = BOX + 2;
  for (int t = threadIdx.x; t < RROW * RSIDE * RSIDE; t += BOX_THREADS) {
    const int r = t / RROW;
    const int j = 1 + r % RSIDE, k = 1 + r / RSIDE;
    const int i = 1 + 2 * (t % RROW) + ((1 + j + k) & 1);
    const int w = (k * SX + j) * SX + i;
    const double xo = sx[w];
    const double nb = sx[w - 1] + sx[w + 1] + sx[w - SX] + sx[w + SX] + sx[w - SX2] + sx[w + SX2];
    const double gs = (nb - h2 * sf[((k - 1) * BOX_F + (j - 1)) * BOX_F + (i - 1)]) * (1.0 / 6.0);
    sx[w] = omega == 1.0 ? gs : xo + omega * (gs - xo);
  }
  __syncthreads();
  // colour 1 on the tile (window sites 2 .. BOX + 1): BOX / 2 per row
  constexpr int BROW = BOX / 2;
  for (int t = threadIdx.x; t < BROW * BOX * BOX; t += BOX_THREADS) {
    const int r = t / BROW;
    const int j = 2 + r % BOX, k = 2 + r / BOX;
    const int i = 2 + 2 * (t % BROW) + ((j + k + 1) & 1);
    const int w = (k * SX + j) * SX + i;
    const double xo = sx[w];
    const double nb = sx[w - 1] + sx[w + 1] + sx[w - SX] + sx[w + SX] + sx[w - SX2] + sx[w + SX2];
    const double gs = (nb - h2 * sf[((k - 1) * BOX_F + (j - 1)) * BOX_F + (i - 1)]) * (1.0 / 6.0);
    sx[w] = omega == 1.0 ? gs : xo + omega * (gs - xo);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < BOX * BOX * BOX; t += BOX_THREADS) {
    const int i = t % BOX, j = (t / BOX) % BOX, k = t / (BOX * BOX);
    xout[idx3(x0 + i, y0 + j, z0 + k, L)] = sx[((k + 2) * SX + (j + 2)) * SX + (i + 2)];
  }
}

// The pre-smoothing of a coarser level with the restriction to the next in
// one launch: the level F arrives from the restriction with its colour-0 half
// sweep done and its colour-1 sites at zero, so its single pre-smoothing
// sweep is the colour-1 half sweep from that zero start (omega (gs - 0)).  A
// workgroup loads the colour-0 sites of its BOX^3 tile of F with a two-site
// ring, and f with a one-site ring, into LDS, relaxes the colour-1 sites of
// the tile and of a one-site ring around it (the ring again by the
// neighbouring workgroups alike), takes the residual at the tile's sites
// and restricts it into the (BOX/2)^3 cells of level C below the tile, as
// restrict_site (with the first colour-0 half sweep of C when omega_red is
// not zero), and writes the tile's colour-1 sites in place: it reads only
// colour-0 sites of F, which no workgroup writes.
__global__ __launch_bounds__(BOX_THREADS) void k_restrict_box(Lvl F, Lvl C,
                                                              const PoissonScalars* ps,
                                                              double omega, double omega_red) {
  __shared__ double sx[BOX_X * BOX_X * BOX_X];
  __shared__ double sf[BOX_F * BOX_F * BOX_F];
  __shared__ double sr[BOX * BOX * BOX];
  const int tiles_x = F.nx / BOX, tiles_y = F.ny / BOX;
  const int b = box_tile(blockIdx.x, gridDim.x);
  const int bxy = b % (tiles_x * tiles_y);
  const int x0 = (bxy % tiles_x) * BOX, y0 = (bxy / tiles_x) * BOX;
  const int z0 = (b / (tiles_x * tiles_y)) * BOX;
  // the colour-0 sites of the iterate window ((i + j + k) even, as x0, y0,
  // z0 are even): BOX_X / 2 per row; all loads issued before the first store
  constexpr int NR = BOX_X / 2 * BOX_X * BOX_X, NF = BOX_F * BOX_F * BOX_F;
  constexpr int PR = (NR + BOX_THREADS - 1) / BOX_THREADS, PF = (NF + BOX_THREADS - 1) / BOX_THREADS;
  double vx[PR], vf[PF];
#pragma unroll
  for (int q = 0; q < PR; ++q) {
    const int t = min((int)threadIdx.x + q * BOX_THREADS, NR - 1);
    const int r = t / (BOX_X / 2);
    const int j = r % BOX_X, k = r / BOX_X;
    const int i = 2 * (t % (BOX_X / 2)) + ((j + k) & 1);
    vx[q] = F.x[idx3(wrap_index(x0 - 2 + i, F.nx), wrap_index(y0 - 2 + j, F.ny),
                     wrap_index(z0 - 2 + k, F.nz), F)];
  }
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const int t = min((int)threadIdx.x + q * BOX_THREADS, NF - 1);
    const int i = t % BOX_F, j = (t / BOX_F) % BOX_F, k = t / (BOX_F * BOX_F);
    vf[q] = F.f[idx3(wrap_index(x0 - 1 + i, F.nx), wrap_index(y0 - 1 + j, F.ny),
                     wrap_index(z0 - 1 + k, F.nz), F)];
  }
  if (ps->done) return;
  constexpr int SX = BOX_X, SX2 = BOX_X * BOX_X;
#pragma unroll
  for (int q = 0; q < PR; ++q) {
    const int t = (int)threadIdx.x + q * BOX_THREADS;
    if (t < NR) {
      const int r = t / (BOX_X / 2);
      const int j = r % BOX_X, k = r / BOX_X;
      sx[(k * SX + j) * SX + 2 * (t % (BOX_X / 2)) + ((j + k) & 1)] = vx[q];
    }
  }
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const int t = (int)threadIdx.x + q * BOX_THREADS;
    if (t < NF) sf[t] = vf[q];   // a coarser level: no shift
  }
  __syncthreads();
  const double h2 = F.h2;
  // colour 1 on the window's sites 1 .. BOX + 2 of every side, from zero
  constexpr int RROW = BOX / 2 + 1, RSIDE = BOX + 2;
  for (int t = threadIdx.x; t < RROW * RSIDE * RSIDE; t += BOX_THREADS) {
    const int r = t / RROW;
    const int j = 1 + r % RSIDE, k = 1 + r / RSIDE;
    const int i = 1 + 2 * (t % RROW) + ((j + k) & 1);
    const int w = (k * SX + j) * SX + i;
    const double xo = 0.0;
    const double nb = sx[w - 1] + sx[w + 1] + sx[w - SX] + sx[w + SX] + sx[w - SX2] + sx[w + SX2];
    const double gs = (nb - h2 * sf[((k - 1) * BOX_F + (j - 1)) * BOX_F + (i - 1)]) * (1.0 / 6.0);
    sx[w] = omega == 1.0 ? gs : xo + omega * (gs - xo);
  }
  __syncthreads();
  // the residual at the tile's sites (restrict_site's expression)
  const double ih2 = 1.0 / h2;
  for (int t = threadIdx.x; t < BOX * BOX * BOX; t += BOX_THREADS) {
    const int i = 2 + t % BOX, j = 2 + (t / BOX) % BOX, k = 2 + t / (BOX * BOX);
    const int w = (k * SX + j) * SX + i;
    const double nb = sx[w - 1] + sx[w + 1] + sx[w - SX] + sx[w + SX] + sx[w - SX2] + sx[w + SX2];
    sr[t] = sf[((k - 1) * BOX_F + (j - 1)) * BOX_F + (i - 1)] - (nb - 6.0 * sx[w]) * ih2;
  }
  __syncthreads();
  // the tile's colour-1 sites back to F.x, and the coarse cells
  constexpr int BROW = BOX / 2;
  for (int t = threadIdx.x; t < BROW * BOX * BOX; t += BOX_THREADS) {
    const int r = t / BROW;
    const int j = r % BOX, k = r / BOX;
    const int i = 2 * (t % BROW) + ((j + k + 1) & 1);
    F.x[idx3(x0 + i, y0 + j, z0 + k, F)] = sx[((k + 2) * SX + (j + 2)) * SX + (i + 2)];
  }
  constexpr int H = BOX / 2;
  for (int t = threadIdx.x; t < H * H * H; t += BOX_THREADS) {
    const int X = t % H, Y = (t / H) % H, Z = t / (H * H);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      s += sr[((2 * Z + ((c >> 2) & 1)) * BOX + 2 * Y + ((c >> 1) & 1)) * BOX + 2 * X + (c & 1)];
    const int X0 = x0 / 2 + X, Y0 = y0 / 2 + Y, Z0 = z0 / 2 + Z;
    const int u = idx3(X0, Y0, Z0, C);
    const double fc = 0.125 * s;
    C.f[u] = fc;
    double xc = 0.0;
    if (omega_red != 0.0 && ((X0 + Y0 + Z0) & 1) == 0) {
      const double gs = (0.0 - C.h2 * (fc + 0.0)) * (1.0 / 6.0);
      xc = omega_red == 1.0 ? gs : 0.0 + omega_red * (gs - 0.0);
    }
    C.x[u] = xc;
  }
}

// --- one full red-black sweep per launch, marching up z -----------------------
// xout = (colour-0 half sweep, then colour-1 half sweep)(xin), out of place.
// A workgroup owns the TX x TY tile at (x0, y0) of the planes z0 .. z1-1
// and keeps five planes of the tile plus a two-site ring in LDS.  At step k it
// relaxes the colour-0 sites of plane k on the tile and a one-site ring (from
// the old colour-1 values of planes k-1, k, k+1), then the colour-1 sites of
// plane k-1 on the tile (whose neighbours are all colour-0 sites, now new),
// and writes plane k-1.  The ring's colour-0 values are recomputed by every
// tile that borders them, from the same old values in the same order, so no
// workgroup waits for another and every site gets the update of the two
// in-place half sweeps (the same formula and summation order; the compiler
// may contract its multiply-adds differently, so the two agree to rounding:
// 4e-11 relative on psi after four steps of the 256x256x512 pore, with the
// same cycle counts).  Each site of xin and f is read once from memory
// (plus the rings and the two planes either side of a chunk, which the
// neighbouring workgroups read too) and xout is written once: 24 bytes per
// site for the sweep, against 48 for two half sweeps over the interleaved
// colours.  The loads run ahead of their use: the right-hand side of a step
// is read during the step before, the iterate planes two steps before.  The
// nz planes are cut into nch chunks (heights differ by at most one plane),
// their number chosen so that the launch runs in as few rounds of the
// workgroups the device holds at once as the chunks' extra steps allow:
// 1 <= nch <= nz; TX divides nx, TY divides ny; all sides even.
// With CORR the sweep is the first post-smoothing sweep of a cycle and takes
// the coarse-grid correction on the way in: each iterate plane gets the
// trilinear interpolation of the coarse iterate C.x (cell-centred, weights
// 3/4 and 1/4 per axis, as prolong_value) added as it is stored in LDS, in
// two stages: the two coarse planes it lies between, over a window of the
// coarse plane around the tile, are combined along z into Ez (one barrier
// phase ahead), and each site then takes its four values of Ez along y and
// x.  The separate prolongation pass (read xin, write xin + P e: 16 bytes
// per site) is saved; xin stays unchanged.
// With NIN the sweep also takes the residual norms of its input (the start of
// a solve, in its first cycle's first sweep): at step k, plane k+1 is still
// unswept in LDS, and each thread keeps the unswept values of its own region
// sites of planes k and k+1 in registers (plane k is being swept in LDS), so
// r = (f + shift) - A xin on the tile of plane k+1 needs only one more load,
// f at those sites; block partials of r^2, (f + shift)^2 and xin as
// k_residual's.
constexpr int SWEEP_THREADS = 256;
constexpr int SWEEP_SLOTS = 5;

template <int TX, int TY, bool CORR = false, bool NIN = false>
struct SweepRegs {
  static constexpr int REGION = (TX + 4) * (TY + 4);
  static constexpr int XPT = (REGION + SWEEP_THREADS - 1) / SWEEP_THREADS;
  static constexpr int RED_ROW = TX / 2 + 1;             // colour-0 sites per ring-1 row
  static constexpr int RED_ITEMS = RED_ROW * (TY + 2);
  static constexpr int RPT = (RED_ITEMS + SWEEP_THREADS - 1) / SWEEP_THREADS;
  static constexpr int PAIR_ITEMS = (TX / 2) * TY;
  static constexpr int BPT = (PAIR_ITEMS + SWEEP_THREADS - 1) / SWEEP_THREADS;
  // coarse window: the coarse cells of the region's sites and their
  // neighbours, columns x0/2 - 2 .. x0/2 + TX/2 + 1, rows likewise
  static constexpr int CWX = TX / 2 + 4, CWY = TY / 2 + 4, CW = CWX * CWY;
  static constexpr int CPT = CORR ? (CW + SWEEP_THREADS - 1) / SWEEP_THREADS : 1;
  double x[XPT];    // an iterate plane (tile and two-site ring), to be stored in LDS
  double fr[RPT];   // f at this thread's colour-0 ring sites of a plane
  double fb[BPT];   // f at this thread's colour-1 tile sites of a plane
  double c0[CPT];   // CORR: the coarse window of the plane's own coarse plane
  double c1[CPT];   //       and of the one above or below it
  double ff[NIN ? XPT : 1];   // NIN: f at this thread's region sites of a plane
};

template <int TX, int TY, bool CORR = false, bool NIN = false>
__global__ __launch_bounds__(SWEEP_THREADS) void k_sweep_z(Lvl L, const double* __restrict__ xin,
                                                           double* __restrict__ xout, int nch,
                                                           const PoissonScalars* ps, int level0,
                                                           double omega, Lvl C,
                                                           double* __restrict__ partials) {
  static_assert(TX % 2 == 0 && TY % 2 == 0, "even tiles");
  static_assert(!(CORR && NIN), "the input norms belong to a pre-smoothing sweep");
  using R = SweepRegs<TX, TY, CORR, NIN>;
  constexpr int RX = TX + 4, RY = TY + 4;
  __shared__ double P[SWEEP_SLOTS][RY][RX];
  __shared__ double Ez[CORR ? R::CW : 1];
  if (ps->done) return;
  const double shift = level0 ? ps->shift : 0.0;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const double h2 = L.h2;
  const double* __restrict__ f = L.f;
  const int tid = threadIdx.x;
  // workgroup -> (tile, chunk): consecutive groups of the launch go to
  // different XCDs, so group b is renumbered to put neighbouring tiles of a
  // chunk on one XCD (whose L2 then serves their shared rings)
  const int ntx = nx / TX, nty = ny / TY;
  const int nblk = gridDim.x;
  int b = blockIdx.x;
  if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  const int tx_i = b % ntx;
  const int rest = b / ntx;
  const int ty_i = rest % nty;
  const int chunk = rest / nty;
  const int x0 = tx_i * TX, y0 = ty_i * TY;
  const int z0 = chunk * nz / nch, z1 = (chunk + 1) * nz / nch;
  const int zb = z0 - 2;                                   // plane of relative index 0

  auto wrapi = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  auto plane_base = [&](int q) {                           // any plane index, wrapped here
    int zq = q % nz;
    if (zq < 0) zq += nz;
    return (long long)zq * ny * nx;
  };
  auto slot = [&](int q) { return (q - zb) % SWEEP_SLOTS; };
  // The loads are issued unconditionally (indexes past the end are clamped,
  // their values never used): loads inside branches would leave the compiler
  // unable to count the ones in flight, and it would then wait for all of
  // them, the loads meant for later steps included, before the first use.
  auto gather_x = [&](int q, double (&r)[R::XPT]) {
    const long long base = plane_base(q);
#pragma unroll
    for (int u = 0; u < R::XPT; ++u) {
      const int t = min(tid + u * SWEEP_THREADS, R::REGION - 1);
      const int j = t / RX, i = t - j * RX;
      r[u] = xin[base + (long long)wrapi(y0 - 2 + j, ny) * nx + wrapi(x0 - 2 + i, nx)];
    }
  };
  // (CORR) site (j, i) of the region lies in the coarse cell of window
  // column (i >> 1) + 1, row (j >> 1) + 1 (x0, y0 even); its neighbour cell
  // along an axis is the next one for an odd and the previous one for an even
  // fine coordinate
  auto store_x = [&](int s, const double (&r)[R::XPT]) {
#pragma unroll
    for (int u = 0; u < R::XPT; ++u) {
      const int t = tid + u * SWEEP_THREADS;
      if (t < R::REGION) {
        const int j = t / RX, i = t - j * RX;
        double v = r[u];
        if constexpr (CORR) {
          const int wx = (i >> 1) + 1, wy = (j >> 1) + 1;
          const int wxn = (i & 1) ? wx + 1 : wx - 1, wyn = (j & 1) ? wy + 1 : wy - 1;
          const double* e0 = Ez + wy * R::CWX;
          const double* e1 = Ez + wyn * R::CWX;
          v += 0.75 * (0.75 * e0[wx] + 0.25 * e0[wxn]) + 0.25 * (0.75 * e1[wx] + 0.25 * e1[wxn]);
        }
        P[s][j][i] = v;
      }
    }
  };
  // (CORR) the coarse window of the two coarse planes fine plane q lies
  // between: its own, q >> 1, and the next one for odd q, the previous one for
  // even q (periodic)
  auto cmod = [](int v, int n) { return ((v % n) + n) % n; };
  auto gather_c = [&](int q, R& r) {
    if constexpr (CORR) {
      const int Z = q >> 1, Zn = (q & 1) ? Z + 1 : Z - 1;
      const long long b0 = (long long)cmod(Z, C.nz) * C.ny * C.nx;
      const long long b1 = (long long)cmod(Zn, C.nz) * C.ny * C.nx;
#pragma unroll
      for (int u = 0; u < R::CPT; ++u) {
        const int t = min(tid + u * SWEEP_THREADS, R::CW - 1);
        const int wy = t / R::CWX, wx = t - wy * R::CWX;
        const long long off = (long long)cmod(y0 / 2 - 2 + wy, C.ny) * C.nx + cmod(x0 / 2 - 2 + wx, C.nx);
        r.c0[u] = C.x[b0 + off];
        r.c1[u] = C.x[b1 + off];
      }
    }
  };
  auto write_ez = [&](const R& r) {
    if constexpr (CORR) {
#pragma unroll
      for (int u = 0; u < R::CPT; ++u) {
        const int t = tid + u * SWEEP_THREADS;
        if (t < R::CW) Ez[t] = 0.75 * r.c0[u] + 0.25 * r.c1[u];
      }
    }
  };
  // colour-0 item t of plane k: ring-1 row j, column i (colour 0 means
  // (x0 - 2 + i) + (y0 - 2 + j) + k even)
  auto red_site = [&](int t, int k, int& j, int& i) {
    const int jj = t / R::RED_ROW, m = t - jj * R::RED_ROW;
    j = 1 + jj;
    i = (((x0 + y0 + k + j) & 1) ? 1 : 2) + 2 * m;
  };
  // colour-1 item t of plane k: tile row jj, pair m; the colour-1 site is the
  // first of the pair when x0 + 2 m + y0 + jj + k is odd
  auto black_first = [&](int jj, int m, int k) { return ((x0 + 2 * m + y0 + jj + k) & 1) != 0; };
  auto gather_fr = [&](int k, double (&r)[R::RPT]) {
    const long long base = plane_base(k);
#pragma unroll
    for (int u = 0; u < R::RPT; ++u) {
      const int t = min(tid + u * SWEEP_THREADS, R::RED_ITEMS - 1);
      int j, i;
      red_site(t, k, j, i);
      r[u] = f[base + (long long)wrapi(y0 - 2 + j, ny) * nx + wrapi(x0 - 2 + i, nx)];
    }
  };
  auto gather_fb = [&](int k, double (&r)[R::BPT]) {
    const long long base = plane_base(k);
#pragma unroll
    for (int u = 0; u < R::BPT; ++u) {
      const int t = min(tid + u * SWEEP_THREADS, R::PAIR_ITEMS - 1);
      const int jj = t / (TX / 2), m = t - jj * (TX / 2);
      r[u] = f[base + (long long)(y0 + jj) * nx + x0 + 2 * m + (black_first(jj, m, k) ? 0 : 1)];
    }
  };
  // (NIN) f at this thread's region sites of plane q, and the unswept
  // values of those sites in planes k and k+1 (xm2, xm1) at step k
  auto gather_ff = [&](int q, R& r) {
    if constexpr (NIN) {
      const long long base = plane_base(q);
#pragma unroll
      for (int u = 0; u < R::XPT; ++u) {
        const int t = min(tid + u * SWEEP_THREADS, R::REGION - 1);
        const int j = t / RX, i = t - j * RX;
        r.ff[u] = f[base + (long long)wrapi(y0 - 2 + j, ny) * nx + wrapi(x0 - 2 + i, nx)];
      }
    }
  };
  double xm1[NIN ? R::XPT : 1], xm2[NIN ? R::XPT : 1];
  double acc[3] = {0.0, 0.0, 0.0};
  // Step k.  cur holds the iterate plane k+2 (stored at the end; with CORR its
  // coarse window, combined into Ez in the first phase; with NIN f of plane
  // k+1 at the thread's region sites), f of the colour-0 sites of plane k and
  // of the colour-1 sites of plane k-1; nxt receives plane k+3 (and its
  // coarse window, or f of plane k+2 at the region sites) and f of planes
  // k+1 (colour 0) and k (colour 1).
  auto step = [&](int k, R& cur, R& nxt) {
    // (near the chunk's end the planes are clamped: loaded, never used)
    gather_x(min(k + 3, z1 + 1), nxt.x);
    gather_c(min(k + 3, z1 + 1), nxt);
    gather_ff(min(k + 2, z1), nxt);
    gather_fr(min(k + 1, z1), nxt.fr);
    gather_fb(max(min(k, z1 - 1), z0), nxt.fb);
    if (k + 2 <= z1 + 1) write_ez(cur);
    const int sk = slot(k), skm = slot(k + SWEEP_SLOTS - 1), skp = slot(k + 1),
              skm2 = slot(k + SWEEP_SLOTS - 2);
#pragma unroll
    for (int u = 0; u < R::RPT; ++u) {
      const int t = tid + u * SWEEP_THREADS;
      if (t < R::RED_ITEMS) {
        int j, i;
        red_site(t, k, j, i);
        const double xo = P[sk][j][i];
        const double nb = P[sk][j][i - 1] + P[sk][j][i + 1] + P[sk][j - 1][i] + P[sk][j + 1][i] +
                          P[skm][j][i] + P[skp][j][i];
        const double gs = (nb - h2 * (cur.fr[u] + shift)) * (1.0 / 6.0);
        P[sk][j][i] = omega == 1.0 ? gs : xo + omega * (gs - xo);
      }
    }
    __syncthreads();
    if (k - 1 >= z0) {
      const long long base = plane_base(k - 1);
#pragma unroll
      for (int u = 0; u < R::BPT; ++u) {
        const int t = tid + u * SWEEP_THREADS;
        if (t < R::PAIR_ITEMS) {
          const int jj = t / (TX / 2), m = t - jj * (TX / 2);
          const int j = 2 + jj, i0 = 2 + 2 * m;
          const bool first = black_first(jj, m, k - 1);
          const int ib = first ? i0 : i0 + 1, ir = first ? i0 + 1 : i0;
          const double xo = P[skm][j][ib];
          const double nb = P[skm][j][ib - 1] + P[skm][j][ib + 1] + P[skm][j - 1][ib] +
                            P[skm][j + 1][ib] + P[skm2][j][ib] + P[sk][j][ib];
          const double gs = (nb - h2 * (cur.fb[u] + shift)) * (1.0 / 6.0);
          const double vb = omega == 1.0 ? gs : xo + omega * (gs - xo);
          const double vr = P[skm][j][ir];
          double2 out;
          out.x = first ? vb : vr;
          out.y = first ? vr : vb;
          *reinterpret_cast<double2*>(xout + base + (long long)(y0 + jj) * nx + x0 + 2 * m) = out;
        }
      }
    }
    if constexpr (NIN) {
      // residual of the unswept plane k+1 on the tile (its slot is not
      // written during step k)
      if (k + 1 >= z0 && k + 1 < z1) {
        const int s1 = slot(k + 1);
        const double ih2 = 1.0 / h2;
#pragma unroll
        for (int u = 0; u < R::XPT; ++u) {
          const int t = tid + u * SWEEP_THREADS;
          const int j = t / RX, i = t - j * RX;
          if (t < R::REGION && j >= 2 && j < TY + 2 && i >= 2 && i < TX + 2) {
            const double nb = P[s1][j][i - 1] + P[s1][j][i + 1] + P[s1][j - 1][i] +
                              P[s1][j + 1][i] + xm2[u] + cur.x[u];
            const double rhs = cur.ff[u] + shift;
            const double res = rhs - (nb - 6.0 * xm1[u]) * ih2;
            acc[0] += res * res;
            acc[1] += rhs * rhs;
            acc[2] += xm1[u];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < R::XPT; ++u) {
        xm2[u] = xm1[u];
        xm1[u] = cur.x[u];
      }
    }
    if (k + 2 <= z1 + 1) store_x(slot(k + 2), cur.x);
    __syncthreads();
  };
  R A, B;
  for (int q = zb; q <= z0; ++q) {                         // planes z0-2, z0-1, z0
    gather_x(q, A.x);
    gather_c(q, A);
    if constexpr (CORR) {
      write_ez(A);
      __syncthreads();
    }
    store_x(slot(q), A.x);
    if constexpr (CORR) __syncthreads();
    if constexpr (NIN) {
#pragma unroll
      for (int u = 0; u < R::XPT; ++u) {
        xm2[u] = xm1[u];
        xm1[u] = A.x[u];
      }
    }
  }
  gather_x(z0 + 1, A.x);
  gather_c(z0 + 1, A);
  gather_ff(z0, A);
  gather_fr(z0 - 1, A.fr);
  __syncthreads();
  int k = z0 - 1;
  for (; k + 1 <= z1; k += 2) {
    step(k, A, B);
    step(k + 1, B, A);
  }
  if (k <= z1) step(k, A, B);
  if constexpr (NIN) block_partials<3>(acc, partials, blockIdx.x, gridDim.x);
}

// --- a full sweep that also takes the residual of its result ---------------
// As k_sweep_z, with a three-site ring: the colour-0 sites are relaxed on the
// tile and two rings, the colour-1 sites on the tile and one ring, so the
// swept values of the tile and its one-site ring are final and the residual
// r = (f + shift) - A x of the result is taken on the tile as the march goes:
// at step k, after the colour-1 sites of plane k-1, the residual of plane k-2
// (from planes k-3, k-2 and k-1).  MODE = SWEEP_RESTRICT adds the residuals
// of each 2 x 2 x 2 block in the order of restrict_site and writes the coarse
// level's right-hand side (and its first colour-0 half sweep, omega_red), so
// the pre-smoothing of the finest level and its restriction are one pass;
// MODE = SWEEP_NORMS adds r^2, (f + shift)^2 and x for the convergence test
// (block partials as k_residual), so the last post-smoothing sweep of a tested
// cycle is its residual pass too.  A chunk computes the colour-1 sites of the
// planes either side of it as well (its neighbours do too), and keeps six
// planes in LDS.  The nz planes are cut into nch chunks of an even number of
// planes (their heights differ by at most two).  nz even, 1 <= nch <= nz / 2;
// TX, TY multiples of 4.
enum : int { SWEEP_RESTRICT = 1, SWEEP_NORMS = 2 };
// Tile of the fused sweeps (64 x ZR_TY) and their workgroup size (a thread
// pair per 2 x 2 block of the tile).
constexpr int ZR_TY = 8;
constexpr int ZR_THREADS = ZR_TY * 32;

template <int TX, int TY>
struct SweepRRegs {
  static constexpr int RX = TX + 6, RY = TY + 6;
  static constexpr int REGION = RX * RY;
  static constexpr int XPT = (REGION + ZR_THREADS - 1) / ZR_THREADS;
  static constexpr int RED_ROW = TX / 2 + 2;              // colour-0 sites per ring-2 row
  static constexpr int RED_ITEMS = RED_ROW * (TY + 4);
  static constexpr int RPT = (RED_ITEMS + ZR_THREADS - 1) / ZR_THREADS;
  static constexpr int BLK_ROW = TX / 2 + 1;              // colour-1 sites per ring-1 row
  static constexpr int BLK_ITEMS = BLK_ROW * (TY + 2);
  static constexpr int BPT = (BLK_ITEMS + ZR_THREADS - 1) / ZR_THREADS;
  static constexpr int CELLS = (TX / 2) * (TY / 2);       // 2 x 2 blocks of the tile
  double x[XPT];     // an iterate plane (tile and three-site ring), to be stored in LDS
  double fr[RPT];    // f at this thread's colour-0 ring-2 sites of a plane
  double fb[BPT];    // f at this thread's colour-1 ring-1 sites of a plane
  double ft[2];      // f at this thread's two tile sites of a plane (a row of its 2 x 2 block)
};

template <int TX, int TY, int MODE>
__global__ __launch_bounds__(ZR_THREADS) void k_sweep_zr(Lvl L, const double* __restrict__ xin,
                                                            double* __restrict__ xout, int nch,
                                                            const PoissonScalars* ps, int level0,
                                                            double omega, Lvl C, double omega_red,
                                                            double* __restrict__ partials) {
  static_assert(TX % 4 == 0 && TY % 4 == 0, "tiles of whole 2 x 2 blocks");
  static_assert(2 * SweepRRegs<TX, TY>::CELLS <= ZR_THREADS, "a 2 x 2 block per thread pair");
  using R = SweepRRegs<TX, TY>;
  constexpr int RX = R::RX, RY = R::RY, NS = 6;
  __shared__ double P[NS][RY][RX];
  if (ps->done) return;
  const double shift = level0 ? ps->shift : 0.0;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const double h2 = L.h2, ih2 = 1.0 / L.h2;
  const double* __restrict__ f = L.f;
  const int tid = threadIdx.x;
  const int ntx = nx / TX, nty = ny / TY, nblk = gridDim.x;
  int b = blockIdx.x;
  if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  const int tx_i = b % ntx, rest = b / ntx, ty_i = rest % nty, chunk = rest / nty;
  const int x0 = tx_i * TX, y0 = ty_i * TY, half = nz >> 1;
  const int z0 = 2 * (chunk * half / nch), z1 = 2 * ((chunk + 1) * half / nch);
  const int zb = z0 - 3;                                    // plane in slot-relative index 0
  auto wrapi = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  auto plane_base = [&](int q) {
    int zq = q % nz;
    if (zq < 0) zq += nz;
    return (long long)zq * ny * nx;
  };
  auto slot = [&](int q) { return (q - zb) % NS; };
  auto gather_x = [&](int q, double (&r)[R::XPT]) {
    const long long base = plane_base(q);
#pragma unroll
    for (int u = 0; u < R::XPT; ++u) {
      const int t = min(tid + u * ZR_THREADS, R::REGION - 1);
      const int j = t / RX, i = t - j * RX;
      r[u] = xin[base + (long long)wrapi(y0 - 3 + j, ny) * nx + wrapi(x0 - 3 + i, nx)];
    }
  };
  auto store_x = [&](int sl, const double (&r)[R::XPT]) {
#pragma unroll
    for (int u = 0; u < R::XPT; ++u) {
      const int t = tid + u * ZR_THREADS;
      if (t < R::REGION) {
        const int j = t / RX, i = t - j * RX;
        P[sl][j][i] = r[u];
      }
    }
  };
  // colour-0 item t of plane k: ring-2 row j in [1, TY + 5), column i
  auto red_site = [&](int t, int k, int& j, int& i) {
    const int jj = t / R::RED_ROW, m = t - jj * R::RED_ROW;
    j = 1 + jj;
    i = (((x0 + y0 + k + j) & 1) ? 1 : 2) + 2 * m;
  };
  // colour-1 item t of plane k: ring-1 row j in [2, TY + 4), column i
  auto black_site = [&](int t, int k, int& j, int& i) {
    const int jj = t / R::BLK_ROW, m = t - jj * R::BLK_ROW;
    j = 2 + jj;
    i = (((x0 + y0 + k + 1 + j) & 1) ? 3 : 2) + 2 * m;
  };
  // tile 2 x 2 block of this thread pair: threads 2c and 2c + 1 take row
  // 3 + 2 cy + (tid & 1) of block c, sites at columns 3 + 2 cx and 4 + 2 cx
  const int cell = min(tid >> 1, R::CELLS - 1);
  const int cx = cell % (TX / 2), cy = cell / (TX / 2), crow = tid & 1;
  const bool has_cell = (tid >> 1) < R::CELLS;
  auto gather_fr = [&](int k, double (&r)[R::RPT]) {
    const long long base = plane_base(k);
#pragma unroll
    for (int u = 0; u < R::RPT; ++u) {
      const int t = min(tid + u * ZR_THREADS, R::RED_ITEMS - 1);
      int j, i;
      red_site(t, k, j, i);
      r[u] = f[base + (long long)wrapi(y0 - 3 + j, ny) * nx + wrapi(x0 - 3 + i, nx)];
    }
  };
  auto gather_fb = [&](int k, double (&r)[R::BPT]) {
    const long long base = plane_base(k);
#pragma unroll
    for (int u = 0; u < R::BPT; ++u) {
      const int t = min(tid + u * ZR_THREADS, R::BLK_ITEMS - 1);
      int j, i;
      black_site(t, k, j, i);
      r[u] = f[base + (long long)wrapi(y0 - 3 + j, ny) * nx + wrapi(x0 - 3 + i, nx)];
    }
  };
  auto gather_ft = [&](int k, double (&r)[2]) {
    const long long base = plane_base(k) + (long long)(y0 + 2 * cy + crow) * nx + x0 + 2 * cx;
    r[0] = f[base];
    r[1] = f[base + 1];
  };
  double acc[3] = {0.0, 0.0, 0.0};   // SWEEP_NORMS
  double rsum = 0.0;                 // SWEEP_RESTRICT: this thread's row of the block so far
  // Step k, in two phases between barriers:
  //   1. colour 0 of plane k (tile and two rings); the tile of plane k-2,
  //      final since step k-1, is written, and the residual of plane k-3
  //      taken (from planes k-4, k-3, k-2);
  //   2. colour 1 of plane k-1 (tile and one ring); plane k+2 is stored, in
  //      the slot of plane k-4, which phase 1 used last.
  // The two parts of phase 1 touch disjoint planes (k-1 .. k+1 and k-4 ..
  // k-2), so one barrier separates the phases.  cur holds plane k+2, f of the
  // colour-0 sites of plane k, of the colour-1 sites of plane k-1 and of this
  // thread's tile row of plane k-3; nxt receives plane k+3 and f of planes
  // k+1, k and k-2 (clamped near the chunk's ends: loaded, never used).
  auto step = [&](int k, R& cur, R& nxt) {
    gather_x(min(k + 3, z1 + 2), nxt.x);
    gather_fr(min(k + 1, z1 + 1), nxt.fr);
    gather_fb(max(min(k, z1), z0 - 1), nxt.fb);
    gather_ft(max(min(k - 2, z1 - 1), z0), nxt.ft);
    const int sk = slot(k), skm = slot(k + NS - 1), skp = slot(k + 1), skm2 = slot(k + NS - 2),
              skm3 = slot(k + NS - 3), skm4 = slot(k + NS - 4);
    // 1a. colour 0 of plane k on the tile and two rings
    if (k <= z1 + 1) {
#pragma unroll
      for (int u = 0; u < R::RPT; ++u) {
        const int t = tid + u * ZR_THREADS;
        if (t < R::RED_ITEMS) {
          int j, i;
          red_site(t, k, j, i);
          const double xo = P[sk][j][i];
          const double nb = P[sk][j][i - 1] + P[sk][j][i + 1] + P[sk][j - 1][i] + P[sk][j + 1][i] +
                            P[skm][j][i] + P[skp][j][i];
          const double gs = (nb - h2 * (cur.fr[u] + shift)) * (1.0 / 6.0);
          P[sk][j][i] = omega == 1.0 ? gs : xo + omega * (gs - xo);
        }
      }
    }
    // 1b. write the tile of plane k-2; the residual of plane k-3
    if (k - 2 >= z0 && k - 2 < z1) {
      const long long base = plane_base(k - 2);
      for (int t = tid; t < (TX / 2) * TY; t += ZR_THREADS) {
        const int jj = t / (TX / 2), m = t - jj * (TX / 2);
        double2 out;
        out.x = P[skm2][3 + jj][3 + 2 * m];
        out.y = P[skm2][3 + jj][4 + 2 * m];
        *reinterpret_cast<double2*>(xout + base + (long long)(y0 + jj) * nx + x0 + 2 * m) = out;
      }
    }
    if (k - 3 >= z0 && k - 3 < z1) {
      if (has_cell) {
        const int j = 3 + 2 * cy + crow;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int i = 3 + 2 * cx + q;
          const double c = P[skm3][j][i];
          const double nb = P[skm3][j][i - 1] + P[skm3][j][i + 1] + P[skm3][j - 1][i] +
                            P[skm3][j + 1][i] + P[skm4][j][i] + P[skm2][j][i];
          const double rhs = cur.ft[q] + shift;
          if (MODE == SWEEP_RESTRICT) {
            rsum += rhs - (nb - 6.0 * c) * ih2;
          } else {
            const double res = rhs - (nb - 6.0 * c);
            acc[0] += res * res;
            acc[1] += rhs * rhs;
            acc[2] += c;
          }
        }
      }
      if (MODE == SWEEP_RESTRICT && ((k - 3) & 1)) {
        // the block's second plane: the coarse cell's right-hand side (the
        // two rows' sums met in the even thread) and its first colour-0 half
        // sweep from the zero start
        const double other = __shfl_xor(rsum, 1, 64);
        if (has_cell && crow == 0) {
          const int X = x0 / 2 + cx, Y = y0 / 2 + cy, Z = (k - 3) >> 1;
          const long long t = ((long long)Z * C.ny + Y) * C.nx + X;
          const double fc = 0.125 * (rsum + other);
          C.f[t] = fc;
          double xc = 0.0;
          if (omega_red != 0.0 && ((X + Y + Z) & 1) == 0) {
            const double gs = (0.0 - C.h2 * (fc + 0.0)) * (1.0 / 6.0);
            xc = omega_red == 1.0 ? gs : 0.0 + omega_red * (gs - 0.0);
          }
          C.x[t] = xc;
        }
        rsum = 0.0;
      }
    }
    __syncthreads();
    // 2. colour 1 of plane k-1 on the tile and one ring (the planes either
    // side of the chunk as well); store plane k+2
    if (k >= z0 && k <= z1 + 1) {
#pragma unroll
      for (int u = 0; u < R::BPT; ++u) {
        const int t = tid + u * ZR_THREADS;
        if (t < R::BLK_ITEMS) {
          int j, i;
          black_site(t, k - 1, j, i);
          const double xo = P[skm][j][i];
          const double nb = P[skm][j][i - 1] + P[skm][j][i + 1] + P[skm][j - 1][i] +
                            P[skm][j + 1][i] + P[skm2][j][i] + P[sk][j][i];
          const double gs = (nb - h2 * (cur.fb[u] + shift)) * (1.0 / 6.0);
          P[skm][j][i] = omega == 1.0 ? gs : xo + omega * (gs - xo);
        }
      }
    }
    if (k + 2 <= z1 + 2) store_x(slot(k + 2), cur.x);
    __syncthreads();
  };
  R A, B;
  for (int q = zb; q <= z0 - 1; ++q) {                      // planes z0-3, z0-2, z0-1
    gather_x(q, A.x);
    store_x(slot(q), A.x);
  }
  gather_x(z0, A.x);
  gather_fr(z0 - 2, A.fr);
  __syncthreads();
  int k = z0 - 2;
  for (; k + 1 <= z1 + 2; k += 2) {
    step(k, A, B);
    step(k + 1, B, A);
  }
  if (k <= z1 + 2) step(k, A, B);
  if (MODE == SWEEP_NORMS) block_partials<3>(acc, partials, blockIdx.x, gridDim.x);
}

// The coarse part of the cycle runs on copies of the coarse levels in LDS:
// level `first` arrives with its right-hand side and a zero iterate in global
// memory, its iterate goes back to global memory at the end.  As on the
// launched levels, the first colour-0 half sweep of a level coming from a
// zero start is done where its right-hand side is written (copy-in,
// restriction); the correction goes up by a prolongation pass (inside one
// workgroup the fused corrected sweep, which recomputes the correction at
// the six neighbours, measured slower).  The coarsest level is solved
// directly when `pinv` is given (its n x n inverse of A + c 11^T / n, which
// returns the mean-free solution of A x = f for a mean-free f), else by
// coarsest_sweeps red-black SOR sweeps.
__global__ __launch_bounds__(1024) void k_coarse_cycle(LvlSet set, int first, PoissonScalars* ps,
                                                       double omega_coarsest, int coarsest_sweeps,
                                                       const double* __restrict__ pinv) {
  static_assert(NU1 >= 1, "the fold needs a pre-smoothing sweep");
  if (ps->done) return;
  if (threadIdx.x == 0) atomicAdd(&ps->cycles, 1);   // read only by later kernels; no wait
  extern __shared__ __align__(16) double lds[];
  __shared__ Lvl L[MAX_LEVELS];
  __shared__ double* s_pinv;   // the coarsest level's inverse, after the levels
  const int last = set.count - 1;
  if (threadIdx.x == 0) {
    double* p = lds;
    for (int l = first; l <= last; ++l) {
      L[l] = set.l[l];
      L[l].x = p;
      L[l].f = p + L[l].n;
      p += 2 * L[l].n;
    }
    s_pinv = p;
  }
  __syncthreads();
  // copy-in, with the inverse (its global reads overlap those of the
  // right-hand side instead of stalling the direct solve); a level that is
  // smoothed here gets its first colour-0 half sweep
  const bool fold_first = first < last;
  const int n_inv = pinv ? int(set.l[last].n * set.l[last].n) : 0;
  {
    const Lvl F = L[first];
    const float inx = 1.0f / F.nx, iny = 1.0f / F.ny;
    const int nf = int(F.n), nt = nf > n_inv ? nf : n_inv;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const double f = t < nf ? set.l[first].f[t] : 0.0;
      const double pv = t < n_inv ? pinv[t] : 0.0;
      if (t < n_inv) s_pinv[t] = pv;
      if (t >= nf) continue;
      F.f[t] = f;
      int x, y;
      const int yz = fdivmod(t, F.nx, inx, x);
      const int z = fdivmod(yz, F.ny, iny, y);
      double x0 = 0.0;
      if (fold_first && ((x + y + z) & 1) == 0) {
        const double gs = (0.0 - F.h2 * (f + 0.0)) * (1.0 / 6.0);
        x0 = MG_OMEGA == 1.0 ? gs : 0.0 + MG_OMEGA * (gs - 0.0);
      }
      F.x[t] = x0;
    }
  }
  __syncthreads();
  for (int l = first; l < last; ++l) {
    // colour 0 of the first pre-smoothing sweep is already done
    block_half(L[l], 1, 0.0, MG_OMEGA);
    for (int s = 1; s < NU1; ++s) {
      block_half(L[l], 0, 0.0, MG_OMEGA);
      block_half(L[l], 1, 0.0, MG_OMEGA);
    }
    block_restrict(L[l], L[l + 1], 0.0, l + 1 < last ? MG_OMEGA : 0.0);
  }
  if (pinv) {
    const Lvl C = L[last];
    const int n = int(C.n);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += s_pinv[t * n + k] * C.f[k];
      C.x[t] = v;
    }
    __syncthreads();
  } else {
    block_smooth(L[last], coarsest_sweeps, 0.0, omega_coarsest);
  }
  for (int l = last - 1; l >= first; --l) {
    block_prolong(L[l], L[l + 1]);
    block_smooth(L[l], NU2_COARSE, 0.0, MG_OMEGA);
  }
  for (int t = threadIdx.x; t < int(L[first].n); t += blockDim.x) set.l[first].x[t] = L[first].x[t];
}

// Cycle count of a V-cycle whose coarsest level is swept on the grid.
__global__ void k_count_cycle(PoissonScalars* ps) {
  if (threadIdx.x == 0 && !ps->done) ps->cycles += 1;
}

SiteGrid colour_launch(const Lvl& L) { return site_grid(L.nx / 2, L.ny, L.nz); }
SiteGrid level_launch(const Lvl& L) { return site_grid(L.nx, L.ny, L.nz); }

}  // namespace

struct ek_ctx::MG {
  std::vector<Lvl> levels;   // level 0 pointers are filled per solve
  int first_coarse = 0;      // first level handled by the single-workgroup kernel
  size_t coarse_lds = 0;     // LDS bytes of that kernel
  double omega_coarsest = 1.0;
  int coarsest_sweeps = COARSEST_SWEEPS;
  const double* pinv = nullptr;   // inverse for the direct coarsest solve, or null
  bool coarse_kernel = true;      // false: the coarsest level does not fit LDS
  // Full sweeps by k_sweep_z (out of place) on the launched levels whose tiles
  // fit: tile (sweep_tx, sweep_ty), sweep_nch chunks along z; 0 = half
  // sweeps.  The finest level sweeps into tmp0 and back, the others into tmp1.
  std::vector<int> sweep_tx, sweep_ty, sweep_nch;
  // Levels without such a plan whose sides BOX divides take one launch per
  // full sweep instead (k_sweep_box, out of place through the same buffers).
  std::vector<char> box;
  double* tmp0 = nullptr;
  double* tmp1 = nullptr;
  double* tmp2 = nullptr;   // the finest level's third iterate buffer
  // the finest level's pre-smoothing sweep also restricts, and a tested
  // cycle's last sweep also takes the residual norms (k_sweep_zr: a 64 x 8
  // tile, zr_chunks chunks of an even number of planes)
  bool fused0 = false;
  int zr_chunks = 0;
  int start_chunks = 0;     // chunks of the first sweep that also takes the start's residual
  // One V-cycle, and one V-cycle followed by the residual test, recorded as
  // graphs for the level-0 pair (b, x) they were recorded with: a replay
  // dispatches the cycle's ~30 dependent launches faster than the launches
  // issued one by one.  They are recorded on a stream of the library's own
  // (the caller's may be the default stream, which cannot be recorded) and
  // replayed on the context's stream.
  hipStream_t record_stream = nullptr;
  hipGraphExec_t cycle = nullptr, cycle_test = nullptr;
  // the first cycle of a solve (more pre-smoothing on the finest level),
  // with the start's residual (cycle_start*: mg_start_in_cycle) or without
  hipGraphExec_t cycle_start = nullptr, cycle_start_test = nullptr;
  hipGraphExec_t cycle_first = nullptr, cycle_first_test = nullptr;
  const double* graph_b = nullptr;
  double* graph_x = nullptr;
  bool graph_failed = false;   // recording is not possible: launch one by one
  // A whole batch of cycles with their tests and the read-back of the
  // solver's scalars into the pinned buffer, as one graph: the cycles of a
  // batch then follow each other without the idle gap of a graph launch
  // (about 13 us each), nor one before the read-back.  Keyed by the cycle
  // count, the first tested cycle and how the batch opens the solve (0: a
  // later batch, 1: the first cycle, 2: the first cycle with the start's
  // residual); at most MAX_BATCH_GRAPHS are kept.
  struct Batch {
    int n, untested, opens;
    hipGraphExec_t exec;
  };
  static constexpr int MAX_BATCH_GRAPHS = 8;
  std::vector<Batch> batches;
  bool batch_failed = false;   // a batch could not be recorded: per-cycle graphs

  void drop_graphs() {
    for (const Batch& bg : batches) (void)hipGraphExecDestroy(bg.exec);
    batches.clear();
    if (cycle) (void)hipGraphExecDestroy(cycle);
    if (cycle_test) (void)hipGraphExecDestroy(cycle_test);
    if (cycle_start) (void)hipGraphExecDestroy(cycle_start);
    if (cycle_start_test) (void)hipGraphExecDestroy(cycle_start_test);
    if (cycle_first) (void)hipGraphExecDestroy(cycle_first);
    if (cycle_first_test) (void)hipGraphExecDestroy(cycle_first_test);
    cycle = cycle_test = cycle_start = cycle_start_test = cycle_first = cycle_first_test = nullptr;
    graph_b = nullptr;
    graph_x = nullptr;
  }
};

bool halvable(int nx, int ny, int nz) {
  return nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0;
}

// optimal SOR factor 2 / (1 + sqrt(1 - rho_J^2)) of a periodic grid
double omega_opt(int nx, int ny, int nz) {
  const int m = std::max(nx, std::max(ny, nz));
  const double rj = (2.0 + std::cos(2.0 * M_PI / m)) / 3.0;
  return 2.0 / (1.0 + std::sqrt(1.0 - rj * rj));
}

size_t ek::mg_workspace_bytes(int nx, int ny, int nz) {
  size_t bytes = 256;
  while (halvable(nx, ny, nz)) {
    nx /= 2;
    ny /= 2;
    nz /= 2;
    bytes += 2 * (((size_t)nx * ny * nz * 8 + 255) & ~size_t(255));
  }
  // the coarsest level's inverse (direct solve)
  bytes += (size_t)COARSEST_DIRECT_MAX * COARSEST_DIRECT_MAX * 8;
  return bytes;
}

// The sweep buffers of the out-of-place full sweeps: the finest level and the
// next (every coarser level fits in the latter).
size_t ek::mg_sweep_bytes(int nx, int ny, int nz) {
  const size_t n0 = (size_t)nx * ny * nz;
  return 3 * 256 + 2 * ((n0 * 8 + 255) & ~size_t(255)) + ((n0 + 7) / 8 * 8 + 255) / 256 * 256;
}

// Workgroups of `kernel` (`threads` threads each) that the device holds at
// once, or 0 when it cannot be asked.
template <typename F>
static long long resident_workgroups(F kernel, int threads = SWEEP_THREADS) {
  int dev = 0, ncu = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess)
    return 0;
  return (long long)std::max(ncu, 0) * std::max(occ, 0);
}

// Chunks along z of a z-marching sweep over `tiles` tiles of a level of nz
// planes, chunks of `unit` planes at a time (1, or 2 for whole 2 x 2 x 2
// blocks): the count whose launch ends after the fewest plane steps when its
// workgroups run in rounds of `slots` (the workgroups the device holds at
// once), a chunk of h planes taking h + `extra` steps; `fallback` when the
// device could not be asked (slots 0).
static int sweep_chunks(long long tiles, int nz, int unit, int extra, long long slots,
                        int fallback) {
  if (slots < 1) return fallback;
  const int units = nz / unit;
  int best = fallback;
  long long best_steps = -1;
  for (int nch = 1; nch <= units; ++nch) {
    const long long rounds = (tiles * nch + slots - 1) / slots;
    const long long steps = rounds * (unit * ((units + nch - 1) / nch) + extra);
    if (best_steps < 0 || steps < best_steps) {
      best_steps = steps;
      best = nch;
    }
  }
  return best;
}

// Inverse of M = A + c 11^T / n for the periodic 7-point operator A of level
// C ((sum of the 6 neighbours - 6 x) / h^2, a neighbour counted twice where a
// side is 2 long), c = -6 / h^2.  A is singular only along the constant
// vector, which M lifts; for a mean-free f, M^-1 f is the mean-free solution
// of A x = f.  Gauss-Jordan elimination with partial pivoting in double;
// false if a pivot vanishes.
static bool coarsest_inverse(const Lvl& C, std::vector<double>& inv) {
  const int n = int(C.n);
  std::vector<double> a((size_t)n * n, 0.0);
  const double c = -6.0 / C.h2;
  for (int z = 0; z < C.nz; ++z)
    for (int y = 0; y < C.ny; ++y)
      for (int x = 0; x < C.nx; ++x) {
        const int r = (z * C.ny + y) * C.nx + x;
        const int nb[6] = {(z * C.ny + y) * C.nx + (x + C.nx - 1) % C.nx,
                           (z * C.ny + y) * C.nx + (x + 1) % C.nx,
                           (z * C.ny + (y + C.ny - 1) % C.ny) * C.nx + x,
                           (z * C.ny + (y + 1) % C.ny) * C.nx + x,
                           (((z + C.nz - 1) % C.nz) * C.ny + y) * C.nx + x,
                           (((z + 1) % C.nz) * C.ny + y) * C.nx + x};
        for (int k = 0; k < 6; ++k) a[(size_t)r * n + nb[k]] += 1.0 / C.h2;
        a[(size_t)r * n + r] -= 6.0 / C.h2;
      }
  for (size_t k = 0; k < a.size(); ++k) a[k] += c / n;
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + col]) > std::fabs(a[(size_t)piv * n + col])) piv = r;
    if (!(std::fabs(a[(size_t)piv * n + col]) > 0.0)) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)piv * n + k], a[(size_t)col * n + k]);
        std::swap(inv[(size_t)piv * n + k], inv[(size_t)col * n + k]);
      }
    const double d = 1.0 / a[(size_t)col * n + col];
    for (int k = 0; k < n; ++k) {
      a[(size_t)col * n + k] *= d;
      inv[(size_t)col * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double m = a[(size_t)r * n + col];
      if (m == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= m * a[(size_t)col * n + k];
        inv[(size_t)r * n + k] -= m * inv[(size_t)col * n + k];
      }
    }
  }
  return true;
}

void ek_ctx::mg_setup() {
  mg = new MG();
  int nx = p.nx, ny = p.ny, nz = p.nz;
  Lvl l0{nx, ny, nz, (long long)nx * ny * nz, 1.0, nullptr, nullptr};
  mg->levels.push_back(l0);
  char* mem = mg_mem + 256;
  double h2 = 1.0;
  while (halvable(nx, ny, nz) && (int)mg->levels.size() < MAX_LEVELS) {
    nx /= 2;
    ny /= 2;
    nz /= 2;
    h2 *= 4.0;
    const long long n = (long long)nx * ny * nz;
    const size_t b = ((size_t)n * 8 + 255) & ~size_t(255);
    Lvl l{nx, ny, nz, n, h2, (double*)mem, (double*)(mem + b)};
    mem += 2 * b;
    mg->levels.push_back(l);
  }
  const int nl = (int)mg->levels.size();
  const Lvl& c = mg->levels.back();
  // LDS of the direct coarsest solve's inverse (reserved when it is planned)
  const size_t inv_bytes = nl > 1 && c.n <= COARSEST_DIRECT_MAX ? (size_t)(c.n * c.n) * 8 : 0;
  int fc = nl - 1;
  size_t bytes = 16 * (size_t)mg->levels[fc].n;
  while (fc > 1 && bytes + 16 * (size_t)mg->levels[fc - 1].n <= COARSE_LDS_BYTES) {
    --fc;
    bytes += 16 * (size_t)mg->levels[fc].n;
  }
  bytes += inv_bytes;
  // LDS of the one-workgroup kernel: up to 64 KiB by default, more where the
  // device grants it; hand it fewer levels until they fit
  auto fits = [](size_t b) {
    if (b <= 64 * 1024) return true;
    if (hipFuncSetAttribute((const void*)k_coarse_cycle, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)std::min<size_t>(b, INT_MAX)) == hipSuccess)
      return true;
    (void)hipGetLastError();
    return false;
  };
  while (nl > 1 && fc < nl - 1 && !fits(bytes)) {
    bytes -= 16 * (size_t)mg->levels[fc].n;
    ++fc;
  }
  mg->first_coarse = fc;
  mg->coarse_lds = bytes;
  // a coarsest level too large for LDS is swept on the grid instead
  mg->coarse_kernel = nl > 1 && fits(bytes);
  // the coarsest level's inverse, after the levels in the workspace
  if (nl > 1 && c.n <= COARSEST_DIRECT_MAX) {
    std::vector<double> inv;
    if (coarsest_inverse(c, inv) &&
        hipMemcpy(mem, inv.data(), inv.size() * 8, hipMemcpyHostToDevice) == hipSuccess)
      mg->pinv = (double*)mem;
    else
      (void)hipGetLastError();
  }
  // full-sweep tiles of the launched levels: the first of 64x8, 64x16 and
  // 32x8 that divides the level and gives 1024 or more workgroups at 8 or
  // more planes per workgroup, else the one with the most workgroups if
  // that is 512 or more (a smaller level keeps the half sweeps, whose
  // launches fill the chip); levels whose post-smoothing is fused with the
  // correction keep the half sweeps too
  mg->sweep_tx.assign(nl, 0);
  mg->sweep_ty.assign(nl, 0);
  mg->sweep_nch.assign(nl, 0);
  if (mg_tmp) {
    char* t = mg_tmp + 256;
    const size_t b0 = (((size_t)p.nx * p.ny * p.nz) * 8 + 255) & ~size_t(255);
    mg->tmp0 = (double*)t;
    mg->tmp2 = (double*)(t + b0 + 256);
    mg->tmp1 = (double*)(t + 2 * b0 + 512);
    for (int l = 0; l < fc; ++l) {
      const Lvl& L = mg->levels[l];
      if (L.n <= FUSED_CORRECTION_MAX_SITES) continue;
      const int cand[3][2] = {{64, 8}, {64, 16}, {32, 8}};
      long long best_wg = 0;
      for (const auto& tc : cand) {
        if (L.nx % tc[0] || L.ny % tc[1] || L.nz % 2) continue;
        const long long tiles = (long long)(L.nx / tc[0]) * (L.ny / tc[1]);
        int zc = L.nz;
        while (zc % 2 == 0 && zc / 2 >= 8 && tiles * (L.nz / zc) < 1024) zc /= 2;
        const long long wg = tiles * (L.nz / zc);
        if (wg > best_wg) {
          best_wg = wg;
          mg->sweep_tx[l] = tc[0];
          mg->sweep_ty[l] = tc[1];
          mg->sweep_nch[l] = L.nz / zc;
        }
        if (wg >= 1024) break;
      }
      if (best_wg < 512) {
        mg->sweep_tx[l] = mg->sweep_ty[l] = mg->sweep_nch[l] = 0;
        continue;
      }
      // then as many chunks as end the launch soonest (a chunk of h planes
      // takes h + 2 steps)
      const int tx = mg->sweep_tx[l], ty = mg->sweep_ty[l];
      const long long slots = tx == 32 ? resident_workgroups(k_sweep_z<32, 8>)
                              : ty == 16 ? resident_workgroups(k_sweep_z<64, 16>)
                                         : resident_workgroups(k_sweep_z<64, 8>);
      mg->sweep_nch[l] = sweep_chunks((long long)(L.nx / tx) * (L.ny / ty), L.nz, 1, 2, slots,
                                      mg->sweep_nch[l]);
    }
    mg->fused0 = fc > 1 && mg->sweep_tx[0] == 64 && mg->sweep_ty[0] == 8 &&
                 mg->levels[0].ny % ZR_TY == 0;
    if (mg->fused0) {
      // chunks of whole 2 x 2 x 2 blocks, h + 5 steps each, as many
      // workgroups at once as both variants hold
      const Lvl& L = mg->levels[0];
      const long long slots =
          std::min(resident_workgroups(k_sweep_zr<64, ZR_TY, SWEEP_RESTRICT>, ZR_THREADS),
                   resident_workgroups(k_sweep_zr<64, ZR_TY, SWEEP_NORMS>, ZR_THREADS));
      mg->zr_chunks = sweep_chunks((long long)(L.nx / 64) * (L.ny / ZR_TY), L.nz, 2, 5, slots,
                                   std::max(1, mg->sweep_nch[0] / 2));
      mg->start_chunks = sweep_chunks((long long)(L.nx / 64) * (L.ny / 8), L.nz, 1, 2,
                                      resident_workgroups(k_sweep_z<64, 8, false, true>),
                                      mg->sweep_nch[0]);
    }
  }
  mg->box.assign(nl, 0);
  for (int l = 0; mg->tmp0 && l < fc; ++l) {
    const Lvl& L = mg->levels[l];
    mg->box[l] = !mg->sweep_tx[l] && L.nx % BOX == 0 && L.ny % BOX == 0 && L.nz % BOX == 0;
  }
  mg->omega_coarsest = omega_opt(c.nx, c.ny, c.nz);
  const double rate = std::max(mg->omega_coarsest - 1.0, 1e-3);
  const double reduction = nl > 1 ? COARSEST_REDUCTION : 1e-10;
  mg->coarsest_sweeps =
      std::min(200, std::max(4, (int)std::ceil(std::log(reduction) / std::log(rate))));
}

void ek_ctx::mg_release() {
  if (mg) {
    mg->drop_graphs();
    if (mg->record_stream) (void)hipStreamDestroy(mg->record_stream);
  }
  delete mg;
  mg = nullptr;
}

// Records the launches that `enqueue` issues on `stream` into an executable
// graph; false (and nothing recorded) when that is not possible.
template <typename F>
static bool record_graph(hipStream_t stream, hipGraphExec_t* out, F enqueue) {
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  enqueue();
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(stream, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return false;
  }
  const bool ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!ok) {
    (void)hipGetLastError();
    *out = nullptr;
  }
  return ok;
}

// The two cycle graphs for (b, x); false leaves the solve on single launches.
bool ek_ctx::mg_graphs(const double* bb, double* x) {
  MG& m = *mg;
  if (!graph_launch || m.graph_failed || m.levels.size() < 2) return false;
  if (m.cycle && m.graph_b == bb && m.graph_x == x) return true;
  m.drop_graphs();
  if (!m.record_stream &&
      hipStreamCreateWithFlags(&m.record_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    m.record_stream = nullptr;
    m.graph_failed = true;
    return false;
  }
  const SiteGrid g = site_grid(p.nx, p.ny, p.nz, bx_sites);
  // the launchers enqueue on `stream`: point it at the recording stream
  const hipStream_t own = stream;
  stream = m.record_stream;
  const bool ok =
      record_graph(stream, &m.cycle, [&] { mg_vcycle(bb, x); }) &&
      record_graph(stream, &m.cycle_test, [&] {
        int nb = 0;
        mg_vcycle(bb, x, &nb);
        const int nr = nb ? nb : launch_residual(x, bb, ps, partials, dims, g, stream);
        // iteration -1: the test reads the cycle count the coarse kernel keeps
        launch_residual_final(partials, nr, p.poisson_tol, -1, 0, ps, stream);
      }) &&
      record_graph(stream, &m.cycle_first, [&] { mg_vcycle(bb, x, nullptr, false, true); }) &&
      record_graph(stream, &m.cycle_first_test, [&] {
        int nb = 0;
        mg_vcycle(bb, x, &nb, false, true);
        const int nr = nb ? nb : launch_residual(x, bb, ps, partials, dims, g, stream);
        launch_residual_final(partials, nr, p.poisson_tol, -1, 0, ps, stream);
      }) &&
      (!mg_start_in_cycle() ||
       (record_graph(stream, &m.cycle_start, [&] { mg_vcycle(bb, x, nullptr, true, true); }) &&
        record_graph(stream, &m.cycle_start_test, [&] {
          int nb = 0;
          mg_vcycle(bb, x, &nb, true, true);
          const int nr = nb ? nb : launch_residual(x, bb, ps, partials, dims, g, stream);
          launch_residual_final(partials, nr, p.poisson_tol, -1, 0, ps, stream);
        })));
  stream = own;
  if (!ok) {
    m.drop_graphs();
    m.graph_failed = true;
    return false;
  }
  m.graph_b = bb;
  m.graph_x = x;
  return true;
}

// The graph of a batch of n cycles (see ek_ctx::MG::Batch), recorded on first
// use; null when the cycle graphs are not in use or it cannot be recorded.
hipGraphExec_t ek_ctx::mg_batch_graph(const double* bb, double* x, int n, int untested, int opens) {
  MG& m = *mg;
  if (!m.cycle || m.graph_b != bb || m.graph_x != x) return nullptr;
  for (const MG::Batch& bg : m.batches)
    if (bg.n == n && bg.untested == untested && bg.opens == opens) return bg.exec;
  if (m.batch_failed || (int)m.batches.size() >= MG::MAX_BATCH_GRAPHS) return nullptr;
  const SiteGrid g = site_grid(p.nx, p.ny, p.nz, bx_sites);
  const hipStream_t own = stream;
  stream = m.record_stream;
  hipGraphExec_t exec = nullptr;
  const bool ok = record_graph(stream, &exec, [&] {
    for (int k = 0; k < n; ++k) {
      const bool test = k >= untested;
      int nb = 0;
      mg_vcycle(bb, x, test ? &nb : nullptr, opens == 2 && k == 0, opens != 0 && k == 0);
      if (!test) continue;
      const int nr = nb ? nb : launch_residual(x, bb, ps, partials, dims, g, stream);
      launch_residual_final(partials, nr, p.poisson_tol, -1, 0, ps, stream);
    }
    (void)hipMemcpyAsync(pinned, ps, sizeof(PoissonScalars), hipMemcpyDeviceToHost, stream);
  });
  stream = own;
  if (!ok) {
    m.batch_failed = true;
    return nullptr;
  }
  m.batches.push_back({n, untested, opens, exec});
  return exec;
}

// One full sweep of level L from xin into xout with the tile of the plan.
static void launch_sweep_z(const Lvl& L, int tx, int ty, int nch, const double* xin, double* xout,
                           const PoissonScalars* ps, int level0, hipStream_t s) {
  const dim3 grid((unsigned)((L.nx / tx) * (L.ny / ty) * nch));
  if (tx == 64 && ty == 16)
    hipLaunchKernelGGL((k_sweep_z<64, 16>), grid, dim3(SWEEP_THREADS), 0, s, L, xin, xout, nch, ps,
                       level0, level0 ? MG_OMEGA_FINEST : MG_OMEGA, L, nullptr);
  else if (tx == 64)
    hipLaunchKernelGGL((k_sweep_z<64, 8>), grid, dim3(SWEEP_THREADS), 0, s, L, xin, xout, nch, ps,
                       level0, level0 ? MG_OMEGA_FINEST : MG_OMEGA, L, nullptr);
  else
    hipLaunchKernelGGL((k_sweep_z<32, 8>), grid, dim3(SWEEP_THREADS), 0, s, L, xin, xout, nch, ps,
                       level0, level0 ? MG_OMEGA_FINEST : MG_OMEGA, L, nullptr);
}

// One full sweep of level L from xin into xout on BOX^3 tiles; with C the
// coarse-grid correction from level C is added on the way in.
static void launch_sweep_box(const Lvl& L, const double* xin, double* xout,
                             const PoissonScalars* ps, int level0, const Lvl* C, hipStream_t s) {
  const dim3 grid((unsigned)((L.nx / BOX) * (L.ny / BOX) * (L.nz / BOX)));
  if (C)
    hipLaunchKernelGGL((k_sweep_box<true>), grid, dim3(BOX_THREADS), 0, s, L, xin, xout, ps, level0,
                       MG_OMEGA, *C, nullptr);
  else
    hipLaunchKernelGGL((k_sweep_box<false>), grid, dim3(BOX_THREADS), 0, s, L, xin, xout, ps,
                       level0, MG_OMEGA, L, nullptr);
}

// The finest level's first pre-smoothing sweep of a solve on BOX^3 tiles with
// the residual norms of its input in `partials`; returns the block count.
static int launch_sweep_box_start(const Lvl& L, const double* xin, double* xout,
                                  const PoissonScalars* ps, double* partials, hipStream_t s) {
  const int nblocks = (L.nx / BOX) * (L.ny / BOX) * (L.nz / BOX);
  hipLaunchKernelGGL((k_sweep_box<false, true>), dim3(nblocks), dim3(BOX_THREADS), 0, s, L, xin,
                     xout, ps, 1, MG_OMEGA, L, partials);
  return nblocks;
}

// The finest level's first pre-smoothing sweep of a solve (64 x 8 tiles) with
// the residual norms of its input in `partials`; returns the block count.
static int launch_sweep_z_start(const Lvl& L, int nch, const double* xin, double* xout,
                                const PoissonScalars* ps, double* partials, hipStream_t s) {
  const int nblocks = (L.nx / 64) * (L.ny / 8) * nch;
  hipLaunchKernelGGL((k_sweep_z<64, 8, false, true>), dim3(nblocks), dim3(SWEEP_THREADS), 0, s, L,
                     xin, xout, nch, ps, 1, MG_OMEGA_FINEST, L, partials);
  return nblocks;
}

// A first post-smoothing sweep with the correction from level C on the way
// in (64 x 8 tiles): xout = sweep(xin + P e).
static void launch_sweep_z_corrected(const Lvl& L, const Lvl& C, int nch, const double* xin,
                                     double* xout, const PoissonScalars* ps, int level0,
                                     hipStream_t s) {
  const dim3 grid((unsigned)((L.nx / 64) * (L.ny / 8) * nch));
  hipLaunchKernelGGL((k_sweep_z<64, 8, true>), grid, dim3(SWEEP_THREADS), 0, s, L, xin, xout, nch,
                     ps, level0, level0 ? MG_OMEGA_FINEST : MG_OMEGA, C, nullptr);
}

// The finest level's full sweep with the residual of its result (restriction
// into level C, or the norms' block partials) in nch chunks along z; returns
// the block count.
static int launch_sweep_zr(const Lvl& L, int nch, const double* xin, double* xout,
                           const PoissonScalars* ps, int mode, const Lvl& C, double omega_red,
                           double* partials, hipStream_t s) {
  const int nblocks = (L.nx / 64) * (L.ny / ZR_TY) * nch;
  if (mode == SWEEP_RESTRICT)
    hipLaunchKernelGGL((k_sweep_zr<64, ZR_TY, SWEEP_RESTRICT>), dim3(nblocks), dim3(ZR_THREADS), 0,
                       s, L, xin, xout, nch, ps, 1, MG_OMEGA_FINEST, C, omega_red, partials);
  else
    hipLaunchKernelGGL((k_sweep_zr<64, ZR_TY, SWEEP_NORMS>), dim3(nblocks), dim3(ZR_THREADS), 0, s,
                       L, xin, xout, nch, ps, 1, MG_OMEGA_FINEST, C, 0.0, partials);
  return nblocks;
}

bool ek_ctx::mg_start_in_cycle() const {
  return mg && ((mg->fused0 && NU1_FUSED >= 2) || (!mg->box.empty() && mg->box[0]));
}

ek_status ek_ctx::mg_vcycle(const double* bb, double* x, int* norm_blocks, bool start, bool first) {
  if (norm_blocks) *norm_blocks = 0;
  std::vector<Lvl>& L = mg->levels;
  L[0].x = x;
  L[0].f = const_cast<double*>(bb);
  const int fc = mg->first_coarse;
  const int nl = (int)L.size();
  if (nl == 1) {   // no coarser level: red-black SOR at the optimal factor
    for (int s = 0; s < mg->coarsest_sweeps; ++s)
      for (int c = 0; c < 2; ++c)
        hipLaunchKernelGGL(k_smooth, colour_launch(L[0]).grid, colour_launch(L[0]).block, 0, stream,
                           L[0], c, ps, 1, mg->omega_coarsest);
    return EK_OK;
  }
  // Levels 1 .. fc-1 arrive from the restriction with their first colour-0
  // half sweep done; the level handed to the coarse kernel arrives at zero.
  // The finest level with a full-sweep plan is pre-smoothed by one full
  // sweep into tmp0 (NU1 = 1), restricted from there, and corrected back
  // into x by the prolongation; with the fused restriction by NU1_FUSED
  // sweeps, which end in tmp0 (corrected into x as before) or in x
  // (corrected in place).
  static_assert(NU1 == 1 && NU2 % 2 == 0 && NU1_FUSED >= 2 && NU1_FUSED_NEXT >= 1,
                "the out-of-place sweeps end in x");
  first = first || start;
  const int nu1_fused = first ? NU1_FUSED : NU1_FUSED_NEXT;
  const int nu1_finest = first ? NU1_FINEST : NU1_FINEST_NEXT;
  const bool pre_in_x = mg->fused0 && nu1_fused % 2 == 0;
  const bool pre0 = mg->sweep_tx[0] != 0;
  for (int l = 0; l < fc; ++l) {
    Lvl F = L[l];
    const double omega_red = (l + 1 < fc && NU1 > 0) ? MG_OMEGA : 0.0;
    if (l > 0 && mg->box[l] && NU1 == 1) {   // its colour-1 half sweep and the restriction
      hipLaunchKernelGGL(k_restrict_box, dim3((unsigned)((F.nx / BOX) * (F.ny / BOX) * (F.nz / BOX))),
                         dim3(BOX_THREADS), 0, stream, F, L[l + 1], ps, MG_OMEGA, omega_red);
      continue;
    }
    if (l == 0 && mg->fused0) {
      // nu1_fused sweeps back and forth between x and tmp0, the last one
      // with the restriction in the same pass
      double* a = x;
      double* b = mg->tmp0;
      for (int s = 0; s + 1 < nu1_fused; ++s) {
        if (s == 0 && start) {   // the start's residual, then its test
          const int nb = launch_sweep_z_start(L[0], mg->start_chunks, a, b, ps, partials, stream);
          launch_residual_final(partials, nb, p.poisson_tol, 0, 1, ps, stream);
        } else {
          launch_sweep_z(L[0], 64, 8, mg->sweep_nch[0], a, b, ps, 1, stream);
        }
        std::swap(a, b);
      }
      launch_sweep_zr(L[0], mg->zr_chunks, a, b, ps, SWEEP_RESTRICT, L[1], omega_red, nullptr,
                      stream);
      continue;
    }
    if (l == 0 && pre0) {
      launch_sweep_z(L[0], mg->sweep_tx[0], mg->sweep_ty[0], mg->sweep_nch[0], x, mg->tmp0, ps, 1,
                     stream);
      F.x = mg->tmp0;
    } else if (l == 0 && mg->box[0]) {
      // nu1_finest full sweeps x -> tmp0 -> x
      static_assert(NU1_FINEST % 2 == 0 && NU1_FINEST_NEXT % 2 == 0, "the box sweeps end in x");
      for (int s = 0; s < nu1_finest; ++s) {
        const double* in = s % 2 ? mg->tmp0 : x;
        double* out = s % 2 ? x : mg->tmp0;
        if (s == 0 && start) {   // the start's residual, then its test
          const int nb = launch_sweep_box_start(L[0], in, out, ps, partials, stream);
          launch_residual_final(partials, nb, p.poisson_tol, 0, 1, ps, stream);
        } else {
          launch_sweep_box(L[0], in, out, ps, 1, nullptr, stream);
        }
      }
    } else {
      for (int s = 0; s < (l == 0 ? nu1_finest : NU1); ++s)
        for (int c = 0; c < 2; ++c) {
          if (l > 0 && s == 0 && c == 0) continue;
          hipLaunchKernelGGL(k_smooth, colour_launch(L[l]).grid, colour_launch(L[l]).block, 0,
                             stream, L[l], c, ps, l == 0 ? 1 : 0, MG_OMEGA);
        }
    }
    hipLaunchKernelGGL(k_restrict, level_launch(L[l + 1]).grid, level_launch(L[l + 1]).block, 0,
                       stream, F, L[l + 1], ps, l == 0 ? 1 : 0, omega_red);
  }
  if (mg->coarse_kernel) {
    LvlSet set{};
    set.count = nl;
    for (int l = 0; l < nl; ++l) set.l[l] = L[l];
    hipLaunchKernelGGL(k_coarse_cycle, dim3(1), dim3(1024), mg->coarse_lds, stream, set, fc, ps,
                       mg->omega_coarsest, mg->coarsest_sweeps, mg->pinv);
  } else {
    // the coarsest level (arriving at zero) by red-black SOR sweeps over the
    // grid at its optimal factor; the cycle is counted as the coarse kernel
    // would count it
    const Lvl& C = L[nl - 1];
    for (int s = 0; s < mg->coarsest_sweeps; ++s)
      for (int c = 0; c < 2; ++c)
        hipLaunchKernelGGL(k_smooth, colour_launch(C).grid, colour_launch(C).block, 0, stream, C, c,
                           ps, 0, mg->omega_coarsest);
    hipLaunchKernelGGL(k_count_cycle, dim3(1), dim3(64), 0, stream, ps);
  }
  // coarse-grid correction: fused into the first post-smoothing sweep on
  // levels up to FUSED_CORRECTION_MAX_SITES, a pass of its own above
  for (int l = fc - 1; l >= 0; --l) {
    if (l == 0 && mg->fused0) {
      // the correction inside the first post-smoothing sweep, from the
      // pre-smoothed iterate (in x or tmp0) into the other of tmp0 and tmp2,
      // then the second sweep back into x (with the test's residual norms)
      static_assert(NU2 == 2, "one sweep after the corrected one");
      const double* pre = pre_in_x ? x : mg->tmp0;
      double* mid = pre_in_x ? mg->tmp0 : mg->tmp2;
      launch_sweep_z_corrected(L[0], L[1], mg->sweep_nch[0], pre, mid, ps, 1, stream);
      if (norm_blocks)
        *norm_blocks = launch_sweep_zr(L[0], mg->zr_chunks, mid, x, ps, SWEEP_NORMS, L[1], 0.0,
                                       partials, stream);
      else
        launch_sweep_z(L[0], 64, 8, mg->sweep_nch[0], mid, x, ps, 1, stream);
      continue;
    }
    if (mg->box[l]) {
      // the correction inside the first of the NU2 full sweeps, x -> tmp -> x
      static_assert(NU2 == 2, "the box sweeps end in x");
      double* tmp = l == 0 ? mg->tmp0 : mg->tmp1;
      launch_sweep_box(L[l], L[l].x, tmp, ps, l == 0 ? 1 : 0, &L[l + 1], stream);
      launch_sweep_box(L[l], tmp, L[l].x, ps, l == 0 ? 1 : 0, nullptr, stream);
      continue;
    }
    if (mg->sweep_tx[l]) {
      // correction (out of place from tmp0 on the finest level), then NU2
      // full sweeps x -> tmp -> x; on 64 x 8 tiles of a coarser level the
      // correction rides on the first of them
      double* tmp = l == 0 ? mg->tmp0 : mg->tmp1;
      const bool corrected = l > 0 && mg->sweep_tx[l] == 64 && mg->sweep_ty[l] == 8;
      if (corrected)
        launch_sweep_z_corrected(L[l], L[l + 1], mg->sweep_nch[l], L[l].x, tmp, ps, 0, stream);
      else if (l == 0 && pre0 && !pre_in_x)
        hipLaunchKernelGGL(k_prolong_to, level_launch(L[1]).grid, level_launch(L[1]).block, 0,
                           stream, L[0], L[1], mg->tmp0, x, ps);
      else
        hipLaunchKernelGGL(k_prolong, level_launch(L[l + 1]).grid, level_launch(L[l + 1]).block, 0,
                           stream, L[l], L[l + 1], ps);
      for (int s = corrected ? 1 : 0; s < NU2; ++s) {
        const bool to_tmp = (s & 1) == 0;
        if (l == 0 && s == NU2 - 1 && norm_blocks && mg->fused0) {   // the test's residual too
          *norm_blocks = launch_sweep_zr(L[0], mg->zr_chunks, tmp, L[0].x, ps, SWEEP_NORMS,
                                         L[1], 0.0, partials, stream);
          continue;
        }
        launch_sweep_z(L[l], mg->sweep_tx[l], mg->sweep_ty[l], mg->sweep_nch[l],
                       to_tmp ? L[l].x : tmp, to_tmp ? tmp : L[l].x, ps, l == 0 ? 1 : 0, stream);
      }
      continue;
    }
    const bool fused = NU2 > 0 && L[l].n <= FUSED_CORRECTION_MAX_SITES;
    if (!fused)
      hipLaunchKernelGGL(k_prolong, level_launch(L[l + 1]).grid, level_launch(L[l + 1]).block, 0,
                         stream, L[l], L[l + 1], ps);
    for (int s = 0; s < NU2; ++s)
      for (int c = 0; c < 2; ++c) {
        if (fused && s == 0)
          hipLaunchKernelGGL(k_corrected_smooth, colour_launch(L[l]).grid, colour_launch(L[l]).block,
                             0, stream, L[l], L[l + 1], c, ps, l == 0 ? 1 : 0, MG_OMEGA);
        else
          hipLaunchKernelGGL(k_smooth, colour_launch(L[l]).grid, colour_launch(L[l]).block, 0,
                             stream, L[l], c, ps, l == 0 ? 1 : 0, MG_OMEGA);
      }
  }
  return EK_OK;
}

// V-cycles until ||b - A psi|| / ||b|| <= tol, tested after every cycle;
// cycles are enqueued ahead of the test in batches and skip themselves once
// the device-side flag is set.
ek_status ek_ctx::mg_solve(const double* bb, double* x, PoissonScalars h, int& iters, double& res,
                          double& res0, bool start_norms) {
  const SiteGrid g = site_grid(p.nx, p.ny, p.nz, bx_sites);
  ek_status st = EK_OK;
  int it = 0;
  int batch = std::max(1, last_iters);
  // the previous solve needed `batch` cycles: the residual is first tested
  // after batch - 1 of them (a solve that converges earlier than that costs
  // one extra cycle, the usual one saves the tests of the early cycles), or
  // in the time loop, whose consecutive solves start alike, only after the
  // batch when the previous step's residual one cycle before its end (its
  // last residual over its mean rate per cycle) lay more than EARLY_MARGIN
  // times above the tolerance
  int untested = std::max(0, batch - 2);
  if (!solo && batch >= 2 && last_res > 0.0 && last_res0 > last_res) {
    const double rate = std::pow(last_res / last_res0, 1.0 / batch);
    if (last_res / rate > EARLY_MARGIN * p.poisson_tol) untested = batch - 1;
  }
  const bool graphs = mg_graphs(bb, x);
  while (!h.done && it < p.poisson_max_iter) {
    const int nrun = std::min(batch, p.poisson_max_iter - it);
    // the batch as one graph where its tests follow the rule alone (a batch
    // that reaches the cycle limit also tests its last cycle)
    hipGraphExec_t bg = graphs && it + nrun < p.poisson_max_iter
                            ? mg_batch_graph(bb, x, nrun, std::min(untested, nrun),
                                             it == 0 ? (start_norms ? 2 : 1) : 0)
                            : nullptr;
    if (bg) {
      const hipError_t e = hipGraphLaunch(bg, stream);
      if (e != hipSuccess) return fail(EK_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
      it += nrun;
      untested = 0;
      st = sync();
      if (st) return st;
      std::memcpy(&h, pinned, sizeof(PoissonScalars));
      batch = 1;
      continue;
    }
    for (int k = 0; k < nrun; ++k) {
      ++it;
      const bool test = k >= untested || it >= p.poisson_max_iter;
      const bool first = it == 1;
      const bool start = start_norms && first;   // the cycle also evaluates the start
      if (graphs) {
        hipGraphExec_t ge = start   ? (test ? mg->cycle_start_test : mg->cycle_start)
                            : first ? (test ? mg->cycle_first_test : mg->cycle_first)
                                    : (test ? mg->cycle_test : mg->cycle);
        const hipError_t e = hipGraphLaunch(ge, stream);
        if (e != hipSuccess) return fail(EK_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        continue;
      }
      int nb = 0;
      st = mg_vcycle(bb, x, test ? &nb : nullptr, start, first);
      if (st) return st;
      if (!test) continue;
      const int nr = nb ? nb : launch_residual(x, bb, ps, partials, dims, g, stream);
      launch_residual_final(partials, nr, p.poisson_tol, it, 0, ps, stream);
    }
    untested = 0;
    st = read_scalars(&h);
    if (st) return st;
    batch = 1;
  }
  res0 = h.rel0;
  res = h.rel;
  if (!h.done) {
    iters = it;
    char buf[160];
    std::snprintf(buf, sizeof buf, "multigrid did not reach %.3g in %d cycles (residual %.3e)",
                  p.poisson_tol, p.poisson_max_iter, h.rel);
    return fail(EK_ENOCONV, buf);
  }
  iters = h.iters;
  if (defer_shift) shift_pending = true;
  else launch_psi_shift(x, ps, 1.0 / double(dims.n), dims, stream);
  return EK_OK;
}
