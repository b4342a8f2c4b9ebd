// Multigrid level description and per-site operations, shared by the
// grid-wide multigrid kernels and the persistent ensemble kernel.
//   level l, spacing h = 2^l:  (sum of 6 neighbours - 6 x) / h^2 = f_l
//   smoother     red-black Gauss-Seidel over-relaxed by MG_OMEGA
//   restriction  f_{l+1} = average of the 8 fine residuals; zeroes x_{l+1}
//   prolongation trilinear cell-centred interpolation (3/4, 1/4 per axis)
#pragma once

#include <hip/hip_runtime.h>

#include "ek_internal.h"

namespace ek {

// Pre- and post-smoothing sweeps of the launched multigrid (one launch per
// half sweep): V(1,2) reaches the tolerance in about the same number of
// cycles as V(2,2) on the pore systems (4.0-4.2 against 4.0 per step from the
// previous solution) with a quarter fewer launches per cycle.  The finest
// level takes more pre-smoothing sweeps (NU1_FINEST, NU1_FUSED in
// kernels_mg.hip): from the extrapolated starts its extra sweeps save whole
// cycles.
constexpr int NU1 = 1, NU2 = 2;
// Relaxation factor of the red-black smoother on every level but the
// coarsest: over-relaxed red-black Gauss-Seidel smooths the 7-point operator
// faster than plain Gauss-Seidel; at 1.25 a V(2,2) cycle cuts the residual of
// the pore systems by about 0.01 instead of 0.05, and 1.25 is also the best
// of 1.15, 1.25 and 1.35 for V(1,2) (the coarsest level uses the optimal SOR
// factor of its own grid).
constexpr double MG_OMEGA = 1.25;
constexpr int MAX_LEVELS = 16;

struct Lvl {
  int nx, ny, nz;
  long long n;
  double h2;
  double* x;
  double* f;
};

struct LvlSet {
  Lvl l[MAX_LEVELS];
  int count;
};

// q = t / d and t - q d for 0 <= t < 2^24 without an integer divide: the
// float quotient is off by at most one, which the remainder test corrects.
__device__ inline int fdivmod(int t, int d, float inv_d, int& rem) {
  int q = int(float(t) * inv_d);
  int r = t - q * d;
  if (r < 0) { --q; r += d; }
  else if (r >= d) { ++q; r -= d; }
  rem = r;
  return q;
}

__device__ inline int idx3(int x, int y, int z, const Lvl& L) {
  return (z * L.ny + y) * L.nx + x;
}

__device__ inline double nbsum(const double* __restrict__ v, int x, int y, int z, const Lvl& L) {
  const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
  return v[idx3(xm, y, z, L)] + v[idx3(xp, y, z, L)] + v[idx3(x, ym, z, L)] +
         v[idx3(x, yp, z, L)] + v[idx3(x, y, zm, L)] + v[idx3(x, y, zp, L)];
}

// --- per-site operations shared by the grid-wide and single-block kernels ---
// (tx, y, z) enumerates the sites of one colour: nx/2 per row
__device__ inline void smooth_site(const Lvl& L, int colour, int tx, int y, int z, double shift,
                                   double omega = 1.0) {
  const int x = 2 * tx + ((colour + y + z) & 1);
  const int r = idx3(x, y, z, L);
  const double xo = L.x[r];   // read with the neighbours, not after their sum
  const double gs = (nbsum(L.x, x, y, z, L) - L.h2 * (L.f[r] + shift)) * (1.0 / 6.0);
  L.x[r] = omega == 1.0 ? gs : xo + omega * (gs - xo);
}

// omega_red != 0: the coarse level's first colour-0 half sweep is done here
// as well (from the zero start it only needs the site's own right-hand side).
// h^2 is a power of two, so multiplying by its reciprocal equals dividing by it.
__device__ inline void restrict_site(const Lvl& F, const Lvl& C, int X, int Y, int Z, double shift,
                                     double omega_red = 0.0) {
  const double ih2 = 1.0 / F.h2;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int x = 2 * X + (k & 1), y = 2 * Y + ((k >> 1) & 1), z = 2 * Z + ((k >> 2) & 1);
    const int r = idx3(x, y, z, F);
    s += (F.f[r] + shift) - (nbsum(F.x, x, y, z, F) - 6.0 * F.x[r]) * ih2;
  }
  const int t = idx3(X, Y, Z, C);
  const double f = 0.125 * s;
  C.f[t] = f;
  double x0 = 0.0;
  if (omega_red != 0.0 && ((X + Y + Z) & 1) == 0) {
    const double gs = (0.0 - C.h2 * (f + 0.0)) * (1.0 / 6.0);
    x0 = omega_red == 1.0 ? gs : 0.0 + omega_red * (gs - 0.0);
  }
  C.x[t] = x0;
}

// Coarse-grid correction at fine site (x, y, z) (trilinear, cell-centred).
__device__ inline double prolong_value(const Lvl& C, int x, int y, int z) {
  const int X = x >> 1, Y = y >> 1, Z = z >> 1;
  const int Xn = (x & 1) ? (X + 1 == C.nx ? 0 : X + 1) : (X == 0 ? C.nx - 1 : X - 1);
  const int Yn = (y & 1) ? (Y + 1 == C.ny ? 0 : Y + 1) : (Y == 0 ? C.ny - 1 : Y - 1);
  const int Zn = (z & 1) ? (Z + 1 == C.nz ? 0 : Z + 1) : (Z == 0 ? C.nz - 1 : Z - 1);
  const double a = 0.75, b = 0.25;
  return a * a * a * C.x[idx3(X, Y, Z, C)] + b * a * a * C.x[idx3(Xn, Y, Z, C)] +
         a * b * a * C.x[idx3(X, Yn, Z, C)] + a * a * b * C.x[idx3(X, Y, Zn, C)] +
         b * b * a * C.x[idx3(Xn, Yn, Z, C)] + b * a * b * C.x[idx3(Xn, Y, Zn, C)] +
         a * b * b * C.x[idx3(X, Yn, Zn, C)] + b * b * b * C.x[idx3(Xn, Yn, Zn, C)];
}

__device__ inline void prolong_site(const Lvl& F, const Lvl& C, int x, int y, int z) {
  F.x[idx3(x, y, z, F)] += prolong_value(C, x, y, z);
}

// The corrections of the 8 fine children of coarse cell (X, Y, Z), each the
// sum of prolong_value term by term, from the cell's 3x3x3 coarse
// neighbourhood read once; the two children in a fine row are adjacent.
// src and dst are fine-level iterates (the same array for the in-place
// correction).
__device__ inline void prolong_cell(const Lvl& F, const Lvl& C, int X, int Y, int Z,
                                    const double* src, double* dst) {
  const int xs[3] = {X == 0 ? C.nx - 1 : X - 1, X, X + 1 == C.nx ? 0 : X + 1};
  const int ys[3] = {Y == 0 ? C.ny - 1 : Y - 1, Y, Y + 1 == C.ny ? 0 : Y + 1};
  const int zs[3] = {Z == 0 ? C.nz - 1 : Z - 1, Z, Z + 1 == C.nz ? 0 : Z + 1};
  double c[3][3][3];   // [z][y][x], centre at [1][1][1]
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) c[k][j][i] = C.x[idx3(xs[i], ys[j], zs[k], C)];
  const double a = 0.75, b = 0.25;
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy) {
      const int zn = oz ? 2 : 0, yn = oy ? 2 : 0;
      const int r0 = idx3(2 * X, 2 * Y + oy, 2 * Z + oz, F);
      const double v0 = src[r0], v1 = src[r0 + 1];
      double e[2];
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const int xn = ox ? 2 : 0;
        e[ox] = a * a * a * c[1][1][1] + b * a * a * c[1][1][xn] + a * b * a * c[1][yn][1] +
                a * a * b * c[zn][1][1] + b * b * a * c[1][yn][xn] + b * a * b * c[zn][1][xn] +
                a * b * b * c[zn][yn][1] + b * b * b * c[zn][yn][xn];
      }
      dst[r0] = v0 + e[0];
      dst[r0 + 1] = v1 + e[1];
    }
}

__device__ inline void prolong_cell(const Lvl& F, const Lvl& C, int X, int Y, int Z) {
  prolong_cell(F, C, X, Y, Z, F.x, F.x);
}

// First post-smoothing sweep with the coarse-grid correction applied on the
// fly (no separate prolongation pass).  Colour 0: the site and its six
// neighbours (colour 1, not yet corrected) are read corrected; colour 1
// (after colour 0): the site is corrected, its neighbours are final.  Equal
// to a prolongation followed by the two half sweeps.
__device__ inline void corrected_smooth_site(const Lvl& L, const Lvl& C, int colour, int tx, int y,
                                             int z, double shift, double omega) {
  const int x = 2 * tx + ((colour + y + z) & 1);
  const int r = idx3(x, y, z, L);
  const double xo = L.x[r] + prolong_value(C, x, y, z);
  double nb = nbsum(L.x, x, y, z, L);
  if (colour == 0) {
    const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
    nb += prolong_value(C, xm, y, z) + prolong_value(C, xp, y, z) + prolong_value(C, x, ym, z) +
          prolong_value(C, x, yp, z) + prolong_value(C, x, y, zm) + prolong_value(C, x, y, zp);
  }
  const double gs = (nb - L.h2 * (L.f[r] + shift)) * (1.0 / 6.0);
  L.x[r] = omega == 1.0 ? gs : xo + omega * (gs - xo);
}

// --- the coarse part of a V-cycle in one workgroup ----------------------------
// The level descriptions are taken by value: in registers the compiler need
// not read them again after every store to the level's arrays (a descriptor
// kept in LDS may alias them).
__device__ inline void block_smooth(const Lvl L, int sweeps, double shift, double omega = 1.0) {
  const int hx = L.nx / 2, nh = hx * L.ny * L.nz;
  const float ihx = 1.0f / hx, iny = 1.0f / L.ny;
  for (int s = 0; s < sweeps; ++s)
    for (int colour = 0; colour < 2; ++colour) {
      for (int t = threadIdx.x; t < nh; t += blockDim.x) {
        int tx, y;
        const int yz = fdivmod(t, hx, ihx, tx);
        const int z = fdivmod(yz, L.ny, iny, y);
        smooth_site(L, colour, tx, y, z, shift, omega);
      }
      __syncthreads();
    }
}

// One colour of a red-black sweep of a whole level by one workgroup.
__device__ inline void block_half(const Lvl L, int colour, double shift, double omega) {
  const int hx = L.nx / 2, nh = hx * L.ny * L.nz;
  const float ihx = 1.0f / hx, iny = 1.0f / L.ny;
  for (int t = threadIdx.x; t < nh; t += blockDim.x) {
    int tx, y;
    const int yz = fdivmod(t, hx, ihx, tx);
    const int z = fdivmod(yz, L.ny, iny, y);
    smooth_site(L, colour, tx, y, z, shift, omega);
  }
  __syncthreads();
}

// Restriction and prolongation of a whole level by one workgroup
// (omega_red as in restrict_site).
__device__ inline void block_restrict(const Lvl F, const Lvl C, double shift,
                                      double omega_red = 0.0) {
  const float inx = 1.0f / C.nx, iny = 1.0f / C.ny;
  for (int t = threadIdx.x; t < int(C.n); t += blockDim.x) {
    int X, Y;
    const int yz = fdivmod(t, C.nx, inx, X);
    const int Z = fdivmod(yz, C.ny, iny, Y);
    restrict_site(F, C, X, Y, Z, shift, omega_red);
  }
  __syncthreads();
}

__device__ inline void block_prolong(const Lvl F, const Lvl C) {
  const float inx = 1.0f / F.nx, iny = 1.0f / F.ny;
  for (int t = threadIdx.x; t < int(F.n); t += blockDim.x) {
    int x, y;
    const int yz = fdivmod(t, F.nx, inx, x);
    const int z = fdivmod(yz, F.ny, iny, y);
    prolong_site(F, C, x, y, z);
  }
  __syncthreads();
}

}  // namespace ek
