// Per-site bodies of the charge pass and of the fused pull-stream + collide
// step, shared by the grid-wide kernels (one thread per site) and by the
// persistent ensemble kernel (a workgroup striding over one replica).
//
// Storage: populations of the three species are structure-of-arrays planes
// f[(s * 19 + p) * N + site], site = (z * ny + y) * nx + x, holding the
// post-collision values of the previous step.  A thread pulls f*_p(r - c_p)
// (halfway bounce-back: f*_opp(p)(r) when r - c_p is solid), which makes every
// read of a plane a shifted but coalesced row and every write aligned.  Values
// are stored as deviations from rest, g_p = f_p - w_p nref^a, so that float32
// keeps the small velocity-carrying part of the populations to full relative
// precision.
#pragma once

#include "ek_internal.h"
#include "md_table.h"
#include "philox.h"

namespace ek {

// Offsets of the rows r - c for one site: index [1 - c] selects minus, same,
// plus.  I is the index type: 32-bit when every element offset within one
// species' 19 planes fits (fewer address instructions), 64-bit otherwise.
template <typename I>
struct NbrT {
  I zo[3], yo[3], xo[3];
};
using Nbr = NbrT<long long>;

template <typename I>
__device__ inline NbrT<I> neighbours_t(int x, int y, int z, const Dims& d) {
  NbrT<I> n;
  const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const I nxy = I(d.nx) * I(d.ny);
  n.zo[0] = I(zm) * nxy; n.zo[1] = I(z) * nxy; n.zo[2] = I(zp) * nxy;
  n.yo[0] = I(ym) * I(d.nx); n.yo[1] = I(y) * I(d.nx); n.yo[2] = I(yp) * I(d.nx);
  n.xo[0] = I(xm); n.xo[1] = I(x); n.xo[2] = I(xp);
  return n;
}
__device__ inline Nbr neighbours(int x, int y, int z, const Dims& d) {
  return neighbours_t<long long>(x, y, z, d);
}

// True when 19 planes of n sites of T can be addressed with 32-bit element
// offsets from a species' base.
template <typename T>
__host__ __device__ inline bool fits_idx32(long long n) {
  return (unsigned long long)n * Q * sizeof(T) < (1ull << 32);
}

// The 19 planes of one species, read through a plain pointer with index
// type I.
template <typename T, typename I>
struct Planes {
  const T* base;
  __device__ Planes(const T* b, I) : base(b) {}
  __device__ T load(I idx) const { return base[idx]; }
};

// Writes of plane p at site r of one species, as non-temporal stores: the
// populations of a step are read again only by the next step's passes, after
// the Poisson solve has streamed its own fields through the caches, so
// keeping them there gains nothing (the stores' streaming hint took the
// 256x256x512 pore's fused step from 3.04 to 2.92 ms, and the chain beside it
// from 1.9 to 1.4 ms).
template <typename T, typename I>
struct PlanesOut {
  T* base;
  I n;
  __device__ PlanesOut(T* b, I nn) : base(b), n(nn) {}
  __device__ void store(int p, I r, T v) const {
    __builtin_nontemporal_store(v, (base + (size_t)p * n) + r);
  }
};

// Pull the 19 post-collision deviations of one species into a site.
template <typename T, typename I>
__device__ inline void pull(const Planes<T, I>& fs, I r, uint32_t m, const NbrT<I>& nb, I N,
                            T (&g)[Q]) {
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    const bool bounce = (m >> p) & 1u;
    const I src = nb.zo[1 - CZ[p]] + nb.yo[1 - CY[p]] + nb.xo[1 - CX[p]];
    const I idx = bounce ? I(OPP[p]) * N + r : I(p) * N + src;
    g[p] = fs.load(idx);
  }
}
template <typename T>
__device__ inline void pull(const T* __restrict__ f, int s, long long r, uint32_t m,
                            const Nbr& nb, long long N, T (&g)[Q]) {
  pull<T, long long>(Planes<T, long long>(f + (size_t)s * Q * N, N), r, m, nb, N, g);
}

// 1 / x: the hardware reciprocal (1 ulp) in float32, division in float64.
template <typename T>
__device__ inline T recip(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);
  else return T(1) / x;
}

// Charge density at site (x, y, z): sum of z^a n^a over the charged species
// (fluid sites), the fixed wall charge and the beads' deposited charge.
// With NEU (insulating walls) solid sites carry nothing and a fluid site adds
// the surface charge of its wall faces (stored at the solid face neighbours,
// `wall_q` then holding Sigma_f).
template <typename T, typename I = long long, bool NEU = false>
__device__ inline double charge_site(const T* __restrict__ f, const uint32_t* __restrict__ mask,
                                     const double* __restrict__ wall_q, const LBParams& lp,
                                     const BeadTableView& bt, int x, int y, int z, const Dims& d) {
  const I N = I(d.n);
  const I r = (I(z) * I(d.ny) + I(y)) * I(d.nx) + I(x);
  const uint32_t m = mask[r];
  double rho = 0.0;
  if (NEU && (m & MASK_SOLID)) return 0.0;
  if (!NEU && (m & MASK_CHARGED)) rho += wall_q[r];
  if (!(m & MASK_SOLID)) {
    const NbrT<I> nb = neighbours_t<I>(x, y, z, d);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (lp.valence[s] == 0.0) continue;
      T g[Q];
      pull<T, I>(Planes<T, I>(f + (size_t)s * Q * d.n, N), r, m, nb, N, g);
      T dn = T(0);
#pragma unroll
      for (int p = 0; p < Q; ++p) dn += g[p];
      rho += lp.valence[s] * (lp.nref[s] + double(dn));
    }
    if constexpr (NEU) {
#pragma unroll
      for (int p = 1; p <= 6; ++p)
        if ((m >> p) & 1u) rho += wall_q[nb.zo[1 - CZ[p]] + nb.yo[1 - CY[p]] + nb.xo[1 - CX[p]]];
    }
  }
  if (m & MASK_BEAD) rho += bt.charge_at(r);
  return rho;
}

// Fused step at one fluid site: pull + bounce-back, moments, field from the
// potential, closed-form implicit drag, BGK collision with the half-force
// (Guo) forcing term, with FLUCT the stochastic term of the populations
// (philox.h), aligned store.  Adds the site's species masses and momentum of
// f(t) to acc[0..5] (float64).  Sites whose link word has one of the `skip`
// bits are left alone; returns whether the site was updated.
template <typename T, typename I = long long, int NA, bool FLUCT = false, bool NEU = false>
__device__ inline bool lb_site(const T* __restrict__ fsrc, T* __restrict__ fdst,
                               const uint32_t* __restrict__ mask, const double* __restrict__ psi,
                               const LBParams& lp, const BeadTableView& bt, int x, int y, int z,
                               const Dims& d, double (&acc)[NA], uint32_t skip = 0u,
                               const NoiseParams* noise = nullptr,
                               const WallView* walls = nullptr) {
  static_assert(NA >= 6, "masses and momentum take six sums");
  const I N = I(d.n);
  const I r = (I(z) * I(d.ny) + I(y)) * I(d.nx) + I(x);
  const uint32_t m = mask[r];
  if (m & (MASK_SOLID | skip)) return false;
  {
    const NbrT<I> nb = neighbours_t<I>(x, y, z, d);
    T g[3][Q];
#pragma unroll
    for (int s = 0; s < 3; ++s)
      pull<T, I>(Planes<T, I>(fsrc + (size_t)s * Q * d.n, N), r, m, nb, N, g[s]);

    // electric field E = -grad psi (central differences) + applied field;
    // with insulating walls a solid face neighbour is replaced by the ghost
    // value psi_r + Sigma_f / eps of its face (bit p of the link word: the
    // neighbour r - c_p is solid; bits 1/2 are -x/+x, 3/4 -y/+y, 5/6 -z/+z)
    T ex, ey, ez;
    if constexpr (NEU) {
      const double pc = psi[r];
      auto side = [&](int bit, I idx) -> double {
        return ((m >> bit) & 1u) ? pc + walls->face_q[idx] * walls->inv_eps : psi[idx];
      };
      ex = T(-0.5 * (side(2, nb.zo[1] + nb.yo[1] + nb.xo[2]) - side(1, nb.zo[1] + nb.yo[1] + nb.xo[0])) + lp.eext[0]);
      ey = T(-0.5 * (side(4, nb.zo[1] + nb.yo[2] + nb.xo[1]) - side(3, nb.zo[1] + nb.yo[0] + nb.xo[1])) + lp.eext[1]);
      ez = T(-0.5 * (side(6, nb.zo[2] + nb.yo[1] + nb.xo[1]) - side(5, nb.zo[0] + nb.yo[1] + nb.xo[1])) + lp.eext[2]);
    } else {
      ex = T(-0.5 * (psi[nb.zo[1] + nb.yo[1] + nb.xo[2]] - psi[nb.zo[1] + nb.yo[1] + nb.xo[0]]) + lp.eext[0]);
      ey = T(-0.5 * (psi[nb.zo[1] + nb.yo[2] + nb.xo[1]] - psi[nb.zo[1] + nb.yo[0] + nb.xo[1]]) + lp.eext[1]);
      ez = T(-0.5 * (psi[nb.zo[2] + nb.yo[1] + nb.xo[1]] - psi[nb.zo[0] + nb.yo[1] + nb.xo[1]]) + lp.eext[2]);
    }

    double kb[3][3];
    const bool has_bead = (m & MASK_BEAD) != 0;
    if (has_bead) bt.force_at(r, kb);

    // moments, force per particle G^a (without the drag) and
    // b^a = j^a / n^a + G^a / 2
    T n[3], dns[3], G[3][3], bv[3][3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      T dn = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        dn += g[s][p];
        if (CX[p]) jx += CX[p] > 0 ? g[s][p] : -g[s][p];
        if (CY[p]) jy += CY[p] > 0 ? g[s][p] : -g[s][p];
        if (CZ[p]) jz += CZ[p] > 0 ? g[s][p] : -g[s][p];
      }
      n[s] = T(lp.nref[s]) + dn;
      dns[s] = dn;
      acc[s] += lp.nref[s] + double(dn);
      acc[3] += double(jx); acc[4] += double(jy); acc[5] += double(jz);
      const T zs = T(lp.valence[s]);
      const T inv_n = recip(n[s]);
      G[s][0] = zs * ex + T(lp.fext[s][0]);
      G[s][1] = zs * ey + T(lp.fext[s][1]);
      G[s][2] = zs * ez + T(lp.fext[s][2]);
      if (has_bead) {
#pragma unroll
        for (int c = 0; c < 3; ++c) G[s][c] += T(kb[s][c]) * inv_n;
      }
      bv[s][0] = jx * inv_n + T(0.5) * G[s][0];
      bv[s][1] = jy * inv_n + T(0.5) * G[s][1];
      bv[s][2] = jz * inv_n + T(0.5) * G[s][2];
    }
    // implicit drag in closed form: with a^a = omega_drag^a / 2,
    // ubar = sum x^a b^a / (1 + a^a) / sum x^a / (1 + a^a),
    // u^a = (b^a + a^a ubar) / (1 + a^a), Phi^a = G^a - omega_drag^a (u^a - ubar)
    const T inv_ntot = recip(n[0] + n[1] + n[2]);
    T ub[3] = {T(0), T(0), T(0)};
    T den = T(0);
    T inv1a[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      inv1a[s] = recip(T(1) + T(0.5 * lp.wdrag[s]));
      const T xs = n[s] * inv_ntot * inv1a[s];
#pragma unroll
      for (int c = 0; c < 3; ++c) ub[c] += xs * bv[s][c];
      den += xs;
    }
    const T inv_den = recip(den);
#pragma unroll
    for (int c = 0; c < 3; ++c) ub[c] *= inv_den;

#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const PlanesOut<T, I> out(fdst + (size_t)s * Q * d.n, N);
      const T as = T(0.5 * lp.wdrag[s]);
      const T wd = T(lp.wdrag[s]);
      T u[3], ph[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u[c] = (bv[s][c] + as * ub[c]) * inv1a[s];
        ph[c] = G[s][c] - wd * (u[c] - ub[c]);
      }
      const T om = T(lp.omega[s]);
      const T half = T(1) - T(0.5) * om;
      const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const T pu = ph[0] * u[0] + ph[1] * u[1] + ph[2] * u[2];
      const T ns = n[s];
      const T dn = dns[s];  // kept from the sum: n - nref would lose it in float32
      T delta[FLUCT ? Q : 1];
      if constexpr (FLUCT) {
#pragma unroll
        for (int p = 0; p < Q; ++p) delta[p] = T(0);
        add_lattice_noise<T>(delta, *noise, s, uint32_t(r), ns);
      }
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        const T cu = T(CX[p]) * u[0] + T(CY[p]) * u[1] + T(CZ[p]) * u[2];
        const T cf = T(CX[p]) * ph[0] + T(CY[p]) * ph[1] + T(CZ[p]) * ph[2];
        const T w = T(weight(p));
        // deviation of the second-order equilibrium (vT2 = 1/3) and forcing
        const T geq = w * (dn + ns * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu));
        const T src = w * ns * (T(3) * cf + T(9) * cu * cf - T(3) * pu);
        T gs = g[s][p] - om * (g[s][p] - geq) + half * src;
        if constexpr (FLUCT) gs += delta[FLUCT ? p : 0];
        out.store(p, r, gs);
      }
    }
  }
  return true;
}

}  // namespace ek
