// Bead-spring chain coupled to the three species by friction (Sec. II.B)
// through the trilinear interpolation / spreading kernel (Sec. II.C): state,
// node table access and the per-step pieces, shared by the single-system
// kernels and the persistent ensemble kernel.
#pragma once

#include <climits>
#include <cmath>

#include "ek_internal.h"
#include "md_table.h"
#include "philox.h"

namespace ek {

constexpr int BOX = 4;          // moment box edge (nodes floor(R0) - 1 .. floor(R0) + 2)
constexpr int BOX3 = BOX * BOX * BOX;
constexpr int WIN = 6;          // flag window edge (nodes floor(R0) - 2 .. floor(R0) + 3)
constexpr int WIN3 = WIN * WIN * WIN;

// Wall reach WR: the bead-wall WCA looks at the wall sites floor(R) - WR ..
// floor(R) + 1 + WR in each axis (an S^3 cube around the bead's cell), which
// holds every site closer than WR + 1 to the bead: WR = 1 for a cut-off
// 2^(1/6) sigma below 2, WR = 2 below 3.  Since the bead stays within one
// cell of its start over a step, the flag window of the step spans
// floor(R0) - 1 - WR .. floor(R0) + 2 + WR, W = 2 WR + 4 sites per axis.
template <int WR>
struct WallGeom {
  static constexpr int S = 2 * WR + 2;
  static constexpr int S3 = S * S * S;
  static constexpr int W = 2 * WR + 4;
  static constexpr int W3 = W * W * W;
};
constexpr int WIN3_MAX = WallGeom<2>::W3;   // per-bead flag storage of a single context
constexpr int MOM = 15;         // x[3] (n^a / n), 1/n^a [3], j[3][3]

enum : int { ERR_BOX = 1, ERR_FLUID = 2, ERR_BOND = 4, ERR_TABLE = 8 };

struct BeadState {
  double* R;          // [maxb][3]
  double* V;          // [maxb][3]
  double* q;          // [maxb]
  int* origin;        // [maxb][3] floor(R0) - 1 of the current step
  double* mom;        // [maxb][BOX3][MOM]
  double* efield;     // [maxb][BOX3][3]
  unsigned char* flags;  // [maxb][W3 of the wall reach]: bit0 fluid, bit1 wall
  int* err;           // error bits
  int* cross = nullptr;  // [maxb][3] plane crossings: first step, last step, net count
};

// Views of the bead state carved from a context's bead memory (host side).
BeadState bead_state_view(char* mem, int max_beads);

__device__ inline int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__device__ inline long long site_of(int x, int y, int z, const Dims& d) {
  return ((long long)wrap(z, d.nz) * d.ny + wrap(y, d.ny)) * d.nx + wrap(x, d.nx);
}

__device__ inline long long ld_i64(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int ld_i32(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Find or insert `site`; flags the site for the lattice kernels.
__device__ inline int table_insert(int* keys, uint32_t* mask, long long site, int* err, int bits) {
  const int slots = 1 << bits;
  int h = hash_slot(site, bits);
  for (int k = 0; k < slots; ++k) {
    const int prev = atomicCAS(&keys[h], -1, int(site));
    if (prev == -1) {
      atomicOr(&mask[site], MASK_BEAD);
      return h;
    }
    if (prev == int(site)) return h;
    h = (h + 1) & (slots - 1);
  }
  atomicOr(err, ERR_TABLE);
  return -1;
}

// Slot of `site` if present (reads that see the atomics of this launch).
__device__ inline int table_find(const int* keys, long long site, int bits) {
  const int slots = 1 << bits;
  int h = hash_slot(site, bits);
  for (int k = 0; k < slots; ++k) {
    const int key = ld_i32(&keys[h]);
    if (key == int(site)) return h;
    if (key < 0) return -1;
    h = (h + 1) & (slots - 1);
  }
  return -1;
}

// Empty table (once, when the context is created: the workspace arrives
// uninitialised).
struct MDParams {
  int n, n_sub;
  double M, k_fene, R0, eps, sigma, gamma;
  double Lx, Ly, Lz;
  // crossing record of the plane z = z_plane (and its periodic images) in
  // bs.cross; `step` is the number of completed steps once this one ends
  int track = 0;
  int step = 0;
  double z_plane = 0.0;
  // bonds: 0 FENE (k_fene, R0) with the WCA between all pairs; 1 harmonic
  // (k_bond, l_bond, Eq. polymermodel) with the WCA only for |i - j| > 1
  int bond = 0;
  double k_bond = 0.0, l_bond = 0.0;
  // thermal noise (philox.h): xi ~ N(0, xi_scale^2) per component and
  // substep, xi_scale = sqrt(2 gamma k_B T / h), from the counter
  // (bead, tstep, substep, 1); tstep = steps completed before this one
  int thermal = 0;
  uint32_t key0 = 0, key1 = 0, tstep = 0;
  double xi_scale = 0.0;
  // coupling kernel: 0 trilinear, 1 the occupation cube of side 2 half_sigma
  // (Eq. totalforcefluid) for the velocity at the bead and the friction
  int theta = 0;
  double half_sigma = 0.5;
  // insulating walls: the field at the bead with the trilinear weights
  // renormalised over the fluid corners (where its charge was deposited)
  int field_fluid = 0;
};

__device__ inline double min_image(double v, double L) { return v - L * rint(v / L); }

// WCA force on a pair at squared distance r2 (factor multiplying the separation).
__device__ inline double wca_coef(double r2, double eps, double sigma) {
  const double rc2 = 1.2599210498948732 * sigma * sigma;   // (2^(1/6) sigma)^2
  if (r2 >= rc2) return 0.0;
  const double s2 = sigma * sigma / r2;
  const double s6 = s2 * s2 * s2;
  return 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
}

// Nearest integer (ties to even, as llrint) of x.  For |x| < 2^51 the sum
// x + 1.5 * 2^52 has a unit in the last place of 1, so its low mantissa bits
// hold the rounded value as an offset from the bits of 1.5 * 2^52; larger
// values take llrint.
__device__ inline long long round_fixed(double x) {
  if (__builtin_expect(fabs(x) < 2251799813685248.0, 1)) {       // 2^51
    const double t = x + 6755399441055744.0;                        // 1.5 * 2^52
    return __double_as_longlong(t) - 0x4338000000000000ll;
  }
  return llrint(x);
}

// Node accumulators for the friction impulse: the context's global table, or
// a table in LDS (sites it has no room for stay in the global table) that is
// flushed to the global one once after the substeps.  Values are int64 fixed
// point, so the sums are exact whatever the order of the additions.
struct GlobalNodes {
  int* keys;
  long long* vals;
  uint32_t* mask;
  int* err;
  int bits;
  __device__ int slot(long long site) { return table_insert(keys, mask, site, err, bits); }
  __device__ double get(int h, int c) const {
    return double(ld_i64(&vals[(size_t)h * SLOT_VALUES + 1 + c])) * (1.0 / FIX_FORCE);
  }
  __device__ void add(int h, int c, long long v) {
    atomicAdd((unsigned long long*)&vals[(size_t)h * SLOT_VALUES + 1 + c], (unsigned long long)v);
  }
};

// LDS probes of an insertion before the site goes to the global table.
constexpr int LDS_PROBES = 32;

// The LDS table has any number of slots (positions h = mulhi(mix(site), slots)
// and linear probing); a site whose probe path holds no free slot within
// LDS_PROBES probes is kept in the global table instead.  Every lane that
// looks up a site walks the same path over slots that, once taken, stay
// taken, so all of them reach the same decision.  Slot codes: h >= 0 the LDS
// slot, h <= -2 the global slot -2 - h, -1 none (the global table is full).
struct LdsNodes {
  int* keys;          // LDS [slots]
  long long* vals;    // LDS [slots][9]
  int slots;
  int* err;
  GlobalNodes global;
  __device__ int slot(long long site) {
    const unsigned long long mix = (unsigned long long)site * 0x9E3779B97F4A7C15ull;
    int h = int(((mix >> 32) * (unsigned long long)slots) >> 32);
    const int probes = slots < LDS_PROBES ? slots : LDS_PROBES;
    for (int k = 0; k < probes; ++k) {
      const int prev = atomicCAS(&keys[h], -1, int(site));
      if (prev == -1 || prev == int(site)) return h;
      h = h + 1 == slots ? 0 : h + 1;
    }
    const int g = global.slot(site);
    return g < 0 ? -1 : -2 - g;
  }
  __device__ double get(int h, int c) const {
    if (h >= 0) return double(vals[h * 9 + c]) * (1.0 / FIX_FORCE);
    return global.get(-2 - h, c);
  }
  __device__ void add(int h, int c, long long v) {
    if (h >= 0) atomicAdd((unsigned long long*)&vals[h * 9 + c], (unsigned long long)v);
    else global.add(-2 - h, c, v);
  }
};

// One workgroup per chain, TPB threads per bead: the lanes of a bead split
// its 8 corners, its pair partners and its wall sites, and combine their
// parts with a butterfly over the TPB lanes (every lane ends with the same
// bits, so all lanes advance the bead identically).  The exchanges are DPP
// lane moves within a row of 16 lanes: xor 1 and xor 2 as quad permutations;
// after those every lane of a quad holds the quad's sum, so the last level
// takes the other quad's sum from the mirrored lane of the group of 8
// (lane l reads lane 7 - l).  A bead's lanes are active together.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int TPB>
__device__ inline double group_sum(double v) {
  static_assert(TPB == 1 || TPB == 2 || TPB == 4 || TPB == 8, "lanes per bead");
  constexpr int XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
  constexpr int XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
  constexpr int HALF_MIRROR = 0x141;  // row_half_mirror (lane l reads lane 7 - l of its 8)
  if constexpr (TPB >= 2) v += dpp_move<XOR1>(v);
  if constexpr (TPB >= 4) v += dpp_move<XOR2>(v);
  if constexpr (TPB >= 8) v += dpp_move<HALF_MIRROR>(v);
  return v;
}

// ---------------------------------------------------------------------------
// Per-step pieces written for a team of threads (tid, nthreads): a whole
// grid of one-thread-per-item launches, or one workgroup.
// ---------------------------------------------------------------------------

// Drop a table's entries and their site flags.
__device__ inline void table_clear_items(int* keys, long long* vals, uint32_t* mask, long long n,
                                         int bits, int tid, int nthreads) {
  for (int h = tid; h < (1 << bits); h += nthreads) {
    const int key = keys[h];
    if (key >= 0 && key < n) {
      atomicAnd(&mask[key], ~MASK_BEAD);
      keys[h] = -1;
#pragma unroll
      for (int c = 0; c < SLOT_VALUES; ++c) vals[(size_t)h * SLOT_VALUES + c] = 0;
    }
  }
}

// Bead charges on the 8 corner nodes with the plain trilinear weights, or
// (fluid_only, insulating walls) with the weights renormalised over the
// fluid corners.
__device__ inline void deposit_items(const BeadState& bs, int n, int* keys, long long* vals,
                                     uint32_t* mask, const Dims& d, int bits, int tid,
                                     int nthreads, bool fluid_only = false) {
  for (int t = tid; t < 8 * n; t += nthreads) {
    const int i = t >> 3, k = t & 7;
    const double* R = bs.R + 3 * i;
    const double fx = floor(R[0]), fy = floor(R[1]), fz = floor(R[2]);
    const double dx = R[0] - fx, dy = R[1] - fy, dz = R[2] - fz;
    const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
    double w = (ox ? dx : 1.0 - dx) * (oy ? dy : 1.0 - dy) * (oz ? dz : 1.0 - dz);
    const long long site = site_of(int(fx) + ox, int(fy) + oy, int(fz) + oz, d);
    if (fluid_only) {
      if (mask[site] & MASK_SOLID) continue;
      double wsum = 0.0;
      for (int k2 = 0; k2 < 8; ++k2) {
        const int px = k2 & 1, py = (k2 >> 1) & 1, pz = (k2 >> 2) & 1;
        if (mask[site_of(int(fx) + px, int(fy) + py, int(fz) + pz, d)] & MASK_SOLID) continue;
        wsum += (px ? dx : 1.0 - dx) * (py ? dy : 1.0 - dy) * (pz ? dz : 1.0 - dz);
      }
      w /= wsum;
    }
    const int h = table_insert(keys, mask, site, bs.err, bits);
    if (h < 0) continue;
    atomicAdd((unsigned long long*)&vals[(size_t)h * SLOT_VALUES],
              (unsigned long long)llrint(bs.q[i] * w * FIX_CHARGE));
  }
}

// Fields of time t around bead i: item t < W3 sets the fluid / wall flags of
// the flag window (W^3 for the wall reach WR), item t < BOX3 the moments and
// field of one node of the 4^3 box.  The box origin is written by item 0.
// With `defer` set, every box node is also flagged MASK_DEFER: the chain's
// friction can only reach nodes of the boxes, so the lattice update of all
// other sites need not wait for it.
// With `walls` (insulating walls) the field at a fluid node takes the ghost
// value psi + Sigma_f / eps for a solid face neighbour, and is 0 at a solid
// node (the beads then interpolate it over fluid corners only).
template <typename T, int WR = 1>
__device__ inline void bead_box_item(const BeadState& bs, int i, int t, const T* __restrict__ f,
                                     const uint32_t* mask,
                                     const double* __restrict__ psi, const LBParams& lp,
                                     const Dims& d, uint32_t* defer = nullptr,
                                     const double* face_q = nullptr, double inv_eps = 0.0) {
  const double* R = bs.R + 3 * i;
  const int bx = int(floor(R[0])) - 1, by = int(floor(R[1])) - 1, bz = int(floor(R[2])) - 1;
  if (t == 0) {
    bs.origin[3 * i] = bx;
    bs.origin[3 * i + 1] = by;
    bs.origin[3 * i + 2] = bz;
  }
  using G = WallGeom<WR>;
  if (t < G::W3) {
    const int wx = t % G::W, wy = (t / G::W) % G::W, wz = t / (G::W * G::W);
    const uint32_t m = mask[site_of(bx - WR + wx, by - WR + wy, bz - WR + wz, d)];
    bs.flags[(size_t)i * G::W3 + t] =
        (unsigned char)(((m & MASK_SOLID) ? 0 : 1) | ((m & MASK_WALL) ? 2 : 0));
  }
  if (t >= BOX3) return;
  const int cx = bx + t % BOX, cy = by + (t / BOX) % BOX, cz = bz + t / (BOX * BOX);
  const long long r = site_of(cx, cy, cz, d);
  if (defer) atomicOr(&defer[r], MASK_DEFER);
  const uint32_t m = mask[r];
  double* mo = bs.mom + ((size_t)i * BOX3 + t) * MOM;
  // all 57 pulls are issued before any sum (registers only, one store pass)
  double v[MOM];
#pragma unroll
  for (int c = 0; c < MOM; ++c) v[c] = 0.0;
  if (!(m & MASK_SOLID)) {
    const int x = wrap(cx, d.nx), y = wrap(cy, d.ny), z = wrap(cz, d.nz);
    T g[3][Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      const bool bounce = (m >> p) & 1u;
      const long long src = bounce ? r : site_of(x - CX[p], y - CY[p], z - CZ[p], d);
      const int q = bounce ? OPP[p] : p;
#pragma unroll
      for (int s = 0; s < 3; ++s) g[s][p] = f[(size_t)(s * Q + q) * d.n + src];
    }
    double n[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      double dn = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        const double gp = double(g[s][p]);
        dn += gp;
        jx += CX[p] * gp;
        jy += CY[p] * gp;
        jz += CZ[p] * gp;
      }
      n[s] = lp.nref[s] + dn;
      v[6 + 3 * s] = jx;
      v[7 + 3 * s] = jy;
      v[8 + 3 * s] = jz;
    }
    const double ntot = n[0] + n[1] + n[2];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      v[3 + s] = 1.0 / n[s];
      v[s] = n[s] / ntot;
    }
  }
#pragma unroll
  for (int c = 0; c < MOM; ++c) mo[c] = v[c];
  double* e = bs.efield + ((size_t)i * BOX3 + t) * 3;
  if (face_q) {
    if (m & MASK_SOLID) {
      e[0] = e[1] = e[2] = 0.0;
      return;
    }
    const double pc = psi[r];
    // bit p of the link word: the neighbour r - c_p is solid (1/2: -x/+x,
    // 3/4: -y/+y, 5/6: -z/+z)
    auto side = [&](int bit, long long idx) {
      return ((m >> bit) & 1u) ? pc + face_q[idx] * inv_eps : psi[idx];
    };
    e[0] = -0.5 * (side(2, site_of(cx + 1, cy, cz, d)) - side(1, site_of(cx - 1, cy, cz, d))) + lp.eext[0];
    e[1] = -0.5 * (side(4, site_of(cx, cy + 1, cz, d)) - side(3, site_of(cx, cy - 1, cz, d))) + lp.eext[1];
    e[2] = -0.5 * (side(6, site_of(cx, cy, cz + 1, d)) - side(5, site_of(cx, cy, cz - 1, d))) + lp.eext[2];
    return;
  }
  e[0] = -0.5 * (psi[site_of(cx + 1, cy, cz, d)] - psi[site_of(cx - 1, cy, cz, d)]) + lp.eext[0];
  e[1] = -0.5 * (psi[site_of(cx, cy + 1, cz, d)] - psi[site_of(cx, cy - 1, cz, d)]) + lp.eext[1];
  e[2] = -0.5 * (psi[site_of(cx, cy, cz + 1, d)] - psi[site_of(cx, cy, cz - 1, d)]) + lp.eext[2];
}

// Pair partners kept per lane: lane l of bead i lists the beads j = l,
// l + TPB, ... within the WCA cut-off plus NB_SKIN at the last build, in
// increasing j, up to NBL of them (a template parameter).  The list is rebuilt
// when any bead has moved more than NB_SKIN / 2 since the build, so every
// pair inside the cut-off stays listed.  Chains of at most SMALL_CHAIN beads
// with eight lanes per bead have room for every candidate
// (NBL = SMALL_CHAIN / 8); longer chains keep up to NB_PER_LANE partners per
// lane and a lane that would list more switches the chain back to all pairs.
// A lane sums the same nonzero pair terms in the same order either way.
constexpr int NB_PER_LANE = 32;
constexpr double NB_SKIN = 0.6;
constexpr int SMALL_CHAIN = 64;

// LDS bytes of the pair lists.
__host__ __device__ inline size_t md_list_bytes(int threads, int nbl) {
  return (size_t)threads * nbl * sizeof(unsigned short);
}

// n_sub substeps of one chain by one workgroup (TPB lanes per bead; the
// threads beyond n * TPB only take part in the barriers).  smem: LDS for the
// bead positions, when LDS is set the node table of lds_slots slots (sites
// that find no room there go to the global table), and with NBL > 0 the pair
// lists (md_list_bytes; with NBL = 0 every lane walks all its candidate
// partners each substep: the persistent ensemble kernel, whose registers the
// lists would spill).  THERMAL = false compiles the bead noise out (the
// ensemble, which runs without thermal fluctuations).
template <bool LDS, int TPB, int NBL, int WR = 1, bool THERMAL = true>
__device__ inline void md_chain(const BeadState& bs, const MDParams& mp, int* gkeys,
                                long long* gvals, uint32_t* mask, const Dims& d, int gbits,
                                int lds_slots, unsigned char* smem) {
  using G = WallGeom<WR>;
  constexpr int WIN = G::W;                                    // flag window edge
  constexpr int CPL = 8 / TPB;                                 // corners per lane
  double* sR = (double*)smem;                                  // [3 * n]
  long long* lvals = (long long*)(smem + (((size_t)mp.n * 24 + 15) & ~size_t(15)));
  const int lslots = LDS ? lds_slots : 0;
  int* lkeys = (int*)(lvals + (size_t)lslots * 9);
  // pair lists: entry k of thread t at nbl[k * blockDim.x + t], after the
  // LDS node table
  constexpr bool NLIST = NBL > 0;
  unsigned short* nbl = (unsigned short*)(lkeys + lslots);
  __shared__ int s_rebuild, s_overflow;
  if (NLIST && threadIdx.x == 0) {
    s_rebuild = 1;
    s_overflow = 0;
  }
  int nb_count = 0;
  double Rb[3] = {0, 0, 0};                 // position at the last list build

  const int i = threadIdx.x / TPB;          // bead
  const int lane = threadIdx.x % TPB;
  const bool live = i < mp.n;
  if (LDS) {
    for (int h = threadIdx.x; h < lslots; h += blockDim.x) {
      lkeys[h] = -1;
      for (int c = 0; c < 9; ++c) lvals[(size_t)h * 9 + c] = 0;
    }
  }
  double R[3] = {0, 0, 0}, V[3] = {0, 0, 0}, q = 0.0;
  int org[3] = {0, 0, 0};
  if (live) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R[c] = bs.R[3 * i + c];
      V[c] = bs.V[3 * i + c];
      org[c] = bs.origin[3 * i + c];
      if (lane == 0) sR[3 * i + c] = R[c];
    }
    q = bs.q[i];
  }
  const double z_start = R[2];   // for the plane crossing record
  __syncthreads();
  GlobalNodes gn{gkeys, gvals, mask, bs.err, gbits};
  LdsNodes ln{lkeys, lvals, lslots, bs.err, gn};

  const double h = 1.0 / mp.n_sub;
  const double hM = h / mp.M;
  const double L[3] = {mp.Lx, mp.Ly, mp.Lz};
  const double iL[3] = {1.0 / mp.Lx, 1.0 / mp.Ly, 1.0 / mp.Lz};
  const double rc2 = 1.2599210498948732 * mp.sigma * mp.sigma;   // (2^(1/6) sigma)^2
  const double s2w = mp.sigma * mp.sigma;
  const double iR02 = 1.0 / (mp.R0 * mp.R0);
  const double* mom = bs.mom + (size_t)(live ? i : 0) * BOX3 * MOM;
  const double* ef = bs.efield + (size_t)(live ? i : 0) * BOX3 * 3;
  const unsigned char* fl = bs.flags + (size_t)(live ? i : 0) * G::W3;
  int cell[3] = {INT_MIN, INT_MIN, INT_MIN};
  int slot[CPL], bidx[CPL];
  double wfl[CPL];
  double fl_all[8];                 // fluid flag of every corner (for the normalisation)
  // With at most two corners per lane the corner data, which is fixed for the
  // whole step (node momenta of time t and the field), and the lane's
  // wall-site flags are kept in registers from the substep the bead enters
  // its cell on; with more corners per lane they are read each substep.
  constexpr bool CACHE = CPL <= 2;   // node momenta too
  constexpr bool CACHE_E = CPL <= 4; // field and wall flags
  constexpr int NWS = G::S3 / TPB;  // wall sites per lane
  static_assert(G::S3 % TPB == 0, "wall sites split evenly over a bead's lanes");
  constexpr int NWB = (NWS + 63) / 64;
  double mo_c[CACHE ? CPL : 1][MOM];
  double e_c[CACHE_E ? CPL : 1][3];
  unsigned long long wall_bits[NWB];
#pragma unroll
  for (int b = 0; b < NWB; ++b) wall_bits[b] = 0;
  // this lane's share of q E(R(t)): the field is interpolated once, with the
  // plain weights at the position where the bead's charge was deposited for
  // this step's solve (the electrostatic forces on ions, walls and beads then
  // cancel exactly, and the bead never feels its own deposited charge)
  double qe[3] = {0.0, 0.0, 0.0};
  const double rl = 1.122462048309373 * mp.sigma + NB_SKIN;      // list radius
  const double rl2 = rl * rl, half_skin2 = 0.25 * NB_SKIN * NB_SKIN;
  for (int sub = 0; sub < mp.n_sub; ++sub) {
    if (NLIST && s_rebuild) {            // the same in every thread (set before the last barrier)
      if (live) {
        nb_count = 0;
        for (int j = lane; j < mp.n; j += TPB) {
          if (j == i || (mp.bond == 1 && (j == i - 1 || j == i + 1))) continue;
          double r2 = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double v = R[c] - sR[3 * j + c];
            const double dv = v - L[c] * rint(v * iL[c]);
            r2 += dv * dv;
          }
          if (r2 < rl2) {
            if (nb_count < NBL) nbl[nb_count * blockDim.x + threadIdx.x] = (unsigned short)j;
            ++nb_count;
          }
        }
        if (nb_count > NBL) s_overflow = 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) Rb[c] = R[c];
      }
      __syncthreads();
      if (threadIdx.x == 0) s_rebuild = 0;
    }
    double wt[CPL];
    double phi[3][3];
    double Rn[3];
#pragma unroll
    for (int a = 0; a < CPL; ++a) wt[a] = 0.0;
    if (live) {
      const int fx = int(floor(R[0])), fy = int(floor(R[1])), fz = int(floor(R[2]));
      const double dx = R[0] - fx, dy = R[1] - fy, dz = R[2] - fz;
      int lx = fx - org[0], ly = fy - org[1], lz = fz - org[2];   // corner 0 in the box
      if (fx != cell[0] || fy != cell[1] || fz != cell[2]) {
        // the bead entered another cell: new corners, their box entries and slots
        cell[0] = fx; cell[1] = fy; cell[2] = fz;
        if (lx < 0 || lx > BOX - 2 || ly < 0 || ly > BOX - 2 || lz < 0 || lz > BOX - 2) {
          if (lane == 0) atomicOr(bs.err, ERR_BOX);
          lx = min(max(lx, 0), BOX - 2);
          ly = min(max(ly, 0), BOX - 2);
          lz = min(max(lz, 0), BOX - 2);
        }
#pragma unroll
        for (int k8 = 0; k8 < 8; ++k8) {
          const int ox = k8 & 1, oy = (k8 >> 1) & 1, oz = (k8 >> 2) & 1;
          const int wi = (lx + ox + WR) + WIN * ((ly + oy + WR) + WIN * (lz + oz + WR));
          fl_all[k8] = (fl[wi] & 1) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int a = 0; a < CPL; ++a) {
          const int k8 = lane * CPL + a;
          const int ox = k8 & 1, oy = (k8 >> 1) & 1, oz = (k8 >> 2) & 1;
          bidx[a] = (lx + ox) + BOX * ((ly + oy) + BOX * (lz + oz));
          // from the flag window, not fl_all[k8]: k8 depends on the lane, and
          // a register array indexed at run time would live in scratch memory
          wfl[a] = (fl[(lx + ox + WR) + WIN * ((ly + oy + WR) + WIN * (lz + oz + WR))] & 1) ? 1.0 : 0.0;
          slot[a] = -1;
          if (wfl[a] != 0.0) {
            const long long site = site_of(fx + ox, fy + oy, fz + oz, d);
            slot[a] = LDS ? ln.slot(site) : gn.slot(site);
          }
          if constexpr (CACHE_E) {
            const double* e = ef + (size_t)bidx[a] * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) e_c[CACHE_E ? a : 0][c] = e[c];
          }
          if constexpr (CACHE) {
            const double* mo = mom + (size_t)bidx[a] * MOM;
#pragma unroll
            for (int c = 0; c < MOM; ++c) {   // read unconditionally: not behind the flag's read
              const double m = mo[c];
              mo_c[CACHE ? a : 0][c] = wfl[a] != 0.0 ? m : 0.0;
            }
          }
        }
        if constexpr (CACHE_E) {
#pragma unroll
          for (int b = 0; b < NWB; ++b) wall_bits[b] = 0;
#pragma unroll
          for (int k = 0; k < NWS; ++k) {
            const int wsite = lane + k * TPB;
            const int wx = wsite % G::S, wy = (wsite / G::S) % G::S, wz = wsite / (G::S * G::S);
            // site floor(R) - WR + w sits at window index (floor(R) - org) + w
            const int ix = lx + wx, iy = ly + wy, iz = lz + wz;
            if (ix < 0 || ix >= WIN || iy < 0 || iy >= WIN || iz < 0 || iz >= WIN) continue;
            if (fl[ix + WIN * (iy + WIN * iz)] & 2) wall_bits[k >> 6] |= 1ull << (k & 63);
          }
        }
      }
      // impulse of earlier substeps on this lane's corners, read before the
      // weights so that the reads overlap their arithmetic (one corner per
      // lane: with more the registers are not spared)
      constexpr bool PRE_K = CPL == 1;
      double kpre[PRE_K ? CPL : 1][9];
      if constexpr (PRE_K) {
#pragma unroll
        for (int a = 0; a < CPL; ++a)
#pragma unroll
          for (int k = 0; k < 9; ++k)
            kpre[a][k] = slot[a] == -1 ? 0.0 : (LDS ? ln.get(slot[a], k) : gn.get(slot[a], k));
      }
      // plain and fluid-renormalised trilinear weights; with the occupation
      // cube, its node indicator per axis (offset 0: d < sigma/2, offset 1:
      // d >= 1 - sigma/2) renormalised over the fluid nodes
      auto cube = [&](int ox, int oy, int oz) {
        const double hs = mp.half_sigma;
        return ((ox ? dx >= 1.0 - hs : dx < hs) && (oy ? dy >= 1.0 - hs : dy < hs) &&
                (oz ? dz >= 1.0 - hs : dz < hs)) ? 1.0 : 0.0;
      };
      double wsum = 0.0, wsum_c = 0.0;
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8) {
        const int ox = k8 & 1, oy = (k8 >> 1) & 1, oz = (k8 >> 2) & 1;
        wsum += fl_all[k8] * (ox ? dx : 1.0 - dx) * (oy ? dy : 1.0 - dy) * (oz ? dz : 1.0 - dz);
        if (mp.theta) wsum_c += fl_all[k8] * cube(ox, oy, oz);
      }
      if (!mp.theta) wsum_c = wsum;
      if (!(wsum_c > 0.0) || !(wsum > 0.0)) {
        if (lane == 0) atomicOr(bs.err, ERR_FLUID);
        wsum = wsum > 0.0 ? wsum : 1.0;
        wsum_c = wsum_c > 0.0 ? wsum_c : 1.0;
      }
      const double iws = 1.0 / wsum_c;
      // this lane's corners: velocities from the node momentum (populations of
      // time t plus the friction impulse of earlier substeps), composition,
      // and on the first substep the electric field with the plain weights
      double acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = 0.0;
#pragma unroll
      for (int a = 0; a < CPL; ++a) {
        const int k8 = lane * CPL + a;
        const int ox = k8 & 1, oy = (k8 >> 1) & 1, oz = (k8 >> 2) & 1;
        const double w = (ox ? dx : 1.0 - dx) * (oy ? dy : 1.0 - dy) * (oz ? dz : 1.0 - dz);
        wt[a] = (mp.theta ? cube(ox, oy, oz) : w) * wfl[a] * iws;
        if (sub == 0) {
          const double* e = CACHE_E ? e_c[CACHE_E ? a : 0] : ef + (size_t)bidx[a] * 3;
          const double we = mp.field_fluid ? w * wfl[a] / wsum : w;
#pragma unroll
          for (int c = 0; c < 3; ++c) qe[c] += q * we * e[c];
        }
        if (wt[a] != 0.0) {
          const double* mo = CACHE ? mo_c[CACHE ? a : 0] : mom + (size_t)bidx[a] * MOM;
#pragma unroll
          for (int s = 0; s < 3; ++s) {
            acc[9 + s] += wt[a] * mo[s];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double kacc =
                  PRE_K ? kpre[PRE_K ? a : 0][3 * s + c]
                        : (slot[a] == -1 ? 0.0 : (LDS ? ln.get(slot[a], 3 * s + c)
                                                    : gn.get(slot[a], 3 * s + c)));
              acc[3 * s + c] += wt[a] * (mo[6 + 3 * s + c] + kacc) * mo[3 + s];
            }
          }
        }
      }
      // this lane's share of the conservative forces
      double F[3] = {0.0, 0.0, 0.0};
      // FENE bonds: the bond to i - 1 on lane 0 and the one to i + 1 on lane
      // 1 (both on lane 0 with one lane per bead); the bonded neighbour's
      // position is read up front with the partners' ones where the registers
      // allow (short chains with the lists)
      constexpr int NBOND = TPB >= 2 ? 1 : 2;        // bonds per bond lane
      const int bond0 = TPB >= 2 ? lane : 0;         // 0: bond to i - 1, 1: to i + 1
      const bool bond_lane = TPB >= 2 ? lane < 2 : true;
      constexpr bool PRE_B = LDS && NLIST;
      double PB[PRE_B ? NBOND : 1][3];
      if constexpr (PRE_B) {
#pragma unroll
        for (int k = 0; k < NBOND; ++k) {
          const int j = min(max(i + 2 * (bond0 + k) - 1, 0), mp.n - 1);
#pragma unroll
          for (int c = 0; c < 3; ++c) PB[PRE_B ? k : 0][c] = sR[3 * j + c];
        }
      }
      auto wca_at = [&](const double* P) {   // WCA with a partner at P
        double dv[3], r2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double v = R[c] - P[c];
          dv[c] = v - L[c] * rint(v * iL[c]);
          r2 += dv[c] * dv[c];
        }
        if (r2 < rc2) {
          const double ir2 = 1.0 / r2;
          const double s6 = s2w * ir2 * s2w * ir2 * s2w * ir2;
          const double coef = 24.0 * mp.eps * (2.0 * s6 * s6 - s6) * ir2;
#pragma unroll
          for (int c = 0; c < 3; ++c) F[c] += coef * dv[c];
        }
      };
      if (NLIST && !s_overflow) {                    // WCA with the listed partners
        // four partners at a time: their indices, then their positions, are
        // read together (one LDS round trip each), the terms are added in
        // list order
        constexpr int CH = 4;
        static_assert(NBL % CH == 0, "list chunks");
        for (int k0 = 0; k0 < nb_count; k0 += CH) {
          int jj[CH];
#pragma unroll
          for (int u = 0; u < CH; ++u)
            jj[u] = k0 + u < nb_count ? int(nbl[(k0 + u) * blockDim.x + threadIdx.x]) : i;
          double P[CH][3];
#pragma unroll
          for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) P[u][c] = sR[3 * jj[u] + c];
#pragma unroll
          for (int u = 0; u < CH; ++u)
            if (k0 + u < nb_count) wca_at(P[u]);
        }
      } else {
        for (int j = lane; j < mp.n; j += TPB)       // WCA between all pairs
          if (j != i && !(mp.bond == 1 && (j == i - 1 || j == i + 1))) {
            const double P[3] = {sR[3 * j], sR[3 * j + 1], sR[3 * j + 2]};
            wca_at(P);
          }
      }
      // WCA against wall-site centres: site k of this lane is lane + k TPB of
      // the S^3 sites around the bead's cell
      auto wall_at = [&](int ax, int ay, int az) {
        const double dv[3] = {R[0] - ax, R[1] - ay, R[2] - az};
        const double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
        if (r2 < rc2) {
          const double ir2 = 1.0 / r2;
          const double s6 = s2w * ir2 * s2w * ir2 * s2w * ir2;
          const double coef = 24.0 * mp.eps * (2.0 * s6 * s6 - s6) * ir2;
#pragma unroll
          for (int c = 0; c < 3; ++c) F[c] += coef * dv[c];
        }
      };
      if constexpr (CACHE_E) {
        // only the wall sites among them, in increasing k
#pragma unroll
        for (int b = 0; b < NWB; ++b)
          for (unsigned long long mb = wall_bits[b]; mb; mb &= mb - 1) {
            const int wsite = lane + (64 * b + __builtin_ctzll(mb)) * TPB;
            wall_at(fx - WR + wsite % G::S, fy - WR + (wsite / G::S) % G::S,
                    fz - WR + wsite / (G::S * G::S));
          }
      } else {
        for (int k = 0; k < NWS; ++k) {
          const int wsite = lane + k * TPB;
          const int wx = wsite % G::S, wy = (wsite / G::S) % G::S, wz = wsite / (G::S * G::S);
          const int ix = lx + wx, iy = ly + wy, iz = lz + wz;
          if (ix < 0 || ix >= WIN || iy < 0 || iy >= WIN || iz < 0 || iz >= WIN) continue;
          if (!(fl[ix + WIN * (iy + WIN * iz)] & 2)) continue;
          wall_at(fx - WR + wx, fy - WR + wy, fz - WR + wz);
        }
      }
      if (bond_lane) {
#pragma unroll
        for (int k = 0; k < NBOND; ++k) {            // FENE bonds
          const int j = i + 2 * (bond0 + k) - 1;
          if (j < 0 || j >= mp.n) continue;
          double dv[3], r2 = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double v = (PRE_B ? PB[PRE_B ? k : 0][c] : sR[3 * j + c]) - R[c];
            dv[c] = v - L[c] * rint(v * iL[c]);
            r2 += dv[c] * dv[c];
          }
          double coef;
          if (mp.bond == 1) {   // harmonic: k (r - l) / r along the bond
            const double r = sqrt(r2);
            coef = r > 0.0 ? mp.k_bond * (r - mp.l_bond) / r : 0.0;
          } else {
            const double x2 = r2 * iR02;
            if (x2 >= 1.0) {
              atomicOr(bs.err, ERR_BOND);
              continue;
            }
            coef = mp.k_fene / (1.0 - x2);
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) F[c] += coef * dv[c];
        }
      }
      // combine the lanes of this bead (the field enters only as q E, so each
      // lane adds its corners' share to its force first)
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] += qe[c];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = group_sum<TPB>(acc[c]);
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] = group_sum<TPB>(F[c]);
      // friction of each species (with the thermal noise shared by the
      // species' number fractions) and the substep update
      double xi[3] = {0.0, 0.0, 0.0};
      if (THERMAL && mp.thermal) {
        const Philox4 w = philox4x32_10(uint32_t(i), mp.tstep, uint32_t(sub), 1u, mp.key0, mp.key1);
        double z[4];
        box_muller4<double>(w, z);
#pragma unroll
        for (int c = 0; c < 3; ++c) xi[c] = mp.xi_scale * z[c];
      }
      double ftot[3] = {F[0], F[1], F[2]};
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          phi[s][c] = mp.gamma * acc[9 + s] * (acc[3 * s + c] - V[c]) + acc[9 + s] * xi[c];
          ftot[c] += phi[s][c];
        }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        V[c] += hM * ftot[c];
        Rn[c] = R[c] + h * V[c];
      }
    }
    __syncthreads();   // every bead has read positions and node momenta of this substep
    if (live) {
#pragma unroll
      for (int a = 0; a < CPL; ++a) {
        if (wt[a] == 0.0 || slot[a] == -1) continue;
        const double g = -h * wt[a] * FIX_FORCE;   // impulse scale of this corner
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const long long v = round_fixed(phi[s][c] * g);
            if (LDS) ln.add(slot[a], 3 * s + c, v);
            else gn.add(slot[a], 3 * s + c, v);
          }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R[c] = Rn[c];
        if (lane == 0) sR[3 * i + c] = Rn[c];
      }
      if (NLIST) {   // moved more than half the skin since the build: rebuild next substep
        double dd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) dd += (R[c] - Rb[c]) * (R[c] - Rb[c]);
        if (dd > half_skin2) s_rebuild = 1;
      }
    }
    // one workgroup advances the chain: the barrier's workgroup-scope ordering
    // (prior atomics completed) is enough for the table's atomic reads, which
    // go to the shared L2
    __syncthreads();
  }
  if (live && lane == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bs.R[3 * i + c] = R[c];
      bs.V[3 * i + c] = V[c];
    }
    if (mp.track && bs.cross) {   // the step moved the bead across an image of the plane
      const double k0 = floor((z_start - mp.z_plane) / mp.Lz);
      const double k1 = floor((R[2] - mp.z_plane) / mp.Lz);
      if (k0 != k1) {
        int* cr = bs.cross + 3 * i;
        if (cr[0] < 0) cr[0] = mp.step;
        cr[1] = mp.step;
        cr[2] += k1 > k0 ? 1 : -1;
      }
    }
  }
  if (LDS) {   // hand the accumulated impulses to the lattice kernels
    __syncthreads();
    for (int hh = threadIdx.x; hh < lslots; hh += blockDim.x) {
      const int key = lkeys[hh];
      if (key < 0) continue;
      const int g = table_insert(gkeys, mask, key, bs.err, gbits);
      if (g < 0) continue;
      for (int c = 0; c < 9; ++c) {
        const long long v = lvals[(size_t)hh * 9 + c];
        if (v) atomicAdd((unsigned long long*)&gvals[(size_t)g * SLOT_VALUES + 1 + c], (unsigned long long)v);
      }
    }
  }
  __syncthreads();
}

}  // namespace ek
