// Bead-spring chain coupled to the three species by friction (Sec. II.B)
// through the trilinear interpolation / spreading kernel (Sec. II.C).
//
// Per lattice step:
//   k_table_clear   drop last step's node table entries and their site flags
//   k_deposit       bead charges q_i W(r - R_i) onto the 8 corner nodes
//   (charge pass, Poisson solve)
//   k_bead_box      per bead, the fields of time t on the 4x4x4 nodes around
//                   it (species density and momentum, electric field) and the
//                   fluid / wall flags on the 6x6x6 nodes around it
//   k_md            one workgroup per chain, one thread per bead: n_sub
//                   substeps of friction + FENE + WCA (pairs and wall) +
//                   electric force, semi-implicit Euler; the friction impulse
//                   is spread onto the nodes after every substep, and the
//                   node velocities seen by later substeps include it
//   (fused lattice step reads the accumulated force density)
//
// Node values are int64 fixed point added with atomics, so the sums do not
// depend on the order in which beads and substeps reach a node.
#include <cmath>
#include <cstring>
#include <vector>

#include "ek_context.h"
#include "reduce.h"

using namespace ek;

namespace {

constexpr int BOX = 4;          // moment box edge (nodes floor(R0) - 1 .. floor(R0) + 2)
constexpr int BOX3 = BOX * BOX * BOX;
constexpr int WIN = 6;          // flag window edge (nodes floor(R0) - 2 .. floor(R0) + 3)
constexpr int WIN3 = WIN * WIN * WIN;
constexpr int MOM = 12;         // n[3], j[3][3]

enum : int { ERR_BOX = 1, ERR_FLUID = 2, ERR_BOND = 4, ERR_TABLE = 8 };

struct BeadState {
  double* R;          // [maxb][3]
  double* V;          // [maxb][3]
  double* q;          // [maxb]
  int* origin;        // [maxb][3] floor(R0) - 1 of the current step
  double* mom;        // [maxb][BOX3][MOM]
  double* efield;     // [maxb][BOX3][3]
  unsigned char* flags;  // [maxb][WIN3]: bit0 fluid, bit1 wall
  int* err;           // error bits
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

BeadState carve(char* mem, int maxb) {
  BeadState s;
  size_t off = 0;
  auto take = [&](size_t b) { char* p = mem + off; off += align256(b); return p; };
  s.R = (double*)take(maxb * 3 * 8 + 8);
  s.V = (double*)take(maxb * 3 * 8 + 8);
  s.q = (double*)take(maxb * 8 + 8);
  s.origin = (int*)take(maxb * 3 * 4 + 4);
  s.mom = (double*)take((size_t)maxb * BOX3 * MOM * 8 + 8);
  s.efield = (double*)take((size_t)maxb * BOX3 * 3 * 8 + 8);
  s.flags = (unsigned char*)take((size_t)maxb * WIN3 + 8);
  s.err = (int*)take(64);
  return s;
}

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
__device__ inline int table_insert(int* keys, uint32_t* mask, long long site, int* err) {
  int h = hash_slot(site);
  for (int k = 0; k < HASH_SLOTS; ++k) {
    const int prev = atomicCAS(&keys[h], -1, int(site));
    if (prev == -1) {
      atomicOr(&mask[site], MASK_BEAD);
      return h;
    }
    if (prev == int(site)) return h;
    h = (h + 1) & (HASH_SLOTS - 1);
  }
  atomicOr(err, ERR_TABLE);
  return -1;
}

// Slot of `site` if present (reads that see the atomics of this launch).
__device__ inline int table_find(const int* keys, long long site) {
  int h = hash_slot(site);
  for (int k = 0; k < HASH_SLOTS; ++k) {
    const int key = ld_i32(&keys[h]);
    if (key == int(site)) return h;
    if (key < 0) return -1;
    h = (h + 1) & (HASH_SLOTS - 1);
  }
  return -1;
}

// Empty table (once, when the context is created: the workspace arrives
// uninitialised).
__global__ __launch_bounds__(256) void k_table_init(int* keys, long long* vals) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= HASH_SLOTS) return;
  keys[h] = -1;
#pragma unroll
  for (int c = 0; c < SLOT_VALUES; ++c) vals[(size_t)h * SLOT_VALUES + c] = 0;
}

__global__ __launch_bounds__(256) void k_table_clear(int* keys, long long* vals, uint32_t* mask,
                                                     long long n) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= HASH_SLOTS) return;
  const int key = keys[h];
  if (key >= 0 && key < n) {
    atomicAnd(&mask[key], ~MASK_BEAD);
    keys[h] = -1;
#pragma unroll
    for (int c = 0; c < SLOT_VALUES; ++c) vals[(size_t)h * SLOT_VALUES + c] = 0;
  }
}

// One thread per (bead, corner): plain trilinear weight of the corner.
__global__ __launch_bounds__(256) void k_deposit(BeadState bs, int n, int* keys, long long* vals,
                                                 uint32_t* mask, Dims d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 8 * n) return;
  const int i = t >> 3, k = t & 7;
  const double* R = bs.R + 3 * i;
  const double fx = floor(R[0]), fy = floor(R[1]), fz = floor(R[2]);
  const double dx = R[0] - fx, dy = R[1] - fy, dz = R[2] - fz;
  const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
  const double w = (ox ? dx : 1.0 - dx) * (oy ? dy : 1.0 - dy) * (oz ? dz : 1.0 - dz);
  const long long site = site_of(int(fx) + ox, int(fy) + oy, int(fz) + oz, d);
  const int h = table_insert(keys, mask, site, bs.err);
  if (h < 0) return;
  atomicAdd((unsigned long long*)&vals[(size_t)h * SLOT_VALUES],
            (unsigned long long)llrint(bs.q[i] * w * FIX_CHARGE));
}

// Per bead: moments and field on the 4^3 box, flags on the 6^3 window.
template <typename T>
__global__ __launch_bounds__(256) void k_bead_box(BeadState bs, const T* __restrict__ f,
                                                  const uint32_t* __restrict__ mask,
                                                  const double* __restrict__ psi, LBParams lp,
                                                  Dims d) {
  const int i = blockIdx.x;
  const double* R = bs.R + 3 * i;
  const int bx = int(floor(R[0])) - 1, by = int(floor(R[1])) - 1, bz = int(floor(R[2])) - 1;
  if (threadIdx.x == 0) {
    bs.origin[3 * i] = bx;
    bs.origin[3 * i + 1] = by;
    bs.origin[3 * i + 2] = bz;
  }
  for (int t = threadIdx.x; t < WIN3; t += blockDim.x) {
    const int wx = t % WIN, wy = (t / WIN) % WIN, wz = t / (WIN * WIN);
    const uint32_t m = mask[site_of(bx - 1 + wx, by - 1 + wy, bz - 1 + wz, d)];
    bs.flags[(size_t)i * WIN3 + t] =
        (unsigned char)(((m & MASK_SOLID) ? 0 : 1) | ((m & MASK_WALL) ? 2 : 0));
  }
  const int t = threadIdx.x;
  if (t >= BOX3) return;
  const int cx = bx + t % BOX, cy = by + (t / BOX) % BOX, cz = bz + t / (BOX * BOX);
  const long long r = site_of(cx, cy, cz, d);
  const uint32_t m = mask[r];
  double* mo = bs.mom + ((size_t)i * BOX3 + t) * MOM;
  for (int c = 0; c < MOM; ++c) mo[c] = 0.0;
  if (!(m & MASK_SOLID)) {
    const int x = wrap(cx, d.nx), y = wrap(cy, d.ny), z = wrap(cz, d.nz);
    for (int s = 0; s < 3; ++s) {
      double dn = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
      for (int p = 0; p < Q; ++p) {
        long long src;
        int q = p;
        if ((m >> p) & 1u) {
          src = r;
          q = OPP[p];
        } else {
          src = site_of(x - CX[p], y - CY[p], z - CZ[p], d);
        }
        const double g = double(f[(size_t)(s * Q + q) * d.n + src]);
        dn += g;
        jx += CX[p] * g;
        jy += CY[p] * g;
        jz += CZ[p] * g;
      }
      mo[s] = lp.nref[s] + dn;
      mo[3 + 3 * s] = jx;
      mo[4 + 3 * s] = jy;
      mo[5 + 3 * s] = jz;
    }
  }
  double* e = bs.efield + ((size_t)i * BOX3 + t) * 3;
  e[0] = -0.5 * (psi[site_of(cx + 1, cy, cz, d)] - psi[site_of(cx - 1, cy, cz, d)]) + lp.eext[0];
  e[1] = -0.5 * (psi[site_of(cx, cy + 1, cz, d)] - psi[site_of(cx, cy - 1, cz, d)]) + lp.eext[1];
  e[2] = -0.5 * (psi[site_of(cx, cy, cz + 1, d)] - psi[site_of(cx, cy, cz - 1, d)]) + lp.eext[2];
}

struct MDParams {
  int n, n_sub;
  double M, k_fene, R0, eps, sigma, gamma;
  double Lx, Ly, Lz;
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

__global__ __launch_bounds__(1024) void k_md(BeadState bs, MDParams mp, int* keys,
                                             long long* vals, uint32_t* mask, Dims d) {
  __shared__ double sR[3 * MAX_BEADS];
  const int i = threadIdx.x;
  const bool live = i < mp.n;
  double R[3] = {0, 0, 0}, V[3] = {0, 0, 0}, q = 0.0;
  int org[3] = {0, 0, 0};
  if (live) {
    for (int c = 0; c < 3; ++c) {
      R[c] = bs.R[3 * i + c];
      V[c] = bs.V[3 * i + c];
      org[c] = bs.origin[3 * i + c];
      sR[3 * i + c] = R[c];
    }
    q = bs.q[i];
  }
  __syncthreads();
  const double h = 1.0 / mp.n_sub;
  const double* mom = bs.mom + (size_t)i * BOX3 * MOM;
  const double* ef = bs.efield + (size_t)i * BOX3 * 3;
  const unsigned char* fl = bs.flags + (size_t)i * WIN3;
  for (int sub = 0; sub < mp.n_sub; ++sub) {
    double wt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long site[8];
    double phi[3][3];
    double Rn[3];
    if (live) {
      const int fx = int(floor(R[0])), fy = int(floor(R[1])), fz = int(floor(R[2]));
      const double dx = R[0] - fx, dy = R[1] - fy, dz = R[2] - fz;
      int lx = fx - org[0], ly = fy - org[1], lz = fz - org[2];   // corner 0 in the box
      if (lx < 0 || lx > BOX - 2 || ly < 0 || ly > BOX - 2 || lz < 0 || lz > BOX - 2) {
        atomicOr(bs.err, ERR_BOX);
        lx = min(max(lx, 0), BOX - 2);
        ly = min(max(ly, 0), BOX - 2);
        lz = min(max(lz, 0), BOX - 2);
      }
      double w[8], wsum = 0.0;
      int bidx[8];
      for (int k = 0; k < 8; ++k) {
        const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
        w[k] = (ox ? dx : 1.0 - dx) * (oy ? dy : 1.0 - dy) * (oz ? dz : 1.0 - dz);
        bidx[k] = (lx + ox) + BOX * ((ly + oy) + BOX * (lz + oz));
        const int wi = (lx + ox + 1) + WIN * ((ly + oy + 1) + WIN * (lz + oz + 1));
        const bool fluid = fl[wi] & 1;
        wt[k] = fluid ? w[k] : 0.0;
        wsum += wt[k];
        site[k] = site_of(fx + ox, fy + oy, fz + oz, d);
      }
      if (!(wsum > 0.0)) {
        atomicOr(bs.err, ERR_FLUID);
        wsum = 1.0;
      }
      for (int k = 0; k < 8; ++k) wt[k] /= wsum;
      // fields at the bead: velocities from the node momentum (populations of
      // time t plus the friction impulse of earlier substeps), composition,
      // electric field with the plain weights
      double u[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, x[3] = {0, 0, 0}, E[3] = {0, 0, 0};
      for (int k = 0; k < 8; ++k) {
        const double* mo = mom + (size_t)bidx[k] * MOM;
        const double* e = ef + (size_t)bidx[k] * 3;
        for (int c = 0; c < 3; ++c) E[c] += w[k] * e[c];
        if (wt[k] == 0.0) continue;
        double kacc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        const int hsl = table_find(keys, site[k]);
        if (hsl >= 0) {
          for (int s = 0; s < 3; ++s)
            for (int c = 0; c < 3; ++c)
              kacc[s][c] = double(ld_i64(&vals[(size_t)hsl * SLOT_VALUES + 1 + 3 * s + c])) *
                           (1.0 / FIX_FORCE);
        }
        const double ntot = mo[0] + mo[1] + mo[2];
        for (int s = 0; s < 3; ++s) {
          x[s] += wt[k] * mo[s] / ntot;
          for (int c = 0; c < 3; ++c) u[s][c] += wt[k] * (mo[3 + 3 * s + c] + kacc[s][c]) / mo[s];
        }
      }
      // conservative forces
      double F[3] = {q * E[0], q * E[1], q * E[2]};
      const double L[3] = {mp.Lx, mp.Ly, mp.Lz};
      for (int nb = -1; nb <= 1; nb += 2) {           // FENE bonds
        const int j = i + nb;
        if (j < 0 || j >= mp.n) continue;
        double dv[3], r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
          dv[c] = min_image(sR[3 * j + c] - R[c], L[c]);
          r2 += dv[c] * dv[c];
        }
        const double x2 = r2 / (mp.R0 * mp.R0);
        if (x2 >= 1.0) {
          atomicOr(bs.err, ERR_BOND);
          continue;
        }
        const double coef = mp.k_fene / (1.0 - x2);
        for (int c = 0; c < 3; ++c) F[c] += coef * dv[c];
      }
      for (int j = 0; j < mp.n; ++j) {                 // WCA between all pairs
        if (j == i) continue;
        double dv[3], r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
          dv[c] = min_image(R[c] - sR[3 * j + c], L[c]);
          r2 += dv[c] * dv[c];
        }
        const double coef = wca_coef(r2, mp.eps, mp.sigma);
        for (int c = 0; c < 3; ++c) F[c] += coef * dv[c];
      }
      // WCA against wall-site centres within the 4^3 nodes around the bead
      for (int wz = 0; wz < 4; ++wz)
        for (int wy = 0; wy < 4; ++wy)
          for (int wx = 0; wx < 4; ++wx) {
            const int ax = fx - 1 + wx, ay = fy - 1 + wy, az = fz - 1 + wz;
            const int ix = ax - org[0] + 1, iy = ay - org[1] + 1, iz = az - org[2] + 1;
            if (ix < 0 || ix >= WIN || iy < 0 || iy >= WIN || iz < 0 || iz >= WIN) continue;
            if (!(fl[ix + WIN * (iy + WIN * iz)] & 2)) continue;
            const double dv[3] = {R[0] - ax, R[1] - ay, R[2] - az};
            const double coef = wca_coef(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2], mp.eps, mp.sigma);
            for (int c = 0; c < 3; ++c) F[c] += coef * dv[c];
          }
      // friction of each species and the substep update
      double ftot[3] = {F[0], F[1], F[2]};
      for (int s = 0; s < 3; ++s)
        for (int c = 0; c < 3; ++c) {
          phi[s][c] = mp.gamma * x[s] * (u[s][c] - V[c]);
          ftot[c] += phi[s][c];
        }
      for (int c = 0; c < 3; ++c) {
        V[c] += h * ftot[c] / mp.M;
        Rn[c] = R[c] + h * V[c];
      }
    }
    __syncthreads();   // every bead has read positions and node momenta of this substep
    if (live) {
      for (int k = 0; k < 8; ++k) {
        if (wt[k] == 0.0) continue;
        const int hsl = table_insert(keys, mask, site[k], bs.err);
        if (hsl < 0) continue;
        for (int s = 0; s < 3; ++s)
          for (int c = 0; c < 3; ++c)
            atomicAdd((unsigned long long*)&vals[(size_t)hsl * SLOT_VALUES + 1 + 3 * s + c],
                      (unsigned long long)llrint(-h * phi[s][c] * wt[k] * FIX_FORCE));
      }
      for (int c = 0; c < 3; ++c) {
        R[c] = Rn[c];
        sR[3 * i + c] = Rn[c];
      }
    }
    __threadfence();
    __syncthreads();
  }
  if (live) {
    for (int c = 0; c < 3; ++c) {
      bs.R[3 * i + c] = R[c];
      bs.V[3 * i + c] = V[c];
    }
  }
}

__global__ void k_err_reset(int* err) {
  if (threadIdx.x == 0) *err = 0;
}

void launch_table_clear(int* keys, long long* vals, uint32_t* mask, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_table_clear, dim3(HASH_SLOTS / 256), dim3(256), 0, s, keys, vals, mask, n);
}

}  // namespace

// ---------------------------------------------------------------------------
size_t ek::bead_state_bytes(int maxb) {
  maxb = maxb < 1 ? 1 : maxb;
  size_t t = 0;
  t += align256(maxb * 3 * 8 + 8) * 2 + align256(maxb * 8 + 8) + align256(maxb * 3 * 4 + 4);
  t += align256((size_t)maxb * BOX3 * MOM * 8 + 8) + align256((size_t)maxb * BOX3 * 3 * 8 + 8);
  t += align256((size_t)maxb * WIN3 + 8) + align256(64);
  return t;
}

void ek::launch_table_init(int* keys, long long* vals, hipStream_t s) {
  hipLaunchKernelGGL(k_table_init, dim3(HASH_SLOTS / 256), dim3(256), 0, s, keys, vals);
}

BeadTableView ek_ctx::bead_view() const {
  BeadTableView v;
  v.keys = keys;
  v.vals = vals;
  return v;
}

ek_status ek_ctx::beads_deposit() {
  BeadState bs = carve(bead_mem, max_beads < 1 ? 1 : max_beads);
  launch_table_clear(keys, vals, mask, dims.n, stream);
  hipLaunchKernelGGL(k_deposit, dim3((8 * n_beads + 255) / 256), dim3(256), 0, stream, bs, n_beads,
                     keys, vals, mask, dims);
  return EK_OK;
}

template <typename T>
ek_status ek_ctx::beads_advance() {
  BeadState bs = carve(bead_mem, max_beads < 1 ? 1 : max_beads);
  const LBParams lp = lb_params();
  hipLaunchKernelGGL(k_bead_box<T>, dim3(n_beads), dim3(256), 0, stream, bs, (const T*)fcur(),
                     mask, psi, lp, dims);
  MDParams mp;
  mp.n = n_beads;
  mp.n_sub = poly.n_sub;
  mp.M = poly.M;
  mp.k_fene = poly.k_fene;
  mp.R0 = poly.R0;
  mp.eps = poly.eps;
  mp.sigma = poly.sigma;
  mp.gamma = poly.gamma;
  mp.Lx = p.nx;
  mp.Ly = p.ny;
  mp.Lz = p.nz;
  const int threads = ((n_beads + 63) / 64) * 64;
  hipLaunchKernelGGL(k_md, dim3(1), dim3(threads), 0, stream, bs, mp, keys, vals, mask, dims);
  return EK_OK;
}
template ek_status ek_ctx::beads_advance<float>();
template ek_status ek_ctx::beads_advance<double>();

ek_status ek_ctx::beads_check() {
  BeadState bs = carve(bead_mem, max_beads < 1 ? 1 : max_beads);
  int e = 0;
  if (hipMemcpy(&e, bs.err, sizeof e, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(EK_EHIP, "reading the bead error flags failed");
  if (e) {
    std::string m = "bead update failed:";
    if (e & ERR_BOX) m += " a bead moved more than one lattice spacing in a step;";
    if (e & ERR_FLUID) m += " a bead has no fluid node around it;";
    if (e & ERR_BOND) m += " a FENE bond reached its maximum extension;";
    if (e & ERR_TABLE) m += " the bead node table is full;";
    return fail(EK_EUNSTABLE, m);
  }
  return EK_OK;
}

extern "C" ek_status ek_set_polymer(ek_ctx* ctx, int32_t n, const double* pos, const double* vel,
                                    const double* charge, const ek_polymer_params* pp) {
  if (!ctx) return EK_EINVAL;
  if (!ctx->have_geometry) return ctx->fail(EK_ESTATE, "set the geometry first");
  if (n < 0 || n > ctx->max_beads) return ctx->fail(EK_EINVAL, "n_beads exceeds max_beads of the context");
  if (n > 0 && (!pos || !vel || !pp)) return ctx->fail(EK_EINVAL, "NULL polymer argument");
  if (n > 0) {
    if (!(pp->M > 0) || pp->n_sub < 1 || !(pp->gamma >= 0) || !(pp->R0 > 0) || !(pp->sigma > 0) ||
        !(pp->eps >= 0) || !(pp->k_fene >= 0))
      return ctx->fail(EK_EINVAL, "invalid polymer parameters");
    if (1.122462048309373 * pp->sigma >= 2.0)
      return ctx->fail(EK_EINVAL, "WCA cut-off must stay below two lattice spacings");
    const Dims d = ctx->dims;
    for (int i = 0; i < n; ++i) {
      for (int c = 0; c < 3; ++c)
        if (!std::isfinite(pos[3 * i + c]) || !std::isfinite(vel[3 * i + c]))
          return ctx->fail(EK_EINVAL, "non-finite bead position or velocity");
      if (i > 0) {
        const double L[3] = {double(d.nx), double(d.ny), double(d.nz)};
        double r2 = 0;
        for (int c = 0; c < 3; ++c) {
          double v = pos[3 * i + c] - pos[3 * (i - 1) + c];
          v -= L[c] * std::rint(v / L[c]);
          r2 += v * v;
        }
        if (r2 >= pp->R0 * pp->R0) return ctx->fail(EK_EINVAL, "a bond is longer than R0");
      }
      bool fluid = false;
      const int fx = (int)std::floor(pos[3 * i]), fy = (int)std::floor(pos[3 * i + 1]),
                fz = (int)std::floor(pos[3 * i + 2]);
      for (int k = 0; k < 8; ++k) {
        const int x = ((fx + (k & 1)) % d.nx + d.nx) % d.nx;
        const int y = ((fy + ((k >> 1) & 1)) % d.ny + d.ny) % d.ny;
        const int z = ((fz + ((k >> 2) & 1)) % d.nz + d.nz) % d.nz;
        if (!ctx->host_solid[((long long)z * d.ny + y) * d.nx + x]) fluid = true;
      }
      if (!fluid) return ctx->fail(EK_EINVAL, "a bead has no fluid node around it");
    }
  }
  BeadState bs = carve(ctx->bead_mem, ctx->max_beads < 1 ? 1 : ctx->max_beads);
  std::vector<double> q(n > 0 ? n : 1, 0.0);
  if (charge)
    for (int i = 0; i < n; ++i) q[i] = charge[i];
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = hipMemcpyAsync(bs.R, pos, n * 3 * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(bs.V, vel, n * 3 * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(bs.q, q.data(), n * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return ctx->fail(EK_EHIP, "copying the polymer failed");
    ctx->poly = *pp;
  }
  // clear a previous chain's node table and error flags
  launch_table_clear(ctx->keys, ctx->vals, ctx->mask, ctx->dims.n, ctx->stream);
  hipLaunchKernelGGL(k_err_reset, dim3(1), dim3(64), 0, ctx->stream, bs.err);
  ctx->n_beads = n;
  ctx->host_q = q;
  return ctx->sync();
}

extern "C" ek_status ek_get_beads(ek_ctx* ctx, double* pos, double* vel) {
  if (!ctx) return EK_EINVAL;
  if (ctx->n_beads == 0) return EK_OK;
  BeadState bs = carve(ctx->bead_mem, ctx->max_beads < 1 ? 1 : ctx->max_beads);
  if (pos && hipMemcpyAsync(pos, bs.R, ctx->n_beads * 3 * 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return ctx->fail(EK_EHIP, "copying bead positions failed");
  if (vel && hipMemcpyAsync(vel, bs.V, ctx->n_beads * 3 * 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return ctx->fail(EK_EHIP, "copying bead velocities failed");
  return ctx->sync();
}
