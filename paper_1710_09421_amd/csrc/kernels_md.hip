// Bead-spring chain coupled to the three species by friction (Sec. II.B)
// through the trilinear interpolation / spreading kernel (Sec. II.C):
// single-system launches and the host side of the chain.  The device code is
// in md_chain.h.
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
#include <climits>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ek_context.h"
#include "md_chain.h"
#include "reduce.h"

using namespace ek;

namespace {

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
  s.flags = (unsigned char*)take((size_t)maxb * WIN3_MAX + 8);
  s.err = (int*)take(64);
  s.cross = (int*)take((size_t)maxb * 3 * 4 + 4);
  return s;
}

// Wall reach of a chain (WallGeom): 1 for a WCA cut-off below two lattice
// spacings, 2 below three.
int wall_reach(double sigma) { return 1.122462048309373 * sigma < 2.0 ? 1 : 2; }

// Empty table (once, when the context is created: the workspace arrives
// uninitialised).
__global__ __launch_bounds__(256) void k_table_init(int* keys, long long* vals, int slots) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= slots) return;
  keys[h] = -1;
#pragma unroll
  for (int c = 0; c < SLOT_VALUES; ++c) vals[(size_t)h * SLOT_VALUES + c] = 0;
}

__global__ __launch_bounds__(256) void k_table_clear(int* keys, long long* vals, uint32_t* mask,
                                                     long long n, int bits) {
  table_clear_items(keys, vals, mask, n, bits, blockIdx.x * blockDim.x + threadIdx.x,
                    gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(256) void k_deposit(BeadState bs, int n, int* keys, long long* vals,
                                                 uint32_t* mask, Dims d, int bits, int fluid_only) {
  deposit_items(bs, n, keys, vals, mask, d, bits, blockIdx.x * blockDim.x + threadIdx.x,
                gridDim.x * blockDim.x, fluid_only != 0);
}

// One block per bead: moments and field on the 4^3 box, flags on the 6^3 window.
template <typename T, int WR>
__global__ __launch_bounds__(256) void k_bead_box(BeadState bs, const T* __restrict__ f,
                                                  uint32_t* mask, const double* __restrict__ psi,
                                                  LBParams lp, Dims d, int defer,
                                                  const double* face_q, double inv_eps) {
  constexpr int items = WallGeom<WR>::W3 > BOX3 ? WallGeom<WR>::W3 : BOX3;
  for (int t = threadIdx.x; t < items; t += blockDim.x)
    bead_box_item<T, WR>(bs, blockIdx.x, t, f, mask, psi, lp, d, defer ? mask : nullptr, face_q,
                         inv_eps);
}

template <bool LDS, int TPB, int NBL, int MAXT, int WR>
__global__ __launch_bounds__(MAXT) void k_md(BeadState bs, MDParams mp, int* gkeys,
                                             long long* gvals, uint32_t* mask, Dims d,
                                             int gbits, int lds_slots) {
  extern __shared__ __align__(16) unsigned char smem[];
  md_chain<LDS, TPB, NBL, WR>(bs, mp, gkeys, gvals, mask, d, gbits, lds_slots, smem);
}

// LDS of one workgroup the chain kernel may use: the device's limit for a
// kernel that asks for it (160 KiB on gfx950), else the default 64 KiB.
constexpr size_t CHAIN_LDS_MAX = 159 * 1024;   // 160 KiB less the static LDS of the kernel
constexpr size_t CHAIN_LDS_DEFAULT = 64 * 1024;

__global__ void k_err_reset(int* err) {
  if (threadIdx.x == 0) *err = 0;
}

// Empty crossing record: no first / last step (-1), net count 0.
__global__ __launch_bounds__(256) void k_cross_reset(int* cross, int maxb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= maxb) return;
  cross[3 * i] = -1;
  cross[3 * i + 1] = -1;
  cross[3 * i + 2] = 0;
}

void launch_table_clear(int* keys, long long* vals, uint32_t* mask, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_table_clear, dim3(HASH_SLOTS / 256), dim3(256), 0, s, keys, vals, mask, n,
                     HASH_BITS);
}

}  // namespace

// ---------------------------------------------------------------------------
size_t ek::bead_state_bytes(int maxb) {
  maxb = maxb < 1 ? 1 : maxb;
  size_t t = 0;
  t += align256(maxb * 3 * 8 + 8) * 2 + align256(maxb * 8 + 8) + align256(maxb * 3 * 4 + 4);
  t += align256((size_t)maxb * BOX3 * MOM * 8 + 8) + align256((size_t)maxb * BOX3 * 3 * 8 + 8);
  t += align256((size_t)maxb * WIN3_MAX + 8) + align256(64);
  t += align256((size_t)maxb * 3 * 4 + 4);   // plane crossing record
  return t;
}

void ek::launch_table_init_bits(int* keys, long long* vals, int bits, hipStream_t s) {
  const int slots = 1 << bits;
  hipLaunchKernelGGL(k_table_init, dim3((slots + 255) / 256), dim3(256), 0, s, keys, vals, slots);
}

void ek::launch_table_init(int* keys, long long* vals, hipStream_t s) {
  hipLaunchKernelGGL(k_table_init, dim3(HASH_SLOTS / 256), dim3(256), 0, s, keys, vals, HASH_SLOTS);
}

BeadState ek::bead_state_view(char* mem, int max_beads) {
  return carve(mem, max_beads < 1 ? 1 : max_beads);
}

const int* ek_ctx::bead_origin() const {
  return carve(bead_mem, max_beads < 1 ? 1 : max_beads).origin;
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
                     keys, vals, mask, dims, HASH_BITS, insulating() ? 1 : 0);
  return EK_OK;
}

template <typename T>
ek_status ek_ctx::beads_advance(bool overlap, hipEvent_t chain_end) {
  BeadState bs = carve(bead_mem, max_beads < 1 ? 1 : max_beads);
  const LBParams lp = lb_params();
  const int wr = wall_reach(poly.sigma);
  auto box = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(n_beads), dim3(256), 0, stream, bs, (const T*)fcur(), mask, psi,
                       lp, dims, overlap ? 1 : 0, insulating() ? wall_q : nullptr, inv_eps());
  };
  if (wr == 1) box(k_bead_box<T, 1>);
  else box(k_bead_box<T, 2>);
  const hipStream_t cs = stream;   // the chain follows the box gather on the context stream
  if (overlap) {
    // the lattice update outside the boxes (launched by the caller on the
    // side stream) may start once the boxes are flagged
    if (!side_stream) {
      if (hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&side_fork, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&side_join, hipEventDisableTiming) != hipSuccess)
        return fail(EK_EHIP, "creating the side stream failed");
    }
    if (hipEventRecord(side_fork, stream) != hipSuccess)
      return fail(EK_EHIP, "recording the side stream's fork failed");
  }
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
  mp.bond = poly.bond;
  mp.k_bond = poly.k_bond;
  mp.l_bond = poly.l_bond;
  mp.track = cross_on ? 1 : 0;
  mp.step = (int)(step_count + 1);
  mp.z_plane = cross_plane;
  mp.theta = poly.coupling == EK_COUPLE_THETA ? 1 : 0;
  mp.half_sigma = 0.5 * poly.sigma;
  mp.field_fluid = insulating() ? 1 : 0;
  if (p.fluctuations) {
    mp.thermal = 1;
    mp.key0 = uint32_t(p.seed & 0xFFFFFFFFull);
    mp.key1 = uint32_t(p.seed >> 32);
    mp.tstep = uint32_t(step_count);
    mp.xi_scale = std::sqrt(2.0 * poly.gamma * p.kT * poly.n_sub);   // h = 1 / n_sub
  }
  // lanes per bead so that a chain fills at most 512 threads (register budget
  // of 256 per thread); chains beyond 512 beads take one lane each
  const int tpb = n_beads <= 64 ? 8 : (n_beads <= 128 ? 4 : (n_beads <= 256 ? 2 : 1));
  const int threads = ((n_beads * tpb + 63) / 64) * 64;
  const size_t sr_bytes = ((size_t)n_beads * 24 + 15) & ~size_t(15);
  // The node table lives in LDS: 16 slots per bead (a load factor of at most
  // 1/2 for eight corners per bead) where they fit beside the positions and
  // the pair lists, else as many as fit (sites past them go to the global
  // table).  Chains of at most SMALL_CHAIN beads list every candidate partner.
  auto md = [&](auto kernel, int nbl) -> ek_status {
    const size_t fixed = sr_bytes + md_list_bytes(threads, nbl);
    auto slots_for = [&](size_t budget) {
      const long long room = budget > fixed ? (long long)((budget - fixed) / (9 * 8 + 4)) : 0;
      return (int)std::min<long long>(16LL * n_beads, room);
    };
    int slots = slots_for(CHAIN_LDS_MAX);
    size_t lds = fixed + (size_t)slots * (9 * 8 + 4);
    if (lds > CHAIN_LDS_DEFAULT &&
        hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess) {
      (void)hipGetLastError();
      slots = slots_for(CHAIN_LDS_DEFAULT);
      lds = fixed + (size_t)slots * (9 * 8 + 4);
    }
    if (slots < 1) return fail(EK_EHIP, "the chain's positions and pair lists do not fit LDS");
    hipLaunchKernelGGL(kernel, dim3(1), dim3(threads), lds, cs, bs, mp, keys, vals, mask, dims,
                       HASH_BITS, slots);
    return EK_OK;
  };
  // the kernel instance for the chain's size and wall reach
  auto launch = [&](auto wr_tag) -> ek_status {
    constexpr int WR = decltype(wr_tag)::value;
    if (tpb == 8) return md(k_md<true, 8, SMALL_CHAIN / 8, 512, WR>, SMALL_CHAIN / 8);
    if (tpb == 4) return md(k_md<true, 4, NB_PER_LANE, 512, WR>, NB_PER_LANE);
    if (tpb == 2) return md(k_md<true, 2, NB_PER_LANE, 512, WR>, NB_PER_LANE);
    if (threads <= 512) return md(k_md<true, 1, NB_PER_LANE, 512, WR>, NB_PER_LANE);
    return md(k_md<true, 1, NB_PER_LANE, 1024, WR>, NB_PER_LANE);
  };
  const ek_status lst = wr == 1 ? launch(std::integral_constant<int, 1>{})
                                : launch(std::integral_constant<int, 2>{});
  if (lst) return lst;
  if (chain_end && hipEventRecord(chain_end, cs) != hipSuccess)
    return fail(EK_EHIP, "recording the chain timer failed");
  return EK_OK;
}
template ek_status ek_ctx::beads_advance<float>(bool, hipEvent_t);
template ek_status ek_ctx::beads_advance<double>(bool, hipEvent_t);

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
    const bool fene = pp->bond == EK_BOND_FENE;
    if (!(pp->M > 0) || pp->n_sub < 1 || !(pp->gamma >= 0) || !(pp->sigma > 0) ||
        !(pp->eps >= 0) || (pp->bond != EK_BOND_FENE && pp->bond != EK_BOND_HARMONIC) ||
        (fene && (!(pp->R0 > 0) || !(pp->k_fene >= 0))) ||
        (!fene && (!(pp->k_bond >= 0) || !(pp->l_bond > 0))))
      return ctx->fail(EK_EINVAL, "invalid polymer parameters");
    if (1.122462048309373 * pp->sigma >= 3.0)
      return ctx->fail(EK_EINVAL, "WCA cut-off must stay below three lattice spacings");
    if (pp->coupling != EK_COUPLE_TRILINEAR && pp->coupling != EK_COUPLE_THETA)
      return ctx->fail(EK_EINVAL, "unknown coupling");
    if (pp->coupling == EK_COUPLE_THETA && !(pp->sigma >= 1.0 && pp->sigma <= 2.0))
      return ctx->fail(EK_EINVAL, "the occupation cube needs 1 <= sigma <= 2");
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
        if (fene && r2 >= pp->R0 * pp->R0) return ctx->fail(EK_EINVAL, "a bond is longer than R0");
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
  // clear a previous chain's node table, error flags and crossing record
  launch_table_clear(ctx->keys, ctx->vals, ctx->mask, ctx->dims.n, ctx->stream);
  hipLaunchKernelGGL(k_err_reset, dim3(1), dim3(64), 0, ctx->stream, bs.err);
  const int mb = ctx->max_beads < 1 ? 1 : ctx->max_beads;
  hipLaunchKernelGGL(k_cross_reset, dim3((mb + 255) / 256), dim3(256), 0, ctx->stream, bs.cross, mb);
  ctx->n_beads = n;
  ctx->host_q = q;
  return ctx->sync();
}

extern "C" ek_status ek_set_crossing_plane(ek_ctx* ctx, double z_plane) {
  if (!ctx) return EK_EINVAL;
  if (!std::isfinite(z_plane)) return ctx->fail(EK_EINVAL, "non-finite crossing plane");
  if (!ctx->bead_mem) return ctx->fail(EK_ESTATE, "the context has no bead storage");
  const int mb = ctx->max_beads < 1 ? 1 : ctx->max_beads;
  BeadState bs = carve(ctx->bead_mem, mb);
  hipLaunchKernelGGL(k_cross_reset, dim3((mb + 255) / 256), dim3(256), 0, ctx->stream, bs.cross, mb);
  ctx->cross_on = true;
  ctx->cross_plane = z_plane;
  return ctx->sync();
}

extern "C" ek_status ek_get_crossings(ek_ctx* ctx, int32_t* first, int32_t* last, int32_t* net) {
  if (!ctx) return EK_EINVAL;
  if (!ctx->cross_on) return ctx->fail(EK_ESTATE, "no crossing plane is set");
  if (ctx->n_beads == 0) return EK_OK;
  const int n = ctx->n_beads;
  BeadState bs = carve(ctx->bead_mem, ctx->max_beads < 1 ? 1 : ctx->max_beads);
  std::vector<int> rec((size_t)n * 3);
  if (hipMemcpyAsync(rec.data(), bs.cross, (size_t)n * 3 * 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return ctx->fail(EK_EHIP, "copying the crossing record failed");
  ek_status st = ctx->sync();
  if (st) return st;
  for (int i = 0; i < n; ++i) {
    if (first) first[i] = rec[3 * i];
    if (last) last[i] = rec[3 * i + 1];
    if (net) net[i] = rec[3 * i + 2];
  }
  return EK_OK;
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
