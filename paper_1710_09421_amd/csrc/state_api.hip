// Checkpoint and resume of a context: everything the time loop of Fig. 1
// carries from one step to the next, in one host buffer.
//
// Layout of a state buffer (little-endian, as written by this library):
//   StateHeader
//   payload, every section starting on an 8-byte boundary:
//     solid     nz*ny*nx bytes (0 fluid, 1 solid)
//     wall_q    nz*ny*nx doubles
//     f         3*19*nz*ny*nx populations of the precision, the current
//               post-collision values stored as deviations from w_p nref
//     psi       nz*ny*nx doubles: the last solution
//     psi_old   nz*ny*nx doubles: the solution before it (extrapolated starts)
//     psi_old2  nz*ny*nx doubles: the one before that (quadratic, cubic start)
//     psi_old3  nz*ny*nx doubles: the one before that (cubic start)
//     q, R, V   n_beads, 3*n_beads, 3*n_beads doubles
//     cross     3*n_beads int32: first step, last step, net count
// The header carries the counters the next steps depend on (step count,
// the previous solve's cycle count that schedules the next solve's residual
// tests, the extrapolation history), the reference densities of the
// deviation storage and a 64-bit checksum of the payload.
#include <cstring>
#include <string>
#include <vector>

#include "ek_context.h"
#include "md_chain.h"

using namespace ek;

namespace {

constexpr char STATE_MAGIC[8] = {'E', 'K', 'S', 'T', 'A', 'T', 'E', '\0'};
constexpr uint32_t STATE_VERSION = 1;

struct StateHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  int32_t nx, ny, nz, precision, warm_start, n_beads;
  int64_t step_count;
  int32_t last_iters, solo_iters, psi_hist, reserved0;
  double last_res, last_res0;
  double nref[3], mass[3], mom[3];
  int32_t cross_on, pad0;
  double cross_plane;
  ek_polymer_params poly;
  uint64_t payload_bytes;
  uint64_t checksum;
};

size_t up8(size_t x) { return (x + 7) & ~size_t(7); }

struct Sections {
  size_t solid, wall_q, f, psi, psi_old, psi_old2, psi_old3, q, R, V, cross, total;
};

Sections sections(const ek_params& p, int n_beads) {
  const size_t n = (size_t)p.nx * p.ny * p.nz;
  const size_t tsz = p.precision == EK_FP64 ? 8 : 4;
  Sections s{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += up8(b); return o; };
  s.solid = take(n);
  s.wall_q = take(n * 8);
  s.f = take(3 * Q * n * tsz);
  s.psi = take(n * 8);
  const int held = extrap_history(p.warm_start);
  s.psi_old = take(held >= 1 ? n * 8 : 0);
  s.psi_old2 = take(held >= 2 ? n * 8 : 0);
  s.psi_old3 = take(held >= 3 ? n * 8 : 0);
  s.q = take((size_t)n_beads * 8);
  s.R = take((size_t)n_beads * 24);
  s.V = take((size_t)n_beads * 24);
  s.cross = take((size_t)n_beads * 12);
  s.total = off;
  return s;
}

// 64-bit checksum over whole 8-byte words plus the tail bytes (the payload
// length is a multiple of 8): xor with the word, multiply by an odd
// constant, rotate.
uint64_t checksum(const unsigned char* p, size_t bytes) {
  uint64_t h = 0x9E3779B97F4A7C15ull ^ bytes;
  const size_t words = bytes / 8;
  for (size_t i = 0; i < words; ++i) {
    uint64_t w;
    std::memcpy(&w, p + 8 * i, 8);
    h = (h ^ w) * 0xFF51AFD7ED558CCDull;
    h = (h << 29) | (h >> 35);
  }
  for (size_t i = words * 8; i < bytes; ++i) h = (h ^ p[i]) * 0xC4CEB9FE1A85EC53ull;
  return h;
}

}  // namespace

extern "C" {

ek_status ek_state_bytes(ek_ctx* ctx, size_t* bytes) {
  if (!ctx) return EK_EINVAL;
  if (!bytes) return ctx->fail(EK_EINVAL, "bytes is NULL");
  *bytes = sizeof(StateHeader) + sections(ctx->p, ctx->n_beads).total;
  return EK_OK;
}

ek_status ek_save_state(ek_ctx* ctx, void* host, size_t bytes) {
  if (!ctx) return EK_EINVAL;
  if (!host) return ctx->fail(EK_EINVAL, "host buffer is NULL");
  if (!ctx->have_geometry || !ctx->have_species[0] || !ctx->have_species[1] || !ctx->have_species[2])
    return ctx->fail(EK_ESTATE, "geometry and all three species densities must be set");
  const Sections s = sections(ctx->p, ctx->n_beads);
  const size_t need = sizeof(StateHeader) + s.total;
  if (bytes < need) return ctx->fail(EK_EINVAL, "state buffer too small (ek_state_bytes)");
  const Dims d = ctx->dims;
  const size_t tsz = ctx->p.precision == EK_FP64 ? 8 : 4;
  unsigned char* pay = (unsigned char*)host + sizeof(StateHeader);
  std::memset(pay, 0, s.total);   // padding bytes enter the checksum
  std::memcpy(pay + s.solid, ctx->host_solid.data(), d.n);
  auto d2h = [&](size_t off, const void* src, size_t nb) {
    return nb == 0 || hipMemcpyAsync(pay + off, src, nb, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
  };
  const BeadState bs = bead_state_view(ctx->bead_mem, ctx->max_beads);
  const size_t nb = (size_t)ctx->n_beads;
  std::memcpy(pay + s.wall_q, ctx->host_wall_q.data(), d.n * 8);
  ctx->settle_psi();
  bool ok = d2h(s.f, ctx->fcur(), 3 * Q * d.n * tsz) && d2h(s.psi, ctx->psi, d.n * 8);
  if (ok && ctx->psi_old) ok = d2h(s.psi_old, ctx->psi_old, d.n * 8);
  if (ok && ctx->psi_old2) ok = d2h(s.psi_old2, ctx->psi_old2, d.n * 8);
  if (ok && ctx->psi_old3) ok = d2h(s.psi_old3, ctx->psi_old3, d.n * 8);
  if (ok && nb) ok = d2h(s.R, bs.R, nb * 24) && d2h(s.V, bs.V, nb * 24) && d2h(s.cross, bs.cross, nb * 12);
  if (!ok) return ctx->fail(EK_EHIP, "copying the state to the host failed");
  ek_status st = ctx->sync();
  if (st) return st;
  if (nb) std::memcpy(pay + s.q, ctx->host_q.data(), nb * 8);

  StateHeader h{};
  std::memcpy(h.magic, STATE_MAGIC, 8);
  h.version = STATE_VERSION;
  h.header_bytes = sizeof(StateHeader);
  h.nx = ctx->p.nx;
  h.ny = ctx->p.ny;
  h.nz = ctx->p.nz;
  h.precision = ctx->p.precision;
  h.warm_start = ctx->p.warm_start;
  h.n_beads = ctx->n_beads;
  h.step_count = ctx->step_count;
  h.last_iters = ctx->last_iters;
  h.solo_iters = ctx->solo_iters;
  h.psi_hist = ctx->psi_hist;
  h.last_res = ctx->last_res;
  h.last_res0 = ctx->last_res0;
  for (int k = 0; k < 3; ++k) {
    h.nref[k] = ctx->nref[k];
    h.mass[k] = ctx->mass[k];
    h.mom[k] = ctx->mom[k];
  }
  h.cross_on = ctx->cross_on ? 1 : 0;
  h.cross_plane = ctx->cross_plane;
  h.poly = ctx->poly;
  h.payload_bytes = s.total;
  h.checksum = checksum(pay, s.total);
  std::memcpy(host, &h, sizeof h);
  return EK_OK;
}

ek_status ek_load_state(ek_ctx* ctx, const void* host, size_t bytes) {
  if (!ctx) return EK_EINVAL;
  if (!host) return ctx->fail(EK_EINVAL, "host buffer is NULL");
  if (bytes < sizeof(StateHeader)) return ctx->fail(EK_EINVAL, "state buffer too small");
  StateHeader h;
  std::memcpy(&h, host, sizeof h);
  if (std::memcmp(h.magic, STATE_MAGIC, 8) != 0 || h.version != STATE_VERSION ||
      h.header_bytes != sizeof(StateHeader))
    return ctx->fail(EK_EINVAL, "not a state buffer of this library version");
  if (h.nx != ctx->p.nx || h.ny != ctx->p.ny || h.nz != ctx->p.nz || h.precision != ctx->p.precision ||
      h.warm_start != ctx->p.warm_start)
    return ctx->fail(EK_EINVAL, "state of another lattice size, precision or warm start");
  if (h.n_beads < 0 || h.n_beads > ctx->max_beads)
    return ctx->fail(EK_EINVAL, "the state's chain exceeds max_beads of the context");
  const Sections s = sections(ctx->p, h.n_beads);
  if (h.payload_bytes != s.total || bytes < sizeof(StateHeader) + s.total)
    return ctx->fail(EK_EINVAL, "state buffer truncated");
  const unsigned char* pay = (const unsigned char*)host + sizeof(StateHeader);
  if (checksum(pay, s.total) != h.checksum) return ctx->fail(EK_EINVAL, "state checksum mismatch");
  const int held = extrap_history(ctx->p.warm_start);
  if (h.psi_hist < 0 || h.psi_hist > (held ? held + 1 : 0) || h.last_iters < 0 || h.solo_iters < 0 || h.step_count < 0)
    return ctx->fail(EK_EINVAL, "state counters out of range");

  // geometry (link words, wall charges; clears populations and counters)
  ek_status st = ek_set_geometry(ctx, pay + s.solid, (const double*)(pay + s.wall_q));
  if (st) return st;
  const Dims d = ctx->dims;
  const size_t tsz = ctx->p.precision == EK_FP64 ? 8 : 4;
  auto h2d = [&](void* dst, size_t off, size_t nb) {
    return nb == 0 || hipMemcpyAsync(dst, pay + off, nb, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
  };
  bool ok = h2d(ctx->fA, s.f, 3 * Q * d.n * tsz) && h2d(ctx->psi, s.psi, d.n * 8);
  if (ok && ctx->psi_old) ok = h2d(ctx->psi_old, s.psi_old, d.n * 8);
  if (ok && ctx->psi_old2) ok = h2d(ctx->psi_old2, s.psi_old2, d.n * 8);
  if (ok && ctx->psi_old3) ok = h2d(ctx->psi_old3, s.psi_old3, d.n * 8);
  if (!ok) return ctx->fail(EK_EHIP, "copying the state to the device failed");
  ctx->cur_is_a = true;
  for (int k = 0; k < 3; ++k) {
    ctx->have_species[k] = true;
    ctx->nref[k] = h.nref[k];
    ctx->mass[k] = h.mass[k];
    ctx->mom[k] = h.mom[k];
  }
  st = ctx->sync();
  if (st) return st;
  // the chain (clears the node table, error flags and crossing record)
  const int nb = h.n_beads;
  st = ek_set_polymer(ctx, nb, nb ? (const double*)(pay + s.R) : nullptr,
                      nb ? (const double*)(pay + s.V) : nullptr,
                      nb ? (const double*)(pay + s.q) : nullptr, nb ? &h.poly : nullptr);
  if (st) return st;
  if (h.cross_on) {
    ctx->cross_on = true;
    ctx->cross_plane = h.cross_plane;
    if (nb) {
      const BeadState bs = bead_state_view(ctx->bead_mem, ctx->max_beads);
      if (!h2d(bs.cross, s.cross, (size_t)nb * 12)) return ctx->fail(EK_EHIP, "copying the crossing record failed");
    }
  }
  ctx->step_count = h.step_count;
  ctx->last_iters = h.last_iters;
  ctx->solo_iters = h.solo_iters;
  ctx->psi_hist = h.psi_hist;
  // the right-hand side of the last solve is not part of the state: the
  // next step forms its own (ek_get_poisson_system waits for it)
  ctx->have_solve = false;
  ctx->last_res = h.last_res;
  ctx->last_res0 = h.last_res0;
  return ctx->sync();
}

}  // extern "C"
