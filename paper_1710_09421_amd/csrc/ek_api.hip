// Host runtime behind the C ABI of ek.h: parameter checks, the device
// workspace, geometry preprocessing, the time loop of one lattice step and
// the Poisson driver.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ek_context.h"
#include "philox.h"

using namespace ek;

namespace {

thread_local std::string g_create_error;

#define EK_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      return ctx->fail(EK_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    }                                                                                \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Message of the last failing call that has no context (ek_last_error(NULL)).
void ek::set_thread_error(const std::string& msg) { g_create_error = msg; }

namespace {

ek_status check_params(const ek_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return EK_EINVAL; }
  if (p->nx < 2 || p->ny < 2 || p->nz < 2 || (p->nx & 1) || (p->ny & 1) || (p->nz & 1)) {
    why = "nx, ny, nz must be even and >= 2 (red-black colouring of the periodic box)";
    return EK_EINVAL;
  }
  if ((long long)p->nx * p->ny * p->nz >= (1LL << 31)) { why = "lattice too large"; return EK_EINVAL; }
  if (p->precision != EK_FP32 && p->precision != EK_FP64) { why = "precision must be EK_FP32 or EK_FP64"; return EK_EINVAL; }
  for (int s = 0; s < 3; ++s) {
    if (!(p->tau[s] > 0.5)) { why = "tau must exceed 1/2"; return EK_EINVAL; }
    if (!(p->omega_drag[s] >= 0.0)) { why = "omega_drag must be >= 0"; return EK_EINVAL; }
  }
  if (!(p->kT > 0.0) || !(p->bjerrum > 0.0)) { why = "kT and bjerrum must be positive"; return EK_EINVAL; }
  if (p->poisson_method != EK_POISSON_SOR && p->poisson_method != EK_POISSON_MG) {
    why = "unknown poisson_method"; return EK_EINVAL;
  }
  if (!(p->poisson_tol > 0.0) || p->poisson_max_iter < 1 || p->poisson_check_every < 1) {
    why = "poisson_tol > 0, poisson_max_iter >= 1 and poisson_check_every >= 1 required";
    return EK_EINVAL;
  }
  if (p->rho_jacobi < 0.0 || p->rho_jacobi >= 1.0) { why = "rho_jacobi must be in [0, 1)"; return EK_EINVAL; }
  if (p->warm_start < EK_WS_ZERO || p->warm_start > EK_WS_EXTRAP3) { why = "unknown warm_start"; return EK_EINVAL; }
  if (p->warm_start == EK_WS_LEARNED && !UNet::shape_ok(p->nx, p->ny, p->nz)) {
    why = "the learned warm start needs nx, ny, nz divisible by 4 (two 2x2x2 poolings)";
    return EK_EINVAL;
  }
  if (p->fluctuations != 0 && p->fluctuations != 1) { why = "fluctuations must be 0 or 1"; return EK_EINVAL; }
  if (p->walls != EK_WALLS_PERIODIC && p->walls != EK_WALLS_INSULATING) { why = "unknown walls"; return EK_EINVAL; }
  if (p->walls == EK_WALLS_INSULATING &&
      (p->poisson_method != EK_POISSON_SOR || p->warm_start == EK_WS_LEARNED)) {
    why = "insulating walls need EK_POISSON_SOR and a start other than EK_WS_LEARNED";
    return EK_EINVAL;
  }
  return EK_OK;
}

// Workspace layout (every block 256-byte aligned).
struct Layout {
  size_t fA, fB, mask, wall_q, psi, b, partials, ps, stats, keys, vals, beads, mg, mgt, net, guess,
      psi_old, psi_old2, psi_old3, total;
};

Layout make_layout(const ek_params* p, int max_beads) {
  const size_t n = (size_t)p->nx * p->ny * p->nz;
  const size_t tsz = p->precision == EK_FP64 ? 8 : 4;
  const SiteGrid g = site_grid(p->nx, p->ny, p->nz);
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.fA = take(3 * Q * n * tsz);
  L.fB = take(3 * Q * n * tsz);
  L.mask = take(n * 4);
  L.wall_q = take(n * 8);
  L.psi = take(n * 8);
  L.b = take(n * 8);
  // block partials of up to 8 components: site-grid or lattice-grid blocks,
  // plus the blocks of the bead-box tail
  const int nbp = std::max(g.nblocks(), lattice_grid(p->nx, p->ny, p->nz).nblocks()) +
                  lb_tail_blocks(std::max(max_beads, 1));
  L.partials = take((size_t)nbp * 8 * 8);
  L.ps = take(sizeof(PoissonScalars));
  L.stats = take(16 * 8);
  L.keys = take((size_t)HASH_SLOTS * 4);
  L.vals = take((size_t)HASH_SLOTS * 10 * 8);
  L.beads = take(bead_state_bytes(max_beads));
  L.mg = take(mg_workspace_bytes(p->nx, p->ny, p->nz));
  L.mgt = take(p->poisson_method == EK_POISSON_MG ? mg_sweep_bytes(p->nx, p->ny, p->nz) : 0);
  const bool learned = p->warm_start == EK_WS_LEARNED;
  L.net = take(learned ? UNet::bytes(p->nx, p->ny, p->nz, false) : 0);
  L.guess = take(learned ? n * 8 : 0);
  const int held = extrap_history(p->warm_start);
  L.psi_old = take(held >= 1 ? n * 8 : 0);
  L.psi_old2 = take(held >= 2 ? n * 8 : 0);
  L.psi_old3 = take(held >= 3 ? n * 8 : 0);
  L.total = off;
  return L;
}

}  // namespace

// ---------------------------------------------------------------------------
ek_status ek_ctx::fail(ek_status st, const std::string& msg) {
  err = msg;
  return st;
}

ek_status ek_ctx::sync() {
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(EK_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return EK_OK;
}

void* ek_ctx::fcur() { return cur_is_a ? fA : fB; }
void* ek_ctx::fnext() { return cur_is_a ? fB : fA; }

LBParams ek_ctx::lb_params() const {
  LBParams lp{};
  for (int s = 0; s < 3; ++s) {
    lp.omega[s] = 1.0 / p.tau[s];
    lp.valence[s] = p.valence[s];
    lp.wdrag[s] = p.omega_drag[s];
    lp.nref[s] = nref[s];
    for (int c = 0; c < 3; ++c) lp.fext[s][c] = p.F_ext[s][c];
    lp.eext[s] = p.E_ext[s];
  }
  return lp;
}

double ek_ctx::inv_eps() const { return 4.0 * M_PI * p.bjerrum * p.kT; }

// Stochastic term of the step that starts after `step` completed steps:
// key from the seed, amplitude m omega (2 - omega) per species with the
// thermal mass m = k_B T / v_T^2 (v_T^2 = 1/3 on D3Q19), and the norms of
// the mode polynomials under the lattice weights.
NoiseParams ek_ctx::noise_params(long long step) const {
  NoiseParams np{};
  np.key0 = uint32_t(p.seed & 0xFFFFFFFFull);
  np.key1 = uint32_t(p.seed >> 32);
  np.step = uint32_t(step);
  const double m = p.kT * 3.0;
  for (int s = 0; s < 3; ++s) {
    const double om = 1.0 / p.tau[s];
    np.amp2[s] = m * om * (2.0 - om);
  }
  for (int k = 4; k < Q; ++k) {
    double n2 = 0.0;
    for (int q = 0; q < Q; ++q) n2 += weight(q) * double(mode_poly(k, q)) * double(mode_poly(k, q));
    np.inv_norm[k - 4] = 1.0 / std::sqrt(n2);
  }
  return np;
}

double ek_ctx::jacobi_radius() const {
  if (p.rho_jacobi > 0.0) return p.rho_jacobi;
  const int m = std::max(p.nx, std::max(p.ny, p.nz));
  return (2.0 + std::cos(2.0 * M_PI / m)) / 3.0;
}

ek_status ek_ctx::read_scalars(PoissonScalars* out) {
  ek_ctx* ctx = this;
  EK_HIP(hipMemcpyAsync(pinned, ps, sizeof(PoissonScalars), hipMemcpyDeviceToHost, stream));
  ek_status st = sync();
  if (st) return st;
  std::memcpy(out, pinned, sizeof(PoissonScalars));
  return EK_OK;
}

// Red-black SOR with the Chebyshev schedule on A psi = b + shift (the shift
// is already in ps).  The residual is tested after every `check_every`
// iterations; iterations are enqueued in batches ahead of the test and turn
// into no-ops once the device-side flag is set.
int ek_ctx::residual_launch(const double* bb, const double* x) {
  const SiteGrid g = site_grid(p.nx, p.ny, p.nz, bx_sites);
  if (insulating()) return launch_residual_neu(x, bb, mask, ps, partials, dims, g, stream);
  return launch_residual(x, bb, ps, partials, dims, g, stream);
}

ek_status ek_ctx::sor_solve(const double* bb, double* x, PoissonScalars h, int& iters, double& res,
                           double& res0) {
  const SiteGrid cg = colour_grid(p.nx, p.ny, p.nz, bx_colour);
  const bool neu = insulating();
  const double rj = jacobi_radius();
  ek_status st = EK_OK;
  int it = 0;
  double omega = 1.0;
  bool first = true;
  const int ce = p.poisson_check_every;
  int batch = std::max(ce, ((last_iters + ce - 1) / ce) * ce);
  while (!h.done && it < p.poisson_max_iter) {
    const int nrun = std::min(batch, p.poisson_max_iter - it);
    for (int k = 0; k < nrun; ++k) {
      for (int colour = 0; colour < 2; ++colour) {
        if (neu) launch_sor_half_neu(x, bb, mask, ps, colour, omega, dims, cg, stream);
        else launch_sor_half(x, bb, ps, colour, omega, dims, cg, stream);
        omega = first ? 1.0 / (1.0 - 0.5 * rj * rj) : 1.0 / (1.0 - 0.25 * rj * rj * omega);
        first = false;
      }
      ++it;
      if (it % ce == 0 || it == p.poisson_max_iter) {
        const int nr = residual_launch(bb, x);
        launch_residual_final(partials, nr, p.poisson_tol, it, 0, ps, stream);
      }
    }
    st = read_scalars(&h);
    if (st) return st;
    batch = ce;
  }
  res0 = h.rel0;
  res = h.rel;
  if (!h.done) {
    iters = it;
    char buf[160];
    std::snprintf(buf, sizeof buf, "Poisson solve did not reach %.3g in %d iterations (residual %.3e)",
                  p.poisson_tol, p.poisson_max_iter, h.rel);
    return fail(EK_ENOCONV, buf);
  }
  iters = h.iters;
  if (neu) launch_psi_shift_neu(x, mask, ps, 1.0 / double(n_fluid), dims, stream);
  else if (defer_shift) shift_pending = true;
  else launch_psi_shift(x, ps, 1.0 / double(dims.n), dims, stream);
  return EK_OK;
}

void ek_ctx::settle_psi() {
  if (!shift_pending) return;
  launch_psi_shift(psi, ps, 1.0 / double(dims.n), dims, stream);
  shift_pending = false;
}

ek_status ek_ctx::initial_residual(const double* bb, const double* x, PoissonScalars* h) {
  const int nr = residual_launch(bb, x);
  launch_residual_final(partials, nr, p.poisson_tol, 0, 1, ps, stream);
  return read_scalars(h);
}

// Learned warm start with fallback.  The residual of the current start x
// (previous step, or what the caller passed) is evaluated first; only when it
// exceeds LEARNED_GATE is the network consulted, its guess's residual
// evaluated, and the smaller of the two starts kept in x with its residual
// state in ps.  A non-finite guess residual always falls back.
ek_status ek_ctx::learned_start(const double* bb, double* x, PoissonScalars* h) {
  ek_ctx* ctx = this;
  const SiteGrid g = site_grid(p.nx, p.ny, p.nz, bx_sites);
  last_fallback = 0;
  last_consulted = 0;
  ek_status st = initial_residual(bb, x, h);
  if (st || h->done || !(h->rel > LEARNED_GATE)) return st;
  last_consulted = 1;
  const PoissonScalars hp = *h;
  launch_ps_rearm(ps, stream);
  net->forward(bb, mask, true, guess);
  const int nr = launch_residual(guess, bb, ps, partials, dims, g, stream);
  launch_residual_final(partials, nr, p.poisson_tol, 0, 1, ps, stream);
  PoissonScalars hl{};
  st = read_scalars(&hl);
  if (st) return st;
  if (hl.rel < hp.rel) {
    EK_HIP(hipMemcpyAsync(x, guess, dims.n * 8, hipMemcpyDeviceToDevice, stream));
    *h = hl;
    return EK_OK;
  }
  last_fallback = 1;
  launch_ps_rearm(ps, stream);
  return initial_residual(bb, x, h);
}

ek_status ek_ctx::poisson(const double* bb, double* x, bool learned, int& iters, double& res,
                          double& res0) {
  PoissonScalars h{};
  last_fallback = 0;
  last_consulted = 0;
  if (!learned && p.poisson_method == EK_POISSON_MG) {
    // the start's residual stays on the device (the cycles test its flag and
    // skip themselves once converged); the host reads it with the first
    // batch's result.  Where the finest level's first sweep can take it, the
    // first cycle does (no pass of its own)
    if (mg_start_in_cycle()) return mg_solve(bb, x, h, iters, res, res0, true);
    const SiteGrid g = site_grid(p.nx, p.ny, p.nz, bx_sites);
    const int nr = launch_residual(x, bb, ps, partials, dims, g, stream);
    launch_residual_final(partials, nr, p.poisson_tol, 0, 1, ps, stream);
    return mg_solve(bb, x, h, iters, res, res0);
  }
  ek_status st = learned ? learned_start(bb, x, &h) : initial_residual(bb, x, &h);
  if (st) return st;
  if (p.poisson_method == EK_POISSON_MG) return mg_solve(bb, x, h, iters, res, res0);
  return sor_solve(bb, x, h, iters, res, res0);
}

ek_status ek_ctx::ensure_events(int n_steps) {
  ek_ctx* ctx = this;
  while ((int)events.size() < 6 * n_steps) {
    hipEvent_t e;
    EK_HIP(hipEventCreate(&e));
    events.push_back(e);
  }
  return EK_OK;
}

void ek_ctx::record(int t, int k) {
  if (timing) (void)hipEventRecord(events[6 * t + k], stream);
}

template <typename T>
ek_status ek_ctx::step_impl(int n_steps) {
  ek_ctx* ctx = this;
  const SiteGrid g = bx_sites ? site_grid(p.nx, p.ny, p.nz, bx_sites) : lattice_grid(p.nx, p.ny, p.nz);
  const int nb = g.nblocks();
  const LBParams lp = lb_params();
  // lattice update beside the chain (box sites after it): see EK_LAUNCH_OVERLAP
  const bool overlap = overlap_md && n_beads > 0 && p.nx >= 4 && p.ny >= 4 && p.nz >= 4;
  const int nb_bulk = lb_step_blocks(g, p.nz);
  const int nb_lb = nb_bulk + (overlap ? lb_tail_blocks(n_beads) : 0);

  if (timing) {
    ek_status st = ensure_events(n_steps);
    if (st) return st;
  }
  WallView wv;
  wv.face_q = wall_q;
  wv.inv_eps = inv_eps();
  const WallView* wvp = insulating() ? &wv : nullptr;
  for (int t = 0; t < n_steps; ++t) {
    const BeadTableView bt = bead_view();
    const NoiseParams noise = noise_params(step_count);
    const NoiseParams* npp = p.fluctuations ? &noise : nullptr;
    record(t, 0);
    // charge density of ions, walls and beads at time t
    if (n_beads > 0) {
      ek_status st = beads_deposit();
      if (st) return st;
    }
    // the charge pass also prepares the extrapolated start: with psi_hist
    // previous solutions held (psi, then the history buffers) it extrapolates
    // with the highest order they allow, up to the order of the warm start,
    // and shifts the history by one (the mode numbers of StartExtrap)
    const int held = extrap_history(p.warm_start);
    int extrap = 0;
    if (held > 0) {
      const int order = std::min(psi_hist - 1, held);  // -1: no solution yet
      static const int keep[3] = {1, 3, 5};            // order < held: history deepens
      static const int top[4] = {0, 2, 4, 6};          // order == held
      if (order >= 0) extrap = order == held ? top[order] : keep[order];
    }
    // (a mean left in psi by the previous solve is removed by the same pass)
    if (extrap == 0) settle_psi();
    launch_charge<T>((const T*)fcur(), mask, wall_q, b, partials, lp, inv_eps(), dims, g, stream, bt,
                     psi, psi_old, extrap, insulating(), psi_old2, psi_old3,
                     shift_pending ? ps : nullptr);
    rotate_history(extrap, psi_old, psi_old2, psi_old3);
    shift_pending = false;
    if (held > 0) psi_hist = std::min(psi_hist + 1, held + 1);
    launch_mean_shift(partials, nb, 1.0 / double(insulating() ? n_fluid : dims.n), inv_eps(), ps,
                      stream, partials + nb, partials_cap - nb);
    record(t, 1);
    if (p.warm_start == EK_WS_ZERO) launch_fill(psi, 0.0, dims.n, stream);
    int iters = 0;
    double res = 0, res0 = 0;
    defer_shift = held > 0 && !insulating();
    ek_status st = poisson(b, psi, p.warm_start == EK_WS_LEARNED, iters, res, res0);
    defer_shift = false;
    if (st) return st;
    last_iters = iters;
    last_res = res;
    last_res0 = res0;
    have_solve = true;
    if (timing) tacc.poisson_iters += iters;
    record(t, 2);
    // beads: n_sub MD substeps with the fields of time t, friction spread
    // (event 5: end of the chain kernel)
    if (n_beads > 0) {
      st = beads_advance<T>(overlap, timing ? events[6 * t + 5] : nullptr);
      if (st) return st;
    }
    // events 3 and 4 are stamped by the fused kernel's own start and end.
    // With the overlap it runs on the side stream from the box gather on,
    // beside the chain (the longer of the two stays on the context stream,
    // which then waits only for a lattice update that has long finished)
    hipStream_t ls = stream;
    if (overlap) {
      EK_HIP(hipStreamWaitEvent(side_stream, side_fork, 0));
      ls = side_stream;
    }
    launch_lb_step<T>((const T*)fcur(), (T*)fnext(), mask, psi, lp, bt, partials, nb_lb,
                      overlap ? MASK_DEFER : 0u, dims, g, ls,
                      timing ? events[6 * t + 3] : nullptr, timing ? events[6 * t + 4] : nullptr,
                      npp, wvp);
    if (overlap) {
      // the box sites after the chain, beside the rest of the lattice update
      // (disjoint sites and partials); their flags are cleared once both end
      launch_lb_tail<T>((const T*)fcur(), (T*)fnext(), mask, psi, lp, bt, bead_origin(), n_beads,
                        partials, nb_bulk, nb_lb, dims, stream, npp, wvp);
      EK_HIP(hipEventRecord(side_join, side_stream));
      EK_HIP(hipStreamWaitEvent(stream, side_join, 0));
      launch_defer_clear(mask, bead_origin(), n_beads, dims, stream);
    }
    launch_sum_partials(partials, nb_lb, stats_dev, timing ? 1 : 0, stream,
                        partials + 7LL * nb_lb, partials_cap - 7LL * nb_lb);
    cur_is_a = !cur_is_a;
    ++step_count;
  }
  ek_status st = sync();
  if (st) return st;
  if (timing) {
    for (int t = 0; t < n_steps; ++t) {
      float ms[4];
      for (int k = 0; k < 4; ++k)
        EK_HIP(hipEventElapsedTime(&ms[k], events[6 * t + k], events[6 * t + k + 1]));
      if (n_beads > 0)   // solve end to chain end (the lattice kernel may start earlier)
        EK_HIP(hipEventElapsedTime(&ms[2], events[6 * t + 2], events[6 * t + 5]));
      tacc.ms_charge += ms[0];
      tacc.ms_poisson += ms[1];
      tacc.ms_md += ms[2];
      tacc.ms_lb += ms[3];
      tacc.n_lb += 1;
      tacc.n_steps += 1;
    }
  }
  double h[6];
  EK_HIP(hipMemcpy(h, stats_dev, sizeof h, hipMemcpyDeviceToHost));
  for (int s = 0; s < 3; ++s) {
    mass[s] = h[s];
    mom[s] = h[3 + s];
    if (!std::isfinite(h[s]) || h[s] < 0.0) return fail(EK_EUNSTABLE, "species mass is not finite or negative");
  }
  if (n_beads > 0) {
    st = beads_check();
    if (st) return st;
  }
  return EK_OK;
}

// Link word of every site (bounce-back bits, solid, wall and charge flags)
// from the host solid mask; returns the number of fluid sites.
long long ek::build_link_words(const uint8_t* solid, const double* wall_q, const Dims& d,
                               std::vector<uint32_t>& m) {
  m.assign(d.n, 0u);
  long long nfluid = 0;
  for (int z = 0; z < d.nz; ++z)
    for (int y = 0; y < d.ny; ++y)
      for (int x = 0; x < d.nx; ++x) {
        const long long r = ((long long)z * d.ny + y) * d.nx + x;
        uint32_t w = 0;
        if (solid[r]) {
          w |= MASK_SOLID;
          for (int q = 1; q < Q; ++q) {
            const int sx = (x + CX[q] + d.nx) % d.nx, sy = (y + CY[q] + d.ny) % d.ny,
                      sz = (z + CZ[q] + d.nz) % d.nz;
            if (!solid[((long long)sz * d.ny + sy) * d.nx + sx]) w |= MASK_WALL;
          }
        } else {
          ++nfluid;
          for (int q = 1; q < Q; ++q) {
            const int sx = (x - CX[q] + d.nx) % d.nx, sy = (y - CY[q] + d.ny) % d.ny,
                      sz = (z - CZ[q] + d.nz) % d.nz;
            if (solid[((long long)sz * d.ny + sy) * d.nx + sx]) w |= 1u << q;
          }
        }
        if (wall_q && wall_q[r] != 0.0) w |= MASK_CHARGED;
        m[r] = w;
      }
  return nfluid;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

ek_status ek_workspace_bytes(const ek_params* p, int32_t max_beads, size_t* bytes) {
  std::string why;
  ek_status st = check_params(p, why);
  if (st) { g_create_error = why; return st; }
  if (!bytes || max_beads < 0 || max_beads > MAX_BEADS) { g_create_error = "bad bytes pointer or max_beads"; return EK_EINVAL; }
  *bytes = make_layout(p, max_beads).total;
  return EK_OK;
}

ek_status ek_create(const ek_params* p, int32_t max_beads, void* dev_ws, size_t ws_bytes,
                    void* hip_stream, ek_ctx** out) {
  std::string why;
  if (!out) { g_create_error = "out is NULL"; return EK_EINVAL; }
  *out = nullptr;
  ek_status st = check_params(p, why);
  if (st) { g_create_error = why; return st; }
  if (max_beads < 0 || max_beads > MAX_BEADS) { g_create_error = "max_beads out of range"; return EK_EINVAL; }
  const Layout L = make_layout(p, max_beads);
  char* ws = (char*)dev_ws;
  bool own = false;
  if (ws) {
    if (ws_bytes < L.total) { g_create_error = "workspace too small"; return EK_ENOMEM; }
    if (((uintptr_t)ws & 255) != 0) { g_create_error = "workspace must be 256-byte aligned"; return EK_EINVAL; }
  } else {
    if (hipMalloc((void**)&ws, L.total) != hipSuccess) { g_create_error = "hipMalloc of the workspace failed"; return EK_ENOMEM; }
    own = true;
  }
  ek_ctx* c = new ek_ctx();
  c->p = *p;
  c->dims = Dims{p->nx, p->ny, p->nz, (long long)p->nx * p->ny * p->nz};
  c->stream = (hipStream_t)hip_stream;
  c->ws = ws;
  c->own_ws = own;
  c->max_beads = max_beads;
  c->fA = ws + L.fA;
  c->fB = ws + L.fB;
  c->mask = (uint32_t*)(ws + L.mask);
  c->wall_q = (double*)(ws + L.wall_q);
  c->psi = (double*)(ws + L.psi);
  c->b = (double*)(ws + L.b);
  c->partials = (double*)(ws + L.partials);
  c->partials_cap = (long long)((L.ps - L.partials) / 8);
  c->ps = (PoissonScalars*)(ws + L.ps);
  c->stats_dev = (double*)(ws + L.stats);
  c->keys = (int*)(ws + L.keys);
  c->vals = (long long*)(ws + L.vals);
  c->bead_mem = ws + L.beads;
  c->mg_mem = ws + L.mg;
  c->mg_tmp = p->poisson_method == EK_POISSON_MG ? ws + L.mgt : nullptr;
  if (hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    if (own) (void)hipFree(ws);
    delete c;
    g_create_error = "hipHostMalloc failed";
    return EK_EHIP;
  }
  c->bx_sites = 0;
  c->bx_colour = 0;
  // the workspace arrives uninitialised: empty the bead node table and zero
  // the link words before any kernel reads them
  launch_table_init(c->keys, c->vals, c->stream);
  if (hipMemsetAsync(c->mask, 0, c->dims.n * 4, c->stream) != hipSuccess ||
      hipMemsetAsync(c->stats_dev, 0, 16 * 8, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipHostFree(c->pinned);
    if (own) (void)hipFree(ws);
    delete c;
    g_create_error = "initialising the workspace failed";
    return EK_EHIP;
  }
  c->mg_setup();
  if (p->warm_start == EK_WS_LEARNED) {
    c->net = new UNet();
    c->net->stream = c->stream;
    c->net->carve(ws + L.net, p->nx, p->ny, p->nz, false);
    c->guess = (double*)(ws + L.guess);
    if (c->net->init_state() != hipSuccess) {
      ek_destroy(c);
      g_create_error = "initialising the network state failed";
      return EK_EHIP;
    }
  }
  const int held = extrap_history(p->warm_start);
  if (held >= 1) c->psi_old = (double*)(ws + L.psi_old);
  if (held >= 2) c->psi_old2 = (double*)(ws + L.psi_old2);
  if (held >= 3) c->psi_old3 = (double*)(ws + L.psi_old3);
  *out = c;
  return EK_OK;
}

void ek_destroy(ek_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->side_stream) {
    (void)hipStreamSynchronize(ctx->side_stream);
    (void)hipStreamDestroy(ctx->side_stream);
  }
  if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
  if (ctx->side_join) (void)hipEventDestroy(ctx->side_join);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  ctx->mg_release();
  delete ctx->net;
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->own_ws) (void)hipFree(ctx->ws);
  delete ctx;
}

const char* ek_last_error(const ek_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

ek_status ek_set_geometry(ek_ctx* ctx, const uint8_t* solid, const double* wall_q) {
  if (!ctx) return EK_EINVAL;
  if (!solid) return ctx->fail(EK_EINVAL, "solid is NULL");
  const Dims d = ctx->dims;
  std::vector<uint32_t> m;
  const long long nfluid = build_link_words(solid, wall_q, d, m);
  if (nfluid == 0) return ctx->fail(EK_EINVAL, "geometry has no fluid site");
  std::vector<double> face_q;
  if (ctx->insulating()) {
    // insulating walls: the charge of a solid site is shared by its faces
    // with the fluid (Sigma_f = q / faces); every fluid site needs a fluid
    // face neighbour (else its potential is undefined)
    face_q.assign(d.n, 0.0);
    for (long long r = 0; r < d.n; ++r) {
      int faces = 0;
      for (int q = 1; q <= 6; ++q) faces += (m[r] >> q) & 1u;    // solid face neighbours
      const bool is_solid = (m[r] & MASK_SOLID) != 0;
      if (!is_solid && faces == 6) return ctx->fail(EK_EINVAL, "a fluid site has no fluid face neighbour");
      if (!is_solid || !wall_q || wall_q[r] == 0.0) continue;
      const int z = int(r / ((long long)d.nx * d.ny)), y = int((r / d.nx) % d.ny), x = int(r % d.nx);
      int open = 0;
      for (int q = 1; q <= 6; ++q) {
        const int sx = (x + CX[q] + d.nx) % d.nx, sy = (y + CY[q] + d.ny) % d.ny,
                  sz = (z + CZ[q] + d.nz) % d.nz;
        open += solid[((long long)sz * d.ny + sy) * d.nx + sx] ? 0 : 1;
      }
      if (open == 0)
        return ctx->fail(EK_EINVAL, "insulating walls: a charged solid site has no face shared with the fluid");
      face_q[r] = wall_q[r] / open;
    }
  }
  EK_HIP(hipMemcpy(ctx->mask, m.data(), d.n * 4, hipMemcpyHostToDevice));
  if (ctx->insulating()) {
    EK_HIP(hipMemcpy(ctx->wall_q, face_q.data(), d.n * 8, hipMemcpyHostToDevice));
  } else if (wall_q) {
    EK_HIP(hipMemcpy(ctx->wall_q, wall_q, d.n * 8, hipMemcpyHostToDevice));
  } else {
    launch_fill(ctx->wall_q, 0.0, d.n, ctx->stream);
  }
  ctx->host_solid.assign(solid, solid + d.n);
  if (wall_q) ctx->host_wall_q.assign(wall_q, wall_q + d.n);
  else ctx->host_wall_q.assign(d.n, 0.0);
  ctx->n_fluid = nfluid;
  const size_t tsz = ctx->p.precision == EK_FP64 ? 8 : 4;
  EK_HIP(hipMemsetAsync(ctx->fA, 0, 3 * Q * d.n * tsz, ctx->stream));
  EK_HIP(hipMemsetAsync(ctx->fB, 0, 3 * Q * d.n * tsz, ctx->stream));
  launch_fill(ctx->psi, 0.0, d.n, ctx->stream);
  ctx->shift_pending = false;
  ctx->cur_is_a = true;
  ctx->have_geometry = true;
  for (int s = 0; s < 3; ++s) ctx->have_species[s] = false;
  ctx->step_count = 0;
  ctx->last_iters = 0;
  ctx->psi_hist = 0;
  ctx->cross_on = false;   // the step count restarts: a crossing record would not match it
  return ctx->sync();
}

ek_status ek_set_species_density(ek_ctx* ctx, int32_t species, const double* n) {
  if (!ctx) return EK_EINVAL;
  if (!ctx->have_geometry) return ctx->fail(EK_ESTATE, "set the geometry first");
  if (species < 0 || species > 2 || !n) return ctx->fail(EK_EINVAL, "bad species or NULL density");
  const Dims d = ctx->dims;
  double sum = 0.0;
  for (long long r = 0; r < d.n; ++r) {
    if (ctx->host_solid[r]) continue;
    if (!std::isfinite(n[r]) || n[r] < 0.0) return ctx->fail(EK_EINVAL, "densities must be finite and >= 0");
    sum += n[r];
  }
  const double nref = sum / double(ctx->n_fluid);
  // stage the density in the free population buffer
  double* stage = (double*)ctx->fnext();
  EK_HIP(hipMemcpyAsync(stage, n, d.n * 8, hipMemcpyHostToDevice, ctx->stream));
  if (ctx->p.precision == EK_FP64)
    launch_init_species<double>((double*)ctx->fcur(), ctx->mask, stage, species, nref, d, ctx->stream);
  else
    launch_init_species<float>((float*)ctx->fcur(), ctx->mask, stage, species, nref, d, ctx->stream);
  ctx->nref[species] = nref;
  ctx->have_species[species] = true;
  return ctx->sync();
}

ek_status ek_step(ek_ctx* ctx, int32_t n_steps) {
  if (!ctx) return EK_EINVAL;
  if (n_steps < 0) return ctx->fail(EK_EINVAL, "n_steps < 0");
  if (!ctx->have_geometry || !ctx->have_species[0] || !ctx->have_species[1] || !ctx->have_species[2])
    return ctx->fail(EK_ESTATE, "geometry and all three species densities must be set");
  if (ctx->p.warm_start == EK_WS_LEARNED && !ctx->net->have_params)
    return ctx->fail(EK_ESTATE, "learned warm start without a model (ek_set_model)");
  if (ctx->p.precision == EK_FP64) return ctx->step_impl<double>(n_steps);
  return ctx->step_impl<float>(n_steps);
}

ek_status ek_set_model(ek_ctx* ctx, const float* params, int32_t n, float out_scale) {
  if (!ctx) return EK_EINVAL;
  if (!ctx->net) return ctx->fail(EK_ESTATE, "context was not created with warm_start = EK_WS_LEARNED");
  if (!params || n != UNET_PARAMS) return ctx->fail(EK_EINVAL, "expected EK_UNET_PARAMS parameters");
  if (!(out_scale > 0.0f) || !std::isfinite(out_scale)) return ctx->fail(EK_EINVAL, "out_scale must be positive");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return ctx->fail(EK_EINVAL, "non-finite parameter");
  EK_HIP(hipMemcpyAsync(ctx->net->params, params, size_t(n) * 4, hipMemcpyHostToDevice, ctx->stream));
  ctx->net->out_scale = out_scale;
  ctx->net->pack();
  ctx->net->have_params = true;
  return ctx->sync();
}

ek_status ek_get_poisson_system(ek_ctx* ctx, double* dev_rhs, double* dev_psi) {
  if (!ctx) return EK_EINVAL;
  if (ctx->insulating()) return ctx->fail(EK_ESTATE, "the context has insulating walls");
  if (!ctx->have_solve) return ctx->fail(EK_ESTATE, "no Poisson solve has run yet");
  ctx->settle_psi();
  if (dev_rhs) launch_rhs_copy(ctx->b, ctx->ps, dev_rhs, ctx->dims.n, ctx->stream);
  if (dev_psi)
    EK_HIP(hipMemcpyAsync(dev_psi, ctx->psi, ctx->dims.n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return ctx->sync();
}

ek_status ek_get_moments(ek_ctx* ctx, int32_t species, double* n, double* u) {
  if (!ctx) return EK_EINVAL;
  if (species < 0 || species > 2) return ctx->fail(EK_EINVAL, "bad species");
  if (!ctx->have_geometry) return ctx->fail(EK_ESTATE, "no geometry");
  const Dims d = ctx->dims;
  double* scratch = (double*)ctx->fnext();   // 4 doubles per site fit in the free buffer
  if (ctx->p.precision == EK_FP64)
    launch_moments<double>((const double*)ctx->fcur(), ctx->mask, species, ctx->nref[species],
                           scratch, scratch + d.n, d, ctx->stream);
  else
    launch_moments<float>((const float*)ctx->fcur(), ctx->mask, species, ctx->nref[species],
                          scratch, scratch + d.n, d, ctx->stream);
  if (n) EK_HIP(hipMemcpyAsync(n, scratch, d.n * 8, hipMemcpyDeviceToHost, ctx->stream));
  if (u) EK_HIP(hipMemcpyAsync(u, scratch + d.n, 3 * d.n * 8, hipMemcpyDeviceToHost, ctx->stream));
  return ctx->sync();
}

ek_status ek_get_potential(ek_ctx* ctx, double* psi) {
  if (!ctx) return EK_EINVAL;
  if (!psi) return ctx->fail(EK_EINVAL, "psi is NULL");
  ctx->settle_psi();
  EK_HIP(hipMemcpyAsync(psi, ctx->psi, ctx->dims.n * 8, hipMemcpyDeviceToHost, ctx->stream));
  return ctx->sync();
}

ek_status ek_get_stats(ek_ctx* ctx, ek_stats* out) {
  if (!ctx || !out) return EK_EINVAL;
  std::memset(out, 0, sizeof *out);
  for (int s = 0; s < 3; ++s) {
    out->mass[s] = ctx->mass[s];
    out->momentum[s] = ctx->mom[s];
  }
  out->step = ctx->step_count;
  out->poisson_iters = ctx->last_iters;
  out->poisson_residual = ctx->last_res;
  out->fallback = ctx->last_fallback;
  out->consulted = ctx->last_consulted;
  out->poisson_residual0 = ctx->last_res0;
  return EK_OK;
}

ek_status ek_set_timing(ek_ctx* ctx, int32_t enable) {
  if (!ctx) return EK_EINVAL;
  ctx->timing = enable != 0;
  ctx->tacc = ek_timing{};
  // the running count of updated lattice sites (stats slot 7)
  static const double zero = 0.0;
  EK_HIP(hipMemcpyAsync(ctx->stats_dev + 7, &zero, sizeof zero, hipMemcpyHostToDevice, ctx->stream));
  return ctx->sync();
}

ek_status ek_set_launch_mode(ek_ctx* ctx, int32_t flags) {
  if (!ctx) return EK_EINVAL;
  if (flags & ~(EK_LAUNCH_GRAPHS | EK_LAUNCH_OVERLAP)) return ctx->fail(EK_EINVAL, "unknown launch flag");
  ctx->graph_launch = (flags & EK_LAUNCH_GRAPHS) != 0;
  ctx->overlap_md = (flags & EK_LAUNCH_OVERLAP) != 0;
  return EK_OK;
}

ek_status ek_get_timing(ek_ctx* ctx, ek_timing* out) {
  if (!ctx || !out) return EK_EINVAL;
  double sites = 0.0;
  EK_HIP(hipMemcpyAsync(&sites, ctx->stats_dev + 7, sizeof sites, hipMemcpyDeviceToHost, ctx->stream));
  const ek_status st = ctx->sync();
  if (st) return st;
  *out = ctx->tacc;
  out->lb_sites = (int64_t)sites;
  return EK_OK;
}

ek_status ek_poisson_solve(ek_ctx* ctx, const double* dev_rho, double* dev_psi,
                           int32_t warm_start, ek_poisson_report* rep) {
  if (!ctx) return EK_EINVAL;
  if (ctx->insulating()) return ctx->fail(EK_ESTATE, "the context has insulating walls");
  if (!dev_rho || !dev_psi) return ctx->fail(EK_EINVAL, "NULL device buffer");
  if (warm_start < EK_WS_ZERO || warm_start > EK_WS_EXTRAP3) return ctx->fail(EK_EINVAL, "unknown warm_start");
  if (warm_start == EK_WS_LEARNED && !(ctx->net && ctx->net->have_params))
    return ctx->fail(EK_ESTATE, "learned warm start without a model (ek_set_model)");
  ctx->settle_psi();   // before ps is reused
  const SiteGrid g = site_grid(ctx->p.nx, ctx->p.ny, ctx->p.nz, ctx->bx_sites);
  launch_rho_to_b(dev_rho, ctx->b, ctx->partials, ctx->inv_eps(), ctx->dims, g, ctx->stream);
  launch_mean_shift(ctx->partials, g.nblocks(), 1.0 / double(ctx->dims.n), ctx->inv_eps(), ctx->ps,
                    ctx->stream);
  if (warm_start == EK_WS_ZERO) launch_fill(dev_psi, 0.0, ctx->dims.n, ctx->stream);
  int iters = 0;
  double res = 0, res0 = 0;
  const int saved = ctx->last_iters;
  ctx->last_iters = ctx->solo_iters;
  ctx->solo = true;
  ek_status st = ctx->poisson(ctx->b, dev_psi, warm_start == EK_WS_LEARNED, iters, res, res0);
  ctx->solo = false;
  ctx->solo_iters = iters;
  if (st == EK_OK) ctx->have_solve = true;
  ctx->last_iters = saved;
  if (rep) {
    rep->iterations = iters;
    rep->residual = res;
    rep->initial_residual = res0;
  }
  if (st) return st;
  return ctx->sync();
}

ek_status ek_poisson_sor_iterations(ek_ctx* ctx, const double* dev_b, double* dev_psi,
                                    int32_t iterations) {
  if (!ctx) return EK_EINVAL;
  if (ctx->insulating()) return ctx->fail(EK_ESTATE, "the context has insulating walls");
  if (!dev_b || !dev_psi || iterations < 0) return ctx->fail(EK_EINVAL, "bad arguments");
  const SiteGrid cg = colour_grid(ctx->p.nx, ctx->p.ny, ctx->p.nz, ctx->bx_colour);
  ctx->settle_psi();   // before ps is reused
  launch_ps_reset(ctx->ps, 0.0, ctx->stream);
  const double rj = ctx->jacobi_radius();
  double omega = 1.0;
  bool first = true;
  for (int it = 0; it < iterations; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      launch_sor_half(dev_psi, dev_b, ctx->ps, colour, omega, ctx->dims, cg, ctx->stream);
      omega = first ? 1.0 / (1.0 - 0.5 * rj * rj) : 1.0 / (1.0 - 0.25 * rj * rj * omega);
      first = false;
    }
  return ctx->sync();
}

}  // extern "C"

template ek_status ek_ctx::step_impl<float>(int);
template ek_status ek_ctx::step_impl<double>(int);
