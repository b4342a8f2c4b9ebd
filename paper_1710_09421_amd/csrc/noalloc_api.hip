// The stand-alone Poisson solve of ek_poisson_solve, by red-black SOR with
// the Chebyshev schedule (Sec. II.C), for callers that cannot allocate: no
// context, no hipMalloc / hipFree / hipHostMalloc, the solver's scratch
// (right-hand side, block partial sums, solver scalars) in one file-scope
// device array.  It launches the same kernels in the same order as a context
// with EK_POISSON_SOR, so both give the same bits.
//
// The array is the library's on every device it runs on and lives until the
// process ends; each call clears what must start at zero.  Calls on one
// device share it: calls that overlap in time on one device (two host
// threads, or two streams) race and give wrong results.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "ek_context.h"

using namespace ek;

namespace {

// Largest lattice of the no-allocation solve (2^21 sites, e.g. 128^3).
constexpr long long NOALLOC_MAX_SITES = 1LL << 21;
// Block partial sums: at most NOALLOC_PARTIALS doubles per reduction.
constexpr long long NOALLOC_PARTIALS = 1LL << 18;
constexpr long long SCRATCH_DOUBLES = NOALLOC_MAX_SITES + NOALLOC_PARTIALS + 64;

// b[NOALLOC_MAX_SITES] | partials[NOALLOC_PARTIALS] | PoissonScalars
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device.  The host-side name of the array is not a device address.
ek_status scratch_on_current_device(double** out, std::string& why) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    why = "no current HIP device";
    return EK_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      why = std::string("hipGetSymbolAddress of the solver scratch failed: ") + hipGetErrorString(e);
      return EK_EHIP;
    }
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return EK_OK;
}

ek_status fail(ek_status st, const std::string& msg) {
  set_thread_error(msg);
  return st;
}

ek_status read_scalars(const PoissonScalars* ps, hipStream_t s, PoissonScalars* out) {
  if (hipMemcpyAsync(out, ps, sizeof(PoissonScalars), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(EK_EHIP, "reading the solver scalars failed");
  return EK_OK;
}

}  // namespace

extern "C" ek_status ek_poisson_solve_noalloc(const ek_params* p, const double* dev_rho,
                                              double* dev_psi, int32_t warm_start,
                                              void* hip_stream, ek_poisson_report* rep) {
  size_t ws = 0;
  if (ek_workspace_bytes(p, 0, &ws) != EK_OK) return EK_EINVAL;   // message already set
  if (p->poisson_method != EK_POISSON_SOR)
    return fail(EK_EINVAL, "the no-allocation solve runs red-black SOR (EK_POISSON_SOR) only");
  if (p->walls != EK_WALLS_PERIODIC)
    return fail(EK_EINVAL, "the no-allocation solve is the periodic problem (EK_WALLS_PERIODIC)");
  if (warm_start != EK_WS_ZERO && warm_start != EK_WS_PREV && warm_start != EK_WS_EXTRAP)
    return fail(EK_EINVAL, "warm_start must be EK_WS_ZERO, EK_WS_PREV or EK_WS_EXTRAP");
  if (!dev_rho || !dev_psi) return fail(EK_EINVAL, "NULL device buffer");
  const Dims d{p->nx, p->ny, p->nz, (long long)p->nx * p->ny * p->nz};
  if (d.n > NOALLOC_MAX_SITES) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "lattice of %lld sites exceeds the no-allocation maximum of %lld",
                  d.n, NOALLOC_MAX_SITES);
    return fail(EK_EINVAL, buf);
  }
  const SiteGrid g = site_grid(p->nx, p->ny, p->nz);
  const SiteGrid cg = colour_grid(p->nx, p->ny, p->nz);
  // the residual reduction writes 3 components over its blocks, the charge
  // reduction 1 over the site grid's blocks
  const long long res_blocks = residual_blocks(d, g);
  if ((long long)g.nblocks() > NOALLOC_PARTIALS || 3 * res_blocks > NOALLOC_PARTIALS)
    return fail(EK_EINVAL, "lattice shape needs more block partials than the scratch holds");

  double* base = nullptr;
  std::string why;
  if (scratch_on_current_device(&base, why) != EK_OK) return fail(EK_EHIP, why);
  double* b = base;
  double* partials = base + NOALLOC_MAX_SITES;
  PoissonScalars* ps = (PoissonScalars*)(base + NOALLOC_MAX_SITES + NOALLOC_PARTIALS);
  const hipStream_t s = (hipStream_t)hip_stream;

  // b = -rho / eps; the mean of rho enters as the scalar shift (k_mean_shift
  // also clears the convergence flags left by the previous call)
  const double inv_eps = 4.0 * M_PI * p->bjerrum * p->kT;
  launch_rho_to_b(dev_rho, b, partials, inv_eps, d, g, s);
  launch_mean_shift(partials, g.nblocks(), 1.0 / double(d.n), inv_eps, ps, s);
  if (warm_start == EK_WS_ZERO) launch_fill(dev_psi, 0.0, d.n, s);
  // residual of the start
  int nr = launch_residual(dev_psi, b, ps, partials, d, g, s);
  launch_residual_final(partials, nr, p->poisson_tol, 0, 1, ps, s);
  PoissonScalars h{};
  ek_status st = read_scalars(ps, s, &h);
  if (st) return st;
  // iterations in batches of check_every, each ended by a residual test;
  // iterations after convergence are skipped on the device
  const double rj = p->rho_jacobi > 0.0
                        ? p->rho_jacobi
                        : (2.0 + std::cos(2.0 * M_PI / std::max(p->nx, std::max(p->ny, p->nz)))) / 3.0;
  const int ce = p->poisson_check_every;
  int it = 0;
  double omega = 1.0;
  bool first = true;
  while (!h.done && it < p->poisson_max_iter) {
    const int nrun = std::min(ce, p->poisson_max_iter - it);
    for (int k = 0; k < nrun; ++k) {
      for (int colour = 0; colour < 2; ++colour) {
        launch_sor_half(dev_psi, b, ps, colour, omega, d, cg, s);
        omega = first ? 1.0 / (1.0 - 0.5 * rj * rj) : 1.0 / (1.0 - 0.25 * rj * rj * omega);
        first = false;
      }
      ++it;
      if (it % ce == 0 || it == p->poisson_max_iter) {
        nr = launch_residual(dev_psi, b, ps, partials, d, g, s);
        launch_residual_final(partials, nr, p->poisson_tol, it, 0, ps, s);
      }
    }
    st = read_scalars(ps, s, &h);
    if (st) return st;
  }
  if (rep) {
    rep->iterations = h.done ? h.iters : it;
    rep->residual = h.rel;
    rep->initial_residual = h.rel0;
  }
  if (!h.done) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "Poisson solve did not reach %.3g in %d iterations (residual %.3e)",
                  p->poisson_tol, p->poisson_max_iter, h.rel);
    return fail(EK_ENOCONV, buf);
  }
  launch_psi_shift(dev_psi, ps, 1.0 / double(d.n), d, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(EK_EHIP, "hipStreamSynchronize failed");
  return EK_OK;
}
