// The ion-density (charge) pass, one thread per site: the charge density that
// the Poisson solve of the step needs (Sec. II.A, the right-hand side of Eq.
// poisson), with the extrapolated start of that solve prepared in the same
// pass.  The per-site density is charge_site of lb_site.h.
#include "ek_internal.h"

#include "lb_site.h"
#include "md_chain.h"
#include "reduce.h"

namespace ek {

namespace {

// Charge pass: n^a at time t for every charged species, rho_e = sum z^a n^a
// + fixed wall charge + bead charge; stores -rho_e / eps and partial sums of
// rho_e (for the mean that the periodic problem removes).  With `start` set
// it also prepares the extrapolated start of the solve at the site, from the
// last solution p = psi and the earlier ones o = old, o2 = old2, o3 = old3
// (time t-1 down to t-4), and the history of the next step (old = p, and
// old2 = o, old3 = o2 where the mode keeps them):
//   mode 1  psi = p                                      old = p
//   mode 2  psi = 2p - o  (linear)                        old = p
//   mode 3  linear, the history deepened                  old = p, old2 = o
//   mode 4  psi = 3p - 3o + o2  (quadratic)               old = p, old2 = o
//   mode 5  quadratic, the history deepened               ... and old3 = o2
//   mode 6  psi = 4p - 6o + 4o2 - o3  (cubic)             ... and old3 = o2
// (the Newton backward-difference forms of the polynomial through the last
// two, three or four solutions, evaluated one step ahead).  Modes 3 to 6
// store only p, in the buffer of the value that drops out (or the unused
// deepest one), and the buffers are renamed afterwards.  With `pending` the
// last solution still carries its mean: p = psi - psum / n (zero for a
// vanishing right-hand side), as k_psi_shift would have left it, and mode 1
// stores that p in psi too.
struct StartExtrap {
  double* psi;
  double* old;
  int mode;
  double* old2;
  double* old3;
  const PoissonScalars* pending;
  double inv_n;
};

template <typename T, typename I, bool NEU>
__global__ __launch_bounds__(BLOCK) void k_charge(const T* __restrict__ f,
                                                  const uint32_t* __restrict__ mask,
                                                  const double* __restrict__ wall_q,
                                                  double* __restrict__ b,
                                                  double* __restrict__ partials, LBParams lp,
                                                  double inv_eps, BeadTableView bt, Dims d,
                                                  StartExtrap start) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int nblocks = gridDim.x * gridDim.y * gridDim.z;
  double acc[1] = {0.0};
  if (x < d.nx && y < d.ny) {
    const double rho = charge_site<T, I, NEU>(f, mask, wall_q, lp, bt, x, y, z, d);
    const long long r = ((long long)z * d.ny + y) * d.nx + x;
    b[r] = -rho * inv_eps;
    acc[0] = rho;
    if (start.mode) {
      double p = start.psi[r];
      if (start.pending) {
        p = mean_removed(p, start.pending, start.inv_n);
        if (start.mode == 1) start.psi[r] = p;
      }
      // the history deepens by rotation: p goes to the buffer that becomes
      // old, which is old for modes 1 and 2, old2 for 3 and 4 and old3 for
      // 5 and 6 (the host then renames the buffers: rotate_history)
      if (start.mode == 2 || start.mode == 3) {
        start.psi[r] = 2.0 * p - start.old[r];
      } else if (start.mode == 4 || start.mode == 5) {
        start.psi[r] = 3.0 * (p - start.old[r]) + start.old2[r];
      } else if (start.mode == 6) {
        start.psi[r] = 4.0 * (p + start.old2[r]) - 6.0 * start.old[r] - start.old3[r];
      }
      double* dst = start.mode <= 2 ? start.old : (start.mode <= 4 ? start.old2 : start.old3);
      dst[r] = p;
    }
  }
  block_partials<1>(acc, partials, bid, nblocks);
}

}  // namespace

template <typename T>
void launch_charge(const T* f, const uint32_t* mask, const double* wall_q, double* b,
                   double* partials, const LBParams& lp, double inv_eps, Dims d,
                   const SiteGrid& g, hipStream_t s, const BeadTableView& bt, double* psi,
                   double* psi_old, int extrap, bool insulating, double* psi_old2,
                   double* psi_old3, const PoissonScalars* pending) {
  const StartExtrap start{psi,      psi_old,  psi_old ? extrap : 0, psi_old2,
                          psi_old3, pending,  1.0 / double(d.n)};
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, g.grid, g.block, 0, s, f, mask, wall_q, b, partials, lp, inv_eps,
                       bt, d, start);
  };
  const bool i32 = fits_idx32<T>(d.n);
  if (insulating) {
    if (i32) go(k_charge<T, uint32_t, true>);
    else go(k_charge<T, long long, true>);
  } else {
    if (i32) go(k_charge<T, uint32_t, false>);
    else go(k_charge<T, long long, false>);
  }
}

#define EK_INST(T)                                                                          \
  template void launch_charge<T>(const T*, const uint32_t*, const double*, double*, double*, \
                                 const LBParams&, double, Dims, const SiteGrid&, hipStream_t,\
                                 const BeadTableView&, double*, double*, int, bool, double*,  \
                                 double*, const PoissonScalars*);
EK_INST(float)
EK_INST(double)

}  // namespace ek
