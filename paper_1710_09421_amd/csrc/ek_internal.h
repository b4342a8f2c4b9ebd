// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ek.h"

namespace ek {

// ---------------------------------------------------------------------------
// D3Q19 velocity set in the order fixed by ek.h: rest, 6 axis links, 12
// face-diagonal links, opposite directions adjacent.
// ---------------------------------------------------------------------------
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
__host__ __device__ constexpr double weight(int p) {
  return p == 0 ? 1.0 / 3.0 : (p <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Per-site link word: bit p (1..18) set when the pull source r - c_p is solid
// (the population is then bounced back from the opposite link of r itself).
constexpr uint32_t MASK_SOLID = 1u << 31;       // the site itself is solid
constexpr uint32_t MASK_CHARGED = 1u << 30;     // the site carries a fixed charge
constexpr uint32_t MASK_BEAD = 1u << 29;        // a bead kernel touches the site
constexpr uint32_t MASK_WALL = 1u << 28;        // solid site next to the fluid (bead-wall WCA)
constexpr uint32_t MASK_DEFER = 1u << 27;       // in a bead's box: updated after the chain

// Fixed-point scales for order-independent (hence deterministic) sums of the
// bead charge and bead force densities accumulated with integer atomics.
constexpr double FIX_CHARGE = 4503599627370496.0;     // 2^52
constexpr double FIX_FORCE = 17592186044416.0;        // 2^44

constexpr int BLOCK = 256;                            // threads per block for site kernels
constexpr int HASH_BITS = 16;
constexpr int HASH_SLOTS = 1 << HASH_BITS;            // bead-touched node table

// Launch shape of a site kernel: blockDim (bx, by) with bx * by == BLOCK,
// grid (ceil(nx / bx), ceil(ny / by), nz).
struct SiteGrid {
  dim3 grid, block;
  int nblocks() const { return int(grid.x * grid.y * grid.z); }
};
SiteGrid site_grid(int nx, int ny, int nz, int bx_pref = 0);
// Launch shape for kernels that visit one colour of the red-black checkerboard:
// threads cover nx/2 sites per row.
SiteGrid colour_grid(int nx, int ny, int nz, int bx_pref = 0);
SiteGrid lattice_grid(int nx, int ny, int nz);

struct Dims {
  int nx, ny, nz;
  long long n;       // nx * ny * nz
};

// Scalars the fused lattice kernel needs, passed by value.
struct LBParams {
  double omega[3];        // 1 / tau
  double valence[3];
  double wdrag[3];        // omega_drag
  double nref[3];         // reference densities of the deviation storage
  double fext[3][3];      // body force per particle
  double eext[3];         // applied field
};

struct BeadTableView;      // md_table.h
struct NoiseParams;        // philox.h
// Insulating walls: the surface charge Sigma_f of the faces of each solid
// site (face_q, in place of the point charges of the periodic problem) and
// 1 / eps for the ghost values psi_r + Sigma_f / eps of the field.
struct WallView {
  const double* face_q = nullptr;
  double inv_eps = 0.0;
};

// Sets the message ek_last_error(NULL) returns on the calling thread.
void set_thread_error(const std::string& msg);

// Link word of every site from the host solid mask; returns the fluid count.
long long build_link_words(const uint8_t* solid, const double* wall_q, const Dims& d,
                           std::vector<uint32_t>& m);

// Device-side scalars of the Poisson solver (one struct in device memory).
struct PoissonScalars {
  double shift;           // mean(rho) / eps, added to the stored -rho/eps
  double r2, b2, psum;    // last residual sums
  double rel;             // last relative residual
  double rel0;            // residual of the warm start
  int done;               // solve converged
  int iters;              // iteration at which it converged
  int zero_rhs;           // right-hand side vanished
  int cycles;             // multigrid cycles run since the flags were cleared
};

// A potential value with the solution's mean removed (zero for a vanishing
// right-hand side): one fused multiply-add, so that the removal after the
// solve and the one the next charge pass does round alike.
__device__ inline double mean_removed(double v, const PoissonScalars* ps, double inv_n) {
  return ps->zero_rhs ? 0.0 : __builtin_fma(-ps->psum, inv_n, v);
}

// ---------------------------------------------------------------------------
// Launchers (kernel files).  All take the stream as last argument.
// ---------------------------------------------------------------------------
template <typename T>
void launch_init_species(T* f, const uint32_t* mask, const double* n_dev, int species,
                         double nref, Dims d, hipStream_t s);
// The renaming of the history buffers after a charge pass in `mode`: p was
// stored in old2 (modes 3, 4) or old3 (5, 6), which becomes old, the others
// move one step deeper.
inline void rotate_history(int mode, double*& old, double*& old2, double*& old3) {
  if (mode == 3 || mode == 4) {
    double* t = old2;
    old2 = old;
    old = t;
  } else if (mode == 5 || mode == 6) {
    double* t = old3;
    old3 = old2;
    old2 = old;
    old = t;
  }
}
// Previous solutions besides psi that an extrapolated start of the solve
// keeps: 1 for the linear, 2 for the quadratic, 3 for the cubic one.
inline int extrap_history(int warm_start) {
  return warm_start == EK_WS_EXTRAP ? 1
         : warm_start == EK_WS_EXTRAP2 ? 2
         : warm_start == EK_WS_EXTRAP3 ? 3
                                       : 0;
}
// With psi_old (an extrapolated start) and extrap != 0 the pass also prepares
// the start and the history of the next step (the modes of StartExtrap; for
// modes 3 to 6 the caller renames the buffers with rotate_history); with
// `pending` (not null) psi still holds the last solution before the removal
// of its mean, which the pass then does first (as launch_psi_shift).
// insulating: the charge of insulating walls (fluid sites only, the wall
// faces' surface charge added to the fluid sites they bound).
template <typename T>
void launch_charge(const T* f, const uint32_t* mask, const double* wall_q, double* b,
                   double* partials, const LBParams& lp, double inv_eps, Dims d,
                   const SiteGrid& g, hipStream_t s, const BeadTableView& bt,
                   double* psi = nullptr, double* psi_old = nullptr, int extrap = 0,
                   bool insulating = false, double* psi_old2 = nullptr,
                   double* psi_old3 = nullptr, const PoissonScalars* pending = nullptr);
// Fused step over the sites without a `skip` bit.  Writes its block partials
// (seven components: masses, momentum, sites updated) first in a layout of
// `nblocks` blocks (lb_step_blocks(g, nz), plus the tail's blocks when a tail
// follows) and returns the number it wrote.  start / stop (may be null) are
// recorded at the kernel's own start and end.
int lb_step_blocks(const SiteGrid& g, int nz);
int lb_tail_blocks(int n_beads);
// With `noise` (not null) the populations get the stochastic term of the
// thermal fluctuations.
template <typename T>
int launch_lb_step(const T* fsrc, T* fdst, const uint32_t* mask, const double* psi,
                   const LBParams& lp, const BeadTableView& bt, double* partials, int nblocks,
                   uint32_t skip, Dims d, const SiteGrid& g, hipStream_t s,
                   hipEvent_t start = nullptr, hipEvent_t stop = nullptr,
                   const NoiseParams* noise = nullptr, const WallView* walls = nullptr);
// The sites flagged MASK_DEFER in the boxes of n_beads beads (box origins of
// the step); partials of blocks first_block .. of the same layout.  The flags
// stay set (launch_defer_clear clears them after the fused step has ended).
template <typename T>
void launch_lb_tail(const T* fsrc, T* fdst, const uint32_t* mask, const double* psi,
                    const LBParams& lp, const BeadTableView& bt, const int* origin, int n_beads,
                    double* partials, int first_block, int nblocks, Dims d, hipStream_t s,
                    const NoiseParams* noise = nullptr, const WallView* walls = nullptr);
void launch_defer_clear(uint32_t* mask, const int* origin, int n_beads, Dims d, hipStream_t s);
template <typename T>
void launch_moments(const T* f, const uint32_t* mask, int species, double nref, double* n_out,
                    double* u_out, Dims d, hipStream_t s);

// out[0..6] = the seven sums of the fused step's partials; count != 0 also
// adds out[6] (sites updated) to the running count out[7].  With `scratch`
// (room: the doubles free there) many partials are first folded by a grid of
// blocks (kernels_sums.hip).
void launch_sum_partials(const double* partials, int nblocks, double* out, int count,
                         hipStream_t s, double* scratch = nullptr, long long room = 0);
void launch_mean_shift(const double* partials, int nblocks, double inv_n, double inv_eps,
                       PoissonScalars* ps, hipStream_t s, double* scratch = nullptr,
                       long long room = 0);

// Poisson (kernels_poisson.hip)
void launch_sor_half(double* psi, const double* b, const PoissonScalars* ps, int colour,
                     double omega, Dims d, const SiteGrid& g, hipStream_t s);
// Returns the number of block partials it writes (for launch_residual_final).
// Blocks (partial sums) of launch_residual for a lattice and its site grid.
int residual_blocks(const Dims& d, const SiteGrid& g);
int launch_residual(const double* psi, const double* b, PoissonScalars* ps, double* partials,
                    Dims d, const SiteGrid& g, hipStream_t s);
void launch_residual_final(const double* partials, int nblocks, double tol, int iter,
                           int initial, PoissonScalars* ps, hipStream_t s);
void launch_psi_shift(double* psi, const PoissonScalars* ps, double inv_n, Dims d,
                      hipStream_t s);
// Insulating walls: the same over the fluid sites only (the link words give
// the solid face neighbours); inv_nf = 1 / number of fluid sites.
void launch_sor_half_neu(double* psi, const double* b, const uint32_t* mask,
                         const PoissonScalars* ps, int colour, double omega, Dims d,
                         const SiteGrid& g, hipStream_t s);
int launch_residual_neu(const double* psi, const double* b, const uint32_t* mask,
                        PoissonScalars* ps, double* partials, Dims d, const SiteGrid& g,
                        hipStream_t s);
void launch_psi_shift_neu(double* psi, const uint32_t* mask, const PoissonScalars* ps,
                          double inv_nf, Dims d, hipStream_t s);
void launch_fill(double* x, double v, long long n, hipStream_t s);
void launch_ps_reset(PoissonScalars* ps, double shift, hipStream_t s);
void launch_ps_rearm(PoissonScalars* ps, hipStream_t s);
void launch_rhs_copy(const double* b, const PoissonScalars* ps, double* out, long long n,
                     hipStream_t s);
void launch_rho_to_b(const double* rho, double* b, double* partials, double inv_eps, Dims d,
                     const SiteGrid& g, hipStream_t s);

}  // namespace ek
