// The context object behind the opaque ek_ctx handle.
#pragma once

#include <string>
#include <vector>

#include "ek_internal.h"
#include "md_table.h"
#include "unet.h"

namespace ek {
constexpr int MAX_BEADS = 1024;        // one workgroup advances a whole chain
size_t bead_state_bytes(int max_beads);
void launch_table_init(int* keys, long long* vals, hipStream_t s);
void launch_table_init_bits(int* keys, long long* vals, int bits, hipStream_t s);
size_t mg_workspace_bytes(int nx, int ny, int nz);
size_t mg_sweep_bytes(int nx, int ny, int nz);
}  // namespace ek

// The learned warm start consults the network only when the relative
// residual of the current start exceeds this value (cold or abruptly changed
// right-hand sides); a start closer than that is kept as it is.
constexpr double LEARNED_GATE = 0.25;

struct ek_ctx {
  ek_params p{};
  ek::Dims dims{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  bool own_ws = false;
  void* pinned = nullptr;              // small pinned host buffer for read-backs

  // device state carved from the workspace
  void* fA = nullptr;
  void* fB = nullptr;
  bool cur_is_a = true;                // fA holds the current post-collision populations
  uint32_t* mask = nullptr;
  double* wall_q = nullptr;
  double* psi = nullptr;
  double* b = nullptr;
  double* partials = nullptr;
  long long partials_cap = 0;          // doubles in the partials buffer
  ek::PoissonScalars* ps = nullptr;
  double* stats_dev = nullptr;
  int* keys = nullptr;                 // bead-touched node table
  long long* vals = nullptr;
  char* bead_mem = nullptr;
  char* mg_mem = nullptr;
  char* mg_tmp = nullptr;              // sweep buffers of the multigrid (or null)

  // host-side state
  std::vector<uint8_t> host_solid;
  std::vector<double> host_wall_q;     // the wall charges as given (for the state)
  long long n_fluid = 0;
  double nref[3] = {0, 0, 0};
  bool have_geometry = false;
  bool have_species[3] = {false, false, false};
  long long step_count = 0;
  int last_iters = 0;
  int solo_iters = 0;
  bool solo = false;   // a stand-alone solve (ek_poisson_solve) is running
  double last_res = 0.0;
  double last_res0 = 0.0;
  int last_fallback = 0;
  int last_consulted = 0;
  bool have_solve = false;             // b, ps and psi hold a finished solve
  // The time loop with an extrapolated start leaves the removal of the
  // solution's mean to the next charge pass, which reads and writes psi
  // anyway (defer_shift set around such a solve; shift_pending: psi still
  // holds the solution before the shift, whose amount ps keeps).
  bool defer_shift = false;
  bool shift_pending = false;
  double mass[3] = {0, 0, 0};
  double mom[3] = {0, 0, 0};
  int bx_sites = 0, bx_colour = 0;     // launch shapes (0 = default)
  std::string err;

  // polymer
  int max_beads = 0;
  int n_beads = 0;
  ek_polymer_params poly{};
  std::vector<double> host_q;
  bool table_dirty = false;
  // bead crossing record of the plane z = cross_plane (when cross_on)
  bool cross_on = false;
  double cross_plane = 0.0;

  // per-phase timers (HIP events on the context stream)
  bool timing = false;
  bool graph_launch = true;            // multigrid cycles replayed from recorded graphs
  bool overlap_md = true;              // lattice update outside the bead boxes beside the chain
  // second stream for the lattice update outside the bead boxes, beside the
  // chain kernel, and its fork / join events (created on first use)
  hipStream_t side_stream = nullptr;
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  // 6 per step: charge, poisson, md, lb start, lb end, chain end
  std::vector<hipEvent_t> events;
  ek_timing tacc{};
  ek_status ensure_events(int n_steps);
  void record(int step_in_call, int k);

  // multigrid
  struct MG;
  MG* mg = nullptr;

  ek_status fail(ek_status st, const std::string& msg);
  ek_status sync();
  void* fcur();
  void* fnext();
  ek::LBParams lb_params() const;
  ek::NoiseParams noise_params(long long step) const;
  bool insulating() const { return p.walls == EK_WALLS_INSULATING; }
  double inv_eps() const;
  double jacobi_radius() const;
  ek_status read_scalars(ek::PoissonScalars* out);
  // The solvers start from x whose residual state h (ps on the device) is
  // already evaluated.
  ek_status sor_solve(const double* b, double* x, ek::PoissonScalars h, int& iters, double& res,
                      double& res0);
  // With start_norms the start's residual has not been evaluated: the first
  // cycle does it (mg_start_in_cycle), before anything else of the cycle.
  ek_status mg_solve(const double* b, double* x, ek::PoissonScalars h, int& iters, double& res,
                     double& res0, bool start_norms = false);
  bool mg_start_in_cycle() const;
  ek_status initial_residual(const double* b, const double* x, ek::PoissonScalars* h);
  // residual kernel of the context's problem (periodic or insulating walls);
  // returns the number of block partials
  int residual_launch(const double* b, const double* x);
  ek_status learned_start(const double* b, double* x, ek::PoissonScalars* h);
  // Removes a pending mean from psi (before psi is read or ps reused).
  void settle_psi();
  void mg_setup();
  void mg_release();
  // One V-cycle; with norm_blocks given, its last finest-level sweep also
  // leaves the residual norms' block partials where the finest level allows
  // it (*norm_blocks = their count, else 0: the caller takes the residual).
  // With first (the first cycle of a solve) the finest level takes more
  // pre-smoothing sweeps; with start (mg_start_in_cycle, implies first) its
  // first sweep also takes the residual of its input, and the start's test
  // follows it.
  ek_status mg_vcycle(const double* b, double* x, int* norm_blocks = nullptr, bool start = false,
                      bool first = false);
  bool mg_graphs(const double* b, double* x);
  hipGraphExec_t mg_batch_graph(const double* b, double* x, int n, int untested, int opens);
  ek_status poisson(const double* b, double* x, bool learned, int& iters, double& res,
                    double& res0);

  // learned warm start (present when p.warm_start == EK_WS_LEARNED)
  ek::UNet* net = nullptr;
  double* guess = nullptr;
  // extrapolated starts (EK_WS_EXTRAP, EK_WS_EXTRAP2, EK_WS_EXTRAP3): psi(t-2),
  // psi(t-3), psi(t-4) as the order needs them, and how many previous step
  // solutions psi and the history hold (0 up to the order + 1)
  double* psi_old = nullptr;
  double* psi_old2 = nullptr;
  double* psi_old3 = nullptr;
  int psi_hist = 0;
  template <typename T>
  ek_status step_impl(int n_steps);

  // beads (kernels_md.hip)
  ek::BeadTableView bead_view() const;
  const int* bead_origin() const;      // box origins of the step's beads (device)
  ek_status beads_deposit();
  // Box gather and chain kernel on the context stream (stamping `chain_end`
  // when given).  With `overlap` the box nodes are flagged MASK_DEFER and
  // side_fork is recorded after the gather, for the lattice update that the
  // caller runs beside the chain on side_stream.
  template <typename T>
  ek_status beads_advance(bool overlap, hipEvent_t chain_end);
  ek_status beads_check();
};
