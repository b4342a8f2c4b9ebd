// Ensemble of uneven replicas in one persistent launch.
//
// One workgroup owns one replica for the whole call: it runs every phase of
// the time step (Fig. 1) on its replica with __syncthreads as the only
// barrier — bead charge deposit, charge pass, multigrid Poisson solve with the
// replica's own convergence test, bead boxes and chain substeps, fused
// collide-and-stream — and loops over the steps.  No workgroup ever waits for
// another, so replicas with more Poisson cycles or longer chains do not hold
// the rest back, and no grid-wide barrier (a device-scope fence, i.e. an L2
// write-back on every XCD) is ever needed.
//
// The per-site and per-team code is shared with the single-system kernels
// (lb_site.h, mg_site.h, md_chain.h), so a replica computes exactly what a
// single context computes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ek_context.h"
#include "lb_site.h"
#include "md_chain.h"
#include "mg_site.h"

using namespace ek;

namespace {

constexpr int ENS_TABLE_BITS = 12;     // node table of a replica: 4096 slots
constexpr int ENS_MAX_BEADS = 64;      // node sums of a chain live in LDS
constexpr int ENS_COARSEST_CAP = 200;
// smoothing sweeps of the in-kernel V-cycle: V(1,2), as the launched solver
// (with the extrapolated start 6.3 against 6.6 ms per step of 64 replicas for
// V(2,2); from the previous solution V(2,2) had been the faster)
constexpr int ENS_NU1 = 1, ENS_NU2 = 2;
// Relaxation factor of the finest level's half sweeps (the coarser levels
// keep MG_OMEGA): 6.62 ms per step of 64 replicas against 6.78 at 1.25, 6.76
// at 1.15 and 7.21 at 1.3 (the first 23 steps from the extrapolated start).
constexpr double ENS_OMEGA_FINEST = 1.2;

enum : int { ST_OK = 0, ST_NOCONV = 1, ST_UNSTABLE = 2, ST_TIMEOUT = 3 };

// A replica is advanced by a team of G workgroups (G = 1, 2 or 4) of one
// cooperative launch: the site-parallel phases on the finest level are split
// over the team, the coarse multigrid levels and the chain run in member 0.
constexpr int ENS_MAX_GROUP = 4;
constexpr long long ENS_SPIN_LIMIT = 1ll << 24;   // ~1 s of s_sleep: then the team aborts

// Team barrier state and reduction partials of one replica (global memory,
// cleared by the host before every launch).  Partials are double-buffered by
// the parity of the reduction count, so a member that has summed reduction k
// can write reduction k + 1 while the others still read k.
struct TeamSync {
  int count;                  // barrier arrivals
  int abort;                  // set when a member waited beyond the spin limit
  int pad[14];
  double part[2][ENS_MAX_GROUP][8];
};

// Per-replica device pointers and parameters.
struct RepDev {
  void* f[2];                 // populations; f[cur] holds the current ones
  TeamSync* sync;
  uint32_t* mask;             // link words (own copy: the bead flag is per replica)
  double* psi;
  double* psi_old;            // psi(t-2) for the extrapolated start, or null
  int psi_hist;               // previous solutions held (0, 1 or 2)
  double* b;
  double* mg;                 // multigrid levels 1.. (x then f per level)
  int* keys;
  long long* vals;
  BeadState bs;
  MDParams mp;
  LBParams lp;
  int n_beads;
  int cur;
  int status;
  int steps;                  // steps completed
  int last_cycles;
  double last_res;
  double last_res0;
  double stats[6];            // species masses and fluid momentum of f(t)
  // wall-clock ticks spent by the team's first workgroup in the phases of
  // all steps so far: charge pass, Poisson solve, chain, collide-and-stream
  unsigned long long phase_ticks[4];
  unsigned long long phase_mark;   // clock at the start of the current phase
};

struct EnsConst {
  Dims d;
  const double* wall_q;
  double inv_eps;
  double tol;
  int max_cycles;
  int n_steps;
  int nlev;
  Lvl lv[MAX_LEVELS];         // sizes and spacings; pointers filled per replica
  size_t lv_off[MAX_LEVELS];  // offsets (doubles) of x in the replica's mg block
  double omega_coarsest;
  int coarsest_sweeps;
  int lds_bits;
  int n_rep;
  int group;                  // workgroups per replica
};

// Sum of one value per thread in a fixed tree order (deterministic).
template <int MAXT>
__device__ inline double team_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = MAXT / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Barrier of the G workgroups of one replica: release this workgroup's
// writes, count in, wait for the other members, acquire theirs.  Returns
// false (in every thread) when the team has aborted.
__device__ inline bool team_sync(TeamSync* ts, int G, int& gen, int* s_ok) {
  __syncthreads();
  if (G == 1) return true;
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    atomicAdd(&ts->count, 1);
    gen += G;
    long long spins = 0;
    while (__hip_atomic_load(&ts->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
      if (__hip_atomic_load(&ts->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (++spins > ENS_SPIN_LIMIT) {
        atomicExch(&ts->abort, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Team-wide sums of NV values: per workgroup in a fixed tree, then the G
// partials in member order, so every member gets the same bits.
template <int MAXT, int NV>
__device__ inline bool team_sums(double (&v)[NV], double* sh, TeamSync* ts, int g, int G, int& gen,
                                 int& nred, int* s_ok) {
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = team_sum<MAXT>(v[k], sh);
  if (G == 1) return true;
  const int set = nred & 1;
  ++nred;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) ts->part[set][g][k] = v[k];
  }
  if (!team_sync(ts, G, gen, s_ok)) return false;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
    for (int m = 0; m < G; ++m) t += ts->part[set][m][k];
    v[k] = t;
  }
  return true;
}

// One colour of a red-black sweep of level L over the team's share of sites.
// (Level descriptions by value: see block_smooth.)
__device__ inline void team_half(const Lvl L, int colour, double shift, double omega, int first,
                                 int stride) {
  const int hx = L.nx / 2, nh = hx * L.ny * L.nz;
  const float ihx = 1.0f / hx, iny = 1.0f / L.ny;
  for (int t = first; t < nh; t += stride) {
    int tx, y;
    const int yz = fdivmod(t, hx, ihx, tx);
    const int z = fdivmod(yz, L.ny, iny, y);
    smooth_site(L, colour, tx, y, z, shift, omega);
  }
}

__device__ inline void team_restrict(const Lvl F, const Lvl C, double shift, int first, int stride) {
  const float inx = 1.0f / C.nx, iny = 1.0f / C.ny;
  for (int t = first; t < int(C.n); t += stride) {
    int X, Y;
    const int yz = fdivmod(t, C.nx, inx, X);
    const int Z = fdivmod(yz, C.ny, iny, Y);
    restrict_site(F, C, X, Y, Z, shift);
  }
}

__device__ inline void team_prolong(const Lvl F, const Lvl C, int first, int stride) {
  const float inx = 1.0f / F.nx, iny = 1.0f / F.ny;
  for (int t = first; t < int(F.n); t += stride) {
    int x, y;
    const int yz = fdivmod(t, F.nx, inx, x);
    const int z = fdivmod(yz, F.ny, iny, y);
    prolong_site(F, C, x, y, z);
  }
}

__device__ inline void site_xyz(int t, const Dims& d, float inx, float iny, int& x, int& y, int& z) {
  const int yz = fdivmod(t, d.nx, inx, x);
  z = fdivmod(yz, d.ny, iny, y);
}

template <typename T, int MAXT, int TPB>
__global__ __launch_bounds__(MAXT) void k_ensemble(RepDev* reps, EnsConst ec) {
  extern __shared__ __align__(16) unsigned char smem[];   // the chain's LDS
  __shared__ double sh[MAXT];
  __shared__ Lvl L[MAX_LEVELS];
  __shared__ int s_status;
  __shared__ int s_ok;
  const int G = ec.group;
  const int g = blockIdx.x / ec.n_rep;                    // member of the replica's team
  RepDev& R = reps[blockIdx.x % ec.n_rep];
  TeamSync* ts = R.sync;
  const Dims d = ec.d;
  const int tid = threadIdx.x;
  const int first = g * MAXT + tid, stride = G * MAXT;   // this thread's share of a team loop
  const int N = int(d.n);
  const float inx = 1.0f / d.nx, iny = 1.0f / d.ny;
  int gen = 0, nred = 0;
  if (tid == 0) {
    for (int l = 0; l < ec.nlev; ++l) {
      L[l] = ec.lv[l];
      L[l].x = l == 0 ? R.psi : R.mg + ec.lv_off[l];
      L[l].f = l == 0 ? R.b : R.mg + ec.lv_off[l] + ec.lv[l].n;
    }
    s_status = R.status;
  }
  __syncthreads();
  const int last = ec.nlev - 1;
  const LBParams& lp = R.lp;   // read where used (uniform loads)
  int cur = R.cur;
  int hist = R.psi_hist;       // every member keeps the same count
// every member takes the same branch: the status depends only on team-wide
// values; a failed barrier ends the team's work
#define TEAM_SYNC()                                   \
  if (!team_sync(ts, G, gen, &s_ok)) {                \
    if (tid == 0) s_status = ST_TIMEOUT;              \
    __syncthreads();                                  \
    break;                                            \
  }
  // phase clock (thread 0 of member 0): each phase ends at a team barrier,
  // so its span is the team's.  The counters are the replica's own words in
  // global memory, not registers of every thread (the 512-thread instance
  // has none to spare) nor static LDS (40 more bytes there moved the
  // kernel's LDS layout and made that instance 50 % slower).
  const bool timer = tid == 0 && g == 0;
  auto lap = [&](int ph) {
    if (timer) {
      const unsigned long long now = wall_clock64();
      R.phase_ticks[ph] += now - R.phase_mark;
      R.phase_mark = now;
    }
  };
  for (int step = 0; step < ec.n_steps; ++step) {
    if (s_status != ST_OK) break;
    if (timer) R.phase_mark = wall_clock64();
    const T* fsrc = (const T*)R.f[cur];
    T* fdst = (T*)R.f[cur ^ 1];
    BeadTableView bt;
    bt.keys = R.keys;
    bt.vals = R.vals;
    bt.bits = ENS_TABLE_BITS;

    // bead charges of time t (member 0)
    if (R.n_beads > 0 && g == 0) {
      table_clear_items(R.keys, R.vals, R.mask, d.n, ENS_TABLE_BITS, tid, MAXT);
      __syncthreads();
      deposit_items(R.bs, R.n_beads, R.keys, R.vals, R.mask, d, ENS_TABLE_BITS, tid, MAXT);
    }
    TEAM_SYNC();
    // charge pass; with the extrapolated start also psi = 2 psi(t-1) - psi(t-2)
    // (the sums' barrier orders it before the solve reads neighbours)
    double rs[1] = {0.0};
    const bool extrap = R.psi_old != nullptr && hist > 0;
    for (int t = first; t < N; t += stride) {
      int x, y, z;
      site_xyz(t, d, inx, iny, x, y, z);
      const double rho = charge_site<T, long long>(fsrc, R.mask, ec.wall_q, lp, bt, x, y, z, d);
      R.b[t] = -rho * ec.inv_eps;
      rs[0] += rho;
      if (extrap) {
        const double p = R.psi[t];
        if (hist >= 2) R.psi[t] = 2.0 * p - R.psi_old[t];
        R.psi_old[t] = p;
      }
    }
    if (R.psi_old != nullptr) hist = hist < 2 ? hist + 1 : 2;
    if (!team_sums<MAXT, 1>(rs, sh, ts, g, G, gen, nred, &s_ok)) {
      if (tid == 0) s_status = ST_TIMEOUT;
      __syncthreads();
      break;
    }
    const double shift = rs[0] / double(N) * ec.inv_eps;
    lap(0);

    // Poisson: multigrid cycles until ||b - A psi|| / ||b|| <= tol
    auto residual = [&](double& rel, double& psum, double& b2) -> bool {
      double v[3] = {0.0, 0.0, 0.0};
      for (int t = first; t < N; t += stride) {
        int x, y, z;
        site_xyz(t, d, inx, iny, x, y, z);
        const double c = R.psi[t];
        const double rhs = R.b[t] + shift;
        const double res = rhs - (nbsum(R.psi, x, y, z, L[0]) - 6.0 * c);
        v[0] += res * res;
        v[1] += rhs * rhs;
        v[2] += c;
      }
      if (!team_sums<MAXT, 3>(v, sh, ts, g, G, gen, nred, &s_ok)) return false;
      b2 = v[1];
      psum = v[2];
      rel = v[1] > 0.0 ? sqrt(v[0] / v[1]) : (v[0] == 0.0 ? 0.0 : INFINITY);
      return true;
    };
    // one colour of the finest level over the team, then a barrier
    auto fine_half = [&](int colour, double omega) -> bool {
      team_half(L[0], colour, shift, omega, first, stride);
      return team_sync(ts, G, gen, &s_ok);
    };
    double rel = 0.0, psum = 0.0, b2 = 0.0;
    bool ok = residual(rel, psum, b2);
    const double rel0 = rel;
    int cycles = 0;
    const bool zero_rhs = b2 == 0.0;
    while (ok && !zero_rhs && rel > ec.tol && cycles < ec.max_cycles) {
      if (last == 0) {
        for (int sw = 0; ok && sw < ec.coarsest_sweeps; ++sw)
          for (int c = 0; ok && c < 2; ++c) ok = fine_half(c, ec.omega_coarsest);
      } else {
        for (int sw = 0; ok && sw < ENS_NU1; ++sw)
          for (int c = 0; ok && c < 2; ++c) ok = fine_half(c, ENS_OMEGA_FINEST);
        if (!ok) break;
        team_restrict(L[0], L[1], shift, first, stride);
        if (!(ok = team_sync(ts, G, gen, &s_ok))) break;
        if (g == 0) {   // the coarse levels in member 0
          for (int l = 1; l < last; ++l) {
            block_smooth(L[l], ENS_NU1, 0.0, MG_OMEGA);
            block_restrict(L[l], L[l + 1], 0.0);
          }
          block_smooth(L[last], ec.coarsest_sweeps, 0.0, ec.omega_coarsest);
          for (int l = last - 1; l >= 1; --l) {
            block_prolong(L[l], L[l + 1]);
            block_smooth(L[l], ENS_NU2, 0.0, MG_OMEGA);
          }
        }
        if (!(ok = team_sync(ts, G, gen, &s_ok))) break;
        team_prolong(L[0], L[1], first, stride);
        if (!(ok = team_sync(ts, G, gen, &s_ok))) break;
        for (int sw = 0; ok && sw < ENS_NU2; ++sw)
          for (int c = 0; ok && c < 2; ++c) ok = fine_half(c, ENS_OMEGA_FINEST);
        if (!ok) break;
      }
      ++cycles;
      ok = residual(rel, psum, b2);
    }
    if (!ok) {
      if (tid == 0) s_status = ST_TIMEOUT;
      __syncthreads();
      break;
    }
    if (!zero_rhs && rel > ec.tol) {
      if (tid == 0) {
        s_status = ST_NOCONV;
        if (g == 0) {
          R.last_cycles = cycles;
          R.last_res = rel;
        }
      }
      __syncthreads();
      break;
    }
    // gauge: mean(psi) = 0
    const double mean = zero_rhs ? 0.0 : psum / double(N);
    for (int t = first; t < N; t += stride) R.psi[t] = zero_rhs ? 0.0 : R.psi[t] - mean;
    TEAM_SYNC();
    lap(1);

    // chain (member 0): fields around the beads, then n_sub substeps
    if (R.n_beads > 0 && g == 0) {
      for (int it = tid; it < R.n_beads * WIN3; it += MAXT)
        bead_box_item(R.bs, it / WIN3, it % WIN3, fsrc, R.mask, R.psi, lp, d);
      __syncthreads();
      md_chain<true, TPB, 0, 1, false>(R.bs, R.mp, R.keys, R.vals, R.mask, d, ENS_TABLE_BITS,
                             1 << ec.lds_bits, smem);
    }
    TEAM_SYNC();
    lap(2);

    // fused collide-and-stream
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int t = first; t < N; t += stride) {
      int x, y, z;
      site_xyz(t, d, inx, iny, x, y, z);
      lb_site<T, long long>(fsrc, fdst, R.mask, R.psi, lp, bt, x, y, z, d, acc);
    }
    if (!team_sums<MAXT, 6>(acc, sh, ts, g, G, gen, nred, &s_ok)) {
      if (tid == 0) s_status = ST_TIMEOUT;
      __syncthreads();
      break;
    }
    cur ^= 1;
    if (tid == 0) {
      if (g == 0) {
        for (int c = 0; c < 6; ++c) R.stats[c] = acc[c];
        R.last_cycles = cycles;
        R.last_res = rel;
        R.last_res0 = rel0;
        R.steps += 1;
      }
      for (int sp = 0; sp < 3; ++sp)
        if (!(acc[sp] >= 0.0) || !isfinite(acc[sp])) s_status = ST_UNSTABLE;
      if (R.n_beads > 0 && *R.bs.err) s_status = ST_UNSTABLE;
    }
    // every member reads the chain's error word before any member clears it
    // in the next step's deposit
    TEAM_SYNC();
    lap(3);
  }
#undef TEAM_SYNC
  if (tid == 0 && g == 0) {
    R.cur = cur;
    R.status = s_status;
    R.psi_hist = hist;
  }
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct ek_ensemble {
  ek_params p{};
  int n_rep = 0;
  int max_beads = 0;
  Dims d{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  bool own = false;
  size_t rep_bytes = 0;
  double* wall_q = nullptr;
  RepDev* reps_dev = nullptr;
  std::vector<RepDev> reps;
  std::vector<uint8_t> solid;
  long long n_fluid = 0;
  bool have_geometry = false;
  std::vector<bool> have_replica;
  EnsConst ec{};
  int threads = 512;
  int group = 1;              // workgroups per replica
  double wall_khz = 0.0;      // rate of the device's wall clock
  std::string err;

  ek_status fail(ek_status st, const std::string& m) {
    err = m;
    return st;
  }
};

namespace {

struct RepLayout {
  size_t fA, fB, mask, psi, psi_old, b, mg, keys, vals, beads, sync, total;
};

RepLayout rep_layout(const ek_params* p, int max_beads) {
  const size_t n = (size_t)p->nx * p->ny * p->nz;
  const size_t tsz = p->precision == EK_FP64 ? 8 : 4;
  RepLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += al256(b); return o; };
  L.fA = take(3 * Q * n * tsz);
  L.fB = take(3 * Q * n * tsz);
  L.mask = take(n * 4);
  L.psi = take(n * 8);
  L.psi_old = take(p->warm_start == EK_WS_EXTRAP ? n * 8 : 0);
  L.b = take(n * 8);
  L.mg = take(mg_workspace_bytes(p->nx, p->ny, p->nz));
  L.keys = take((size_t(1) << ENS_TABLE_BITS) * 4);
  L.vals = take((size_t(1) << ENS_TABLE_BITS) * SLOT_VALUES * 8);
  L.beads = take(bead_state_bytes(max_beads));
  L.sync = take(sizeof(TeamSync));
  L.total = off;
  return L;
}

BeadState carve_beads(char* mem, int maxb) {
  maxb = maxb < 1 ? 1 : maxb;
  BeadState s;
  size_t off = 0;
  auto take = [&](size_t b) { char* q = mem + off; off += al256(b); return q; };
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

size_t shared_bytes(int n_rep) { return al256(sizeof(RepDev) * (size_t)n_rep) + 256; }

ek_status check(const ek_params* p, int n_rep, int max_beads, std::string& why) {
  if (!p) { why = "params is NULL"; return EK_EINVAL; }
  size_t dummy = 0;
  if (ek_workspace_bytes(p, 0, &dummy) != EK_OK) { why = ek_last_error(nullptr); return EK_EINVAL; }
  if (n_rep < 1 || n_rep > 4096) { why = "n_rep must be in [1, 4096]"; return EK_EINVAL; }
  if (max_beads < 0 || max_beads > ENS_MAX_BEADS) { why = "max_beads must be in [0, 64]"; return EK_EINVAL; }
  // float64 populations are switched off in the persistent kernel: that path
  // has no oracle parity on record since its team rewrites
  if (p->precision != EK_FP32) { why = "the ensemble stores float32 populations only (EK_FP32)"; return EK_EINVAL; }
  if (p->fluctuations != 0) { why = "the ensemble runs without thermal fluctuations"; return EK_EINVAL; }
  if (p->walls != EK_WALLS_PERIODIC) { why = "the ensemble solves the periodic Poisson problem only"; return EK_EINVAL; }
  return EK_OK;
}

thread_local std::string g_ens_error;

int lds_bits_for(int max_beads) {
  int bits = 6;
  while ((1 << bits) < 16 * std::max(1, max_beads)) ++bits;
  return bits;
}

// LDS of the chain (positions and node table; the ensemble runs the chain
// without pair lists)
size_t md_lds_bytes(int max_beads) {
  const size_t sr = ((size_t)std::max(1, max_beads) * 24 + 15) & ~size_t(15);
  return sr + ((size_t)1 << lds_bits_for(max_beads)) * (9 * 8 + 4);
}

template <typename T>
ek_status launch_ensemble(ek_ensemble* e, int n_steps, int threads, int group) {
  EnsConst ec = e->ec;
  ec.n_steps = n_steps;
  ec.n_rep = e->n_rep;
  ec.group = group;
  const size_t lds = md_lds_bytes(e->max_beads);
  // barrier counters start at zero in every launch
  for (int r = 0; r < e->n_rep; ++r)
    if (hipMemsetAsync(e->reps[r].sync, 0, sizeof(TeamSync), e->stream) != hipSuccess)
      return e->fail(EK_EHIP, "clearing the team barriers failed");
  auto go = [&](auto kernel) -> ek_status {
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
      return e->fail(EK_EHIP, "cannot raise the LDS limit of the ensemble kernel");
    if (group == 1) {
      hipLaunchKernelGGL(kernel, dim3(e->n_rep), dim3(threads), lds, e->stream, e->reps_dev, ec);
      if (hipGetLastError() != hipSuccess) return e->fail(EK_EHIP, "ensemble launch failed");
      return EK_OK;
    }
    // teams of workgroups wait for each other: all of them must be resident,
    // which a cooperative launch guarantees (or refuses)
    RepDev* reps = e->reps_dev;
    void* args[] = {(void*)&reps, (void*)&ec};
    const hipError_t err = hipLaunchCooperativeKernel((const void*)kernel, dim3(e->n_rep * group),
                                                      dim3(threads), args, (unsigned)lds, e->stream);
    if (err != hipSuccess) {
      (void)hipGetLastError();
      return e->fail(EK_EHIP, std::string("cooperative ensemble launch refused: ") + hipGetErrorString(err));
    }
    return EK_OK;
  };
  if (group != 1 && group != 2 && group != 4) return e->fail(EK_EINVAL, "group must be 1, 2 or 4");
  if (threads == 256) return go(k_ensemble<T, 256, 4>);
  if (threads == 512) return go(k_ensemble<T, 512, 8>);
  if (threads == 1024) return go(k_ensemble<T, 1024, 8>);
  return e->fail(EK_EINVAL, "threads must be 256, 512 or 1024");
}

ek_status upload(ek_ensemble* e) {
  if (hipMemcpyAsync(e->reps_dev, e->reps.data(), sizeof(RepDev) * e->n_rep, hipMemcpyHostToDevice,
                     e->stream) != hipSuccess)
    return e->fail(EK_EHIP, "copying replica descriptors failed");
  return EK_OK;
}

ek_status download(ek_ensemble* e) {
  if (hipMemcpyAsync(e->reps.data(), e->reps_dev, sizeof(RepDev) * e->n_rep, hipMemcpyDeviceToHost,
                     e->stream) != hipSuccess ||
      hipStreamSynchronize(e->stream) != hipSuccess)
    return e->fail(EK_EHIP, "reading replica descriptors failed");
  return EK_OK;
}

ek_status run_steps(ek_ensemble* e, int n_steps, int threads, int group) {
  if (n_steps == 0) return EK_OK;
  ek_status st = upload(e);
  if (st) return st;
  st = e->p.precision == EK_FP64 ? launch_ensemble<double>(e, n_steps, threads, group)
                                 : launch_ensemble<float>(e, n_steps, threads, group);
  if (st) return st;
  st = download(e);
  if (st) return st;
  for (int r = 0; r < e->n_rep; ++r) {
    const RepDev& R = e->reps[r];
    char buf[200];
    if (R.status == ST_NOCONV) {
      std::snprintf(buf, sizeof buf, "replica %d: multigrid did not reach %.3g in %d cycles (residual %.3e)",
                    r, e->p.poisson_tol, R.last_cycles, R.last_res);
      return e->fail(EK_ENOCONV, buf);
    }
    if (R.status == ST_UNSTABLE) {
      std::snprintf(buf, sizeof buf, "replica %d: non-finite mass or failed chain update", r);
      return e->fail(EK_EUNSTABLE, buf);
    }
    if (R.status == ST_TIMEOUT) {
      std::snprintf(buf, sizeof buf, "replica %d: a workgroup of its team waited beyond the limit", r);
      return e->fail(EK_EHIP, buf);
    }
  }
  return EK_OK;
}

}  // namespace

extern "C" {

ek_status ek_ensemble_workspace_bytes(const ek_params* base, int32_t n_rep, int32_t max_beads,
                                      size_t* bytes) {
  std::string why;
  if (check(base, n_rep, max_beads, why) != EK_OK || !bytes) {
    g_ens_error = bytes ? why : "bytes is NULL";
    return EK_EINVAL;
  }
  const size_t n = (size_t)base->nx * base->ny * base->nz;
  *bytes = shared_bytes(n_rep) + al256(n * 8) + (size_t)n_rep * rep_layout(base, max_beads).total;
  return EK_OK;
}

ek_status ek_ensemble_create(const ek_params* base, int32_t n_rep, int32_t max_beads,
                             void* dev_ws, size_t ws_bytes, void* hip_stream, ek_ensemble** out) {
  if (!out) { g_ens_error = "out is NULL"; return EK_EINVAL; }
  *out = nullptr;
  size_t need = 0;
  ek_status st = ek_ensemble_workspace_bytes(base, n_rep, max_beads, &need);
  if (st) return st;
  char* ws = (char*)dev_ws;
  bool own = false;
  if (ws) {
    if (ws_bytes < need) { g_ens_error = "workspace too small"; return EK_ENOMEM; }
    if (((uintptr_t)ws & 255) != 0) { g_ens_error = "workspace must be 256-byte aligned"; return EK_EINVAL; }
  } else {
    if (hipMalloc((void**)&ws, need) != hipSuccess) { g_ens_error = "hipMalloc failed"; return EK_ENOMEM; }
    own = true;
  }
  ek_ensemble* e = new ek_ensemble();
  e->p = *base;
  e->p.poisson_method = EK_POISSON_MG;
  e->n_rep = n_rep;
  e->max_beads = max_beads;
  e->d = Dims{base->nx, base->ny, base->nz, (long long)base->nx * base->ny * base->nz};
  e->stream = (hipStream_t)hip_stream;
  e->ws = ws;
  e->own = own;
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess)
      e->wall_khz = khz;
    else
      (void)hipGetLastError();
  }
  e->reps_dev = (RepDev*)ws;
  e->wall_q = (double*)(ws + shared_bytes(n_rep));
  const RepLayout RL = rep_layout(base, max_beads);
  e->rep_bytes = RL.total;
  char* base_rep = ws + shared_bytes(n_rep) + al256(e->d.n * 8);
  // multigrid hierarchy (same construction as the single-system solver)
  EnsConst& ec = e->ec;
  ec.d = e->d;
  ec.wall_q = e->wall_q;
  ec.inv_eps = 4.0 * M_PI * base->bjerrum * base->kT;
  ec.tol = base->poisson_tol;
  ec.max_cycles = base->poisson_max_iter;
  {
    int nx = base->nx, ny = base->ny, nz = base->nz, l = 0;
    size_t off = 0;
    double h2 = 1.0;
    ec.lv[0] = Lvl{nx, ny, nz, (long long)nx * ny * nz, 1.0, nullptr, nullptr};
    ec.lv_off[0] = 0;
    while (nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0 && l + 1 < MAX_LEVELS) {
      nx /= 2; ny /= 2; nz /= 2; h2 *= 4.0; ++l;
      ec.lv[l] = Lvl{nx, ny, nz, (long long)nx * ny * nz, h2, nullptr, nullptr};
      ec.lv_off[l] = off;
      off += 2 * (size_t)ec.lv[l].n;
    }
    ec.nlev = l + 1;
    const Lvl& c = ec.lv[l];
    const int m = std::max(c.nx, std::max(c.ny, c.nz));
    const double rj = (2.0 + std::cos(2.0 * M_PI / m)) / 3.0;
    ec.omega_coarsest = 2.0 / (1.0 + std::sqrt(1.0 - rj * rj));
    const double rate = std::max(ec.omega_coarsest - 1.0, 1e-3);
    // coarsest level solved to 1e-3 inside a cycle (see kernels_mg.hip); a
    // box that cannot be coarsened is solved by these sweeps alone
    const double reduction = ec.nlev > 1 ? 1e-3 : 1e-10;
    ec.coarsest_sweeps = std::min(ENS_COARSEST_CAP,
                                  std::max(4, (int)std::ceil(std::log(reduction) / std::log(rate))));
    if (off * 8 + 256 > mg_workspace_bytes(base->nx, base->ny, base->nz)) {
      if (own) (void)hipFree(ws);
      delete e;
      g_ens_error = "multigrid layout mismatch";
      return EK_EINVAL;
    }
  }
  ec.lds_bits = lds_bits_for(max_beads);
  e->reps.resize(n_rep);
  e->have_replica.assign(n_rep, false);
  for (int r = 0; r < n_rep; ++r) {
    char* m = base_rep + (size_t)r * RL.total;
    RepDev& R = e->reps[r];
    std::memset(&R, 0, sizeof R);
    R.f[0] = m + RL.fA;
    R.f[1] = m + RL.fB;
    R.mask = (uint32_t*)(m + RL.mask);
    R.psi = (double*)(m + RL.psi);
    R.psi_old = base->warm_start == EK_WS_EXTRAP ? (double*)(m + RL.psi_old) : nullptr;
    R.b = (double*)(m + RL.b);
    R.mg = (double*)(m + RL.mg + 256);
    R.keys = (int*)(m + RL.keys);
    R.vals = (long long*)(m + RL.vals);
    R.bs = carve_beads(m + RL.beads, max_beads);
    R.sync = (TeamSync*)(m + RL.sync);
  }
  *out = e;
  return EK_OK;
}

void ek_ensemble_destroy(ek_ensemble* e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->stream);
  if (e->own) (void)hipFree(e->ws);
  delete e;
}

const char* ek_ensemble_last_error(const ek_ensemble* e) {
  return e ? e->err.c_str() : g_ens_error.c_str();
}

ek_status ek_ensemble_set_geometry(ek_ensemble* e, const uint8_t* solid, const double* wall_q) {
  if (!e) return EK_EINVAL;
  if (!solid) return e->fail(EK_EINVAL, "solid is NULL");
  std::vector<uint32_t> m;
  const long long nfluid = build_link_words(solid, wall_q, e->d, m);
  if (nfluid == 0) return e->fail(EK_EINVAL, "geometry has no fluid site");
  const size_t n = e->d.n;
  const size_t tsz = e->p.precision == EK_FP64 ? 8 : 4;
  for (int r = 0; r < e->n_rep; ++r) {
    RepDev& R = e->reps[r];
    if (hipMemcpyAsync(R.mask, m.data(), n * 4, hipMemcpyHostToDevice, e->stream) != hipSuccess ||
        hipMemsetAsync(R.f[0], 0, 3 * Q * n * tsz, e->stream) != hipSuccess ||
        hipMemsetAsync(R.f[1], 0, 3 * Q * n * tsz, e->stream) != hipSuccess ||
        hipMemsetAsync(R.psi, 0, n * 8, e->stream) != hipSuccess ||
        hipMemsetAsync(R.bs.err, 0, 64, e->stream) != hipSuccess)
      return e->fail(EK_EHIP, "initialising a replica failed");
    launch_table_init_bits(R.keys, R.vals, ENS_TABLE_BITS, e->stream);
    R.cur = 0;
    R.status = ST_OK;
    R.steps = 0;
    R.n_beads = 0;
    R.psi_hist = 0;
  }
  if (wall_q) {
    if (hipMemcpyAsync(e->wall_q, wall_q, n * 8, hipMemcpyHostToDevice, e->stream) != hipSuccess)
      return e->fail(EK_EHIP, "copying the wall charge failed");
  } else {
    launch_fill(e->wall_q, 0.0, n, e->stream);
  }
  e->solid.assign(solid, solid + n);
  e->n_fluid = nfluid;
  e->have_geometry = true;
  e->have_replica.assign(e->n_rep, false);
  if (hipStreamSynchronize(e->stream) != hipSuccess) return e->fail(EK_EHIP, "synchronise failed");
  return EK_OK;
}

ek_status ek_ensemble_set_replica(ek_ensemble* e, int32_t r, const double* E_ext, const double* n0,
                                  int32_t n_beads, const double* pos, const double* vel,
                                  const double* charge, const ek_polymer_params* pp) {
  if (!e) return EK_EINVAL;
  if (!e->have_geometry) return e->fail(EK_ESTATE, "set the geometry first");
  if (r < 0 || r >= e->n_rep || !E_ext || !n0) return e->fail(EK_EINVAL, "bad replica arguments");
  if (n_beads < 0 || n_beads > e->max_beads) return e->fail(EK_EINVAL, "n_beads exceeds max_beads");
  if (n_beads > 0 && (!pos || !vel || !pp || pp->n_sub < 1 || !(pp->M > 0) || !(pp->sigma > 0) ||
                      1.122462048309373 * pp->sigma >= 2.0 ||
                      (pp->bond != EK_BOND_FENE && pp->bond != EK_BOND_HARMONIC) ||
                      (pp->bond == EK_BOND_FENE && !(pp->R0 > 0)) ||
                      (pp->bond == EK_BOND_HARMONIC && (!(pp->k_bond >= 0) || !(pp->l_bond > 0))) ||
                      (pp->coupling != EK_COUPLE_TRILINEAR && pp->coupling != EK_COUPLE_THETA) ||
                      (pp->coupling == EK_COUPLE_THETA && !(pp->sigma >= 1.0 && pp->sigma <= 2.0))))
    return e->fail(EK_EINVAL, "bad chain arguments");
  const Dims d = e->d;
  const size_t n = d.n;
  RepDev& R = e->reps[r];
  LBParams lp{};
  for (int s = 0; s < 3; ++s) {
    double sum = 0.0;
    for (size_t i = 0; i < n; ++i) {
      const double v = n0[s * n + i];
      if (e->solid[i]) continue;
      if (!std::isfinite(v) || v < 0.0) return e->fail(EK_EINVAL, "densities must be finite and >= 0");
      sum += v;
    }
    lp.nref[s] = sum / double(e->n_fluid);
    lp.omega[s] = 1.0 / e->p.tau[s];
    lp.valence[s] = e->p.valence[s];
    lp.wdrag[s] = e->p.omega_drag[s];
    for (int c = 0; c < 3; ++c) lp.fext[s][c] = e->p.F_ext[s][c];
    lp.eext[s] = E_ext[s];
  }
  R.lp = lp;
  // populations at rest, staged through the other buffer
  for (int s = 0; s < 3; ++s) {
    double* stage = (double*)R.f[1];
    if (hipMemcpyAsync(stage, n0 + s * n, n * 8, hipMemcpyHostToDevice, e->stream) != hipSuccess)
      return e->fail(EK_EHIP, "copying densities failed");
    if (e->p.precision == EK_FP64)
      launch_init_species<double>((double*)R.f[0], R.mask, stage, s, lp.nref[s], d, e->stream);
    else
      launch_init_species<float>((float*)R.f[0], R.mask, stage, s, lp.nref[s], d, e->stream);
    if (hipStreamSynchronize(e->stream) != hipSuccess) return e->fail(EK_EHIP, "initialising populations failed");
  }
  R.cur = 0;
  R.status = ST_OK;
  R.steps = 0;
  R.n_beads = n_beads;
  R.psi_hist = 0;
  if (n_beads > 0) {
    std::vector<double> q(n_beads, 0.0);
    if (charge) std::copy(charge, charge + n_beads, q.begin());
    if (hipMemcpyAsync(R.bs.R, pos, n_beads * 3 * 8, hipMemcpyHostToDevice, e->stream) != hipSuccess ||
        hipMemcpyAsync(R.bs.V, vel, n_beads * 3 * 8, hipMemcpyHostToDevice, e->stream) != hipSuccess ||
        hipMemcpyAsync(R.bs.q, q.data(), n_beads * 8, hipMemcpyHostToDevice, e->stream) != hipSuccess ||
        hipMemsetAsync(R.bs.err, 0, 64, e->stream) != hipSuccess ||
        hipStreamSynchronize(e->stream) != hipSuccess)
      return e->fail(EK_EHIP, "copying the chain failed");
    MDParams& mp = R.mp;
    mp.n = n_beads;
    mp.n_sub = pp->n_sub;
    mp.M = pp->M;
    mp.k_fene = pp->k_fene;
    mp.R0 = pp->R0;
    mp.eps = pp->eps;
    mp.sigma = pp->sigma;
    mp.gamma = pp->gamma;
    mp.Lx = d.nx;
    mp.Ly = d.ny;
    mp.Lz = d.nz;
    mp.bond = pp->bond;
    mp.k_bond = pp->k_bond;
    mp.l_bond = pp->l_bond;
    mp.theta = pp->coupling == EK_COUPLE_THETA ? 1 : 0;
    mp.half_sigma = 0.5 * pp->sigma;
  }
  e->have_replica[r] = true;
  return EK_OK;
}

ek_status ek_ensemble_step(ek_ensemble* e, int32_t n_steps) {
  if (!e) return EK_EINVAL;
  if (n_steps < 0) return e->fail(EK_EINVAL, "n_steps < 0");
  for (int r = 0; r < e->n_rep; ++r)
    if (!e->have_replica[r]) return e->fail(EK_ESTATE, "every replica must be set first");
  return run_steps(e, n_steps, e->threads, e->group);
}

ek_status ek_ensemble_set_threads(ek_ensemble* e, int32_t threads) {
  if (!e) return EK_EINVAL;
  if (threads != 256 && threads != 512 && threads != 1024)
    return e->fail(EK_EINVAL, "threads must be 256, 512 or 1024");
  e->threads = threads;
  return EK_OK;
}

ek_status ek_ensemble_autotune(ek_ensemble* e, int32_t steps, ek_tune_result* out) {
  if (!e) return EK_EINVAL;
  if (steps < 1) return e->fail(EK_EINVAL, "steps < 1");
  for (int r = 0; r < e->n_rep; ++r)
    if (!e->have_replica[r]) return e->fail(EK_ESTATE, "every replica must be set first");
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return e->fail(EK_EHIP, "hipEventCreate failed");
  // Every candidate is timed in two interleaved passes and keeps its faster
  // time: the replicas are still relaxing while the tuner runs (the Poisson
  // solves get cheaper from step to step), and a single pass in a fixed order
  // would favour whichever candidate comes last.
  constexpr int NT = 3, NG = 3, PASSES = 2;
  const int threads_c[NT] = {256, 512, 1024};
  const int groups_c[NG] = {1, 2, 4};
  double per_c[NT][NG];
  bool fits[NT][NG];
  for (int i = 0; i < NT; ++i)
    for (int j = 0; j < NG; ++j) {
      per_c[i][j] = INFINITY;
      fits[i][j] = true;
    }
  ek_status st = EK_OK;
  for (int pass = 0; pass < PASSES && !st; ++pass)
    for (int i = 0; i < NT && !st; ++i)
      for (int j = 0; j < NG && !st; ++j) {
        if (!fits[i][j]) continue;
        const int cand = threads_c[i], grp = groups_c[j];
        if (pass == 0) {
          st = run_steps(e, 1, cand, grp);    // first launch of a variant: not timed
          if (st == EK_EHIP && grp > 1 && e->err.find("cooperative") != std::string::npos) {
            st = EK_OK;                        // this team size does not fit the device
            fits[i][j] = false;
            continue;
          }
          if (st) break;
        }
        (void)hipEventRecord(a, e->stream);
        st = run_steps(e, steps, cand, grp);
        (void)hipEventRecord(b, e->stream);
        if (st) break;
        (void)hipEventSynchronize(b);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        per_c[i][j] = std::min(per_c[i][j], double(ms) / steps);
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st) return st;
  int best = e->threads, best_group = e->group;
  double best_ms = INFINITY;
  for (int i = 0; i < NT; ++i)
    for (int j = 0; j < NG; ++j)
      if (fits[i][j] && per_c[i][j] < best_ms) {
        best_ms = per_c[i][j];
        best = threads_c[i];
        best_group = groups_c[j];
      }
  e->threads = best;
  e->group = best_group;
  if (out) {
    out->threads = best;
    out->group = best_group;
    out->ms_per_step = best_ms;
  }
  return EK_OK;
}

ek_status ek_ensemble_set_group(ek_ensemble* e, int32_t group) {
  if (!e) return EK_EINVAL;
  if (group != 1 && group != 2 && group != 4) return e->fail(EK_EINVAL, "group must be 1, 2 or 4");
  e->group = group;
  return EK_OK;
}

ek_status ek_ensemble_get_moments(ek_ensemble* e, int32_t r, int32_t species, double* n, double* u) {
  if (!e) return EK_EINVAL;
  if (r < 0 || r >= e->n_rep || species < 0 || species > 2) return e->fail(EK_EINVAL, "bad arguments");
  const RepDev& R = e->reps[r];
  const Dims d = e->d;
  double* scratch = (double*)R.f[R.cur ^ 1];
  if (e->p.precision == EK_FP64)
    launch_moments<double>((const double*)R.f[R.cur], R.mask, species, R.lp.nref[species], scratch,
                           scratch + d.n, d, e->stream);
  else
    launch_moments<float>((const float*)R.f[R.cur], R.mask, species, R.lp.nref[species], scratch,
                          scratch + d.n, d, e->stream);
  if ((n && hipMemcpyAsync(n, scratch, d.n * 8, hipMemcpyDeviceToHost, e->stream) != hipSuccess) ||
      (u && hipMemcpyAsync(u, scratch + d.n, 3 * d.n * 8, hipMemcpyDeviceToHost, e->stream) != hipSuccess) ||
      hipStreamSynchronize(e->stream) != hipSuccess)
    return e->fail(EK_EHIP, "reading moments failed");
  return EK_OK;
}

ek_status ek_ensemble_get_potential(ek_ensemble* e, int32_t r, double* psi) {
  if (!e) return EK_EINVAL;
  if (r < 0 || r >= e->n_rep || !psi) return e->fail(EK_EINVAL, "bad arguments");
  if (hipMemcpyAsync(psi, e->reps[r].psi, e->d.n * 8, hipMemcpyDeviceToHost, e->stream) != hipSuccess ||
      hipStreamSynchronize(e->stream) != hipSuccess)
    return e->fail(EK_EHIP, "reading the potential failed");
  return EK_OK;
}

ek_status ek_ensemble_get_beads(ek_ensemble* e, int32_t r, double* pos, double* vel) {
  if (!e) return EK_EINVAL;
  if (r < 0 || r >= e->n_rep) return e->fail(EK_EINVAL, "bad replica");
  const RepDev& R = e->reps[r];
  if (R.n_beads == 0) return EK_OK;
  if ((pos && hipMemcpyAsync(pos, R.bs.R, R.n_beads * 24, hipMemcpyDeviceToHost, e->stream) != hipSuccess) ||
      (vel && hipMemcpyAsync(vel, R.bs.V, R.n_beads * 24, hipMemcpyDeviceToHost, e->stream) != hipSuccess) ||
      hipStreamSynchronize(e->stream) != hipSuccess)
    return e->fail(EK_EHIP, "reading beads failed");
  return EK_OK;
}

ek_status ek_ensemble_phase_times(ek_ensemble* e, int32_t r, double* ms) {
  if (!e || !ms) return EK_EINVAL;
  if (r < 0 || r >= e->n_rep) return e->fail(EK_EINVAL, "bad replica");
  if (!(e->wall_khz > 0)) return e->fail(EK_EHIP, "the device's wall-clock rate is unknown");
  for (int ph = 0; ph < 4; ++ph) ms[ph] = double(e->reps[r].phase_ticks[ph]) / e->wall_khz;
  return EK_OK;
}

ek_status ek_ensemble_get_stats(ek_ensemble* e, int32_t r, ek_stats* out) {
  if (!e || !out) return EK_EINVAL;
  if (r < 0 || r >= e->n_rep) return e->fail(EK_EINVAL, "bad replica");
  const RepDev& R = e->reps[r];
  std::memset(out, 0, sizeof *out);
  for (int c = 0; c < 3; ++c) {
    out->mass[c] = R.stats[c];
    out->momentum[c] = R.stats[3 + c];
  }
  out->step = R.steps;
  out->poisson_iters = R.last_cycles;
  out->poisson_residual = R.last_res;
  out->poisson_residual0 = R.last_res0;
  return EK_OK;
}

}  // extern "C"
