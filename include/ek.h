/*
 * ek.h - C ABI of the electrokinetic lattice-Boltzmann / MD time step on
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Datar, Fyta, Marini Bettolo Marconi, Melchionna, "Electrokinetic
 * Lattice Boltzmann solver coupled to Molecular Dynamics"):
 *   - a ternary mixture: neutral solvent (species 0), cations (1), anions (2),
 *     point-like, unit masses, valences z^a, uniform permittivity
 *     (Sec. II.A, species and moments);
 *   - D3Q19 kinetic scheme with BGK relaxation towards a second-order
 *     equilibrium (Eq. kernelf), forcing term S (Eq. kernelg) added with the
 *     half-step (Guo) shift, inter-species drag (Eq. Fidef), propagation with
 *     halfway bounce-back on solid walls (Sec. II.C);
 *   - Poisson equation for the potential of ions, wall charges and bead
 *     charges (Eq. poisson), solved by red-black SOR with Chebyshev
 *     acceleration (Sec. II.C) or by red-black multigrid;
 *   - Langevin beads of a bead-spring chain coupled to the species by
 *     friction through a trilinear interpolation / spreading kernel, advanced
 *     with MD substeps (Sec. II.B, Eq. polymermodel);
 *   - the time loop of Fig. 1: moments, charge, Poisson, forces, beads,
 *     collision and propagation.
 *
 * Conventions for every entry point:
 *   - Every function returns ek_status (EK_OK = 0, errors < 0); nothing
 *     throws across the ABI.  ek_last_error() gives a message for the last
 *     failing call on a context (or on the calling thread for ek_create).
 *   - Lattice fields are C-ordered [z][y][x] (x fastest), nz*ny*nx values.
 *     Vector fields are [3][z][y][x] with components (x, y, z).
 *   - Population order p = 0..18: rest, +x, -x, +y, -y, +z, -z, (+x+y),
 *     (-x-y), (+x-y), (-x+y), (+x+z), (-x-z), (+x-z), (-x+z), (+y+z), (-y-z),
 *     (+y-z), (-y+z).
 *   - "host" pointers are ordinary CPU memory owned by the caller and are only
 *     read or written during the call; "device" pointers are GPU memory owned
 *     by the caller.  The library never frees caller memory.
 *   - A context is used by one host thread at a time.  All GPU work is
 *     enqueued on the HIP stream given at creation; calls that return host
 *     data synchronise that stream.
 *   - Units: lattice units, unit spacing, time step, particle mass and proton
 *     charge; k_B T = v_T^2 = 1/3 by default.
 */
#ifndef EK_H
#define EK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EK_OK = 0,
  EK_EINVAL = -1,      /* invalid argument; the context state is unchanged   */
  EK_EHIP = -2,        /* a HIP runtime call failed                           */
  EK_ENOCONV = -3,     /* Poisson solve did not reach its tolerance; the step
                          stops before the collision, the populations stay at
                          the last completed step                              */
  EK_EUNSTABLE = -4,   /* non-finite or negative species mass, a stretched
                          bond or a bead without fluid around it               */
  EK_ESTATE = -5,      /* call out of order (e.g. step before geometry)       */
  EK_ENOMEM = -6       /* workspace too small or allocation failed           */
} ek_status;

enum { EK_FP32 = 0, EK_FP64 = 1 };                 /* population storage type */
enum { EK_POISSON_SOR = 0, EK_POISSON_MG = 1 };    /* Poisson method          */
/* Start of each step's Poisson solve: zero; the previous step's solution
 * (Sec. II.C); the learned guess (see ek_set_model); the linear
 * extrapolation in time 2 psi(t-1) - psi(t-2) of the two previous steps'
 * solutions (the previous solution on the first two steps after
 * ek_set_geometry); or the quadratic one 3 psi(t-1) - 3 psi(t-2) + psi(t-3)
 * (linear on the third step, the previous solution before); or the cubic one
 * 4 psi(t-1) - 6 psi(t-2) + 4 psi(t-3) - psi(t-4) (quadratic on the fourth
 * step, linear on the third, the previous solution before).  The solver
 * finishes every start to the same tolerance. */
enum {
  EK_WS_ZERO = 0,
  EK_WS_PREV = 1,
  EK_WS_LEARNED = 2,
  EK_WS_EXTRAP = 3,
  EK_WS_EXTRAP2 = 4,
  EK_WS_EXTRAP3 = 5
};

/* Problem statement (Sec. II.A-C).  Copied at ek_create. */
typedef struct {
  int32_t nx, ny, nz;          /* lattice size; each even (red-black colouring
                                  of the periodic box); all axes periodic     */
  int32_t precision;           /* EK_FP32 or EK_FP64 populations; the
                                  collision runs in the same type              */
  double valence[3];           /* z^a: solvent, cation, anion                  */
  double tau[3];               /* BGK relaxation time per species (> 1/2),
                                  omega_visc = 1 / tau                         */
  double omega_drag[3];        /* drag rates omega_drag^a of Eq. Fidef         */
  double kT;                   /* k_B T (= v_T^2 of the lattice, 1/3)          */
  double bjerrum;              /* Bjerrum length l_B; eps = 1/(4 pi l_B kT)    */
  double E_ext[3];             /* applied field: force z^a E on ions, q E on
                                  beads                                        */
  double F_ext[3][3];          /* body force per particle [species][xyz]      */
  int32_t poisson_method;      /* EK_POISSON_SOR or EK_POISSON_MG              */
  double poisson_tol;          /* stop when ||b - A psi|| / ||b|| <= tol       */
  int32_t poisson_max_iter;    /* SOR iterations or multigrid cycles           */
  int32_t poisson_check_every; /* residual test every k iterations (>= 1)      */
  double rho_jacobi;           /* Jacobi radius for the Chebyshev schedule;
                                  0 selects (2 + cos(2 pi / max(n))) / 3       */
  int32_t warm_start;          /* EK_WS_ZERO, EK_WS_PREV, EK_WS_LEARNED
                                  (ek_set_model; sizes multiples of 4) or
                                  EK_WS_EXTRAP (one more float64 field in
                                  the workspace), EK_WS_EXTRAP2 (two more)
                                  or EK_WS_EXTRAP3 (three more)           */
  uint64_t seed;               /* key of the thermal noise (64 bits)           */
  int32_t fluctuations;        /* 0: none; 1: thermal fluctuations (Sec. II.A
                                  and II.C): the stochastic term Delta of
                                  Eq. kernelf2 on the populations and the
                                  Langevin noise on the beads (Sec. II.B), at
                                  temperature kT, from the counter-based
                                  generator described below                   */
  int32_t walls;               /* EK_WALLS_PERIODIC: Eq. poisson on the whole
                                  periodic box, wall charges as point charges
                                  on solid sites; EK_WALLS_INSULATING: the
                                  Neumann condition -grad psi . n = Sigma/eps
                                  of insulating walls (see below)             */
} ek_params;

/* Insulating walls (ek_params.walls = EK_WALLS_INSULATING; the boundary
 * condition stated after Eq. poisson): the potential lives on the fluid sites
 * only.  The charge wall_q of a solid site (ek_set_geometry) is its surface
 * charge, divided equally over its faces shared with fluid sites (a charged
 * solid site without such a face is EK_EINVAL); each face's flux Sigma_f/eps
 * enters the balance of the fluid cell it bounds.  The fluid mean of the
 * charge is removed and the fluid mean of psi fixed at 0 (psi is 0 on solid
 * sites); the field at a fluid site is the central difference with
 * psi + Sigma_f/eps in place of a solid face neighbour.  Bead charges are
 * deposited, and the field interpolated at the beads, with the trilinear
 * weights renormalised over the fluid corners.  Needs EK_POISSON_SOR (the
 * paper's red-black SOR, over the fluid sites) and a start other than
 * EK_WS_LEARNED; ek_poisson_solve, ek_poisson_sor_iterations and
 * ek_get_poisson_system, which work on the periodic problem, return
 * EK_ESTATE for such a context; the ensemble refuses it. */
enum { EK_WALLS_PERIODIC = 0, EK_WALLS_INSULATING = 1 };

/* Thermal fluctuations (ek_params.fluctuations = 1).
 * Populations (Sec. II.C): after the collision every fluid site gets, per
 * species a, Delta_p = sqrt(m n^a omega (2 - omega)) w_p sum_{k=4}^{18}
 * chi_kp N_k, where n^a is the site's density before the collision (taken
 * as 0 if negative), omega = 1 / tau^a, m = kT / v_T^2 the thermal mass
 * (v_T^2 = 1/3), and chi_k the D3Q19 mode vectors orthonormal under
 * sum_p w_p chi_kp chi_lp: the polynomials 1; cx, cy, cz; c^2 - 1;
 * 3 cx^2 - c^2; cy^2 - cz^2; cx cy; cy cz; cx cz; (3 c^2 - 5) cx, cy, cz;
 * (cy^2 - cz^2) cx; (cz^2 - cx^2) cy; (cx^2 - cy^2) cz; 3 c^4 - 6 c^2 + 1;
 * (2 c^2 - 3)(3 cx^2 - c^2); (2 c^2 - 3)(cy^2 - cz^2), each divided by its
 * norm.  Delta conserves mass and momentum.
 * Beads (Sec. II.B): each substep h = 1 / n_sub adds xi ~ N(0, 2 gamma kT / h)
 * per component to the friction, shared among the species by their number
 * fractions at the bead (the fluid gets the opposite impulse).
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011) with key (seed mod
 * 2^32, seed div 2^32); word x -> uniform (x + 1/2) / 2^32; words (0, 1) and
 * (2, 3) -> two normals each by Box-Muller, sqrt(-2 ln u1) (cos 2 pi u2,
 * sin 2 pi u2).  N_4..N_18 of species a at site r ((z ny + y) nx + x) in the
 * step that follows t completed steps: the first 15 normals of the counters
 * (r, t, 4 a + j, 0), j = 0..3.  Bead i, step t, substep s: normals 0..2 of
 * counter (i, t, s, 1).  The ensemble runs without fluctuations.
 *
 * ek_philox: the library's device generator for given counters, for callers
 * that reproduce or check the noise: host counters[4 n] (c0..c3 per draw),
 * host words[4 n] (may be NULL) receives the Philox words and host
 * normals[4 n] (may be NULL) the four float64 normals of each draw.  Uses a
 * temporary device buffer; runs on hip_stream and synchronises it.  EK_EINVAL
 * for n < 0, n > 2^24 or NULL counters. */
ek_status ek_philox(const uint32_t* counters, int32_t n, uint64_t seed, uint32_t* words,
                    double* normals, void* hip_stream);

/* Bead-spring chain (Sec. II.B): bonds between chain neighbours, repulsive
 * WCA between bead pairs and between beads and boundary solid sites,
 * friction gamma with the species, n_sub MD substeps per lattice step.
 * Bonds: EK_BOND_FENE, U = -k R0^2 / 2 ln(1 - (r / R0)^2) with the WCA between
 * all pairs; or EK_BOND_HARMONIC, the bonded term of Eq. polymermodel,
 * U = k_bond (r - l_bond)^2 / 2, with the WCA only between beads more than
 * one apart along the chain. */
enum { EK_BOND_FENE = 0, EK_BOND_HARMONIC = 1 };
/* Friction coupling of beads and fluid: the trilinear kernel of Sec. II.C
 * (velocity and composition interpolated, friction spread, with the weights
 * renormalised over the fluid corners), or the occupation cube theta_i of
 * Eq. totalforcefluid: the lattice nodes r with R - sigma/2 < r <= R + sigma/2
 * in every axis, equal weights renormalised over the fluid ones (needs
 * 1 <= sigma <= 2, so that they are corners of the bead's cell).  The bead
 * charge and the field at the bead keep the trilinear weights either way. */
enum { EK_COUPLE_TRILINEAR = 0, EK_COUPLE_THETA = 1 };
typedef struct {
  double M;                    /* bead mass                                    */
  double k_fene, R0;           /* FENE spring constant and maximum extension   */
  double eps, sigma;           /* WCA energy and diameter                      */
  double gamma;                /* friction coefficient                         */
  int32_t n_sub;               /* MD substeps per lattice step (>= 1)          */
  int32_t bond;                /* EK_BOND_FENE or EK_BOND_HARMONIC             */
  double k_bond, l_bond;       /* harmonic spring constant (>= 0) and rest
                                  length (> 0)                                 */
  int32_t coupling;            /* EK_COUPLE_TRILINEAR or EK_COUPLE_THETA       */
} ek_polymer_params;

typedef struct {
  double mass[3];              /* sum of n^a over the lattice (float64)        */
  double momentum[3];          /* total fluid momentum sum_a j^a               */
  int64_t step;                /* completed lattice steps                      */
  int32_t poisson_iters;       /* iterations (or cycles) of the last solve     */
  double poisson_residual;     /* relative residual of the last solve          */
  int32_t fallback;            /* 1 if the last solve consulted the network
                                  and rejected its guess                       */
  int32_t consulted;           /* 1 if the last solve consulted the network    */
  double poisson_residual0;    /* relative residual of the last solve's start  */
} ek_stats;

typedef struct {
  int32_t iterations;          /* SOR iterations or multigrid cycles           */
  double residual;             /* final relative residual (float64)            */
  double initial_residual;     /* relative residual of the warm start          */
} ek_poisson_report;

/* Workspace needed for these parameters and up to max_beads beads (bytes).
 * Returns EK_EINVAL for invalid parameters. */
ek_status ek_workspace_bytes(const ek_params* p, int32_t max_beads, size_t* bytes);

/* Create a context.  dev_ws: device buffer of at least ek_workspace_bytes()
 * bytes that holds all device state (the library then allocates no device
 * memory), or NULL to let the library allocate it.  hip_stream: a
 * hipStream_t (NULL = default stream).  *out receives the context. */
ek_status ek_create(const ek_params* p, int32_t max_beads, void* dev_ws, size_t ws_bytes,
                    void* hip_stream, struct ek_ctx** out);
void ek_destroy(struct ek_ctx* ctx);
const char* ek_last_error(const struct ek_ctx* ctx);

/* Geometry (walls, Sec. II.A): host solid[nz*ny*nx] (0 fluid, 1 solid) and
 * optional host wall_q[nz*ny*nx], the fixed charges of the wall (placed on
 * solid sites; NULL = none).  Resets populations to zero. */
ek_status ek_set_geometry(struct ek_ctx* ctx, const uint8_t* solid, const double* wall_q);

/* Species density at rest: populations f_p = w_p n at every fluid site
 * (host n[nz*ny*nx]; values on solid sites are ignored). */
ek_status ek_set_species_density(struct ek_ctx* ctx, int32_t species, const double* n);

/* Polymer: host pos[3*n] and vel[3*n] (x, y, z per bead, unwrapped
 * coordinates, nodes at integer positions), host charge[n] (NULL = all 0). */
ek_status ek_set_polymer(struct ek_ctx* ctx, int32_t n_beads, const double* pos,
                         const double* vel, const double* charge,
                         const ek_polymer_params* pp);

/* Advance n_steps lattice steps (Fig. 1).  Returns after the stream is
 * synchronised.  On EK_ENOCONV / EK_EUNSTABLE the step in progress is not
 * applied. */
ek_status ek_step(struct ek_ctx* ctx, int32_t n_steps);

/* Density n^a and bare velocity j^a / n^a of the current populations
 * (host outputs, float64; either pointer may be NULL; zero on solid sites). */
ek_status ek_get_moments(struct ek_ctx* ctx, int32_t species, double* n, double* u);

/* Potential of the last solve, mean zero (host psi[nz*ny*nx]). */
ek_status ek_get_potential(struct ek_ctx* ctx, double* psi);

/* Bead positions and velocities (host, 3 doubles per bead). */
ek_status ek_get_beads(struct ek_ctx* ctx, double* pos, double* vel);

/* Pore observables (Sec. IV.B, ionic current and conductance; Sec. IV.C,
 * the time at which each bead passes the pore's mid-plane).
 *
 * ek_plane_flux: particles of each species that the streaming which formed
 * the current densities (those of ek_get_moments) carried across the link
 * plane between z and z + 1 (periodic: z = nz - 1 pairs with 0): populations
 * moving +z count +1, those moving -z count -1, bounced-back links (fluid to
 * solid) carry nothing.  out[0..2]: species 0, 1, 2; out[3]: the charge,
 * sum of valence[a] * out[a], i.e. the ionic current through the plane in
 * charge per time step.  Host output of 4 doubles; EK_EINVAL for z outside
 * [0, nz) or a NULL output; EK_ESTATE before the species are set.  The sums
 * are float64 in a fixed order (deterministic). */
ek_status ek_plane_flux(struct ek_ctx* ctx, int32_t z, double* out);

/* Bead crossing record of the plane z = z_plane (lattice units; its periodic
 * images z_plane + k nz count too).  Setting the plane enables the record and
 * clears it; ek_set_polymer clears it as well, and ek_set_geometry (which
 * restarts the step count) ends it until a plane is set again.  A bead crosses the plane in a
 * step when floor((Z - z_plane) / nz) differs between its z coordinate Z at
 * the start and at the end of the step (both float64).  EK_EINVAL for a
 * non-finite z_plane. */
ek_status ek_set_crossing_plane(struct ek_ctx* ctx, double z_plane);

/* Per bead (host arrays of n_beads int32, any may be NULL): the first and
 * the last step that crossed the plane, counted as the number of steps the
 * context had completed when that step ended (-1: none yet), and the net
 * number of crossings (+1 in +z, -1 in -z).  EK_ESTATE if no plane is set. */
ek_status ek_get_crossings(struct ek_ctx* ctx, int32_t* first, int32_t* last, int32_t* net);

ek_status ek_get_stats(struct ek_ctx* ctx, ek_stats* out);

/* Checkpoint and resume (the time loop of Fig. 1 carries the populations,
 * the potential and the beads from one step to the next; this is not in the
 * paper).  The state holds the geometry (solid mask, wall charges), the
 * current populations, the last Poisson solution (and the one before it with
 * EK_WS_EXTRAP), the chain (parameters, charges, positions, velocities), the
 * crossing plane and record, and the counters the next steps depend on (step
 * count, the previous solve's cycle count, which schedules the next solve's
 * residual tests); a network set with ek_set_model, the launch mode and the
 * timers are not part of it, nor are the ek_params: loading it into a
 * context created with the same ek_params (lattice size, precision and warm
 * start must match, which is checked; max_beads at least the state's chain)
 * and stepping on gives bit for bit the results the saved context would have
 * given, while a context with other physical parameters (field, relaxation
 * times, ...) continues the state under its own.
 *
 * ek_state_bytes: size of the state of the context as it stands (it grows
 *   with the chain).
 * ek_save_state: writes the state into host[bytes]; EK_EINVAL if NULL or
 *   smaller than ek_state_bytes, EK_ESTATE before the geometry and all three
 *   species are set.  Synchronises the stream.
 * ek_load_state: replaces the context's state by host[bytes]; EK_EINVAL (the
 *   context untouched) for a buffer that is not such a state, is truncated,
 *   fails its checksum or belongs to other parameters; EK_EHIP if a copy
 *   fails part way (the context then needs a new geometry or state). */
ek_status ek_state_bytes(struct ek_ctx* ctx, size_t* bytes);
ek_status ek_save_state(struct ek_ctx* ctx, void* host, size_t bytes);
ek_status ek_load_state(struct ek_ctx* ctx, const void* host, size_t bytes);

/* Standalone Poisson solve on device buffers: dev_rho[nz*ny*nx] charge
 * density, dev_psi[nz*ny*nx] warm start on entry and solution (mean zero) on
 * return, both float64.  Uses the context's method, tolerance and iteration
 * limit; warm_start EK_WS_ZERO clears dev_psi first, EK_WS_PREV,
 * EK_WS_EXTRAP, EK_WS_EXTRAP2 and EK_WS_EXTRAP3 start from dev_psi as given (a stand-alone
 * solve has no history to extrapolate), EK_WS_LEARNED consults the network (EK_ESTATE
 * without a model); other values give EK_EINVAL.  The context's own fields
 * (populations, potential) are not touched. */
ek_status ek_poisson_solve(struct ek_ctx* ctx, const double* dev_rho, double* dev_psi,
                           int32_t warm_start, ek_poisson_report* rep);

/* For callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * stand-alone solve of ek_poisson_solve without a context.  p gives the
 * lattice size, bjerrum, kT and the solver settings (poisson_method must be
 * EK_POISSON_SOR: red-black SOR with the Chebyshev schedule, Sec. II.C;
 * poisson_tol, poisson_max_iter, poisson_check_every, rho_jacobi); dev_rho
 * and dev_psi are float64 device buffers of nz*ny*nx values as in
 * ek_poisson_solve (dev_psi: the start on entry unless warm_start is
 * EK_WS_ZERO, the mean-free solution on return); warm_start EK_WS_ZERO,
 * EK_WS_PREV or EK_WS_EXTRAP (the latter two start from dev_psi as given);
 * work is enqueued on hip_stream (a hipStream_t, NULL = default stream),
 * which is synchronised before the call returns; rep may be NULL.  For the
 * same parameters and inputs the result equals ek_poisson_solve's on a
 * context created with them, bit for bit.
 * The solver's scratch (right-hand side, block partial sums, solver scalars)
 * is one static device array of the library, about 18.5 MB on each device
 * the call runs on, held until the process ends: lattices of at most 2^21
 * sites (EK_EINVAL beyond, with a message in ek_last_error(NULL)).  The call
 * allocates nothing (no hipMalloc, hipFree or hipHostMalloc).  Calls that
 * overlap on one device (several host threads or streams) share that array
 * and race.  Errors: EK_EINVAL for invalid parameters or NULL buffers (no
 * work enqueued), EK_ENOCONV when poisson_max_iter iterations do not reach
 * the tolerance (dev_psi then holds the last iterate), EK_EHIP for a failing
 * HIP call; ek_last_error(NULL) gives the message. */
ek_status ek_poisson_solve_noalloc(const ek_params* p, const double* dev_rho, double* dev_psi,
                                   int32_t warm_start, void* hip_stream, ek_poisson_report* rep);

/* Exactly `iterations` red-black SOR iterations (Chebyshev schedule restarted)
 * on A psi = b with no convergence test and no mean removal: dev_b and
 * dev_psi are float64 device buffers; used to compare iterates. */
ek_status ek_poisson_sor_iterations(struct ek_ctx* ctx, const double* dev_b, double* dev_psi,
                                    int32_t iterations);

/* Per-phase GPU time, measured with HIP events for each phase of every step
 * while enabled: the charge pass and the Poisson solve between events
 * recorded around them on the context's stream, the bead update from the end
 * of the solve to the end of the chain kernel, the fused lattice kernel
 * (whose launch count is n_lb) between events stamped at its own start and
 * end.  With the overlap of EK_LAUNCH_OVERLAP the lattice kernel runs while
 * the chain advances and leaves the sites of the bead boxes to a small
 * launch after it; lb_sites counts the fluid sites the timed lattice
 * launches updated.  Used by the benchmark to price kernels against the
 * hardware roofline. */
typedef struct {
  double ms_charge, ms_poisson, ms_md, ms_lb;
  int64_t n_steps;              /* steps measured                               */
  int64_t n_lb;                 /* fused lattice kernel launches measured       */
  int64_t poisson_iters;        /* Poisson iterations (or cycles) summed        */
  int64_t lb_sites;             /* fluid sites updated by those launches        */
} ek_timing;

/* enable != 0 starts (and zeroes) the per-phase timers; 0 stops them. */
ek_status ek_set_timing(struct ek_ctx* ctx, int32_t enable);
ek_status ek_get_timing(struct ek_ctx* ctx, ek_timing* out);

/* Launch modes (flags, both set by default).
 * EK_LAUNCH_GRAPHS: each multigrid V-cycle (EK_POISSON_MG), with or without
 *   its residual test, is recorded once as a HIP graph (on a stream the
 *   library creates; the caller's stream may be the default stream) and
 *   replayed on the context's stream; the graphs are recorded again when the
 *   solve's psi buffer changes.  Without it the same kernels are launched one
 *   by one, in the same order, with bit-identical results.  When recording
 *   fails the context keeps to single launches.
 * EK_LAUNCH_OVERLAP: with a polymer, the fused lattice kernel updates every
 *   site outside the beads' 4x4x4 boxes (the only nodes the friction
 *   reaches) on a second stream of the library's while the chain kernel runs
 *   on the context's stream; the box sites follow in a small launch once
 *   both are done.  Every
 *   site is updated by the same arithmetic either way (bit-identical fields
 *   and beads); only the order of the float64 mass and momentum sums
 *   differs.  Needs nx, ny, nz >= 4, else the kernels run one after the other.
 * A context whose stream the caller is recording itself cannot run a step
 * (the step reads convergence flags back to the host). */
enum { EK_LAUNCH_GRAPHS = 1, EK_LAUNCH_OVERLAP = 2 };
ek_status ek_set_launch_mode(struct ek_ctx* ctx, int32_t flags);

/* ---------------------------------------------------------------------------
 * Learned warm start of the Poisson solve.  The paper solves Eq. poisson
 * iteratively from scratch or from the previous step (Sec. II.C); this library
 * adds a small 3-D convolutional network N that guesses the solution, which
 * the iterative solver then finishes to the same tolerance.  With
 * b' = b - mean(b) and s the RMS of b', the guess is
 *     psi0 = s * out_scale * N(b' / s, solid)
 * (the Poisson equation is linear, so one network serves every charge scale).
 * N: 3x3x3 conv 2->16, ReLU, 2x2x2 average pool, 3x3x3 conv 16->32, ReLU,
 * pool, 3x3x3 conv 32->64, ReLU, 1x1x1 conv 64->32, nearest upsample plus the
 * 32-channel activation, ReLU, 1x1x1 conv 32->16, upsample plus the
 * 16-channel activation, ReLU, 3x3x3 conv 16->1; all convolutions periodic,
 * bfloat16 activations, float32 accumulation on the matrix cores.
 * Parameters: EK_UNET_PARAMS float32 values, per layer in the order above the
 * weights [taps][c_in][c_out] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1) for output
 * site r reading input site r + (dx, dy, dz)) followed by the bias [c_out].
 * Lattice sizes must be multiples of 4.
 * ------------------------------------------------------------------------- */
#define EK_UNET_PARAMS 73137

/* Use a trained network in a context created with warm_start =
 * EK_WS_LEARNED (else EK_ESTATE).  Each solve then evaluates the residual of
 * the previous solution (or of the start passed to ek_poisson_solve); if its
 * relative residual exceeds 1/4 (a cold or abruptly changed right-hand side)
 * the network's guess is evaluated too and the start with the smaller
 * residual is kept (ek_stats.consulted, ek_stats.fallback report which).
 * host params[EK_UNET_PARAMS]; out_scale > 0. */
ek_status ek_set_model(struct ek_ctx* ctx, const float* params, int32_t n, float out_scale);

/* The last solved system: dev_rhs[nz*ny*nx] receives its right-hand side b
 * with the mean removed, dev_psi[nz*ny*nx] its solution (mean zero); float64
 * device buffers, either may be NULL.  EK_ESTATE before the first solve.
 * Training pairs for the network are read this way. */
ek_status ek_get_poisson_system(struct ek_ctx* ctx, double* dev_rhs, double* dev_psi);

/* Stand-alone network on caller-owned device buffers (training and tests). */
typedef struct ek_unet ek_unet;

/* Device workspace for an nx*ny*nz lattice; training != 0 adds the backward
 * activations, the gradient and the Adam moments. */
ek_status ek_unet_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t training,
                                  size_t* bytes);
/* dev_ws as in ek_create (NULL: the library allocates it). */
ek_status ek_unet_create(int32_t nx, int32_t ny, int32_t nz, int32_t training, void* dev_ws,
                         size_t ws_bytes, void* hip_stream, ek_unet** out);
void ek_unet_destroy(ek_unet* net);
const char* ek_unet_last_error(const ek_unet* net);

/* Parameters from host memory; also clears the gradient and Adam moments. */
ek_status ek_unet_set_params(ek_unet* net, const float* params, int32_t n, float out_scale);
ek_status ek_unet_get_params(ek_unet* net, float* params, int32_t n, float* out_scale);

/* dev_guess = s * out_scale * N((dev_b - mean) / s, dev_solid): dev_b and
 * dev_guess float64, dev_solid one byte per site (nonzero = solid). */
ek_status ek_unet_forward(ek_unet* net, const double* dev_b, const uint8_t* dev_solid,
                          double* dev_guess);

/* Forward pass, loss L = mean over sites of (N(...) - target / (s *
 * out_scale))^2 and backward pass; dL/dparams is ADDED to the gradient and L
 * to the loss accumulator.  Enqueued only (no synchronisation). */
ek_status ek_unet_accumulate(ek_unet* net, const double* dev_b, const uint8_t* dev_solid,
                             const double* dev_target);
ek_status ek_unet_get_gradient(ek_unet* net, float* grad, int32_t n);
ek_status ek_unet_zero_gradient(ek_unet* net);

/* One Adam step (Kingma and Ba) with gradient grad_scale * accumulated
 * gradient, which is then cleared.  Enqueued only. */
ek_status ek_unet_adam_step(ek_unet* net, float lr, float beta1, float beta2, float eps,
                            float grad_scale);

/* Mean of the losses accumulated since the last read, and their count;
 * resets the accumulator. */
ek_status ek_unet_read_loss(ek_unet* net, double* mean_loss, int64_t* count);

/* ---------------------------------------------------------------------------
 * Ensemble: uneven replicas of one geometry (translocation replicas with their
 * own salt noise, applied field and chain, Sec. IV.A) advanced together by ONE
 * persistent kernel launch per ek_ensemble_step call: a team of 1, 2 or 4
 * workgroups per replica runs the whole time loop of Fig. 1 for that replica
 * (charge pass, multigrid Poisson solve with its own convergence test, chain
 * substeps, fused lattice step), so replicas with more Poisson cycles or
 * longer chains never hold the others back.  The Poisson method is
 * multigrid, started from the previous solution, or from the extrapolated
 * one when the base warm_start is EK_WS_EXTRAP (other values: the previous
 * solution); all other parameters come from the base ek_params except the
 * applied field.
 * ------------------------------------------------------------------------- */
typedef struct ek_ensemble ek_ensemble;

typedef struct {
  int32_t threads;             /* workgroup size of the persistent kernel      */
  int32_t group;               /* workgroups per replica                       */
  double ms_per_step;          /* measured time per ensemble step              */
} ek_tune_result;

/* Device workspace for n_rep replicas with chains of up to max_beads beads
 * (max_beads <= 64: each chain's node sums live in LDS). */
ek_status ek_ensemble_workspace_bytes(const ek_params* base, int32_t n_rep, int32_t max_beads,
                                      size_t* bytes);
/* base->precision must be EK_FP32 (float64 populations are refused with
 * EK_EINVAL, here and in ek_ensemble_workspace_bytes). */
ek_status ek_ensemble_create(const ek_params* base, int32_t n_rep, int32_t max_beads,
                             void* dev_ws, size_t ws_bytes, void* hip_stream, ek_ensemble** out);
void ek_ensemble_destroy(ek_ensemble* ens);
const char* ek_ensemble_last_error(const ek_ensemble* ens);

/* Shared geometry of all replicas (host arrays as in ek_set_geometry). */
ek_status ek_ensemble_set_geometry(ek_ensemble* ens, const uint8_t* solid, const double* wall_q);

/* Replica r: applied field E_ext[3], host densities n0[3][nz*ny*nx]
 * (solvent, cation, anion; populations at rest), and its chain (n_beads may
 * be 0; pos, vel [3*n_beads], charge [n_beads]; pp as in ek_set_polymer). */
ek_status ek_ensemble_set_replica(ek_ensemble* ens, int32_t r, const double* E_ext,
                                  const double* n0, int32_t n_beads, const double* pos,
                                  const double* vel, const double* charge,
                                  const ek_polymer_params* pp);

/* n_steps steps of every replica in one persistent launch; returns after the
 * stream is synchronised.  EK_ENOCONV if a replica's Poisson solve did not
 * reach the tolerance in poisson_max_iter cycles, EK_EUNSTABLE if a replica's
 * mass became non-finite or its chain failed (ek_ensemble_last_error names
 * the replica). */
ek_status ek_ensemble_step(ek_ensemble* ens, int32_t n_steps);

ek_status ek_ensemble_get_moments(ek_ensemble* ens, int32_t r, int32_t species, double* n,
                                  double* u);
ek_status ek_ensemble_get_potential(ek_ensemble* ens, int32_t r, double* psi);
ek_status ek_ensemble_get_beads(ek_ensemble* ens, int32_t r, double* pos, double* vel);
ek_status ek_ensemble_get_stats(ek_ensemble* ens, int32_t r, ek_stats* out);

/* Time spent by replica r's team in the phases of every step it has taken
 * since the ensemble was created (the persistent kernel's own clock:
 * thread 0 of the team's first workgroup reads the device wall clock at the
 * team barriers that end the phases), in milliseconds: ms[0] the bead deposit
 * and charge pass (Eq. poisson's right-hand side), ms[1] the Poisson solve
 * and gauge, ms[2] the chain (Sec. II.B), ms[3] the fused collide-and-stream
 * (Eq. kernelf2) with its sums.  Host array of 4; reads the values as of the
 * last ek_ensemble_step / ek_ensemble_autotune.  EK_EINVAL for a bad r or a
 * NULL ms; EK_EHIP when the device reports no wall-clock rate. */
ek_status ek_ensemble_phase_times(ek_ensemble* ens, int32_t r, double* ms);

/* Workgroup size of the persistent kernel (256, 512 or 1024). */
ek_status ek_ensemble_set_threads(ek_ensemble* ens, int32_t threads);

/* Workgroups per replica (1, 2 or 4).  With more than one, the replica's
 * site-parallel phases on the finest level (charge pass, finest multigrid
 * level, gauge, collide-and-stream) are split over a team of workgroups of one
 * cooperative launch that meet at barriers; the coarse multigrid levels and
 * the chain run in the team's first workgroup.  Sums are taken per
 * workgroup, then over the team in a fixed order, so results do not depend
 * on timing (but may differ in the last bits between team sizes).  A launch
 * the device cannot make co-resident is refused with EK_EHIP. */
ek_status ek_ensemble_set_group(ek_ensemble* ens, int32_t group);

/* Autotuner: times `steps` ensemble steps with every candidate workgroup size
 * and team size, in two interleaved passes over the candidates, each keeping
 * its faster pass (the replicas advance by 1 + 2 `steps` steps per candidate,
 * like a warm-up; team sizes the device refuses are skipped), and keeps the
 * fastest; *out (may be NULL) receives the choice and its time. */
ek_status ek_ensemble_autotune(ek_ensemble* ens, int32_t steps, ek_tune_result* out);

#ifdef __cplusplus
}
#endif
#endif /* EK_H */
