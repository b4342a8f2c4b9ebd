"""Python binding of the C ABI in include/ek.h (ctypes).

Only argument marshalling lives here: every step of the method runs in the
HIP kernels of libek.so.  PyTorch supplies the device workspace (a uint8 CUDA
tensor) and the HIP stream.  If libek.so is missing the import fails; there is
no CPU fallback.
"""
import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_uint64, c_void_p, c_size_t

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libek.so")

EK_OK, EK_EINVAL, EK_EHIP, EK_ENOCONV, EK_EUNSTABLE, EK_ESTATE, EK_ENOMEM = 0, -1, -2, -3, -4, -5, -6
EK_FP32, EK_FP64 = 0, 1
EK_POISSON_SOR, EK_POISSON_MG = 0, 1
EK_LAUNCH_GRAPHS, EK_LAUNCH_OVERLAP = 1, 2
EK_WS_ZERO, EK_WS_PREV, EK_WS_LEARNED, EK_WS_EXTRAP, EK_WS_EXTRAP2, EK_WS_EXTRAP3 = 0, 1, 2, 3, 4, 5

_STATUS = {0: "EK_OK", -1: "EK_EINVAL", -2: "EK_EHIP", -3: "EK_ENOCONV", -4: "EK_EUNSTABLE",
           -5: "EK_ESTATE", -6: "EK_ENOMEM"}


class ek_params(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("precision", c_int32),
                ("valence", c_double * 3), ("tau", c_double * 3), ("omega_drag", c_double * 3),
                ("kT", c_double), ("bjerrum", c_double), ("E_ext", c_double * 3),
                ("F_ext", (c_double * 3) * 3), ("poisson_method", c_int32),
                ("poisson_tol", c_double), ("poisson_max_iter", c_int32),
                ("poisson_check_every", c_int32), ("rho_jacobi", c_double),
                ("warm_start", c_int32), ("seed", c_uint64), ("fluctuations", c_int32),
                ("walls", c_int32)]


class ek_polymer_params(ctypes.Structure):
    _fields_ = [("M", c_double), ("k_fene", c_double), ("R0", c_double), ("eps", c_double),
                ("sigma", c_double), ("gamma", c_double), ("n_sub", c_int32), ("bond", c_int32),
                ("k_bond", c_double), ("l_bond", c_double), ("coupling", c_int32)]


EK_BOND_FENE, EK_BOND_HARMONIC = 0, 1
EK_COUPLE_TRILINEAR, EK_COUPLE_THETA = 0, 1
EK_WALLS_PERIODIC, EK_WALLS_INSULATING = 0, 1


def _coupling_code(coupling):
    return {"trilinear": EK_COUPLE_TRILINEAR, "theta": EK_COUPLE_THETA}.get(coupling, coupling)


def _bond_code(bond):
    return {"fene": EK_BOND_FENE, "harmonic": EK_BOND_HARMONIC}.get(bond, bond)


class ek_stats(ctypes.Structure):
    _fields_ = [("mass", c_double * 3), ("momentum", c_double * 3), ("step", c_int64),
                ("poisson_iters", c_int32), ("poisson_residual", c_double), ("fallback", c_int32),
                ("consulted", c_int32), ("poisson_residual0", c_double)]


class ek_timing(ctypes.Structure):
    _fields_ = [("ms_charge", c_double), ("ms_poisson", c_double), ("ms_md", c_double),
                ("ms_lb", c_double), ("n_steps", c_int64), ("n_lb", c_int64),
                ("poisson_iters", c_int64), ("lb_sites", c_int64)]


class ek_tune_result(ctypes.Structure):
    _fields_ = [("threads", c_int32), ("group", c_int32), ("ms_per_step", c_double)]


class ek_poisson_report(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("residual", c_double), ("initial_residual", c_double)]


class EKError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1710_09421_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER
    sig = {
        "ek_workspace_bytes": (c_int32, [P(ek_params), c_int32, P(c_size_t)]),
        "ek_create": (c_int32, [P(ek_params), c_int32, c_void_p, c_size_t, c_void_p, P(c_void_p)]),
        "ek_destroy": (None, [c_void_p]),
        "ek_last_error": (ctypes.c_char_p, [c_void_p]),
        "ek_set_geometry": (c_int32, [c_void_p, c_void_p, c_void_p]),
        "ek_set_species_density": (c_int32, [c_void_p, c_int32, c_void_p]),
        "ek_set_polymer": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                     P(ek_polymer_params)]),
        "ek_step": (c_int32, [c_void_p, c_int32]),
        "ek_get_moments": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
        "ek_get_potential": (c_int32, [c_void_p, c_void_p]),
        "ek_get_beads": (c_int32, [c_void_p, c_void_p, c_void_p]),
        "ek_plane_flux": (c_int32, [c_void_p, c_int32, c_void_p]),
        "ek_set_crossing_plane": (c_int32, [c_void_p, ctypes.c_double]),
        "ek_get_crossings": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "ek_get_stats": (c_int32, [c_void_p, P(ek_stats)]),
        "ek_philox": (c_int32, [c_void_p, c_int32, ctypes.c_uint64, c_void_p, c_void_p, c_void_p]),
        "ek_state_bytes": (c_int32, [c_void_p, P(c_size_t)]),
        "ek_save_state": (c_int32, [c_void_p, c_void_p, c_size_t]),
        "ek_load_state": (c_int32, [c_void_p, c_void_p, c_size_t]),
        "ek_poisson_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, P(ek_poisson_report)]),
        "ek_poisson_sor_iterations": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32]),
        "ek_poisson_solve_noalloc": (c_int32, [P(ek_params), c_void_p, c_void_p, c_int32, c_void_p,
                                               P(ek_poisson_report)]),
        "ek_set_timing": (c_int32, [c_void_p, c_int32]),
        "ek_set_launch_mode": (c_int32, [c_void_p, c_int32]),
        "ek_get_timing": (c_int32, [c_void_p, P(ek_timing)]),
        "ek_set_model": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.c_float]),
        "ek_get_poisson_system": (c_int32, [c_void_p, c_void_p, c_void_p]),
        "ek_unet_workspace_bytes": (c_int32, [c_int32, c_int32, c_int32, c_int32, P(c_size_t)]),
        "ek_unet_create": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_size_t,
                                     c_void_p, P(c_void_p)]),
        "ek_unet_destroy": (None, [c_void_p]),
        "ek_unet_last_error": (ctypes.c_char_p, [c_void_p]),
        "ek_unet_set_params": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.c_float]),
        "ek_unet_get_params": (c_int32, [c_void_p, c_void_p, c_int32, P(ctypes.c_float)]),
        "ek_unet_forward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "ek_unet_accumulate": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "ek_unet_get_gradient": (c_int32, [c_void_p, c_void_p, c_int32]),
        "ek_unet_zero_gradient": (c_int32, [c_void_p]),
        "ek_unet_adam_step": (c_int32, [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, ctypes.c_float]),
        "ek_unet_read_loss": (c_int32, [c_void_p, P(ctypes.c_double), P(ctypes.c_int64)]),
        "ek_ensemble_workspace_bytes": (c_int32, [P(ek_params), c_int32, c_int32, P(c_size_t)]),
        "ek_ensemble_create": (c_int32, [P(ek_params), c_int32, c_int32, c_void_p, c_size_t, c_void_p,
                                         P(c_void_p)]),
        "ek_ensemble_destroy": (None, [c_void_p]),
        "ek_ensemble_last_error": (ctypes.c_char_p, [c_void_p]),
        "ek_ensemble_set_geometry": (c_int32, [c_void_p, c_void_p, c_void_p]),
        "ek_ensemble_set_replica": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                              c_void_p, c_void_p, P(ek_polymer_params)]),
        "ek_ensemble_step": (c_int32, [c_void_p, c_int32]),
        "ek_ensemble_get_moments": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
        "ek_ensemble_get_potential": (c_int32, [c_void_p, c_int32, c_void_p]),
        "ek_ensemble_get_beads": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
        "ek_ensemble_get_stats": (c_int32, [c_void_p, c_int32, P(ek_stats)]),
        "ek_ensemble_set_threads": (c_int32, [c_void_p, c_int32]),
        "ek_ensemble_autotune": (c_int32, [c_void_p, c_int32, P(ek_tune_result)]),
        "ek_ensemble_phase_times": (c_int32, [c_void_p, c_int32, c_void_p]),
        "ek_ensemble_set_group": (c_int32, [c_void_p, c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _ptr(a):
    return a.ctypes.data_as(c_void_p)


def poisson_solve_noalloc(params, rho, psi, warm_start=EK_WS_PREV, stream=None):
    """ek_poisson_solve_noalloc: rho, psi float64 CUDA tensors of the lattice
    shape (psi updated in place); no context, nothing allocated."""
    import torch
    lib_ = lib()
    s = stream if stream is not None else torch.cuda.current_stream()
    rep = ek_poisson_report()
    st = lib_.ek_poisson_solve_noalloc(byref(params), c_void_p(rho.data_ptr()),
                                       c_void_p(psi.data_ptr()), warm_start,
                                       c_void_p(s.cuda_stream), byref(rep))
    if st != EK_OK:
        msg = lib_.ek_last_error(None)
        raise EKError(st, msg.decode() if msg else "")
    return dict(iterations=rep.iterations, residual=rep.residual,
                initial_residual=rep.initial_residual)


def philox(counters, seed, stream=None):
    """ek_philox: the device generator's words and float64 normals for
    counters [n, 4] (uint32) under the 64-bit seed."""
    import torch
    lib_ = lib()
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    words = np.empty_like(c)
    z = np.empty(c.shape, dtype=np.float64)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib_.ek_philox(_ptr(c), c.shape[0], int(seed), _ptr(words), _ptr(z),
                        c_void_p(s.cuda_stream))
    if st != EK_OK:
        msg = lib_.ek_last_error(None)
        raise EKError(st, msg.decode() if msg else "")
    return words, z


def make_params(shape, precision=EK_FP32, valence=(0.0, 1.0, -1.0), tau=(1.0, 1.0, 1.0),
                omega_drag=(1.0, 1.0, 1.0), kT=1.0 / 3.0, bjerrum=0.7, E_ext=(0.0, 0.0, 0.0),
                F_ext=None, poisson_method=EK_POISSON_SOR, poisson_tol=1e-8,
                poisson_max_iter=100000, poisson_check_every=1, rho_jacobi=0.0,
                warm_start=EK_WS_PREV, fluctuations=0, seed=0, walls=EK_WALLS_PERIODIC):
    nz, ny, nx = shape
    p = ek_params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.precision = precision
    for s in range(3):
        p.valence[s] = valence[s]
        p.tau[s] = tau[s]
        p.omega_drag[s] = omega_drag[s]
        p.E_ext[s] = E_ext[s]
        for c in range(3):
            p.F_ext[s][c] = 0.0 if F_ext is None else float(F_ext[s][c])
    p.kT, p.bjerrum = kT, bjerrum
    p.poisson_method, p.poisson_tol = poisson_method, poisson_tol
    p.poisson_max_iter, p.poisson_check_every = poisson_max_iter, poisson_check_every
    p.rho_jacobi, p.warm_start = rho_jacobi, warm_start
    p.seed, p.fluctuations = int(seed), int(fluctuations)
    p.walls = {"periodic": EK_WALLS_PERIODIC, "insulating": EK_WALLS_INSULATING}.get(walls, walls)
    return p


class Context:
    """One simulation context on the current CUDA (HIP) device and stream."""

    def __init__(self, params, max_beads=0, stream=None):
        import torch
        self._lib = lib()
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        nbytes = c_size_t()
        self._check(self._lib.ek_workspace_bytes(byref(params), max_beads, byref(nbytes)), None)
        # 256-byte alignment: over-allocate and offset
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        self._check(self._lib.ek_create(byref(params), max_beads, c_void_p(base + off),
                                        nbytes.value, c_void_p(self.stream.cuda_stream),
                                        byref(h)), None)
        self._h = h

    def _check(self, st, h):
        if st != EK_OK:
            msg = self._lib.ek_last_error(h)
            raise EKError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ek_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ---------------------------------------------------------------
    def set_geometry(self, solid, wall_q=None):
        s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        w = None if wall_q is None else np.ascontiguousarray(wall_q, dtype=np.float64).reshape(self.shape)
        self._check(self._lib.ek_set_geometry(self._h, _ptr(s), None if w is None else _ptr(w)), self._h)

    def set_species_density(self, species, n):
        a = np.ascontiguousarray(n, dtype=np.float64).reshape(self.shape)
        self._check(self._lib.ek_set_species_density(self._h, species, _ptr(a)), self._h)

    def set_polymer(self, pos, vel, charge, M=1.0, k_fene=30.0, R0=1.5, eps=1.0, sigma=1.0,
                    gamma=20.0, n_sub=40, bond="fene", k_bond=0.0, l_bond=0.0,
                    coupling="trilinear"):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        q = np.ascontiguousarray(charge, dtype=np.float64)
        pp = ek_polymer_params(M, k_fene, R0, eps, sigma, gamma, n_sub, _bond_code(bond), k_bond,
                               l_bond, _coupling_code(coupling))
        self._check(self._lib.ek_set_polymer(self._h, pos.shape[0], _ptr(pos), _ptr(vel), _ptr(q),
                                             byref(pp)), self._h)

    # -- run -----------------------------------------------------------------
    def step(self, n=1):
        self._check(self._lib.ek_step(self._h, n), self._h)

    # -- outputs -------------------------------------------------------------
    def moments(self, species):
        n = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        self._check(self._lib.ek_get_moments(self._h, species, _ptr(n), _ptr(u)), self._h)
        return n, u

    def potential(self):
        psi = np.empty(self.shape)
        self._check(self._lib.ek_get_potential(self._h, _ptr(psi)), self._h)
        return psi

    def beads(self, n_beads):
        pos = np.empty((n_beads, 3))
        vel = np.empty((n_beads, 3))
        self._check(self._lib.ek_get_beads(self._h, _ptr(pos), _ptr(vel)), self._h)
        return pos, vel

    def plane_flux(self, z):
        """Particles of species 0, 1, 2 carried across the link plane between z
        and z + 1 by the streaming that formed the current densities, and the
        charge they carry (the ionic current in charge per step)."""
        out = np.empty(4)
        self._check(self._lib.ek_plane_flux(self._h, int(z), _ptr(out)), self._h)
        return out

    def set_crossing_plane(self, z_plane):
        self._check(self._lib.ek_set_crossing_plane(self._h, float(z_plane)), self._h)

    def crossings(self, n_beads):
        """Per bead: first and last step that crossed the plane (-1: none) and
        the net crossing count (+1 per crossing in +z)."""
        rec = np.empty((3, n_beads), dtype=np.int32)
        self._check(self._lib.ek_get_crossings(self._h, _ptr(rec[0]), _ptr(rec[1]), _ptr(rec[2])),
                    self._h)
        return rec[0], rec[1], rec[2]

    def stats(self):
        s = ek_stats()
        self._check(self._lib.ek_get_stats(self._h, byref(s)), self._h)
        return dict(mass=np.array(s.mass[:]), momentum=np.array(s.momentum[:]), step=s.step,
                    poisson_iters=s.poisson_iters, poisson_residual=s.poisson_residual,
                    poisson_residual0=s.poisson_residual0, fallback=s.fallback,
                    consulted=s.consulted)

    def state_bytes(self):
        nbytes = c_size_t()
        self._check(self._lib.ek_state_bytes(self._h, byref(nbytes)), self._h)
        return nbytes.value

    def save_state(self):
        """The context's state (ek_save_state) as a numpy uint8 array."""
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        self._check(self._lib.ek_save_state(self._h, _ptr(buf), buf.size), self._h)
        return buf

    def load_state(self, buf):
        a = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._lib.ek_load_state(self._h, _ptr(a), a.size), self._h)

    def set_timing(self, enable=True):
        self._check(self._lib.ek_set_timing(self._h, 1 if enable else 0), self._h)

    def set_launch_mode(self, graphs=True, overlap=True):
        flags = (EK_LAUNCH_GRAPHS if graphs else 0) | (EK_LAUNCH_OVERLAP if overlap else 0)
        self._check(self._lib.ek_set_launch_mode(self._h, flags), self._h)

    def timing(self):
        t = ek_timing()
        self._check(self._lib.ek_get_timing(self._h, byref(t)), self._h)
        return {k: getattr(t, k) for k, _ in ek_timing._fields_}

    def poisson_solve(self, rho, psi, warm_start=EK_WS_PREV):
        """rho, psi: float64 CUDA tensors of the lattice shape (psi updated in place)."""
        rep = ek_poisson_report()
        self._check(self._lib.ek_poisson_solve(self._h, c_void_p(rho.data_ptr()),
                                               c_void_p(psi.data_ptr()), warm_start, byref(rep)),
                    self._h)
        return dict(iterations=rep.iterations, residual=rep.residual,
                    initial_residual=rep.initial_residual)

    def set_model(self, params, out_scale):
        """Trained network parameters (EK_UNET_PARAMS floats) for the learned warm start."""
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._lib.ek_set_model(self._h, _ptr(a), a.size, float(out_scale)), self._h)

    def poisson_system(self, rhs, psi):
        """Copy the last solved system into float64 CUDA tensors: rhs (mean removed), psi."""
        self._check(self._lib.ek_get_poisson_system(
            self._h, None if rhs is None else c_void_p(rhs.data_ptr()),
            None if psi is None else c_void_p(psi.data_ptr())), self._h)

    def sor_iterations(self, b, psi, iterations):
        self._check(self._lib.ek_poisson_sor_iterations(self._h, c_void_p(b.data_ptr()),
                                                        c_void_p(psi.data_ptr()), iterations),
                    self._h)


def from_workload(wl, precision=EK_FP32, poisson_method=EK_POISSON_SOR, poisson_tol=None,
                  poisson_check_every=1, warm_start=EK_WS_PREV, **kw):
    """Context initialised with a workload's geometry, densities and polymer."""
    nb = 0 if wl.beads_R is None else wl.beads_R.shape[0]
    p = make_params(wl.shape, precision=precision, valence=wl.valence, tau=wl.tau,
                    omega_drag=wl.omega_drag, bjerrum=wl.bjerrum, E_ext=wl.E_ext,
                    poisson_method=poisson_method,
                    poisson_tol=wl.poisson_tol if poisson_tol is None else poisson_tol,
                    poisson_check_every=poisson_check_every, warm_start=warm_start, **kw)
    ctx = Context(p, max_beads=nb)
    ctx.set_geometry(wl.solid, wl.wall_q)
    for s in range(3):
        ctx.set_species_density(s, wl.n0[s])
    if nb:
        pp = wl.polymer
        ctx.set_polymer(wl.beads_R, wl.beads_V, pp["q"], M=pp["M"], k_fene=pp["k_fene"],
                        R0=pp["R0"], eps=pp["eps"], sigma=pp["sigma"], gamma=pp["gamma"],
                        n_sub=pp["n_sub"], bond=pp.get("bond", "fene"), k_bond=pp.get("k_bond", 0.0),
                        coupling=pp.get("coupling", "trilinear"),
                        l_bond=pp.get("l_bond", 0.0))
    return ctx


class Ensemble:
    """Replicas of one geometry advanced by one persistent launch per step call."""

    def __init__(self, params, n_rep, max_beads=0, stream=None):
        import torch
        self._lib = lib()
        self.params = params
        self.n_rep = n_rep
        self.shape = (params.nz, params.ny, params.nx)
        self.n_beads = [0] * n_rep
        nbytes = c_size_t()
        self._check(self._lib.ek_ensemble_workspace_bytes(byref(params), n_rep, max_beads,
                                                          byref(nbytes)), None)
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        self._check(self._lib.ek_ensemble_create(byref(params), n_rep, max_beads,
                                                 c_void_p(base + off), nbytes.value,
                                                 c_void_p(self.stream.cuda_stream), byref(h)), None)
        self._h = h

    def _check(self, st, h):
        if st != EK_OK:
            msg = self._lib.ek_ensemble_last_error(h)
            raise EKError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ek_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, solid, wall_q=None):
        s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        w = None if wall_q is None else np.ascontiguousarray(wall_q, dtype=np.float64).reshape(self.shape)
        self._check(self._lib.ek_ensemble_set_geometry(self._h, _ptr(s), None if w is None else _ptr(w)),
                    self._h)

    def set_replica(self, r, E_ext, n0, pos=None, vel=None, charge=None, M=1.0, k_fene=30.0, R0=1.5,
                    eps=1.0, sigma=1.0, gamma=20.0, n_sub=40, bond="fene", k_bond=0.0, l_bond=0.0,
                    coupling="trilinear"):
        E = np.ascontiguousarray(E_ext, dtype=np.float64)
        n = np.ascontiguousarray(n0, dtype=np.float64).reshape((3,) + self.shape)
        nb = 0 if pos is None else int(np.asarray(pos).shape[0])
        args = [None, None, None, None]
        if nb:
            pos = np.ascontiguousarray(pos, dtype=np.float64)
            vel = np.ascontiguousarray(vel, dtype=np.float64)
            q = np.ascontiguousarray(charge, dtype=np.float64)
            pp = ek_polymer_params(M, k_fene, R0, eps, sigma, gamma, n_sub, _bond_code(bond),
                                   k_bond, l_bond, _coupling_code(coupling))
            args = [_ptr(pos), _ptr(vel), _ptr(q), byref(pp)]
        self._check(self._lib.ek_ensemble_set_replica(self._h, r, _ptr(E), _ptr(n), nb, *args),
                    self._h)
        self.n_beads[r] = nb

    def step(self, n=1):
        self._check(self._lib.ek_ensemble_step(self._h, n), self._h)

    def set_threads(self, threads):
        self._check(self._lib.ek_ensemble_set_threads(self._h, threads), self._h)

    def set_group(self, group):
        """Workgroups per replica (1, 2 or 4)."""
        self._check(self._lib.ek_ensemble_set_group(self._h, group), self._h)

    def autotune(self, steps=2):
        res = ek_tune_result()
        self._check(self._lib.ek_ensemble_autotune(self._h, steps, byref(res)), self._h)
        return dict(threads=res.threads, group=res.group, ms_per_step=res.ms_per_step)

    def moments(self, r, species):
        n = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        self._check(self._lib.ek_ensemble_get_moments(self._h, r, species, _ptr(n), _ptr(u)), self._h)
        return n, u

    def potential(self, r):
        psi = np.empty(self.shape)
        self._check(self._lib.ek_ensemble_get_potential(self._h, r, _ptr(psi)), self._h)
        return psi

    def beads(self, r):
        nb = self.n_beads[r]
        pos = np.empty((nb, 3))
        vel = np.empty((nb, 3))
        if nb:
            self._check(self._lib.ek_ensemble_get_beads(self._h, r, _ptr(pos), _ptr(vel)), self._h)
        return pos, vel

    def phase_times(self, r):
        """ek_ensemble_phase_times: ms spent by replica r's team in the charge
        pass, the Poisson solve, the chain and the collide-and-stream of all
        its steps so far."""
        ms = np.empty(4)
        self._check(self._lib.ek_ensemble_phase_times(self._h, r, _ptr(ms)), self._h)
        return dict(charge=ms[0], poisson=ms[1], chain=ms[2], lb=ms[3])

    def stats(self, r):
        s = ek_stats()
        self._check(self._lib.ek_ensemble_get_stats(self._h, r, byref(s)), self._h)
        return dict(mass=np.array(s.mass[:]), momentum=np.array(s.momentum[:]), step=s.step,
                    poisson_iters=s.poisson_iters, poisson_residual=s.poisson_residual)


def ensemble_from_workloads(wls, precision=EK_FP32, poisson_tol=1e-8, poisson_max_iter=200,
                            max_beads=None, warm_start=EK_WS_PREV):
    """Ensemble whose replicas are the given workloads (same geometry)."""
    w0 = wls[0]
    for w in wls:
        assert w.shape == w0.shape and np.array_equal(w.solid, w0.solid), "replicas share the geometry"
    nb = [0 if w.beads_R is None else w.beads_R.shape[0] for w in wls]
    p = make_params(w0.shape, precision=precision, valence=w0.valence, tau=w0.tau,
                    omega_drag=w0.omega_drag, bjerrum=w0.bjerrum, poisson_method=EK_POISSON_MG,
                    poisson_tol=poisson_tol, poisson_max_iter=poisson_max_iter,
                    warm_start=warm_start)
    ens = Ensemble(p, len(wls), max_beads=max(nb) if max_beads is None else max_beads)
    ens.set_geometry(w0.solid, w0.wall_q)
    for r, w in enumerate(wls):
        if nb[r]:
            pp = w.polymer
            ens.set_replica(r, w.E_ext, w.n0, w.beads_R, w.beads_V, pp["q"], M=pp["M"],
                            k_fene=pp["k_fene"], R0=pp["R0"], eps=pp["eps"], sigma=pp["sigma"],
                            gamma=pp["gamma"], n_sub=pp["n_sub"], bond=pp.get("bond", "fene"),
                            k_bond=pp.get("k_bond", 0.0), l_bond=pp.get("l_bond", 0.0),
                            coupling=pp.get("coupling", "trilinear"))
        else:
            ens.set_replica(r, w.E_ext, w.n0)
    return ens


UNET_PARAMS = 73137


class UNet:
    """Stand-alone warm-start network on the current device and stream; all
    field arguments are CUDA tensors of the lattice shape (b, target float64,
    solid uint8)."""

    def __init__(self, shape, training=True, stream=None):
        import torch
        self._lib = lib()
        self.shape = tuple(shape)
        nz, ny, nx = self.shape
        nbytes = c_size_t()
        self._check(self._lib.ek_unet_workspace_bytes(nx, ny, nz, int(training), byref(nbytes)), None)
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        self._check(self._lib.ek_unet_create(nx, ny, nz, int(training), c_void_p(base + off),
                                             nbytes.value, c_void_p(self.stream.cuda_stream),
                                             byref(h)), None)
        self._h = h

    def _check(self, st, h):
        if st != EK_OK:
            msg = self._lib.ek_unet_last_error(h)
            raise EKError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ek_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, out_scale=1.0):
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._lib.ek_unet_set_params(self._h, _ptr(a), a.size, float(out_scale)), self._h)

    def params(self):
        a = np.empty(UNET_PARAMS, dtype=np.float32)
        sc = ctypes.c_float()
        self._check(self._lib.ek_unet_get_params(self._h, _ptr(a), a.size, byref(sc)), self._h)
        return a, sc.value

    def forward(self, b, solid, guess):
        self._check(self._lib.ek_unet_forward(self._h, c_void_p(b.data_ptr()),
                                              c_void_p(solid.data_ptr()),
                                              c_void_p(guess.data_ptr())), self._h)

    def accumulate(self, b, solid, target):
        self._check(self._lib.ek_unet_accumulate(self._h, c_void_p(b.data_ptr()),
                                                 c_void_p(solid.data_ptr()),
                                                 c_void_p(target.data_ptr())), self._h)

    def gradient(self):
        a = np.empty(UNET_PARAMS, dtype=np.float32)
        self._check(self._lib.ek_unet_get_gradient(self._h, _ptr(a), a.size), self._h)
        return a

    def zero_gradient(self):
        self._check(self._lib.ek_unet_zero_gradient(self._h), self._h)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        self._check(self._lib.ek_unet_adam_step(self._h, lr, beta1, beta2, eps, grad_scale), self._h)

    def read_loss(self):
        m = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self._lib.ek_unet_read_loss(self._h, byref(m), byref(n)), self._h)
        return m.value, n.value
