"""One time step of the electrokinetic LB-MD scheme, in the order of the
algorithm sketched in Fig. 1 and described at the end of Sec. II.C:

  moments -> charge density -> Poisson -> forces -> interpolate the fluid to
  the beads -> advance the beads (n_sub MD substeps) -> spread the bead forces
  back -> collide (with the stochastic term when fluctuations are on) ->
  propagate.

State kept between steps: pre-collision populations f(t) [3, 19, Z, Y, X],
the potential of the last solve (warm start of the next one), bead positions
and velocities.  Everything is float64.

Units (reading of Sec. II.C): lattice units with unit spacing, time step,
particle mass and proton charge; k_B T = m v_T^2 = 1/3; the permittivity
follows from the Bjerrum length, eps = 1 / (4 pi l_B k_B T).
"""
from dataclasses import dataclass, field

import numpy as np

from . import lb, md, noise, poisson
from . import d3q19 as L


@dataclass
class Params:
    valence: tuple = (0.0, 1.0, -1.0)            # z^a of solvent, cation, anion
    tau: tuple = (1.0, 1.0, 1.0)                 # BGK relaxation times, omega_visc = 1 / tau
    omega_drag: tuple = (1.0, 1.0, 1.0)          # drag rates of Eq. Fidef
    kT: float = L.VT2                            # k_B T = m v_T^2
    bjerrum: float = 0.7                         # Bjerrum length in lattice units
    E_ext: tuple = (0.0, 0.0, 0.0)               # applied field
    F_ext: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))  # body force per particle [species, xyz]
    poisson_tol: float = 1e-10
    poisson_max_iter: int = 100000
    rho_j: float = None                          # Jacobi radius for the Chebyshev schedule
    fluctuations: bool = False                   # thermal noise on populations and beads
    walls: str = "periodic"                      # Poisson domain: "periodic" whole box with
                                                 # wall charges on solid sites, or "neumann":
                                                 # insulating walls (fluid sites only)
    seed: int = 0                                # key of the counter-based generator

    @property
    def eps(self):
        return 1.0 / (4.0 * np.pi * self.bjerrum * self.kT)


def polymer_params(n_beads, q=-1.0, M=1.0, k_fene=30.0, R0=1.5, eps=1.0, sigma=1.0,
                   gamma=20.0, n_sub=40, bond="fene", k_bond=0.0, l_bond=0.0,
                   coupling="trilinear"):
    """bond "fene" (k_fene, R0) or "harmonic" (k_bond, l_bond: Eq. polymermodel);
    coupling "trilinear" or "theta" (the occupation cube of Eq. totalforcefluid)."""
    return dict(M=M, q=np.full(n_beads, q, dtype=np.float64), k_fene=k_fene, R0=R0,
                eps=eps, sigma=sigma, gamma=gamma, n_sub=n_sub, bond=bond, k_bond=k_bond,
                l_bond=l_bond, coupling=coupling)


class Simulation:
    """Plain float64 reference of the method on a periodic box.

    solid: bool [Z, Y, X]; wall_q: float [Z, Y, X] fixed charges (on
    boundary solid sites); n0: [3, Z, Y, X] initial species densities (zero on
    solid sites); beads: optional (R [N, 3], V [N, 3], polymer dict).
    """

    def __init__(self, params, solid, wall_q, n0, beads=None):
        self.p = params
        self.solid = np.asarray(solid, dtype=bool)
        self.fluid = ~self.solid
        self.wall_q = np.asarray(wall_q, dtype=np.float64)
        self.shape = self.solid.shape
        self.f = lb.init_equilibrium(np.asarray(n0, dtype=np.float64), self.solid)
        self.psi = np.zeros(self.shape)
        self.t = 0
        self.last_iters = 0
        self.last_residual = 0.0
        if beads is not None:
            R, V, poly = beads
            self.R = np.array(R, dtype=np.float64)
            self.V = np.array(V, dtype=np.float64)
            self.poly = poly
            self.walls = md.wall_sites(self.solid)
        else:
            self.R = None

    # -- pieces of one step -------------------------------------------------
    @property
    def neumann(self):
        return self.p.walls == "neumann"

    def charge_density(self, n):
        """Charge of ions and beads, plus the wall charges on solid sites for
        the periodic whole-box problem (insulating walls carry theirs as the
        surface flux of their faces, poisson.neumann_rhs)."""
        z = np.asarray(self.p.valence, dtype=np.float64)
        rho = np.einsum("s,szyx->zyx", z, n)
        if not self.neumann:
            rho = rho + self.wall_q
        if self.R is not None:
            rho = rho + md.deposit_charge(self.R, self.poly["q"], self.shape,
                                          fluid=self.fluid if self.neumann else None)
        return rho

    def solve_potential(self, rho_e):
        if self.neumann:
            b = poisson.neumann_rhs(rho_e, self.wall_q, self.solid, self.p.eps)
            psi, it, rr = poisson.sor_neumann(b, self.psi, self.fluid, self.p.poisson_tol,
                                              self.p.poisson_max_iter, self.p.rho_j)
        else:
            b = poisson.rhs_from_charge(rho_e, self.p.eps)
            psi, it, rr = poisson.sor_red_black_chebyshev(
                b, self.psi, self.p.poisson_tol, self.p.poisson_max_iter, self.p.rho_j)
        self.last_iters, self.last_residual = it, rr
        return psi

    def field(self):
        if self.neumann:
            return poisson.electric_field_neumann(self.psi, self.solid, self.wall_q, self.p.eps,
                                                  self.p.E_ext)
        return poisson.electric_field(self.psi, self.p.E_ext)

    def step(self):
        n, j = lb.moments(self.f)
        rho_e = self.charge_density(n)
        self.psi = self.solve_potential(rho_e)
        E = self.field()

        S = n.shape[0]
        z = np.asarray(self.p.valence, dtype=np.float64)
        G = z[:, None, None, None, None] * E[None] + \
            np.asarray(self.p.F_ext, dtype=np.float64)[:, :, None, None, None]
        thermal = (self.p.seed, self.t, self.p.kT) if self.p.fluctuations else None
        if self.R is not None:
            self.R, self.V, K = md.md_substeps(self.R, self.V, n, j, E, self.fluid,
                                               self.walls, self.poly, thermal=thermal,
                                               field_on_fluid=self.neumann)
            nsafe = np.where(self.fluid[None], n, 1.0)
            G = G + K / nsafe[:, None]
        tau = np.asarray(self.p.tau, dtype=np.float64)
        delta = None
        if self.p.fluctuations:
            delta = np.stack([noise.lattice_noise(n[s], 1.0 / tau[s], self.p.kT, s, self.t,
                                                  self.p.seed) for s in range(S)])
        fstar, _, _ = lb.collide(self.f, G, tau,
                                 np.asarray(self.p.omega_drag, dtype=np.float64), self.fluid,
                                 noise=delta)
        self.f = lb.stream(fstar, self.solid)
        self.t += 1

    def run(self, steps):
        for _ in range(steps):
            self.step()

    # -- observables ----------------------------------------------------------
    def densities(self):
        n, _ = lb.moments(self.f)
        return n

    def velocities(self):
        """Bare species velocities j^a / n^a of f(t) (zero on solid sites)."""
        n, j = lb.moments(self.f)
        nsafe = np.where(self.fluid[None], n, 1.0)
        return np.where(self.fluid[None, None], j / nsafe[:, None], 0.0)

    def mass(self):
        return self.f.sum(axis=(1, 2, 3, 4))

    def momentum(self):
        _, j = lb.moments(self.f)
        return j.sum(axis=(0, 2, 3, 4))
