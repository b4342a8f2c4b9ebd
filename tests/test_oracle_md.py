"""Pins of the bead dynamics and of the bead-lattice coupling (Sec. II.B and
the interpolation kernels of Sec. II.C): forces are minus the gradient of the
stated energies, pair forces obey Newton's third law, the kernel is a
partition of unity that reproduces linear fields, friction alone decays
geometrically, and the fluid + bead momentum is conserved."""
import numpy as np
import pytest

from oracle import md, lb, poisson, step
from paper_1710_09421_amd import workloads

RNG = np.random.default_rng(2)
BOX = np.array([12.0, 10.0, 14.0])


def chain(n, bond=0.97, seed=3):
    rng = np.random.default_rng(seed)
    R = [np.array([5.0, 5.0, 7.0])]
    while len(R) < n:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        c = R[-1] + bond * v
        if all(np.linalg.norm(c - r) > 1.0 for r in R[:-1]):
            R.append(c)
    return np.array(R)


def numerical_gradient(fun, R, h=1e-6):
    g = np.zeros_like(R)
    for i in range(R.shape[0]):
        for a in range(3):
            Rp = R.copy(); Rp[i, a] += h
            Rm = R.copy(); Rm[i, a] -= h
            g[i, a] = (fun(Rp) - fun(Rm)) / (2 * h)
    return g


def test_fene_force_is_minus_energy_gradient():
    R = chain(8)
    F = md.fene_forces(R, BOX, 30.0, 1.5)
    g = numerical_gradient(lambda X: md.fene_energy(X, BOX, 30.0, 1.5), R)
    assert np.allclose(F, -g, rtol=1e-6, atol=1e-6)
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-12)


def test_wca_force_is_minus_energy_gradient():
    R = chain(10, bond=0.9)
    R += RNG.normal(scale=0.05, size=R.shape)
    F = md.wca_pair_forces(R, BOX, 1.0, 1.0)
    assert np.any(F != 0)
    g = numerical_gradient(lambda X: md.wca_energy(X, BOX, 1.0, 1.0), R)
    assert np.allclose(F, -g, rtol=1e-5, atol=1e-5)
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-10)


def test_wca_vanishes_beyond_cutoff_and_uses_minimum_image():
    R = np.array([[0.2, 5.0, 5.0], [11.6, 5.0, 5.0]])     # 0.6 apart across x = 0
    F = md.wca_pair_forces(R, BOX, 1.0, 1.0)
    assert F[0, 0] > 0 and F[1, 0] < 0
    R2 = np.array([[2.0, 5.0, 5.0], [2.0 + 1.13, 5.0, 5.0]])
    assert not md.wca_pair_forces(R2, BOX, 1.0, 1.0).any()


def test_wall_force_is_minus_energy_gradient():
    solid = np.zeros((14, 10, 12), dtype=bool)
    solid[:3] = True
    walls = md.wall_sites(solid)
    # the slab z = 0..2 touches fluid at z = 2 and, through the periodic face, at z = 0
    assert set(walls[:, 2].tolist()) == {0.0, 2.0}
    assert walls.shape[0] == 2 * 10 * 12
    R = np.array([[4.3, 3.2, 3.05], [6.1, 7.7, 3.4], [1.0, 1.0, 8.0]])
    F = md.wall_forces(R, walls, BOX, 1.0, 1.0)
    g = numerical_gradient(lambda X: md.wall_energy(X, walls, BOX, 1.0, 1.0), R)
    assert np.allclose(F, -g, rtol=1e-5, atol=1e-5)
    assert F[0, 2] > 0 and not F[2].any()


def test_trilinear_partition_of_unity_and_linear_reproduction():
    shape = (10, 12, 14)
    R = RNG.uniform(1.0, 8.0, size=(20, 3))
    idx, w = md.trilinear(R, shape)
    assert np.allclose(w.sum(axis=1), 1.0, rtol=1e-15)
    zz, yy, xx = np.indices(shape).astype(float)
    lin = 0.3 + 1.7 * xx - 0.4 * yy + 2.2 * zz
    val = (w * md.gather(lin, idx)).sum(axis=1)
    assert np.allclose(val, 0.3 + 1.7 * R[:, 0] - 0.4 * R[:, 1] + 2.2 * R[:, 2], rtol=1e-13)


def test_deposit_conserves_charge():
    shape = (10, 12, 14)
    R = RNG.uniform(0.0, 20.0, size=(9, 3))
    q = RNG.uniform(-1, 1, size=9)
    rho = md.deposit_charge(R, q, shape)
    assert rho.sum() == pytest.approx(q.sum(), rel=1e-13)


def _quiescent_fields(shape, n_solvent=1.0, n_ion=0.01):
    n = np.stack([np.full(shape, n_solvent), np.full(shape, n_ion), np.full(shape, n_ion)])
    j = np.zeros((3, 3) + shape)
    E = np.zeros((3,) + shape)
    return n, j, E


def test_friction_relaxes_bead_and_node_together():
    """A bead sitting exactly on a node of a fluid at rest, with no other
    force: the bead and that node exchange momentum each substep, so the
    relative velocity decays as (1 - gamma h (1/M + 1/n))^s (two-body
    relaxation with the node's total density n) while M V + n u is kept.
    Velocities are tiny so that the bead stays on the node to 1e-8."""
    shape = (8, 8, 8)
    n, j, E = _quiescent_fields(shape)
    fluid = np.ones(shape, dtype=bool)
    R = np.array([[3.0, 4.0, 2.0]])
    V0 = np.array([[0.1, -0.05, 0.02]]) * 1e-6
    M, gamma, n_sub = 2.0, 5.0, 10
    poly = dict(M=M, q=np.zeros(1), k_fene=30.0, R0=1.5, eps=1.0, sigma=1.0, gamma=gamma, n_sub=n_sub)
    R1, V1, K = md.md_substeps(R, V0, n, j, E, fluid, np.zeros((0, 3)), poly)
    h = 1.0 / n_sub
    ntot = n[:, 0, 0, 0].sum()
    u_node = K[:, :, 2, 4, 3].sum(axis=0) / ntot
    assert np.allclose(V1[0] - u_node, V0[0] * (1 - gamma * h * (1 / M + 1 / ntot)) ** n_sub, rtol=1e-6)
    # the fluid receives exactly the impulse the bead lost
    assert np.allclose(K.sum(axis=(0, 2, 3, 4)), -M * (V1 - V0)[0], rtol=1e-12)
    assert np.abs(K[:, :, 2, 4, 3]).sum() > 0.999 * np.abs(K).sum()


def test_fluid_plus_bead_momentum_is_conserved():
    """Periodic box, no walls, no applied field, neutral beads, charged ions:
    total momentum of the three species plus the beads stays at its initial
    value (the electrostatic forces cancel by the force-balance identity and
    the friction is exchanged exactly)."""
    shape = (8, 8, 12)
    rng = np.random.default_rng(5)
    n0 = np.stack([np.ones(shape), 0.01 * (1 + 0.05 * rng.uniform(-1, 1, shape)),
                   0.01 * (1 + 0.05 * rng.uniform(-1, 1, shape))])
    R = chain(6, seed=4)
    V = rng.normal(scale=0.02, size=R.shape)
    poly = step.polymer_params(6, q=0.0, gamma=20.0, n_sub=40)
    p = step.Params(poisson_tol=1e-12)
    sim = step.Simulation(p, np.zeros(shape, dtype=bool), np.zeros(shape), n0,
                          beads=(R, V, poly))

    def total():
        return sim.momentum() + poly["M"] * sim.V.sum(axis=0)
    P0 = total()
    sim.run(6)
    assert np.allclose(total(), P0, atol=1e-11)
    assert np.abs(sim.V).max() > 0


def test_bead_and_uniform_flow_reach_common_velocity():
    """A bead at rest on a node of a uniformly moving fluid: bead and node
    relax to the common velocity of the two-body system."""
    shape = (8, 8, 8)
    n, j, E = _quiescent_fields(shape)
    u0 = np.array([0.01, -0.02, 0.005]) * 1e-6
    j = n[:, None] * u0[None, :, None, None, None]
    fluid = np.ones(shape, dtype=bool)
    M, gamma, n_sub = 1.0, 20.0, 40
    poly = dict(M=M, q=np.zeros(1), k_fene=30.0, R0=1.5, eps=1.0, sigma=1.0, gamma=gamma, n_sub=n_sub)
    R1, V1, K = md.md_substeps(np.array([[4.0, 4.0, 4.0]]), np.zeros((1, 3)), n, j, E, fluid,
                               np.zeros((0, 3)), poly)
    ntot = n[:, 0, 0, 0].sum()
    common = ntot * u0 / (M + ntot)
    decay = (1 - gamma / n_sub * (1 / M + 1 / ntot)) ** n_sub
    u_node = u0 + K[:, :, 4, 4, 4].sum(axis=0) / ntot
    assert np.allclose(V1[0] - u_node, -u0 * decay, rtol=1e-6, atol=1e-14)
    assert np.allclose(M * V1[0] + ntot * u_node, ntot * u0, rtol=1e-6)
    assert np.allclose(V1[0], common, rtol=1e-6)


def test_harmonic_bond_force_is_minus_energy_gradient():
    """Bonded term of Eq. polymermodel, U = k (r - l_bond)^2 / 2."""
    R = chain(8)
    F = md.harmonic_forces(R, BOX, 25.0, 1.0)
    g = numerical_gradient(lambda X: md.harmonic_energy(X, BOX, 25.0, 1.0), R)
    assert np.allclose(F, -g, rtol=1e-6, atol=1e-6)
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-12)
    pair = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 4.5]])      # r = 1.5 across no boundary
    assert md.harmonic_energy(pair, BOX, 4.0, 1.0) == pytest.approx(0.5, rel=1e-14)
    assert np.allclose(md.harmonic_forces(pair, BOX, 4.0, 1.0), [[0, 0, 2.0], [0, 0, -2.0]])


def test_wca_skips_bonded_neighbours_only():
    """With the harmonic bonds the WCA acts only for |i - j| > 1: a chain whose
    only close pairs are neighbours feels none, and a folded chain feels
    exactly the pair force of its close non-neighbours."""
    straight = np.array([[1.0, 1.0, 1.0], [1.9, 1.0, 1.0], [2.8, 1.0, 1.0]])
    assert np.abs(md.wca_pair_forces(straight, BOX, 1.0, 1.0)).max() > 1.0
    assert np.abs(md.wca_pair_forces(straight, BOX, 1.0, 1.0, skip_bonded=True)).max() == 0.0
    folded = np.array([[1.0, 1.0, 1.0], [1.9, 1.0, 1.0], [1.5, 1.7, 1.0]])   # 0-2 at 0.86
    F = md.wca_pair_forces(folded, BOX, 1.0, 1.0, skip_bonded=True)
    F02 = md.wca_pair_forces(folded[[0, 2]], BOX, 1.0, 1.0)
    assert np.allclose(F[[0, 2]], F02, rtol=1e-14) and np.all(F[1] == 0.0)
    assert md.wca_energy(folded, BOX, 1.0, 1.0, skip_bonded=True) == pytest.approx(
        md.wca_energy(folded[[0, 2]], BOX, 1.0, 1.0), rel=1e-14)


def test_free_harmonic_dimer_oscillates_at_sqrt_2k_over_m():
    """Two beads joined by a harmonic bond, no friction, field or WCA: the
    separation y = r - l obeys the semi-implicit Euler map of an oscillator
    with w^2 = 2 k / M (reduced mass M / 2), v' = v - h w^2 y, y' = y + h v',
    whose exact solution from y_0 = a, v_0 = 0 is
    y_n = a cos(n th) - a (h w)^2 / 2 / sin(th) sin(n th), cos(th) = 1 - (h w)^2 / 2
    (the continuous a cos(w t) to first order in h w)."""
    shape = (8, 8, 8)
    n, j, E = _quiescent_fields(shape)
    fluid = np.ones(shape, dtype=bool)
    k, M, l, a = 2.0, 1.0, 1.0, 0.1
    R = np.array([[3.0, 4.0, 4.0], [3.0 + l + a, 4.0, 4.0]])
    V = np.zeros((2, 3))
    poly = dict(M=M, q=np.zeros(2), k_fene=0.0, R0=1.5, eps=0.0, sigma=1.0, gamma=0.0,
                n_sub=400, bond="harmonic", k_bond=k, l_bond=l)
    w = np.sqrt(2 * k / M)
    hw = w / poly["n_sub"]
    th = np.arccos(1 - hw * hw / 2)
    for t in range(1, 4):
        R, V, K = md.md_substeps(R, V, n, j, E, fluid, np.zeros((0, 3)), poly)
        sep = R[1, 0] - R[0, 0]
        m = t * poly["n_sub"]
        y = a * np.cos(m * th) - a * hw * hw / 2 / np.sin(th) * np.sin(m * th)
        assert sep == pytest.approx(l + y, abs=1e-10), t
        assert sep == pytest.approx(l + a * np.cos(w * t), abs=0.01 * a), t
    assert np.allclose(R[:, 1:], [[4.0, 4.0], [4.0, 4.0]]) and np.abs(K).max() == 0.0


def _field_probe_polymer(q):
    """Beads that feel only the electric force over one substep of unit
    length: no bonds (k = 0 with a far maximum extension), no WCA (eps = 0),
    no friction, unit mass, so that V(after) - V(before) = q E(R)."""
    return dict(M=1.0, q=np.asarray(q, dtype=np.float64), k_fene=0.0, R0=1e3, eps=0.0,
                sigma=1.0, gamma=0.0, n_sub=1)


def test_electrostatic_forces_balance_with_charged_beads_beside_a_wall():
    """Newton's third law of the lattice electrostatics (Sec. II.A, Eq.
    poisson with the central-difference field): the forces charge x field on
    the ions, the fixed wall charges and the beads sum to zero, because the
    beads' charge is deposited with the same plain trilinear weights that
    interpolate the field at the beads and sum_r rho_e grad_h psi = 0 for the
    periodic 7-point problem.  The beads sit beside the charged slab with
    solid corners, where interpolating the field with the weights
    renormalised over fluid corners (those of the fluid velocity) would give
    another force; the bead force is q E, not -q E."""
    shape = (12, 8, 10)
    solid = np.zeros(shape, dtype=bool)
    solid[4:7] = True
    rng = np.random.default_rng(21)
    walls = workloads.boundary_sites(solid.astype(np.uint8))
    wall_q = np.where(walls, -0.02, 0.0)
    fluid = ~solid
    n0 = np.stack([np.where(fluid, 1.0, 0.0),
                   np.where(fluid, 0.01 * (1 + 0.2 * rng.uniform(-1, 1, shape)), 0.0),
                   np.where(fluid, 0.01 * (1 + 0.2 * rng.uniform(-1, 1, shape)), 0.0)])
    # corners at z = 6 (solid) and 7, z = 3 and 4 (solid), one bead in the bulk
    R = np.array([[2.3, 3.6, 6.4], [6.7, 1.2, 3.25], [4.5, 5.5, 9.1]])
    q = np.array([-0.7, 0.4, -1.1])
    poly = _field_probe_polymer(q)
    sim = step.Simulation(step.Params(poisson_tol=1e-13), solid, wall_q, n0,
                          beads=(R, np.zeros_like(R), poly))
    n, j = lb.moments(sim.f)
    psi = sim.solve_potential(sim.charge_density(n))
    E = poisson.electric_field(psi, (0.0, 0.0, 0.0))
    z = np.asarray(sim.p.valence)
    F_ions = np.einsum("s,szyx,kzyx->k", z, n, E)
    F_wall = np.einsum("zyx,kzyx->k", wall_q, E)
    R1, V1, K = md.md_substeps(R, np.zeros_like(R), n, j, E, fluid, sim.walls, poly)
    F_beads = V1                                          # M = 1, one substep of h = 1
    assert not np.abs(K).any()                            # no friction: nothing to the fluid
    scale = np.abs(F_ions).max() + np.abs(F_wall).max() + np.abs(F_beads).max()
    assert np.abs(F_beads).max() > 1e-2 * scale           # the beads carry a real share
    assert np.allclose(F_ions + F_wall + F_beads.sum(axis=0), 0.0, atol=1e-10 * scale)
    # the configuration tells the plain weights from renormalised ones
    idx, w = md.trilinear(R, shape)
    fl = md.gather(fluid, idx).astype(np.float64)
    assert np.all(fl[:2].sum(axis=1) < 8) and fl[2].sum() == 8
    wt = w * fl / (w * fl).sum(axis=1, keepdims=True)
    E_renorm = (wt[None] * md.gather(E, idx)).sum(axis=-1).T
    assert np.abs(q[:, None] * E_renorm - F_beads).max() > 1e-4 * scale


def test_fluid_plus_charged_bead_momentum_is_conserved():
    """Periodic box, no walls, no applied field, charged beads among charged
    ions, 40 substeps per step: the electrostatic forces on ions and beads
    cancel (same identity as above; the beads feel the field where their
    charge was deposited), the friction is exchanged exactly, so fluid + bead
    momentum stays at its initial value while the beads are pushed around by
    the field."""
    shape = (8, 8, 12)
    rng = np.random.default_rng(15)
    n0 = np.stack([np.ones(shape), 0.01 * (1 + 0.05 * rng.uniform(-1, 1, shape)),
                   0.01 * (1 + 0.05 * rng.uniform(-1, 1, shape))])
    R = chain(6, seed=4)
    V = rng.normal(scale=0.02, size=R.shape)
    poly = step.polymer_params(6, q=-0.5, gamma=20.0, n_sub=40)
    poly["q"] = np.array([-0.5, 0.3, -0.8, -0.2, 0.6, -0.5])
    sim = step.Simulation(step.Params(poisson_tol=1e-12), np.zeros(shape, dtype=bool),
                          np.zeros(shape), n0, beads=(R, V, poly))

    def total():
        return sim.momentum() + poly["M"] * sim.V.sum(axis=0)
    P0 = total()
    sim.run(6)
    assert np.allclose(total(), P0, atol=1e-11)
    # the beads' charge does move momentum between beads and ions
    neutral = step.Simulation(step.Params(poisson_tol=1e-12), np.zeros(shape, dtype=bool),
                              np.zeros(shape), n0,
                              beads=(R, V, dict(poly, q=np.zeros(6))))
    neutral.run(6)
    assert np.abs(sim.V - neutral.V).max() > 1e-4


def test_lone_charged_bead_accelerates_along_qE():
    """One charged bead with no friction in a neutral, uniform electrolyte
    under an applied field: its own deposited charge exerts no force on it
    (the periodic lattice Green's function composed with the central
    difference is antisymmetric), so over one lattice step V changes by
    exactly q E_ext / M (Sec. II.B, conservative force of the charge)."""
    shape = (8, 10, 12)
    E_ext = (0.01, -0.02, 0.03)
    n0 = np.stack([np.ones(shape), np.full(shape, 0.01), np.full(shape, 0.01)])
    R = np.array([[4.3, 6.8, 5.55]])
    q = -0.5
    M = 2.0
    poly = dict(_field_probe_polymer([q]), M=M)
    sim = step.Simulation(step.Params(E_ext=E_ext, poisson_tol=1e-13),
                          np.zeros(shape, dtype=bool), np.zeros(shape), n0,
                          beads=(R, np.zeros_like(R), poly))
    sim.step()
    assert np.allclose(sim.V[0], q * np.asarray(E_ext) / M, rtol=1e-9, atol=1e-15)


def test_sigma_two_pair_and_wall_forces_are_minus_energy_gradients():
    """The translocation set-up's beads (sigma = 2, cut-off 2.245 beyond two
    lattice spacings, epsilon = k_B T): WCA pair and bead-wall forces are
    minus the gradients of their energies, including wall sites two cells
    away, and vanish beyond the cut-off."""
    sigma, eps = 2.0, 1.0 / 3.0
    R = np.array([[3.0, 3.0, 5.0], [5.1, 3.2, 5.0], [4.0, 4.9, 6.1], [7.0, 3.0, 5.1]])
    F = md.wca_pair_forces(R, BOX, eps, sigma, skip_bonded=True)
    g = numerical_gradient(lambda X: md.wca_energy(X, BOX, eps, sigma, skip_bonded=True), R)
    assert np.allclose(F, -g, rtol=1e-5, atol=1e-6) and np.abs(F).max() > 0.1
    solid = np.zeros((14, 10, 12), dtype=bool)
    solid[:3] = True
    walls = md.wall_sites(solid)
    Rw = np.array([[4.3, 3.2, 4.1], [6.1, 7.7, 5.3], [1.0, 1.0, 8.0]])    # 2.1 and 3.3 above z = 2
    Fw = md.wall_forces(Rw, walls, BOX, eps, sigma)
    gw = numerical_gradient(lambda X: md.wall_energy(X, walls, BOX, eps, sigma), Rw)
    assert np.allclose(Fw, -gw, rtol=1e-5, atol=1e-6)
    assert Fw[0, 2] > 0 and not Fw[1].any() and not Fw[2].any()
