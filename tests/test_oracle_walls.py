"""Pins of the insulating-wall (Neumann) variant of the Poisson problem
(the boundary condition after Eq. poisson) and of the occupation-cube
coupling theta_i of Eq. totalforcefluid.

Neumann: in a slit between two insulating walls with surface charges
Sigma_1, Sigma_2 and a uniform counter-charge the potential is a parabola
that the finite-volume scheme reproduces exactly at the cell centres, and so
is its field (the ghost value psi + Sigma / eps carries the wall's flux); the
operator is conservative (no flux through walls) and symmetric; SOR reaches
the solution of the dense system assembled face by face on a tiny pore box;
the face charges add up to the wall charge.

theta: the cube nodes are exactly the lattice nodes with
R - sigma/2 < node <= R + sigma/2 per axis (enumerated), one node for
sigma = 1 and the eight cell corners for sigma = 2, equal weights; bead and
fluid exchange momentum exactly through them."""
import numpy as np
import pytest

from oracle import md
from oracle import poisson as P
from oracle import step

EPS = 0.341


def _slit(H, nx=6, ny=4):
    Z = H + 2
    solid = np.zeros((Z, ny, nx), dtype=bool)
    solid[0] = True
    solid[H + 1] = True
    return solid


def test_neumann_slit_potential_and_field_are_the_exact_parabola():
    H = 12
    solid = _slit(H)
    s1, s2 = -0.05, 0.02                                  # bottom and top walls
    wall_q = np.zeros(solid.shape)
    wall_q[0], wall_q[H + 1] = s1, s2                     # one fluid face per solid site
    rho0 = -(s1 + s2) / H                                  # neutral
    rho = np.where(~solid, rho0, 0.0)
    b = P.neumann_rhs(rho, wall_q, solid, EPS)
    psi, it, rr = P.sor_neumann(b, np.zeros(solid.shape), ~solid, 1e-13, 100000)
    z = np.arange(H + 2, dtype=np.float64)
    # psi'' = -rho0 / eps; bottom wall at z = 1/2 with normal +z: psi'(1/2) = -s1 / eps
    exact = -rho0 / (2 * EPS) * (z - 0.5) ** 2 - s1 / EPS * (z - 0.5)
    exact = exact[1:H + 1] - exact[1:H + 1].mean()
    for y in range(solid.shape[1]):
        assert np.allclose(psi[1:H + 1, y, 3], exact, atol=1e-13 * np.abs(exact).max())
    # the top wall's condition follows: psi'(H + 1/2) = +s2 / eps
    dpsi_top = -rho0 / EPS * H - s1 / EPS
    assert dpsi_top == pytest.approx(s2 / EPS, rel=1e-12)
    E = P.electric_field_neumann(psi, solid, wall_q, EPS, (0.0, 0.0, 0.0))
    Ez = rho0 / EPS * (z - 0.5) + s1 / EPS
    assert np.allclose(E[2][1:H + 1, 2, 1], Ez[1:H + 1], atol=1e-12 * np.abs(Ez).max())
    assert np.abs(E[:2]).max() < 1e-12 and not E[:, 0].any() and not E[:, H + 1].any()


def _pore_box(shape=(8, 6, 6)):
    solid = np.zeros(shape, dtype=bool)
    solid[3:5] = True
    solid[3:5, 2:4, 2:4] = False                          # a 2 x 2 pore through the slab
    return solid


def test_neumann_operator_is_conservative_and_symmetric():
    solid = _pore_box()
    fluid = ~solid
    rng = np.random.default_rng(1)
    a = rng.normal(size=solid.shape)
    b = rng.normal(size=solid.shape)
    La = P.neumann_laplacian(a, fluid)
    Lb = P.neumann_laplacian(b, fluid)
    assert abs(La.sum()) < 1e-12                          # no flux leaves the fluid
    assert (a * Lb)[fluid].sum() == pytest.approx((b * La)[fluid].sum(), rel=1e-12)
    assert not La[solid].any()
    assert (a * La)[fluid].sum() < 0                      # negative semi-definite


def test_neumann_sor_reaches_the_dense_solution():
    """The system assembled face by face (a loop over fluid sites and their
    six neighbours), with the gauge fixed by the fluid mean, solved
    directly: SOR's converged potential equals it."""
    solid = _pore_box()
    fluid = ~solid
    Z, Y, X = solid.shape
    rng = np.random.default_rng(2)
    wall_q = np.where(solid & (P.open_faces(fluid) > 0), rng.uniform(-0.03, 0.0, solid.shape), 0.0)
    rho = np.where(fluid, rng.normal(scale=0.01, size=solid.shape), 0.0)
    b = P.neumann_rhs(rho, wall_q, solid, EPS)
    ids = -np.ones(solid.shape, dtype=int)
    ids[fluid] = np.arange(fluid.sum())
    m = int(fluid.sum())
    A = np.zeros((m + 1, m))
    for z in range(Z):
        for y in range(Y):
            for x in range(X):
                if not fluid[z, y, x]:
                    continue
                i = ids[z, y, x]
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    j = ids[(z + dz) % Z, (y + dy) % Y, (x + dx) % X]
                    if j >= 0:
                        A[i, j] += 1.0
                        A[i, i] -= 1.0
    A[m] = 1.0                                            # zero fluid mean
    rhs = np.concatenate([b[fluid], [0.0]])
    direct = np.linalg.lstsq(A, rhs, rcond=None)[0]
    psi, it, rr = P.sor_neumann(b, np.zeros(solid.shape), fluid, 1e-13, 100000)
    assert rr <= 1e-13
    assert np.allclose(psi[fluid], direct, atol=1e-11 * np.abs(direct).max())
    # the wall charge enters as face flux: sum of the right-hand side before
    # the mean removal is ions + walls
    sig = P.face_charge(wall_q, solid)
    assert (sig * P.open_faces(fluid)).sum() == pytest.approx(wall_q.sum(), rel=1e-13)


def test_face_charge_refuses_charges_without_a_fluid_face():
    solid = _pore_box()
    wall_q = np.zeros(solid.shape)
    wall_q[3, 0, 0] = -0.01                               # touches fluid only through edges? no:
    # (3, 0, 0) has the fluid layer z = 2 as a face neighbour; bury a charge instead
    solid2 = solid.copy()
    solid2[2:6] = True
    solid2[2:6, 2:4, 2:4] = False
    q2 = np.zeros(solid.shape)
    q2[4, 0, 0] = -0.01
    with pytest.raises(ValueError):
        P.face_charge(q2, solid2)
    assert P.face_charge(wall_q, solid)[3, 0, 0] == pytest.approx(-0.01)


@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0])
def test_theta_cube_nodes_by_enumeration(sigma):
    rng = np.random.default_rng(int(sigma * 10))
    shape = (12, 10, 8)
    R = rng.uniform(2.0, 7.0, size=(50, 3))
    R[0] = [3.0, 4.0, 5.0]                                 # on a node
    R[1] = [3.5, 4.5, 5.5]                                 # a cell centre
    idx, w = md.theta_weights(R, shape, sigma)
    for i in range(R.shape[0]):
        inside = set()
        for n in np.ndindex(5, 5, 5):
            node = np.floor(R[i]) - 2 + np.array(n)
            if np.all((node - R[i] > -sigma / 2) & (node - R[i] <= sigma / 2)):
                inside.add(tuple(np.mod(node, [8, 10, 12]).astype(int)))
        got = {tuple(idx[i, k]) for k in range(8) if w[i, k] > 0}
        assert got == inside, (i, R[i])
        assert np.all((w[i] == 0) | (w[i] == 1))
    if sigma == 1.0:
        assert np.all(w.sum(axis=1) == 1)
    if sigma == 2.0:
        assert np.all(w.sum(axis=1) == 8)


def test_theta_coupling_exchanges_momentum_exactly():
    """A bead off the nodes with the theta cube of side 2: each of the eight
    corners takes the same share of the friction, and fluid + bead momentum
    is exact; the trilinear kernel shares it unequally."""
    shape = (8, 8, 8)
    n = np.stack([np.ones(shape), np.full(shape, 0.01), np.full(shape, 0.01)])
    j = np.zeros((3, 3) + shape)
    E = np.zeros((3,) + shape)
    fluid = np.ones(shape, dtype=bool)
    R = np.array([[3.2, 4.3, 2.1]])
    V0 = np.array([[0.01, -0.02, 0.005]])
    base = dict(M=1.0, q=np.zeros(1), k_fene=0.0, R0=1e3, eps=0.0, sigma=2.0, gamma=5.0, n_sub=10)
    out = {}
    for kern in ("theta", "trilinear"):
        R1, V1, K = md.md_substeps(R, V0, n, j, E, fluid, np.zeros((0, 3)), dict(base, coupling=kern))
        assert np.allclose(K.sum(axis=(0, 2, 3, 4)), -(V1 - V0)[0], rtol=1e-12, atol=1e-17)
        corners = K.sum(axis=0)[:, 2:4, 4:6, 3:5].reshape(3, -1)
        out[kern] = corners
    c = out["theta"]
    assert np.allclose(c, c[:, :1], rtol=1e-12)           # equal shares
    assert not np.allclose(out["trilinear"], out["trilinear"][:, :1], rtol=1e-3)


def test_theta_chain_conserves_momentum_in_a_periodic_box():
    shape = (8, 8, 12)
    rng = np.random.default_rng(5)
    n0 = np.stack([np.ones(shape), 0.01 * (1 + 0.05 * rng.uniform(-1, 1, shape)),
                   0.01 * (1 + 0.05 * rng.uniform(-1, 1, shape))])
    R = np.array([[3.0, 4.0, 5.0], [3.95, 4.1, 5.1], [4.9, 4.3, 5.0]])
    poly = step.polymer_params(3, q=-0.5, coupling="theta")
    sim = step.Simulation(step.Params(poisson_tol=1e-12), np.zeros(shape, dtype=bool),
                          np.zeros(shape), n0, beads=(R, rng.normal(scale=0.02, size=R.shape), poly))

    def total():
        return sim.momentum() + sim.V.sum(axis=0)
    P0 = total()
    sim.run(5)
    assert np.allclose(total(), P0, atol=1e-12)


def test_neumann_pore_with_chain_conserves_mass_and_charge_balance():
    """A charged pore with insulating walls, an applied field and a chain:
    species masses stay exact, the potential is mean-free over the fluid and
    zero in the solid, and the bead charge lands on fluid sites only."""
    from paper_1710_09421_amd import workloads
    wl = workloads.pore_system((16, 12, 12), 4, 3, 0.01, 0.01, -0.01, 4, 3, steps=10,
                               charge_sites="faces")
    p = step.Params(E_ext=wl.E_ext, poisson_tol=1e-11, walls="neumann")
    sim = step.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0,
                          beads=(wl.beads_R, wl.beads_V, wl.polymer))
    m0 = sim.mass()
    sim.run(5)
    fluid = wl.solid == 0
    assert np.allclose(sim.mass(), m0, rtol=1e-13)
    assert abs(sim.psi[fluid].mean()) < 1e-14 and not sim.psi[~fluid].any()
    dep = md.deposit_charge(sim.R, sim.poly["q"], wl.shape, fluid=fluid)
    assert not dep[~fluid].any() and dep.sum() == pytest.approx(sim.poly["q"].sum(), rel=1e-13)
