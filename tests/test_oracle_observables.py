"""Pins of the pore observables' oracle (Sec. IV.B ionic current through a
plane, Sec. IV.C bead passage through the pore's mid-plane) to facts that do
not come from the oracle itself: the first moment of a uniform equilibrium,
a brute-force count over every link of a tiny box, particle conservation
through a real oracle step, and crossing times of trajectories with a known
answer."""
import itertools

import numpy as np

from oracle import d3q19 as L
from oracle import observables as obs
from oracle import step as ostep
from paper_1710_09421_amd import workloads


def test_uniform_equilibrium_flux_is_n_u_z_times_area():
    """For uniform populations the crossing ones of every plane sum to
    sum_p c_pz f_p = n u_z per column (first moment of the D3Q19 equilibrium:
    sum_p w_p c_p c_p = 1/3 I, so n (1 + 3 c.u + ...) has first moment n u)."""
    Z, Y, X = 5, 4, 6
    n = np.array([1.0, 0.012, 0.008])
    u = np.array([[0.01, -0.02, 0.03], [0.0, 0.0, -0.04], [0.05, 0.01, 0.02]])
    f = np.empty((3, L.Q, Z, Y, X))
    for s in range(3):
        for p in range(L.Q):
            cu = float(L.C[p] @ u[s])
            f[s, p] = L.W[p] * n[s] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * float(u[s] @ u[s]))
    solid = np.zeros((Z, Y, X), dtype=bool)
    for z in range(Z):
        flux = obs.plane_flux(f, solid, z)
        assert np.allclose(flux, n * u[:, 2] * X * Y, rtol=1e-12, atol=1e-15), (z, flux)


def test_plane_flux_matches_a_brute_force_link_count():
    """Random post-collision populations on a 6x5x4 box with random solid
    sites: stream them by explicit loops, then compare the oracle's flux of
    the streamed state with a direct count of the populations that moved
    from a fluid site on one side of the plane to a fluid site on the other."""
    rng = np.random.default_rng(7)
    Z, Y, X = 6, 5, 4
    solid = rng.uniform(size=(Z, Y, X)) < 0.3
    fstar = rng.uniform(0.0, 1.0, size=(3, L.Q, Z, Y, X)) * (~solid)[None, None]
    # propagation by loops: f_p(r) = f*_p(r - c_p) from a fluid source, the
    # bounced population otherwise (only the streamed entries matter here)
    f = np.zeros_like(fstar)
    for z, y, x in itertools.product(range(Z), range(Y), range(X)):
        if solid[z, y, x]:
            continue
        for p in range(L.Q):
            cx, cy, cz = L.C[p]
            zs, ys, xs = (z - cz) % Z, (y - cy) % Y, (x - cx) % X
            f[:, p, z, y, x] = fstar[:, L.OPP[p], z, y, x] if solid[zs, ys, xs] else fstar[:, p, zs, ys, xs]
    for zp in range(Z):
        count = np.zeros(3)
        for z, y, x in itertools.product(range(Z), range(Y), range(X)):
            if solid[z, y, x]:
                continue
            for p in range(L.Q):
                cx, cy, cz = L.C[p]
                zd, yd, xd = (z + cz) % Z, (y + cy) % Y, (x + cx) % X
                if solid[zd, yd, xd]:
                    continue
                if cz == 1 and z == zp:
                    count += fstar[:, p, z, y, x]
                elif cz == -1 and z == (zp + 1) % Z:
                    count -= fstar[:, p, z, y, x]
        assert np.allclose(obs.plane_flux(f, solid, zp), count, rtol=1e-13, atol=1e-13), zp


def test_slab_particle_change_equals_net_flux_through_a_real_step():
    """Pore system with a charged chain, walls and an applied field: over
    one oracle step (collision conserves every species' particles per site,
    propagation moves them) the change of the particles in the planes
    z1 + 1 .. z2 equals flux(z1) - flux(z2) of the streamed state, also for
    a slab that wraps through z = 0."""
    wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.02, -0.01, 8, 31, steps=100)
    p = ostep.Params(valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                     bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_tol=1e-10)
    sim = ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0,
                           beads=(wl.beads_R, wl.beads_V, wl.polymer))
    solid = wl.solid.astype(bool)
    Z = solid.shape[0]
    sim.run(3)
    for _ in range(2):
        f0 = sim.f.copy()
        sim.step()
        for z1, z2 in ((3, 11), (9, 14), (Z - 1, 4), (Z - 5, 2)):
            planes = [(z1 + 1 + k) % Z for k in range((z2 - z1) % Z)]
            before = f0[:, :, planes].sum(axis=(1, 2, 3, 4))
            after = sim.f[:, :, planes].sum(axis=(1, 2, 3, 4))
            net = obs.plane_flux(sim.f, solid, z1) - obs.plane_flux(sim.f, solid, z2)
            assert np.allclose(after - before, net, rtol=0, atol=1e-12 * before.max()), (z1, z2)
            # the planes chosen do carry a current (the check is not 0 = 0)
            assert np.abs(net[1:]).max() > 1e-9 or np.abs(obs.plane_flux(sim.f, solid, z1)[1:]).max() > 1e-9


def test_charge_current_weights_species_by_valence():
    assert obs.charge_current(np.array([5.0, 2.0, 3.0]), (0.0, 1.0, -1.0)) == -1.0
    assert obs.charge_current(np.array([5.0, 2.0, 3.0]), (0.0, 2.0, -1.0)) == 1.0


def test_bead_crossings_of_known_trajectories():
    Lz = 10.0
    t = np.arange(0, 9, dtype=np.float64)
    z = np.stack([
        1.3 + 0.25 * t,                 # up through 2.0 at t = 3 (z = 2.05)
        2.5 - 0.3 * t,                  # down through 2.0 at t = 2 (z = 1.9)
        11.75 + 0.1 * t,                # up through the image 12.0 at t = 3 (12.05)
        1.9 + 0.2 * np.minimum(t, 1) - 0.2 * np.clip(t - 4, 0, 1),   # up at 1, down at 5
        5.0 + 0.1 * t,                  # never crosses 2.0 or 12.0
        -8.05 + 0.1 * t,                # up through the image -8.0 at t = 1
    ], axis=1)
    first, last, net = obs.bead_crossings(z, 2.0, Lz)
    assert first.tolist() == [3, 2, 3, 1, -1, 1]
    assert last.tolist() == [3, 2, 3, 5, -1, 1]
    assert net.tolist() == [1, -1, 1, 0, 0, 1]
