"""GPU parity of the pore observables (Sec. IV.B ionic current through a
plane, Sec. IV.C bead passage through the pore's mid-plane) against the
float64 oracle, through the C ABI, plus the properties that hold at any size
(particle conservation of a slab, the crossing rule applied to the chain's
own positions)."""
import numpy as np
import pytest

from oracle import observables as obs
from oracle import step as ostep
from paper_1710_09421_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def pore_with_chain(seed=31, E_z=0.02):
    return workloads.pore_system((32, 24, 24), 6, 4, 0.01, E_z, -0.01, 8, seed, steps=100)


def oracle_sim(wl, tol):
    p = ostep.Params(valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                     bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_tol=tol)
    return ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0,
                            beads=(wl.beads_R, wl.beads_V, wl.polymer))


def crossing_scale(f, solid, z):
    """Sum of |crossing populations| of the plane (the error scale of a flux)."""
    Z = solid.shape[0]
    return np.abs(f[:, :, [z, (z + 1) % Z]]).sum(axis=(1, 2, 3, 4))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-5)])
def test_plane_flux_matches_oracle(ek, precision, tol):
    wl = pore_with_chain()
    prec = ek.EK_FP64 if precision == "fp64" else ek.EK_FP32
    ptol = 1e-10 if precision == "fp64" else 1e-8
    ctx = ek.from_workload(wl, precision=prec, poisson_tol=ptol, poisson_check_every=1)
    sim = oracle_sim(wl, ptol)
    solid = wl.solid.astype(bool)
    Z = solid.shape[0]
    for chunk in (1, 19):
        ctx.step(chunk)
        sim.run(chunk)
        for z in (0, 5, Z // 2 - 1, Z // 2, Z - 1):
            got = ctx.plane_flux(z)
            ref = obs.plane_flux(sim.f, solid, z)
            scale = crossing_scale(sim.f, solid, z)
            err = np.abs(got[:3] - ref) / scale
            print(precision, sim.t, z, got, ref, err)
            assert err.max() < tol, (z, got, ref)
            q = obs.charge_current(ref, wl.valence)
            assert abs(got[3] - q) < tol * scale[1:].sum(), (z, got[3], q)


def test_plane_flux_conserves_particles_single_pore_64x64x128(ek):
    """Full single-pore box in float64: over each step the particles of every
    species in a slab of planes change by exactly the net flux through its
    two bounding planes (one of them wrapping through z = 0)."""
    wl = workloads.single_pore()
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-8, poisson_max_iter=200)
    Z = ctx.shape[0]
    ctx.step(2)

    def slab(planes):
        return np.array([ctx.moments(s)[0][planes].sum() for s in range(3)])

    cases = [(20, 70), (Z - 3, 10), (50, 64)]
    for _ in range(2):
        before = [slab([(z1 + 1 + k) % Z for k in range((z2 - z1) % Z)]) for z1, z2 in cases]
        ctx.step(1)
        for (z1, z2), b in zip(cases, before):
            planes = [(z1 + 1 + k) % Z for k in range((z2 - z1) % Z)]
            a = slab(planes)
            net = ctx.plane_flux(z1)[:3] - ctx.plane_flux(z2)[:3]
            print(z1, z2, a - b, net)
            assert np.allclose(a - b, net, rtol=0, atol=1e-10 * b.max()), (z1, z2, a - b, net)


def test_bead_crossings_match_oracle(ek):
    wl = pore_with_chain(seed=33, E_z=0.05)
    n = wl.beads_R.shape[0]
    Lz = float(wl.solid.shape[0])
    T = 30
    sim = oracle_sim(wl, 1e-10)
    hist = [sim.R[:, 2].copy()]
    for _ in range(T):
        sim.step()
        hist.append(sim.R[:, 2].copy())
    hist = np.array(hist)
    # a plane half way through the largest one-step move of any bead: that
    # crossing is decided with a wide margin on both sides
    dz = np.abs(np.diff(hist, axis=0))
    k, i = np.unravel_index(np.argmax(dz), dz.shape)
    z_plane = 0.5 * (hist[k, i] + hist[k + 1, i])
    first, last, net = obs.bead_crossings(hist, z_plane, Lz)
    assert first[i] >= 1 and dz[k, i] > 1e-4
    d = (hist - z_plane) / Lz
    margin = np.min(np.abs(d - np.round(d)), axis=0) * Lz     # distance to the nearest image

    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_tol=1e-10, poisson_check_every=1)
    with pytest.raises(ek.EKError):
        ctx.crossings(n)                       # no plane set yet
    ctx.set_crossing_plane(z_plane)
    ctx.step(10)
    ctx.step(T - 10)                           # the step count runs on across calls
    g_first, g_last, g_net = ctx.crossings(n)
    print(z_plane, first, last, net, g_first, g_last, g_net, margin)
    sure = margin > 1e-6
    assert sure[i]
    assert np.array_equal(g_first[sure], first[sure])
    assert np.array_equal(g_last[sure], last[sure])
    assert np.array_equal(g_net[sure], net[sure])
    # the rest: a valid record either way
    assert np.all((g_first <= g_last) & ((g_first < 0) == (g_last < 0)))
    # setting the polymer again clears the record; a new geometry ends it
    ctx.set_polymer(wl.beads_R, wl.beads_V, wl.polymer["q"])
    c_first, c_last, c_net = ctx.crossings(n)
    assert np.all(c_first == -1) and np.all(c_last == -1) and np.all(c_net == 0)
    ctx.set_geometry(wl.solid, wl.wall_q)
    with pytest.raises(ek.EKError):
        ctx.crossings(n)


def test_crossings_follow_the_chain_single_pore_64x64x128(ek):
    """The default benchmark configuration (float32 populations, lattice
    update beside the chain): the record equals the crossing rule applied to
    the chain's own positions read after every step."""
    wl = workloads.single_pore()
    n = wl.beads_R.shape[0]
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-8, poisson_max_iter=200, warm_start=ek.EK_WS_EXTRAP)
    Lz = float(ctx.shape[0])
    ctx.step(5)
    R0, _ = ctx.beads(n)
    z_plane = float(np.median(R0[:, 2]))       # a plane through the chain: several beads cross
    ctx.set_crossing_plane(z_plane)
    hist = [R0[:, 2].copy()]
    for _ in range(40):
        ctx.step(1)
        hist.append(ctx.beads(n)[0][:, 2].copy())
    first, last, net = obs.bead_crossings(np.array(hist), z_plane, Lz)
    g_first, g_last, g_net = ctx.crossings(n)
    # steps are counted from the context's start (5 steps before the plane)
    exp_first = np.where(first >= 0, first + 5, -1)
    exp_last = np.where(last >= 0, last + 5, -1)
    print(z_plane, g_first, exp_first, g_net)
    assert np.array_equal(g_first, exp_first)
    assert np.array_equal(g_last, exp_last)
    assert np.array_equal(g_net, net)


def test_observable_errors(ek):
    wl = pore_with_chain()
    ctx = ek.from_workload(wl, precision=ek.EK_FP32)
    Z = ctx.shape[0]
    for z in (-1, Z):
        with pytest.raises(ek.EKError):
            ctx.plane_flux(z)
    with pytest.raises(ek.EKError):
        ctx.set_crossing_plane(float("nan"))
    with pytest.raises(ek.EKError):
        ctx.crossings(wl.beads_R.shape[0])
    out = ctx.plane_flux(Z - 1)                # before any step: the initial state's streaming
    assert np.all(np.isfinite(out))
