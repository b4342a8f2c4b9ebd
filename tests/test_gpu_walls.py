"""Insulating walls (the Neumann condition after Eq. poisson) and the
occupation-cube coupling theta_i (Eq. totalforcefluid) on the GPU against the
float64 oracle, element by element:

* a pore with insulating charged walls (charge on the solid sites sharing a
  face with the fluid), an applied field and an 8-bead chain, red-black SOR
  over the fluid: float64 after 20 steps (1e-8), float32 after 100 steps
  (1e-5), with the trilinear and with the theta coupling;
* theta coupling in the periodic problem, float64, cube sides 1 and 1.5
  (single beads for 1.5, whose WCA would burst the FENE chain);
* refusals: multigrid, the learned start, the periodic-only entry points, a
  charged solid site without a fluid face.
"""
import numpy as np
import pytest

from oracle import step as ostep
from paper_1710_09421_amd import workloads
from tests.parity import density_error, field_error, velocity_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def _wl(charge_sites="faces", n_beads=8):
    return workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, n_beads, 32, steps=100,
                                 charge_sites=charge_sites)


def _oracle(wl, walls, coupling="trilinear", tol=1e-11):
    p = ostep.Params(valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                     bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_tol=tol, walls=walls)
    beads = None
    if wl.beads_R is not None:
        beads = (wl.beads_R, wl.beads_V, dict(wl.polymer, coupling=coupling))
    return ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0, beads=beads)


def _errors(ctx, sim, wl):
    fluid = wl.solid == 0
    n_ref, u_ref = sim.densities(), sim.velocities()
    err = {}
    for s in range(3):
        n, u = ctx.moments(s)
        err[f"n{s}"] = density_error(n, n_ref[s], fluid)
        err[f"u{s}"] = velocity_error(u, u_ref[s], fluid)
    err["psi"] = field_error(ctx.potential(), sim.psi)
    if wl.beads_R is not None:
        nb = wl.beads_R.shape[0]
        R, V = ctx.beads(nb)
        err["R"] = float(np.abs(R - sim.R).max())
        err["V"] = float(np.abs(V - sim.V).max() / np.abs(sim.V).max())
    return err


def _ctx(ek, wl, precision, walls, coupling="trilinear", tol=1e-11, **kw):
    wl = workloads.Workload(**{**wl.__dict__, "polymer": dict(wl.polymer, coupling=coupling)})
    return ek.from_workload(wl, precision=precision, poisson_method=ek.EK_POISSON_SOR,
                            poisson_tol=tol, walls=walls, **kw)


@pytest.mark.parametrize("coupling", ["trilinear", "theta"])
def test_insulating_pore_fp64_matches_oracle(ek, coupling):
    wl = _wl()
    ctx = _ctx(ek, wl, ek.EK_FP64, "insulating", coupling)
    sim = _oracle(wl, "neumann", coupling)
    ctx.step(20)
    sim.run(20)
    err = _errors(ctx, sim, wl)
    print(coupling, err)
    assert max(err.values()) < 1e-8, err
    psi = ctx.potential()
    fluid = wl.solid == 0
    assert not psi[~fluid].any() and abs(psi[fluid].mean()) < 1e-14
    # insulating walls change the answer: the periodic problem differs
    per = _ctx(ek, workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 32,
                                         charge_sites="faces"), ek.EK_FP64, "periodic", coupling)
    per.step(20)
    assert np.abs(per.potential() - psi)[fluid].max() > 1e-3 * np.abs(psi).max()


def test_insulating_pore_fp32_theta_matches_oracle_after_100_steps(ek):
    wl = _wl()
    ctx = _ctx(ek, wl, ek.EK_FP32, "insulating", "theta", tol=1e-9, poisson_check_every=4,
               warm_start=ek.EK_WS_EXTRAP)
    sim = _oracle(wl, "neumann", "theta")
    ctx.step(100)
    sim.run(100)
    err = _errors(ctx, sim, wl)
    print(err)
    assert max(err.values()) < 1e-5, err


@pytest.mark.parametrize("sigma", [1.0, 1.5])
def test_theta_coupling_periodic_fp64_matches_oracle(ek, sigma):
    if sigma == 1.0:
        wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 33, steps=20)
    else:
        wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 1, 34, steps=20)
        wl.beads_V = np.array([[0.02, -0.01, 0.015]])
    wl.polymer = dict(wl.polymer, sigma=sigma)
    ctx = _ctx(ek, wl, ek.EK_FP64, "periodic", "theta")
    sim = _oracle(wl, "periodic", "theta")
    ctx.step(20)
    sim.run(20)
    err = _errors(ctx, sim, wl)
    print(sigma, err)
    assert max(err.values()) < 1e-8, err


def test_insulating_walls_refusals(ek):
    lib = ek.lib()
    import ctypes
    nbytes = ctypes.c_size_t()
    for kw in (dict(poisson_method=ek.EK_POISSON_MG), dict(warm_start=ek.EK_WS_LEARNED)):
        p = ek.make_params((32, 24, 24), walls="insulating", **kw)
        assert lib.ek_workspace_bytes(ctypes.byref(p), 0, ctypes.byref(nbytes)) == ek.EK_EINVAL
    wl = _wl(n_beads=0)
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, walls="insulating")
    rho = torch.zeros(wl.shape, dtype=torch.float64, device="cuda")
    psi = torch.zeros_like(rho)
    with pytest.raises(ek.EKError) as e:
        ctx.poisson_solve(rho, psi)
    assert e.value.status == ek.EK_ESTATE
    # wall charges on solid sites that touch the fluid only along edges
    edges = _wl(charge_sites="links", n_beads=0)
    bad = ek.Context(ek.make_params(edges.shape, walls="insulating"))
    with pytest.raises(ek.EKError) as e:
        bad.set_geometry(edges.solid, edges.wall_q)
    assert e.value.status == ek.EK_EINVAL
    # the state of an insulating context round-trips (its wall charges as given)
    ctx.step(3)
    buf = ctx.save_state()
    other = ek.Context(ctx.params)
    other.load_state(buf)
    ctx.step(2)
    other.step(2)
    assert np.array_equal(ctx.potential(), other.potential())
