"""Launch modes give the same results as plain launches one after the other.

Graphs: multigrid cycles replayed from recorded HIP graphs give the same bits
as the same kernels launched one by one: every replay is compared with the
eager result, with the program's own eager work (charge pass, chain, lattice
step) and host synchronisations between the replays, and after the graphs are
recorded again for another psi buffer.

Overlap: the lattice update of the sites outside the bead boxes, run beside
the chain kernel, plus the update of the box sites after it, gives the same
fields and beads bit for bit as the whole lattice kernel after the chain; the
float64 mass sums agree to rounding (their order differs); every fluid site is
updated once per step."""
import dataclasses

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


def _pair(ek, wl):
    ctxs = []
    for graphs in (True, False):
        c = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                             poisson_tol=1e-8, poisson_max_iter=200)
        c.set_launch_mode(graphs=graphs, overlap=True)
        ctxs.append(c)
    return ctxs


def _same_state(a, b, n_beads):
    assert np.array_equal(a.potential(), b.potential())
    for s in range(3):
        na, ua = a.moments(s)
        nb, ub = b.moments(s)
        assert np.array_equal(na, nb) and np.array_equal(ua, ub)
    if n_beads:
        assert np.array_equal(a.beads(n_beads)[0], b.beads(n_beads)[0])


@pytest.mark.parametrize("size", ["small", "single-pore"])
def test_replayed_cycles_match_single_launches(ek, size):
    if size == "small":
        wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 32, steps=8)
        nbd, steps = 8, 8
    else:
        wl = workloads.single_pore()
        nbd, steps = 32, 5
    g, e = _pair(ek, wl)
    for t in range(steps):
        g.step(1)
        e.step(1)
        sg, se = g.stats(), e.stats()
        print(size, t, sg["poisson_iters"], se["poisson_iters"], sg["poisson_residual"])
        assert sg["poisson_iters"] == se["poisson_iters"] >= 1
        assert sg["poisson_residual"] == se["poisson_residual"] <= 1e-8
        assert np.array_equal(sg["mass"], se["mass"])
        _same_state(g, e, nbd)


def test_fused_finest_level_replays_match_single_launches(ek):
    """A 128 x 128 x 256 pore, whose finest level runs the sweeps marching up
    z on 64 x 8 tiles (32 tiles x 32 chunks) with the fused restriction,
    correction and norms, and takes the start's residual in the first cycle:
    the first-cycle and later-cycle graphs give the same bits, cycle counts
    and initial residuals as the same launches one by one."""
    wl = workloads.pore_system((256, 128, 128), 12, 8, 0.01, 0.01, -0.01, 8, 34, steps=4)
    g, e = _pair(ek, wl)
    for t in range(4):
        g.step(1)
        e.step(1)
        sg, se = g.stats(), e.stats()
        print(t, sg["poisson_iters"], sg["poisson_residual0"], sg["poisson_residual"])
        assert sg["poisson_iters"] == se["poisson_iters"] >= 1
        assert sg["poisson_residual0"] == se["poisson_residual0"]
        assert sg["poisson_residual"] == se["poisson_residual"] <= 1e-8
        assert np.array_equal(sg["mass"], se["mass"])
        _same_state(g, e, 8)


def test_replay_follows_the_psi_buffer(ek):
    """Stand-alone solves into caller buffers between steps: the graphs are
    recorded again for each buffer and the iteration counts kept on the
    device match the host's."""
    wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 33, steps=4)
    g, e = _pair(ek, wl)
    rng = np.random.default_rng(3)
    rho = torch.tensor(rng.normal(size=wl.shape) * 0.01, dtype=torch.float64, device="cuda")
    for t in range(3):
        g.step(1)
        e.step(1)
        outs = []
        for c in (g, e):
            p1 = torch.zeros(wl.shape, dtype=torch.float64, device="cuda")
            p2 = torch.zeros(wl.shape, dtype=torch.float64, device="cuda")
            r1 = c.poisson_solve(rho, p1, ek.EK_WS_ZERO)
            r2 = c.poisson_solve(rho * 1.001, p2, ek.EK_WS_ZERO)
            r3 = c.poisson_solve(rho * 1.002, p2, ek.EK_WS_PREV)
            outs.append((r1, r2, r3, p1.cpu().numpy(), p2.cpu().numpy()))
        (g1, g2, g3, gp1, gp2), (e1, e2, e3, ep1, ep2) = outs
        print(t, g1, g3, e3)
        assert g1 == e1 and g2 == e2 and g3 == e3
        assert g3["iterations"] < g2["iterations"]
        assert np.array_equal(gp1, ep1) and np.array_equal(gp2, ep2)
        _same_state(g, e, 8)


def _wrapping_chain():
    """8^3 periodic box with a 4-bead chain across the x = 0 boundary: the
    boxes of neighbouring beads overlap and wrap around the box."""
    wl = workloads.plain_box(8, seed=5, steps=6)
    R = np.array([[7.55, 4.0, 4.0], [0.52, 4.05, 4.0], [1.49, 4.15, 4.05], [2.45, 4.35, 4.15]])
    V = np.array([[0.01, 0.0, 0.0], [0.0, 0.01, 0.0], [0.0, 0.0, 0.01], [-0.01, 0.0, 0.0]])
    return dataclasses.replace(wl, name="plain-8^3-wrapping-chain", beads_R=R, beads_V=V,
                               polymer=ostep.polymer_params(4, q=-0.1), E_ext=(0.0, 0.0, 0.01))


@pytest.mark.parametrize("size", ["wrapping", "small", "single-pore"])
def test_overlapped_lattice_update_matches_serial(ek, size):
    if size == "wrapping":
        wl, steps = _wrapping_chain(), 6
    elif size == "small":
        wl, steps = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 34, steps=8), 8
    else:
        wl, steps = workloads.single_pore(), 5
    nbd = wl.beads_R.shape[0]
    ctxs = []
    for overlap in (True, False):
        c = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                             poisson_tol=1e-8, poisson_max_iter=200)
        c.set_launch_mode(graphs=True, overlap=overlap)
        c.set_timing(True)
        ctxs.append(c)
    o, s = ctxs
    for t in range(steps):
        o.step(1)
        s.step(1)
        so, ss = o.stats(), s.stats()
        assert so["poisson_iters"] == ss["poisson_iters"]
        assert np.allclose(so["mass"], ss["mass"], rtol=1e-13, atol=0), (so["mass"], ss["mass"])
        assert np.allclose(so["momentum"], ss["momentum"], rtol=1e-12, atol=1e-15)
        _same_state(o, s, nbd)
    to, ts = o.timing(), s.timing()
    fluid = wl.fluid_sites
    print(size, to["lb_sites"] / steps, ts["lb_sites"] / steps, fluid, to["ms_lb"], ts["ms_lb"])
    assert ts["lb_sites"] == steps * fluid
    deferred = steps * fluid - to["lb_sites"]
    assert 0 < deferred <= steps * 64 * nbd


def test_wrapping_chain_with_overlap_matches_oracle(ek):
    """The overlapped update against the float64 oracle (float64 populations)
    for the chain across the periodic boundary."""
    wl = _wrapping_chain()
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_tol=1e-10, poisson_check_every=1)
    p = ostep.Params(valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                     bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_tol=1e-10)
    sim = ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0,
                           beads=(wl.beads_R, wl.beads_V, wl.polymer))
    ctx.step(6)
    sim.run(6)
    fluid = wl.solid == 0
    err = {}
    for s in range(3):
        n, u = ctx.moments(s)
        err[f"n{s}"] = density_error(n, sim.densities()[s], fluid)
        err[f"u{s}"] = velocity_error(u, sim.velocities()[s], fluid)
    err["psi"] = field_error(ctx.potential(), sim.psi)
    err["R"] = float(np.abs(ctx.beads(4)[0] - sim.R).max())
    print(err)
    assert max(err.values()) < 1e-8, err
