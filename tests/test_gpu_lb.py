"""GPU parity of the lattice step and the Poisson solver against the float64
oracle, through the C ABI.

Bars: float64 populations agree with the oracle to rounding (1e-9); float32
populations (stored as deviations from rest) agree to 1e-5 in densities and
velocities after 100 steps (the stated tolerance), and the Poisson residual of
the GPU potential, recomputed by the oracle in float64, meets the solver's
tolerance.
"""
import numpy as np
import pytest

from oracle import lb as olb
from oracle import poisson as opoisson
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


def oracle_sim(wl, tol, max_iter=100000):
    p = ostep.Params(valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                     bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_tol=tol,
                     poisson_max_iter=max_iter)
    beads = None
    if wl.beads_R is not None:
        beads = (wl.beads_R, wl.beads_V, wl.polymer)
    return ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0, beads=beads)


def compare(ctx, sim, fluid):
    out = {}
    n_ref = sim.densities()
    u_ref = sim.velocities()
    for s in range(3):
        n, u = ctx.moments(s)
        out[f"n{s}"] = density_error(n, n_ref[s], fluid)
        out[f"u{s}"] = velocity_error(u, u_ref[s], fluid)
    out["psi"] = field_error(ctx.potential(), sim.psi)
    return out


def test_plain_box_fp64_matches_oracle(ek):
    """Plain periodic box (32^3, salt noise, no walls, no field), float64,
    red-black SOR to 1e-10 with a residual test after every iteration."""
    wl = workloads.plain_box(32, steps=50)
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_tol=1e-10, poisson_check_every=1)
    sim = oracle_sim(wl, 1e-10)
    for chunk in (1, 9, 40):
        ctx.step(chunk)
        sim.run(chunk)
        st = ctx.stats()
        assert st["poisson_iters"] == sim.last_iters
        err = compare(ctx, sim, wl.solid == 0)
        print(sim.t, err, st["poisson_iters"], np.abs(sim.velocities()).max(axis=(1, 2, 3, 4)))
        assert max(err[k] for k in ("n0", "n1", "n2", "psi")) < 1e-9, err
        # the uncharged solvent barely moves in a field-free box (|u| ~ 1e-9),
        # so its relative velocity error is a ratio of rounding to a tiny scale
        assert max(err[k] for k in ("u0", "u1", "u2")) < 1e-5, err
    m0 = wl.n0.sum(axis=(1, 2, 3))
    assert np.allclose(st["mass"], m0, rtol=1e-13)


@pytest.mark.parametrize("iterations", [1, 2, 7, 25])
def test_sor_iterates_match_oracle(ek, iterations):
    shape = (16, 12, 20)
    rng = np.random.default_rng(9)
    rho = rng.normal(size=shape)
    b = opoisson.rhs_from_charge(rho, 0.341)
    psi0 = rng.normal(size=shape) * 0.1
    p = ek.make_params(shape, precision=ek.EK_FP64)
    ctx = ek.Context(p)
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    pt = torch.tensor(psi0, dtype=torch.float64, device="cuda")
    ctx.sor_iterations(bt, pt, iterations)
    ref, _, _ = opoisson.sor_red_black_chebyshev(b, psi0, 0.0, 0, iterations=iterations)
    got = pt.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape,tol,check", [((32, 32, 64), 1e-8, 1), ((24, 16, 48), 1e-10, 4)])
def test_poisson_solve_meets_tolerance(ek, shape, tol, check):
    rng = np.random.default_rng(3)
    rho = rng.normal(size=shape) * 0.01
    p = ek.make_params(shape, precision=ek.EK_FP64, poisson_tol=tol, poisson_check_every=check)
    ctx = ek.Context(p)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    pt = torch.zeros(shape, dtype=torch.float64, device="cuda")
    rep = ctx.poisson_solve(rt, pt, ek.EK_WS_ZERO)
    psi = pt.cpu().numpy()
    eps = 1.0 / (4 * np.pi * 0.7 / 3.0)
    b = opoisson.rhs_from_charge(rho, eps)
    assert opoisson.relative_residual(psi, b) <= tol
    assert rep["residual"] == pytest.approx(opoisson.relative_residual(psi, b), rel=1e-6)
    assert abs(psi.mean()) < 1e-12 * np.abs(psi).max()
    ref, it, _ = opoisson.sor_red_black_chebyshev(b, np.zeros(shape), tol, 100000)
    if check == 1:
        assert rep["iterations"] == it
    assert field_error(psi, ref) < 1e3 * tol


def pore(beads=0):
    return workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, beads, 21, steps=100)


def test_pore_fp32_matches_oracle_after_100_steps(ek):
    wl = pore()
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_tol=1e-8, poisson_check_every=1)
    sim = oracle_sim(wl, 1e-8)
    ctx.step(100)
    sim.run(100)
    err = compare(ctx, sim, wl.solid == 0)
    print(err)
    assert max(err[k] for k in err if k != "psi") < 1e-5, err
    eps = 1.0 / (4 * np.pi * 0.7 / 3.0)
    assert err["psi"] < 1e-5
    # the GPU potential solves the GPU charge density to the tolerance; check it
    # against the oracle's charge density of the GPU densities
    n = [ctx.moments(s)[0] for s in range(3)]
    rho = n[1] - n[2] + wl.wall_q
    b = opoisson.rhs_from_charge(rho, eps)
    # the GPU solved the system of the previous step's densities; one step
    # changes rho by little, so the residual against this b stays small
    assert opoisson.relative_residual(ctx.potential(), b) < 1e-3


@pytest.mark.parametrize("start", ["extrapolated", "quadratic", "cubic"])
def test_pore_fp32_multigrid_extrapolated_starts_match_oracle(ek, start):
    """The extrapolated starts of the solve (the linear, quadratic and cubic
    polynomials in time through the last two, three, four solutions) change
    where the multigrid begins, not where it ends: 100 steps agree with the
    oracle's previous-solution SOR at the same tolerance."""
    wl = pore()
    ws = {"extrapolated": ek.EK_WS_EXTRAP, "quadratic": ek.EK_WS_EXTRAP2,
          "cubic": ek.EK_WS_EXTRAP3}[start]
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-9, poisson_max_iter=200, warm_start=ws)
    sim = oracle_sim(wl, 1e-10)
    ctx.step(100)
    sim.run(100)
    err = compare(ctx, sim, wl.solid == 0)
    print(start, err, ctx.stats()["poisson_residual0"])
    assert max(err.values()) < 1e-5, err


def test_pore_fp64_matches_oracle(ek):
    wl = pore()
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_tol=1e-10, poisson_check_every=1)
    sim = oracle_sim(wl, 1e-10)
    ctx.step(30)
    sim.run(30)
    err = compare(ctx, sim, wl.solid == 0)
    print(err)
    assert max(err.values()) < 1e-8, err


@pytest.mark.parametrize("nx", [128, 256])
def test_whole_row_blocks_match_oracle(ek, nx):
    """Rows of 128 and 256 sites: the charge pass and the fused step then run
    on blocks of whole x-rows (one row per block), with the pore's bounce-back
    links, periodic wrap in x inside the block and 16 / 8 planes of rows."""
    wl = workloads.pore_system((16, 8, nx), 4, 2, 0.01, 0.01, -0.01, 0, 23, steps=12)
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_tol=1e-10, poisson_check_every=1)
    sim = oracle_sim(wl, 1e-10)
    ctx.step(12)
    sim.run(12)
    err = compare(ctx, sim, wl.solid == 0)
    print(nx, err)
    assert max(err.values()) < 1e-8, err


def test_fp32_mass_conserved_and_deterministic(ek):
    wl = pore()
    runs = []
    for _ in range(2):
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_tol=1e-8, poisson_check_every=4)
        ctx.step(150)
        st = ctx.stats()
        m0 = wl.n0.sum(axis=(1, 2, 3))
        # float32 storage rounds every stored deviation g (|g| <~ 5e-3 for the
        # ions next to the wall) to 2^-24 relative: a random walk of about
        # sqrt(150 steps * 19 * 1.5e4 sites) * 3e-10 ~ 2e-6 in a mass of ~150
        assert np.allclose(st["mass"], m0, rtol=1e-7), (st["mass"], m0)
        runs.append([ctx.moments(s) for s in range(3)] + [ctx.potential()])
        ctx.close()
    for a, b in zip(runs[0][:3], runs[1][:3]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(runs[0][3], runs[1][3])


def test_no_convergence_leaves_state(ek):
    wl = pore()
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_tol=1e-8)
    ctx.step(2)
    before = ctx.moments(1)
    ctx.params.poisson_max_iter = 1
    ctx2 = ek.from_workload(wl, precision=ek.EK_FP32, poisson_tol=1e-14, poisson_max_iter=1)
    with pytest.raises(ek.EKError) as e:
        ctx2.step(1)
    assert e.value.status == ek.EK_ENOCONV
    assert ctx2.stats()["step"] == 0
    n, u = ctx2.moments(1)
    assert np.allclose(n[wl.solid == 0], wl.n0[1][wl.solid == 0], rtol=1e-6)
    assert before[0].shape == n.shape


def test_invalid_arguments(ek):
    p = ek.make_params((8, 8, 8))
    ctx = ek.Context(p)
    with pytest.raises(ek.EKError) as e:
        ctx.step(1)
    assert e.value.status == ek.EK_ESTATE
    with pytest.raises(ek.EKError) as e:
        ctx.set_species_density(3, np.ones((8, 8, 8)))
    assert e.value.status in (ek.EK_EINVAL, ek.EK_ESTATE)
    ctx.set_geometry(np.zeros((8, 8, 8), np.uint8))
    with pytest.raises(ek.EKError) as e:
        ctx.set_species_density(0, -np.ones((8, 8, 8)))
    assert e.value.status == ek.EK_EINVAL
    with pytest.raises(ek.EKError) as e:
        ctx._check(ctx._lib.ek_set_launch_mode(ctx._h, 4), ctx._h)      # unknown launch flag
    assert e.value.status == ek.EK_EINVAL
    rho = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    psi = torch.zeros_like(rho)
    with pytest.raises(ek.EKError) as e:
        ctx.poisson_solve(rho, psi, warm_start=7)                           # unknown start
    assert e.value.status == ek.EK_EINVAL
    with pytest.raises(ek.EKError) as e:
        ctx.poisson_solve(rho, psi, warm_start=ek.EK_WS_LEARNED)           # no model
    assert e.value.status in (ek.EK_ESTATE, ek.EK_EINVAL)
