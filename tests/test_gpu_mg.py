"""Red-black multigrid solves the same discrete Poisson problem as the
paper's red-black SOR: its solution meets the residual tolerance when the
oracle recomputes the residual in float64, and agrees with the oracle's SOR
solution within the error that tolerance allows."""
import numpy as np
import pytest

from oracle import poisson as opoisson
from oracle import step as ostep
from paper_1710_09421_amd import workloads
from tests.parity import density_error, field_error, velocity_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 1.0 / (4 * np.pi * 0.7 / 3.0)


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


# (8, 16, 32): the finest level's 8^3-tile sweeps span a whole side, whose
# window then wraps onto the tile itself
@pytest.mark.parametrize("shape", [(128, 64, 64), (32, 32, 32), (48, 16, 24), (4, 2, 2), (6, 10, 14),
                                   (8, 16, 32)])
def test_multigrid_meets_tolerance(ek, shape):
    rng = np.random.default_rng(sum(shape))
    rho = rng.normal(size=shape) * 0.01
    p = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG,
                       poisson_tol=1e-8, poisson_max_iter=400)
    ctx = ek.Context(p)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    pt = torch.zeros(shape, dtype=torch.float64, device="cuda")
    rep = ctx.poisson_solve(rt, pt, ek.EK_WS_ZERO)
    psi = pt.cpu().numpy()
    b = opoisson.rhs_from_charge(rho, EPS)
    rr = opoisson.relative_residual(psi, b)
    print(shape, rep, rr)
    assert rr <= 1e-8
    assert abs(psi.mean()) < 1e-12 * np.abs(psi).max()
    if min(shape) >= 8:
        assert rep["iterations"] <= 12           # about a decade per V(1,2) cycle
    ref, _, _ = opoisson.sor_red_black_chebyshev(b, np.zeros(shape), 1e-12, 100000)
    assert field_error(psi, ref) < 1e3 * 1e-8


def test_multigrid_128_cubed_meets_tolerance(ek):
    """A 128^3 box (2^21 sites on the finest level).  Reference: the exact
    periodic solution of the 7-point problem by FFT (the SOR oracle is too slow
    at this size)."""
    shape = (128, 128, 128)
    rng = np.random.default_rng(5)
    rho = rng.normal(size=shape) * 0.01
    p = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG,
                       poisson_tol=1e-8, poisson_max_iter=400)
    ctx = ek.Context(p)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    pt = torch.zeros(shape, dtype=torch.float64, device="cuda")
    rep = ctx.poisson_solve(rt, pt, ek.EK_WS_ZERO)
    psi = pt.cpu().numpy()
    b = opoisson.rhs_from_charge(rho, EPS)
    rr = opoisson.relative_residual(psi, b)
    print(rep, rr)
    assert rr <= 1e-8 and rep["iterations"] <= 12
    k = [2 * np.pi * np.fft.fftfreq(n) for n in shape]
    lam = (2 * np.cos(k[0])[:, None, None] + 2 * np.cos(k[1])[None, :, None] +
           2 * np.cos(k[2])[None, None, :] - 6.0)
    lam[0, 0, 0] = 1.0
    bh = np.fft.fftn(b)
    bh[0, 0, 0] = 0.0
    ref = np.real(np.fft.ifftn(bh / lam))
    assert field_error(psi, ref) < 1e3 * 1e-8


def fft_solution(b):
    """Exact mean-free periodic solution of the 7-point problem A psi = b."""
    k = [2 * np.pi * np.fft.fftfreq(n) for n in b.shape]
    lam = (2 * np.cos(k[0])[:, None, None] + 2 * np.cos(k[1])[None, :, None] +
           2 * np.cos(k[2])[None, None, :] - 6.0)
    lam[0, 0, 0] = 1.0
    bh = np.fft.fftn(b)
    bh[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(bh / lam))


@pytest.mark.parametrize("shape", [(256, 128, 128), (128, 64, 64)])
def test_start_residual_taken_in_the_first_cycle(ek, shape):
    """Boxes whose finest level's first sweep takes the start's residual
    inside the first cycle (256 x 128 x 128: sweeps marching up z on 64 x 8
    tiles; 128 x 64 x 64: one launch per sweep on 8^3 tiles): the initial
    residual reported for a rough start is the host's residual of that
    start, and a start that already meets the tolerance (the exact solution
    plus a constant) leaves the solve at zero cycles with that start, its
    mean removed."""
    rng = np.random.default_rng(9)
    rho = rng.normal(size=shape) * 0.01
    p = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG,
                       poisson_tol=1e-8, poisson_max_iter=400)
    ctx = ek.Context(p)
    b = opoisson.rhs_from_charge(rho, EPS)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    start = rng.normal(size=shape) * 0.05
    pt = torch.tensor(start, dtype=torch.float64, device="cuda")
    rep = ctx.poisson_solve(rt, pt, ek.EK_WS_PREV)
    want = opoisson.relative_residual(start, b)
    print(rep, want)
    assert rep["initial_residual"] == pytest.approx(want, rel=1e-10)
    assert opoisson.relative_residual(pt.cpu().numpy(), b) <= 1e-8
    exact = fft_solution(b) + 0.25
    pt = torch.tensor(exact, dtype=torch.float64, device="cuda")
    rep = ctx.poisson_solve(rt, pt, ek.EK_WS_PREV)
    print(rep)
    assert rep["iterations"] == 0
    assert rep["initial_residual"] <= 1e-8
    assert np.abs(pt.cpu().numpy() - (exact - exact.mean())).max() < 1e-12


@pytest.mark.parametrize("shape", [(128, 64, 64), (256, 128, 128)])
def test_multigrid_stops_at_the_cycle_limit(ek, shape):
    """A tolerance no cycle count reaches: the solve runs exactly
    poisson_max_iter cycles (the batches before the limit replayed as
    recorded graphs, the last one launched cycle by cycle with its test) and
    reports EK_ENOCONV with that count; psi holds the iterate it reached,
    whose residual the oracle confirms is far below the start's."""
    rng = np.random.default_rng(sum(shape) + 7)
    rho = rng.normal(size=shape) * 0.01
    p = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG,
                       poisson_tol=1e-30, poisson_max_iter=3)
    ctx = ek.Context(p)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    pt = torch.zeros(shape, dtype=torch.float64, device="cuda")
    with pytest.raises(ek.EKError) as e:
        ctx.poisson_solve(rt, pt, ek.EK_WS_ZERO)
    print(e.value)
    assert e.value.status == ek.EK_ENOCONV
    assert "in 3 cycles" in str(e.value)
    b = opoisson.rhs_from_charge(rho, EPS)
    assert opoisson.relative_residual(pt.cpu().numpy(), b) < 1e-3


@pytest.mark.parametrize("shape", [(36, 36, 36), (44, 44, 44)])
def test_multigrid_with_a_large_coarsest_level(ek, shape):
    """Boxes whose sides stop halving early: the coarsest level of 36^3 is
    18^3 = 5,832 sites (more than the one-workgroup coarse kernel reads ahead
    per thread), that of 44^3 is 22^3 = 10,648 sites (more than one
    workgroup's LDS holds, so it is swept on the grid).  Both must still
    reach the tolerance, in graph replay and in single launches."""
    rng = np.random.default_rng(sum(shape) + 1)
    rho = rng.normal(size=shape) * 0.01
    b = opoisson.rhs_from_charge(rho, EPS)
    ref = fft_solution(b)
    for graphs in (True, False):
        p = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-8, poisson_max_iter=400)
        ctx = ek.Context(p)
        ctx.set_launch_mode(graphs=graphs, overlap=True)
        rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
        pt = torch.zeros(shape, dtype=torch.float64, device="cuda")
        rep = ctx.poisson_solve(rt, pt, ek.EK_WS_ZERO)
        psi = pt.cpu().numpy()
        rr = opoisson.relative_residual(psi, b)
        print(shape, graphs, rep, rr)
        assert rr <= 1e-8 and rep["iterations"] <= 12
        assert field_error(psi, ref) < 1e3 * 1e-8


def test_multigrid_warm_start_needs_fewer_cycles(ek):
    shape = (64, 32, 32)
    rng = np.random.default_rng(5)
    rho = rng.normal(size=shape) * 0.01
    p = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG, poisson_tol=1e-8)
    ctx = ek.Context(p)
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    pt = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cold = ctx.poisson_solve(rt, pt, ek.EK_WS_ZERO)
    rt2 = rt * (1.0 + 1e-4 * torch.randn_like(rt))
    warm = ctx.poisson_solve(rt2, pt, ek.EK_WS_PREV)
    assert warm["iterations"] < cold["iterations"]
    assert warm["initial_residual"] < 1e-2


@pytest.mark.parametrize("start", ["previous", "extrapolated"])
def test_pore_fp32_with_multigrid_matches_oracle(ek, start):
    """Each step's solve starts from the previous solution, or from the linear
    extrapolation of the two previous ones; the oracle starts SOR from the
    previous solution.  Both finish to 1e-8."""
    wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 32, steps=100)
    ws = ek.EK_WS_PREV if start == "previous" else ek.EK_WS_EXTRAP
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-8, warm_start=ws)
    p = ostep.Params(E_ext=wl.E_ext, poisson_tol=1e-8)
    sim = ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0,
                           beads=(wl.beads_R, wl.beads_V, wl.polymer))
    ctx.step(100)
    sim.run(100)
    fluid = wl.solid == 0
    n_ref, u_ref = sim.densities(), sim.velocities()
    err = {}
    for s in range(3):
        n, u = ctx.moments(s)
        err[f"n{s}"] = density_error(n, n_ref[s], fluid)
        err[f"u{s}"] = velocity_error(u, u_ref[s], fluid)
    err["psi"] = field_error(ctx.potential(), sim.psi)
    err["R"] = float(np.abs(ctx.beads(8)[0] - sim.R).max())
    print(err)
    assert max(err.values()) < 1e-5, err


def test_extrapolated_start_needs_fewer_cycles(ek):
    """Single pore, 60 steps after 10: the extrapolated start begins closer to
    the solution than the previous one and needs no more multigrid cycles per
    step; every solve meets the tolerance."""
    wl = workloads.single_pore()
    cycles, res0 = {}, {}
    for name, ws in (("previous", ek.EK_WS_PREV), ("extrapolated", ek.EK_WS_EXTRAP)):
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                               poisson_tol=1e-8, poisson_max_iter=200, warm_start=ws)
        ctx.step(10)
        ctx.set_timing(True)
        r0 = []
        for _ in range(60):
            ctx.step(1)
            st = ctx.stats()
            assert st["poisson_residual"] <= 1e-8
            r0.append(st["poisson_residual0"])
        cycles[name] = ctx.timing()["poisson_iters"] / 60
        res0[name] = float(np.median(r0))
        ctx.close()
    print(cycles, res0)
    assert res0["extrapolated"] < 0.5 * res0["previous"]
    assert cycles["extrapolated"] <= cycles["previous"]


def _ahead_weights(m):
    """Weights of the values at times -1, -2, .., -m in the value at time 0 of
    the polynomial of degree m - 1 through them (Lagrange's form)."""
    t = -np.arange(1, m + 1, dtype=float)
    w = np.ones(m)
    for j in range(m):
        for i in range(m):
            if i != j:
                w[j] *= (0.0 - t[i]) / (t[j] - t[i])
    return w


@pytest.mark.parametrize("start,points", [("extrapolated", 2), ("quadratic", 3), ("cubic", 4)])
def test_extrapolated_start_is_the_polynomial_through_the_last_solutions(ek, start, points):
    """Step k's solve starts from the polynomial in time through the last
    min(k - 1, points) solutions, evaluated one step ahead (zero on the first
    step after the geometry): the residual of that field against step k's
    right-hand side, formed here on the host from the solutions read back,
    is the initial residual the solver reports."""
    wl = workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 32, steps=12)
    ws = {"extrapolated": ek.EK_WS_EXTRAP, "quadratic": ek.EK_WS_EXTRAP2,
          "cubic": ek.EK_WS_EXTRAP3}[start]
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-12, poisson_max_iter=200, warm_start=ws)
    rhs = torch.empty(wl.shape, dtype=torch.float64, device="cuda")
    psi = torch.empty_like(rhs)
    hist = []
    for k in range(1, 10):
        ctx.step(1)
        ctx.poisson_system(rhs, psi)
        b = rhs.cpu().numpy()
        m = min(k - 1, points)
        guess = np.zeros(wl.shape)
        for w, old in zip(_ahead_weights(m), hist[::-1]):
            guess += w * old
        want = opoisson.relative_residual(guess, b)
        got = ctx.stats()["poisson_residual0"]
        print(k, m, got, want)
        assert got == pytest.approx(want, rel=1e-7), (k, got, want)
        hist.append(ctx.potential())
    ctx.close()
