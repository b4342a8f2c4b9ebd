"""The no-allocation Poisson solve (ek_poisson_solve_noalloc) against the
context's stand-alone solve (ek_poisson_solve) with the same red-black SOR
settings: bit for bit the same potential, iteration count and residuals, on
two calls in a row of which the second is smaller (the static scratch keeps
the first call's contents), from a zero and from a given start; invalid
requests are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def _params(ek, shape, tol=1e-10, check_every=3):
    return ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_SOR,
                          poisson_tol=tol, poisson_max_iter=20000, poisson_check_every=check_every)


def _solve_both(ek, shape, seed, warm):
    rng = np.random.default_rng(seed)
    rho = torch.tensor(rng.normal(size=shape), dtype=torch.float64, device="cuda")
    start = torch.tensor(rng.normal(size=shape) * 0.1, dtype=torch.float64, device="cuda")
    p = _params(ek, shape)
    ctx = ek.Context(p)
    psi_ctx = start.clone()
    rep_ctx = ctx.poisson_solve(rho, psi_ctx, warm_start=warm)
    psi_na = start.clone() if warm != ek.EK_WS_ZERO else torch.full_like(start, 7.0)
    rep_na = ek.poisson_solve_noalloc(p, rho, psi_na, warm_start=warm)
    torch.cuda.synchronize()
    ctx.close()
    return psi_ctx.cpu().numpy(), rep_ctx, psi_na.cpu().numpy(), rep_na


@pytest.mark.parametrize("warm", ["zero", "previous"])
def test_noalloc_solve_equals_context_solve_twice_second_smaller(ek, warm):
    ws = ek.EK_WS_ZERO if warm == "zero" else ek.EK_WS_PREV
    for shape, seed in (((32, 24, 20), 5), ((16, 12, 8), 6)):
        psi_ctx, rep_ctx, psi_na, rep_na = _solve_both(ek, shape, seed, ws)
        assert rep_na["iterations"] == rep_ctx["iterations"] > 0
        assert rep_na["residual"] == rep_ctx["residual"] <= 1e-10
        assert rep_na["initial_residual"] == rep_ctx["initial_residual"]
        assert np.array_equal(psi_na, psi_ctx), shape
        assert abs(psi_na.mean()) < 1e-12


def test_noalloc_refuses_invalid_requests(ek):
    lib = ek.lib()
    shape = (16, 12, 8)
    rho = torch.zeros(shape, dtype=torch.float64, device="cuda")
    psi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    mg = ek.make_params(shape, precision=ek.EK_FP64, poisson_method=ek.EK_POISSON_MG)
    with pytest.raises(ek.EKError) as e:
        ek.poisson_solve_noalloc(mg, rho, psi)
    assert e.value.status == ek.EK_EINVAL and "SOR" in str(e.value)
    big = _params(ek, (256, 128, 128))            # 2^22 sites
    with pytest.raises(ek.EKError) as e:
        ek.poisson_solve_noalloc(big, rho, psi)
    assert e.value.status == ek.EK_EINVAL and "maximum" in str(e.value)
    with pytest.raises(ek.EKError) as e:
        ek.poisson_solve_noalloc(_params(ek, shape), rho, psi, warm_start=ek.EK_WS_LEARNED)
    assert e.value.status == ek.EK_EINVAL
    # a vanishing charge gives the zero potential at once
    rep = ek.poisson_solve_noalloc(_params(ek, shape), rho, psi.fill_(3.0))
    assert rep["iterations"] == 0 and float(psi.abs().max()) == 0.0
