"""The learned Poisson warm start end to end on the GPU, with the committed
network (trained on 2000 pairs of 64 x 64 x 128 pore systems by the library's
own kernels): held-out fields are solved by multigrid to the same 1e-8
residual from a zero start, from the network's guess, from the previous
step's solution, and from the previous solution with the network consulted.
The test records what the network gains over the method without it (cycles
and wall time of each start) and checks what the design guarantees: the
same tolerance is reached, the fallback never lets the learned start cost
cycles, the gate skips the network when the previous solution is already
close, and a corrupted network is rejected."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek, learned
    ek.lib()
    return ek, learned


@pytest.fixture(scope="module")
def held(mods):
    _, learned = mods
    return learned.generate(2, 3, 1, seed=4242, first=20, log=lambda s: None)


def test_learned_start_on_held_out_fields(mods, held):
    ek, learned = mods
    params, scale, info = learned.load_model()
    assert params.size == ek.UNET_PARAMS and info["n_traj"] * info["per_traj"] == 2000
    summary, rows = learned.evaluate(params, scale, held, repeats=1, log=lambda s: None)
    print(json.dumps(summary, indent=1))
    for r in rows:
        for k, v in r.items():
            if isinstance(v, dict):
                assert v["residual"] <= 1e-8, (r["index"], k, v)
    assert summary["learned"]["cycles"] <= summary["zero"]["cycles"]
    assert summary["learned"]["consulted"] == summary["learned"]["n"]       # cold: always asked
    assert summary["previous+learned"]["consulted"] == 0                   # close start: gated
    assert summary["previous+learned"]["cycles"] == summary["previous"]["cycles"]
    # the solutions agree to what the common tolerance allows
    assert max(r["learned"]["max_diff_vs_zero_start"] for r in rows) < 1e-6


def test_training_improved_the_guess(mods, held):
    """The trained network's guess is closer to the solution than that of the
    same network at its initial weights (what training gained); its error is
    printed, and is far from that of a solve: the potential of these systems
    is set by charges well outside the network's receptive field."""
    ek, learned = mods
    params, scale, _ = learned.load_model()
    net = ek.UNet(tuple(held["rhs"].shape[1:]), training=False)
    guess = torch.empty_like(held["rhs"][0])

    def errors(p):
        net.set_params(p, scale)
        out = []
        for i in range(held["rhs"].shape[0]):
            net.forward(held["rhs"][i], held["solid"][i], guess)
            g = guess - guess.mean()
            ref = held["psi"][i]
            out.append(float(torch.linalg.vector_norm(g - ref) / torch.linalg.vector_norm(ref)))
        return np.array(out)
    trained = errors(params)
    untrained = errors(learned.init_params(0))
    print("relative L2 error of the guess: trained", trained, "untrained", untrained)
    assert np.all(np.isfinite(trained))
    assert trained.mean() < 0.5 * untrained.mean()


def test_corrupted_network_is_rejected(mods, held):
    ek, learned = mods
    params, scale, _ = learned.load_model()
    shape = tuple(held["rhs"].shape[1:])
    p = ek.make_params((shape[0], shape[1], shape[2]), poisson_method=ek.EK_POISSON_MG,
                       poisson_tol=1e-8, poisson_max_iter=400, warm_start=ek.EK_WS_LEARNED)
    ctx = ek.Context(p)
    ctx.set_geometry(held["solid"][0].cpu().numpy())
    ctx.set_model(params * 40.0, scale)
    rho = -held["rhs"][0] / learned.INV_EPS
    psi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    rep = ctx.poisson_solve(rho, psi, ek.EK_WS_LEARNED)
    st = ctx.stats()
    assert st["consulted"] == 1 and st["fallback"] == 1
    assert rep["initial_residual"] == pytest.approx(1.0) and rep["residual"] <= 1e-8


def test_learned_mode_in_the_time_loop(mods):
    """Single pore (64 x 64 x 128, 32-bead chain): the network is consulted on
    the cold first step only, and the trajectory matches the previous-step
    start to the solver tolerance."""
    ek, learned = mods
    from paper_1710_09421_amd import workloads
    params, scale, _ = learned.load_model()
    wl = workloads.single_pore()
    out = {}
    for ws in (ek.EK_WS_PREV, ek.EK_WS_LEARNED):
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                               poisson_tol=1e-8, poisson_max_iter=200, warm_start=ws)
        if ws == ek.EK_WS_LEARNED:
            ctx.set_model(params, scale)
        consulted = []
        for _ in range(10):
            ctx.step(1)
            consulted.append(ctx.stats()["consulted"])
        out[ws] = (ctx.potential(), ctx.moments(1)[0], consulted)
        ctx.close()
    psi_p, n_p, _ = out[ek.EK_WS_PREV]
    psi_l, n_l, cons = out[ek.EK_WS_LEARNED]
    assert cons[0] == 1 and sum(cons[1:]) == 0
    assert np.abs(psi_l - psi_p).max() <= 1e-6 * np.abs(psi_p).max()
    assert np.abs(n_l - n_p).max() <= 1e-6 * np.abs(n_p).max()
