"""Multigrid cycles replayed from recorded HIP graphs give the same bits as the
same kernels launched one by one: every replay is compared with the eager
result, with the program's own eager work (charge pass, chain, lattice step)
and host synchronisations between the replays, and after the graphs are
recorded again for another psi buffer."""
import numpy as np
import pytest

from paper_1710_09421_amd import workloads

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
        c.set_graph_launch(graphs)
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
