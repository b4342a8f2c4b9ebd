"""The translocation set-up of Sec. IV.A on the GPU against the float64
oracle: harmonic bonds of rest length 2 with the WCA of sigma = 2 between
non-neighbours (Eq. polymermodel, cut-off 2.245 beyond two lattice
spacings, so the chain kernel looks at wall sites two cells from the bead),
bead charge -0.1, Bjerrum length 1.4, one MD step per lattice step, a
membrane pierced by a pore of diameter 12 with a charged pore wall, the
chain starting at the pore entrance.

* a 32 x 32 x 64 box with a 16-site membrane and a 12-bead chain, float64,
  20 steps element by element (1e-8);
* the full 96 x 96 x 160 set-up with its 100-bead chain, float32 and
  multigrid to 1e-8 as the benchmark runs: 5 steps against the oracle's
  stored state (tests/golden/make_single_pore_golden.py, 1e-5), then 200
  more steps with mass conserved and the bonds near their rest length.
"""
import os

import numpy as np
import pytest

from oracle import step as ostep
from paper_1710_09421_amd import workloads
from tests.parity import density_error, field_error, velocity_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "translocation_96x96x160_5steps.npz")


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def test_small_translocation_box_fp64_matches_oracle(ek):
    wl = workloads.paper_translocation(shape=(64, 32, 32), membrane=16, n_beads=12)
    ctx = ek.from_workload(wl, precision=ek.EK_FP64, poisson_tol=1e-11)
    p = ostep.Params(valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                     bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_tol=1e-11)
    sim = ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0,
                           beads=(wl.beads_R, wl.beads_V, wl.polymer))
    ctx.step(20)
    sim.run(20)
    fluid = wl.solid == 0
    n_ref, u_ref = sim.densities(), sim.velocities()
    err = {}
    for s in range(3):
        n, u = ctx.moments(s)
        err[f"n{s}"] = density_error(n, n_ref[s], fluid)
        err[f"u{s}"] = velocity_error(u, u_ref[s], fluid)
    err["psi"] = field_error(ctx.potential(), sim.psi)
    R, V = ctx.beads(12)
    err["R"] = float(np.abs(R - sim.R).max())
    err["V"] = float(np.abs(V - sim.V).max() / np.abs(sim.V).max())
    print(err)
    assert max(err.values()) < 1e-8, err


def test_full_translocation_setup_matches_stored_oracle(ek):
    ref = np.load(GOLDEN)
    wl = workloads.paper_translocation()
    assert tuple(ref["shape"]) == wl.shape
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-8, poisson_max_iter=200, poisson_check_every=4,
                           warm_start=ek.EK_WS_EXTRAP)
    steps = int(ref["steps"][0])
    ctx.step(steps)
    idx = ref["sites"]
    err = {}
    for s in range(3):
        n, u = ctx.moments(s)
        err[f"n{s}"] = float(np.max(np.abs(n.ravel()[idx] - ref["n"][s]) / ref["n"][s]))
        err[f"u{s}"] = float(np.max(np.abs(u.reshape(3, -1)[:, idx] - ref["u"][s]))
                             / ref["u_scale"][s])
    err["psi"] = float(np.max(np.abs(ctx.potential().ravel()[idx] - ref["psi"]))
                       / ref["psi_scale"][0])
    R, V = ctx.beads(100)
    err["R"] = float(np.abs(R - ref["R"]).max())
    err["V"] = float(np.abs(V - ref["V"]).max() / np.abs(ref["V"]).max())
    print(err)
    assert max(err.values()) < 1e-5, err
    m0 = np.asarray(ctx.stats()["mass"])
    ctx.step(200)
    assert np.allclose(np.asarray(ctx.stats()["mass"]), m0, rtol=1e-9)
    R, _ = ctx.beads(100)
    bonds = np.linalg.norm(np.diff(R, axis=0), axis=1)
    assert 1.6 < bonds.min() and bonds.max() < 2.4, (bonds.min(), bonds.max())
