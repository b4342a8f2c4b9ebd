"""Parity at the shapes and in the launch configuration the benchmark runs:
float32 populations, multigrid to 1e-8 from the extrapolated start, the
lattice update beside the chain with the bead-box tail after it, cycles
replayed from graphs, 100 steps, element by element against the float64
oracle at the 1e-5 bar (densities pointwise, velocities relative to the
largest velocity of the species, the potential relative to its largest
value, bead positions absolute).

* A 256 x 8 x 24 pore box with an 8-bead chain: rows of 256 sites, so the
  lattice and charge kernels run the instance the 256 x 256 x 512 pore runs
  (whole-row blocks, 32-bit indices).
* The 64 x 64 x 128 single pore with its 32-bead chain.
Both against the oracle's state after 100 steps, stored by
tests/golden/make_single_pore_golden.py (8,000 sampled fluid sites, the
largest |u| and |psi| over the box, beads, species masses): the oracle needs
1.5-2.5 s per step at these shapes.
"""
import os

import numpy as np
import pytest

from paper_1710_09421_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def bench_context(ek, wl):
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=1e-8, poisson_max_iter=200, poisson_check_every=4,
                           warm_start=ek.EK_WS_EXTRAP)
    ctx.set_launch_mode(graphs=True, overlap=True)
    return ctx


CASES = {
    "whole-row-256x8x24": ("whole_row_256x8x24_100steps.npz",
                           lambda: workloads.pore_system((24, 8, 256), 4, 3, 0.01, 0.01, -0.01,
                                                         8, 77)),
    "single-pore-64x64x128": ("single_pore_64x64x128_100steps.npz", workloads.single_pore),
}


@pytest.mark.parametrize("case", list(CASES))
def test_matches_stored_oracle_after_100_steps(ek, case):
    fname, make = CASES[case]
    ref = np.load(os.path.join(GOLDEN, fname))
    wl = make()
    assert tuple(ref["shape"]) == wl.shape
    ctx = bench_context(ek, wl)
    ctx.step(int(ref["steps"][0]))
    idx = ref["sites"]
    err = {}
    for s in range(3):
        n, u = ctx.moments(s)
        err[f"n{s}"] = float(np.max(np.abs(n.ravel()[idx] - ref["n"][s]) / ref["n"][s]))
        err[f"u{s}"] = float(np.max(np.abs(u.reshape(3, -1)[:, idx] - ref["u"][s]))
                             / ref["u_scale"][s])
    err["psi"] = float(np.max(np.abs(ctx.potential().ravel()[idx] - ref["psi"]))
                       / ref["psi_scale"][0])
    R, V = ctx.beads(wl.beads_R.shape[0])
    err["R"] = float(np.abs(R - ref["R"]).max())
    err["V"] = float(np.abs(V - ref["V"]).max() / np.abs(ref["V"]).max())
    mass = np.asarray(ctx.stats()["mass"])
    err["mass"] = float(np.max(np.abs(mass - ref["mass"]) / ref["mass"]))
    print(case, err)
    assert max(err.values()) < 1e-5, err
    assert ctx.stats()["step"] == int(ref["steps"][0])
