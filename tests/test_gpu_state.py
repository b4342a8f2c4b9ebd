"""Checkpoint and resume (ek_save_state / ek_load_state): the time loop of
Fig. 1 carries populations, potential and beads from step to step; a state
saved after k steps and loaded into a fresh context continues bit for bit as
the uninterrupted run, and invalid buffers are refused with the context left
as it was."""
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


def _workload():
    return workloads.pore_system((32, 24, 24), 6, 4, 0.01, 0.01, -0.01, 8, 41, steps=100)


def _context(ek, wl, warm_start, precision=None, max_beads=None):
    ctx = ek.from_workload(wl, precision=ek.EK_FP32 if precision is None else precision,
                           poisson_method=ek.EK_POISSON_MG, poisson_tol=1e-8,
                           poisson_max_iter=200, warm_start=warm_start)
    return ctx


def _fresh(ek, wl, warm_start, precision=None, max_beads=8):
    """A context of the same parameters with nothing set but its geometry."""
    p = ek.make_params(wl.shape, precision=ek.EK_FP32 if precision is None else precision,
                       valence=wl.valence, tau=wl.tau, omega_drag=wl.omega_drag,
                       bjerrum=wl.bjerrum, E_ext=wl.E_ext, poisson_method=ek.EK_POISSON_MG,
                       poisson_tol=1e-8, poisson_max_iter=200, warm_start=warm_start)
    return ek.Context(p, max_beads=max_beads)


def _snapshot(ctx, n_beads, cross=True):
    out = {"psi": ctx.potential()}
    for s in range(3):
        out[f"n{s}"], out[f"u{s}"] = ctx.moments(s)
    out["R"], out["V"] = ctx.beads(n_beads)
    if cross:
        out["cross"] = np.array(ctx.crossings(n_beads))
    st = ctx.stats()
    out["step"] = np.array([st["step"]])
    out["mass"] = np.asarray(st["mass"])
    out["iters"] = np.array([st["poisson_iters"]])
    return out


@pytest.mark.parametrize("start", ["extrapolated", "quadratic", "cubic", "previous"])
def test_resume_is_bitwise_equal_to_the_uninterrupted_run(ek, start):
    wl = _workload()
    ws = {"extrapolated": ek.EK_WS_EXTRAP, "quadratic": ek.EK_WS_EXTRAP2,
          "cubic": ek.EK_WS_EXTRAP3}.get(start, ek.EK_WS_PREV)
    zp = float(wl.beads_R[:, 2].mean())
    full = _context(ek, wl, ws)
    full.set_crossing_plane(zp)
    full.step(100)
    ref = _snapshot(full, 8)

    first = _context(ek, wl, ws)
    first.set_crossing_plane(zp)
    first.step(50)
    buf = first.save_state()
    first.close()
    resumed = _fresh(ek, wl, ws)
    resumed.load_state(buf)
    assert resumed.stats()["step"] == 50
    resumed.step(50)
    got = _snapshot(resumed, 8)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    assert ref["step"][0] == 100


def test_state_round_trip_in_place_and_save_is_repeatable(ek):
    wl = _workload()
    ctx = _context(ek, wl, ek.EK_WS_EXTRAP)
    ctx.step(20)
    a = ctx.save_state()
    b = ctx.save_state()
    assert np.array_equal(a, b)
    ctx.step(5)
    ctx.load_state(a)
    assert np.array_equal(ctx.save_state(), a)


def test_invalid_states_are_refused_and_leave_the_context(ek):
    wl = _workload()
    ctx = _context(ek, wl, ek.EK_WS_EXTRAP)
    ctx.step(10)
    good = ctx.save_state()
    before = _snapshot(ctx, 8, cross=False)
    lib = ek.lib()
    small = np.empty(good.size - 1, dtype=np.uint8)
    assert lib.ek_save_state(ctx._h, small.ctypes.data, small.size) == ek.EK_EINVAL
    assert lib.ek_save_state(ctx._h, None, good.size) == ek.EK_EINVAL
    assert lib.ek_load_state(ctx._h, None, good.size) == ek.EK_EINVAL
    assert lib.ek_load_state(ctx._h, good.ctypes.data, good.size - 1) == ek.EK_EINVAL
    assert b"truncated" in lib.ek_last_error(ctx._h)
    bad = good.copy()
    bad[-100] ^= 1                                   # a population bit
    assert lib.ek_load_state(ctx._h, bad.ctypes.data, bad.size) == ek.EK_EINVAL
    assert b"checksum" in lib.ek_last_error(ctx._h)
    bad = good.copy()
    bad[0] = ord("X")
    assert lib.ek_load_state(ctx._h, bad.ctypes.data, bad.size) == ek.EK_EINVAL
    after = _snapshot(ctx, 8, cross=False)
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    # another precision, another warm start, a context too small for the chain
    for other in (_fresh(ek, wl, ek.EK_WS_EXTRAP, precision=ek.EK_FP64),
                  _fresh(ek, wl, ek.EK_WS_PREV),
                  _fresh(ek, wl, ek.EK_WS_EXTRAP, max_beads=4)):
        with pytest.raises(ek.EKError) as e:
            other.load_state(good)
        assert e.value.status == ek.EK_EINVAL
    # another lattice size
    wl2 = workloads.pore_system((32, 24, 26), 6, 4, 0.01, 0.01, -0.01, 8, 41)
    with pytest.raises(ek.EKError):
        _fresh(ek, wl2, ek.EK_WS_EXTRAP).load_state(good)
    # nothing to save before the species are set
    with pytest.raises(ek.EKError) as e:
        _fresh(ek, wl, ek.EK_WS_EXTRAP).save_state()
    assert e.value.status == ek.EK_ESTATE
