"""Uneven replicas (own salt noise, field and chain) advanced by the
persistent ensemble kernel: each replica agrees with the float64 oracle and
with a single-context run of the same workload, replicas do not influence
each other, and the autotuner picks a working launch shape."""
import numpy as np
import pytest

from oracle import step as ostep
from paper_1710_09421_amd import workloads
from tests.parity import density_error, field_error, velocity_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (32, 24, 24)


@pytest.fixture(scope="module")
def ek():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1710_09421_amd import ek as binding
    binding.lib()
    return binding


def replica(seed, E_z, n_beads):
    return workloads.pore_system(SHAPE, 6, 4, 0.01, E_z, -0.01, n_beads, seed,
                                 bead_q=workloads.STABLE_BEAD_CHARGE, steps=30)


def replicas():
    return [replica(101, 0.01, 8), replica(102, 0.05, 16), replica(103, 0.02, 0),
            replica(104, 0.08, 12)]


def oracle_sim(wl, tol):
    p = ostep.Params(E_ext=wl.E_ext, poisson_tol=tol)
    beads = None if wl.beads_R is None else (wl.beads_R, wl.beads_V, wl.polymer)
    return ostep.Simulation(p, wl.solid.astype(bool), wl.wall_q, wl.n0, beads=beads)


def errors(get_moments, get_psi, sim, wl):
    fluid = wl.solid == 0
    out = {}
    n_ref, u_ref = sim.densities(), sim.velocities()
    for s in range(3):
        n, u = get_moments(s)
        out[f"n{s}"] = density_error(n, n_ref[s], fluid)
        out[f"u{s}"] = velocity_error(u, u_ref[s], fluid)
    out["psi"] = field_error(get_psi(), sim.psi)
    return out


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_replicas_match_oracle_fp32(ek, threads):
    wls = replicas()
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8)
    ens.set_threads(threads)
    ens.step(20)
    for r in (0, 3):
        sim = oracle_sim(wls[r], 1e-8)
        sim.run(20)
        err = errors(lambda s: ens.moments(r, s), lambda: ens.potential(r), sim, wls[r])
        R, _ = ens.beads(r)
        err["R"] = float(np.abs(R - sim.R).max())
        print(threads, r, err)
        assert max(err.values()) < 1e-5, (r, err)
    for r in range(4):
        assert ens.stats(r)["step"] == 20


@pytest.mark.skip(reason="faulted the GPU once with a since-removed buffer-resource variant of the "
                         "lattice body whose cause was never shown; the ensemble now refuses float64 "
                         "populations (EK_EINVAL), so this case stays off the GPU")
def test_replica_fp64_matches_oracle(ek):
    wls = replicas()[:2]
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP64, poisson_tol=1e-10)
    ens.step(10)
    sim = oracle_sim(wls[1], 1e-10)
    sim.run(10)
    err = errors(lambda s: ens.moments(1, s), lambda: ens.potential(1), sim, wls[1])
    err["R"] = float(np.abs(ens.beads(1)[0] - sim.R).max())
    print(err)
    assert max(err.values()) < 1e-8, err


@pytest.mark.parametrize("start", ["previous", "extrapolated"])
def test_replicas_match_single_contexts(ek, start):
    """Replicas against single contexts with the same start of each solve."""
    wls = replicas()
    ws = ek.EK_WS_PREV if start == "previous" else ek.EK_WS_EXTRAP
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8, warm_start=ws)
    ens.step(15)
    for r, wl in enumerate(wls):
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                               poisson_tol=1e-8, warm_start=ws)
        ctx.step(15)
        for s in range(3):
            n_e, u_e = ens.moments(r, s)
            n_c, u_c = ctx.moments(s)
            fluid = wl.solid == 0
            assert density_error(n_e, n_c, fluid) < 1e-6
            assert velocity_error(u_e, u_c, fluid) < 1e-6
        assert field_error(ens.potential(r), ctx.potential()) < 1e-6
        ctx.close()


@pytest.mark.parametrize("group", [1, 4])
def test_replica_species_mass_is_conserved(ek, group):
    """The per-replica sums of species mass (float64 over the whole replica)
    equal the initial masses."""
    wls = replicas()
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8)
    ens.set_group(group)
    ens.step(5)
    for r, wl in enumerate(wls):
        fluid = wl.solid == 0
        m0 = np.array([wl.n0[s][fluid].sum() for s in range(3)])
        m = ens.stats(r)["mass"]
        print(r, m / m0 - 1.0)
        assert np.all(np.abs(m / m0 - 1.0) < 1e-7), (r, m, m0)


def test_replicas_are_independent(ek):
    a, b = replica(201, 0.03, 10), replica(202, 0.07, 0)
    ens = ek.ensemble_from_workloads([a, b, a], precision=ek.EK_FP32)
    ens.step(12)
    for s in range(3):
        n0, u0 = ens.moments(0, s)
        n2, u2 = ens.moments(2, s)
        assert np.array_equal(n0, n2) and np.array_equal(u0, u2)
    assert np.array_equal(ens.beads(0)[0], ens.beads(2)[0])
    n1, _ = ens.moments(1, 1)
    assert not np.array_equal(n1, ens.moments(0, 1)[0])


@pytest.mark.parametrize("group,start", [(2, "previous"), (4, "previous"), (4, "extrapolated")])
def test_replica_teams_match_oracle_fp32(ek, group, start):
    """Each replica advanced by a team of workgroups meeting at barriers; the
    solves start from the previous solution or its extrapolation (the oracle
    starts from the previous one; both finish to 1e-8)."""
    wls = replicas()
    ws = ek.EK_WS_PREV if start == "previous" else ek.EK_WS_EXTRAP
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8, warm_start=ws)
    ens.set_threads(512)
    ens.set_group(group)
    ens.step(20)
    for r in (0, 3):
        sim = oracle_sim(wls[r], 1e-8)
        sim.run(20)
        err = errors(lambda s: ens.moments(r, s), lambda: ens.potential(r), sim, wls[r])
        R, _ = ens.beads(r)
        err["R"] = float(np.abs(R - sim.R).max())
        print(group, r, err)
        assert max(err.values()) < 1e-5, (r, err)
    for r in range(4):
        assert ens.stats(r)["step"] == 20


def test_replica_teams_agree_with_single_workgroups(ek):
    """Team sizes differ only in the order of the fixed-order sums."""
    wls = replicas()
    out = []
    for group in (1, 2, 4):
        ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8)
        ens.set_threads(256)
        ens.set_group(group)
        ens.step(10)
        out.append([(ens.moments(r, 1)[0], ens.potential(r)) for r in range(4)])
        ens.close()
    for k in (1, 2):
        for r in range(4):
            n1, p1 = out[0][r]
            nk, pk = out[k][r]
            fluid = wls[r].solid == 0
            assert density_error(nk, n1, fluid) < 1e-6
            assert field_error(pk, p1) < 1e-6


def test_replica_teams_are_deterministic(ek):
    wls = replicas()
    res = []
    for _ in range(2):
        ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8)
        ens.set_group(4)
        ens.step(6)
        res.append((ens.moments(3, 2), ens.beads(3), ens.potential(3)))
        ens.close()
    (na, ua), (Ra, Va), pa = res[0]
    (nb, ub), (Rb, Vb), pb = res[1]
    assert np.array_equal(na, nb) and np.array_equal(ua, ub) and np.array_equal(pa, pb)
    assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb)


def test_autotune_picks_a_candidate(ek):
    ens = ek.ensemble_from_workloads(replicas(), precision=ek.EK_FP32)
    res = ens.autotune(steps=2)
    assert res["threads"] in (256, 512, 1024) and res["group"] in (1, 2, 4)
    assert res["ms_per_step"] > 0
    ens.step(2)
    for r in range(4):   # 3 workgroup sizes x 3 team sizes x (1 + 2 + 2) steps, then 2
        assert ens.stats(r)["step"] == 9 * (1 + 2 + 2) + 2


def test_no_convergence_names_the_replica(ek):
    ens = ek.ensemble_from_workloads(replicas(), precision=ek.EK_FP32, poisson_tol=1e-14,
                                     poisson_max_iter=1)
    with pytest.raises(ek.EKError) as e:
        ens.step(1)
    assert e.value.status == ek.EK_ENOCONV and "replica" in str(e.value)


def test_harmonic_replicas_match_single_contexts(ek):
    """Replicas whose chains have the harmonic bonds of Eq. polymermodel (the
    persistent kernel's all-pairs WCA skips bonded neighbours)."""
    wls = replicas()[:2]
    for w in wls:
        w.polymer.update(bond="harmonic", k_bond=40.0, l_bond=1.0)
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8)
    ens.step(10)
    for r, wl in enumerate(wls):
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                               poisson_tol=1e-8)
        ctx.step(10)
        fluid = wl.solid == 0
        for s in range(3):
            n_e, _ = ens.moments(r, s)
            n_c, _ = ctx.moments(s)
            assert np.max(np.abs(n_e - n_c)[fluid] / n_c[fluid]) < 1e-6, (r, s)
        R_e, _ = ens.beads(r)
        R_c, _ = ctx.beads(wl.beads_R.shape[0])
        assert np.abs(R_e - R_c).max() < 1e-6, r


def test_phase_times(ek):
    """ek_ensemble_phase_times: the persistent kernel's own clock of the four
    phases grows with the steps taken and its sum stays below the host's
    wall time around the call; a bad replica index is rejected."""
    import time
    import torch
    ens = ek.ensemble_from_workloads(replicas(), precision=ek.EK_FP32)
    ens.step(1)
    before = [ens.phase_times(r) for r in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(3)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    for r in range(4):
        after = ens.phase_times(r)
        grew = {k: after[k] - before[r][k] for k in after}
        assert all(v > 0.0 for v in grew.values()), grew
        assert sum(grew.values()) <= wall_ms * 1.01 + 0.05, (grew, wall_ms)
    with pytest.raises(ek.EKError) as e:
        ens.phase_times(4)
    assert e.value.status == ek.EK_EINVAL
    ens.close()
