"""Throughput of the electrokinetic LB-MD time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload large|single-pore|ensemble|plain] [--no-extra]

A step is one pass of the whole hot path on the workload: charge pass,
Poisson solve to the stated tolerance, bead update (when the workload has a
chain) and the fused three-species collide-and-stream.  The timed region runs
K steps with every input resident in GPU memory; the metric is lattice-site
updates per second summed over the three species (MLUPS per species-step).

The default workload is the large pore: 256 x 256 x 512 sites, a slab 20
sites thick pierced by a pore of radius 10, salt 0.005, E_z = 0.02 and one
chain of 256 beads (float32 populations, 15.3 GB of them, multigrid to a
relative residual of 1e-8 in float64).  Unless --no-extra is given the same
line also carries the 64 x 64 x 128 single pore with its 32-bead chain
(`single_pore_64x64x128`, with the learned-warm-start comparison) and the
64-replica ensemble of 48 x 48 x 96 pores in one persistent launch
(`ensemble_64x48x48x96`), each measured the same way.

The JSON line also carries:
  roofline      the fused lattice kernel priced against HBM bandwidth, from
                its average duration measured with HIP events stamped at
                the kernel's own start and end on the stream it runs on (the
                library's second stream, beside the chain) during the timed
                region, and its algorithmic bytes per launch (populations
                read and written once, the link word of every site, the
                potential of every updated site); `traffic` is the HBM bytes
                per launch from the committed counter passes at this
                workload, or null when the kernel changed since;
                `copy_kernel` the bandwidth a plain 2 GiB device-to-device
                copy reaches in the same process (the practical peak);
  cpu_baseline  the float64 oracle timed on the host, one thread, on a
                bounded sample of the same workload: a 64 x 64 x 128
                periodic window around the pore with the chain inside it,
                stepped for about 20 s; its per-site rate is reported as the
                rate of the whole workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 * 2 ** 20   # MI355X last-level cache in front of HBM
LB_SOURCES = [os.path.join(ROOT, "paper_1710_09421_amd", "csrc", f)
              for f in ("kernels_lb.hip", "lb_site.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lb_step_traffic.json")


def progress(msg):
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def lb_source_hash():
    """sha256 over the sources of the fused lattice kernel."""
    h = hashlib.sha256()
    for path in LB_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload_name, precision):
    """HBM bytes per launch of the fused lattice kernel from the committed
    rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, scaled by the factor a
    plain copy kernel of known size gives), or None when no run matches this
    workload or the kernel source has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for r in rec.get("runs", []):
        if (r.get("workload") == workload_name and r.get("dtype") == precision
                and r.get("kernel_source_sha256") == lb_source_hash()):
            return r["hbm_bytes_per_launch"]
    return None


def copy_bandwidth(gib=2.0, reps=5):
    """Read + write bandwidth of a plain device-to-device copy of `gib` GiB
    (torch copy_, far beyond the 256 MB Infinity Cache): the practical peak a
    streaming kernel meets on this machine, reported beside the published one."""
    import torch
    n = int(gib * 2 ** 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        dst.copy_(src)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    del src, dst
    return round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)


def build_workload(name):
    from paper_1710_09421_amd import workloads
    if name == "single-pore":
        return workloads.single_pore()
    if name == "large":
        return workloads.large_system()
    if name == "plain":
        return workloads.plain_box(32)
    if name == "single-pore-open":
        return workloads.pore_system((128, 64, 64), 10, 5, 0.01, 0.01, -0.01, 0, 12)
    raise SystemExit(f"unknown workload {name}")


def lb_bytes_per_launch(wl, precision_bytes, fluid_updated=None):
    """Algorithmic bytes of one fused lattice launch: 57 populations read and
    written at every fluid site it updates, the 4-byte link word of every site
    and the float64 potential at every updated site (its neighbours come from
    cache).  With a polymer the launch leaves the sites of the bead boxes to a
    small launch after the chain kernel: fluid_updated is the library's count
    of the sites it did update (per launch)."""
    fluid = wl.fluid_sites if fluid_updated is None else fluid_updated
    return int(round(fluid * (2 * 57 * precision_bytes + 8) + wl.sites * 4))


def cpu_baseline(wl, budget_s=20.0):
    """Oracle (float64 NumPy, one thread) on a bounded sample of the workload:
    a periodic window of at most 64 x 64 x 128 sites centred on the pore (the
    slab, the wall charges, the salt of those sites and the part of the chain
    inside it), one untimed step, then as many timed steps as fit in about
    `budget_s` seconds.  Returns the per-site rate in species-MLUPS."""
    from threadpoolctl import threadpool_limits
    from oracle import step as ostep
    from paper_1710_09421_amd import workloads
    Z, Y, X = wl.shape
    shape = (min(Z, 128), min(Y, 64), min(X, 64))
    sample = wl if shape == wl.shape else workloads.periodic_window(
        wl, shape, ((Z - shape[0]) // 2, (Y - shape[1]) // 2, (X - shape[2]) // 2))
    with threadpool_limits(1):
        p = ostep.Params(valence=sample.valence, tau=sample.tau, omega_drag=sample.omega_drag,
                         bjerrum=sample.bjerrum, E_ext=sample.E_ext,
                         poisson_tol=sample.poisson_tol)
        beads = None if sample.beads_R is None else (sample.beads_R, sample.beads_V,
                                                     sample.polymer)
        sim = ostep.Simulation(p, sample.solid.astype(bool), sample.wall_q, sample.n0,
                               beads=beads)
        t0 = time.perf_counter()
        sim.step()
        first = time.perf_counter() - t0
        steps = max(1, min(20, int(budget_s / max(first, 1e-3))))
        t0 = time.perf_counter()
        sim.run(steps)
        dt = time.perf_counter() - t0
    nb = 0 if sample.beads_R is None else sample.beads_R.shape[0]
    return {"value": round(3 * sample.sites * steps / dt / 1e6, 4),
            "unit": "MLUPS (species-steps)", "cores": 1, "kind": "oracle",
            "sample": f"{steps} timed steps (after 1 untimed) of the {sample.name} "
                      f"({sample.sites} sites, {nb} beads), float64 NumPy, 1 thread, "
                      f"{dt:.1f} s; the sample's rate per site is reported as the "
                      f"workload's"}


def learned_comparison():
    """Poisson solves to 1e-8 by multigrid from the learned start against the
    plain starts, outside the timed region: cold held-out fields (zero start
    vs the network's guess, network time included) and warm pairs (previous
    solution, with and without the network consulted), then the single-pore
    time loop with the previous-step, the extrapolated and the learned start."""
    from paper_1710_09421_amd import learned
    if not os.path.exists(learned.DEFAULT_MODEL):
        return None
    params, scale, info = learned.load_model()
    held = learned.generate(2, 4, 1, seed=90210, first=20, log=lambda s: None)
    summary, _ = learned.evaluate(params, scale, held, repeats=3, log=lambda s: None)
    progress(f"learned start on held-out fields: {json.dumps(summary)}")
    from paper_1710_09421_amd import ek
    sor, _ = learned.evaluate(params, scale, held, repeats=1, log=lambda s: None,
                              method=ek.EK_POISSON_SOR)
    progress(f"learned start with the red-black SOR finisher: {json.dumps(sor)}")
    sim = learned.simulate(params, scale, steps=100, warmup=10, log=lambda s: None)
    progress(f"learned start in the time loop: {json.dumps(sim)}")
    r = lambda x: round(x, 4)
    out = {"tolerance": 1e-8, "finisher": "red-black multigrid (V(4,2) on the finest level)",
           "model": f"{info['n_traj'] * info['per_traj']} pairs, {info['epochs']} epochs"}
    for k, v in summary.items():
        out[k] = {"solves": v["n"], "cycles": r(v["cycles"]), "ms": r(v["ms"]),
                  "initial_residual": float(f"{v['initial_residual']:.3e}"),
                  "network_consulted": v["consulted"], "network_rejected": v["fallbacks"]}
    out["sor_finisher"] = {k: {"solves": v["n"], "iterations": r(v["cycles"]), "ms": r(v["ms"]),
                               "initial_residual": float(f"{v['initial_residual']:.3e}"),
                               "network_consulted": v["consulted"],
                               "network_rejected": v["fallbacks"]}
                           for k, v in sor.items()}
    out["time_loop"] = {k: {"poisson_ms_per_step": r(v["ms_poisson_per_step"]),
                            "cycles_per_step": r(v["cycles_per_step"]),
                            "network_consulted_steps": v["consulted_steps"]}
                        for k, v in sim.items()}
    return out


def measure_context(wl, args, steps, warmup):
    """Time `steps` steps of one context on the workload (after `warmup`
    untimed ones); returns the fields of the JSON line for it."""
    import torch
    from paper_1710_09421_amd import ek
    progress(f"workload {wl.name}: {wl.sites} sites")
    prec = ek.EK_FP32 if args.precision == "fp32" else ek.EK_FP64
    method = ek.EK_POISSON_SOR if args.poisson == "sor" else ek.EK_POISSON_MG
    start = {"extrapolated": ek.EK_WS_EXTRAP, "quadratic": ek.EK_WS_EXTRAP2,
             "cubic": ek.EK_WS_EXTRAP3}.get(args.start, ek.EK_WS_PREV)
    ctx = ek.from_workload(wl, precision=prec, poisson_method=method,
                           poisson_check_every=args.check_every,
                           poisson_max_iter=200 if method == ek.EK_POISSON_MG else 100000,
                           warm_start=start)
    progress("context ready")
    for k in range(warmup):
        ctx.step(1)
        if k < 3 or k == warmup - 1:
            st = ctx.stats()
            progress(f"warmup step {k + 1}: poisson {st['poisson_iters']} iterations, "
                     f"residual {st['poisson_residual']:.2e}")
    torch.cuda.synchronize()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    progress(f"timed {steps} steps in {dt:.3f} s")
    tm = ctx.timing()
    st = ctx.stats()
    ctx.close()
    torch.cuda.synchronize()

    pbytes = 4 if prec == ek.EK_FP32 else 8
    lb_ms = tm["ms_lb"] / max(tm["n_lb"], 1)
    lb_sites = tm["lb_sites"] / max(tm["n_lb"], 1) if tm["lb_sites"] > 0 else None
    lb_bytes = lb_bytes_per_launch(wl, pbytes, lb_sites)
    achieved = lb_bytes / (lb_ms * 1e-3) / 1e9
    dtype = "f32" if prec == ek.EK_FP32 else "f64"
    # both population buffers (3 species x 19): when they fit the last-level
    # cache the lattice kernel's bytes need not come from HBM
    pop_bytes = 2 * 57 * pbytes * wl.sites
    roof = {
        "kernel": "k_lb_step (fused pull-stream + collide, 3 species)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "bytes_per_launch": lb_bytes,
        "fluid_sites_per_launch": None if lb_sites is None else round(lb_sites, 1),
        "avg_launch_ms": round(lb_ms, 5),
        "traffic": measured_traffic(wl.name, dtype),
    }
    if pop_bytes <= INFINITY_CACHE_BYTES:
        roof["cache_resident"] = (f"the populations ({pop_bytes / 1e6:.0f} MB) fit the "
                                  f"{INFINITY_CACHE_BYTES // 2 ** 20} MiB Infinity Cache: not an "
                                  f"HBM roofline figure")
    return {
        "value": round(3 * wl.sites * steps / dt / 1e6, 1),
        "ms_per_step": round(dt / steps * 1e3, 4),
        "dtype": dtype,
        "config": {
            "workload": wl.name,
            "sites": wl.sites,
            "fluid_sites": wl.fluid_sites,
            "species": 3,
            "beads": 0 if wl.beads_R is None else int(wl.beads_R.shape[0]),
            "poisson": f"{args.poisson} to {wl.poisson_tol:g} (fp64 residual) from the "
                       f"{args.start} start, "
                       f"mean {tm['poisson_iters'] / max(tm['n_steps'], 1):.2f} iterations/step",
            "phase_ms_per_step": {
                "charge": round(tm["ms_charge"] / steps, 4),
                "poisson": round(tm["ms_poisson"] / steps, 4),
                "md": round(tm["ms_md"] / steps, 4),
                "lb": round(lb_ms, 4),
            },
            "mass_drift": [float(x) for x in (st["mass"] / wl.n0.sum(axis=(1, 2, 3)) - 1.0)],
        },
        "roofline": roof,
    }


def measure_ensemble(args, steps):
    """64 uneven replicas of the 48 x 48 x 96 pore system in one persistent
    launch per call; the autotuner picks the workgroup size and the number of
    workgroups per replica during warm-up."""
    import numpy as np
    import torch
    from paper_1710_09421_amd import ek, workloads
    n_rep = 64
    wls = [workloads.ensemble_replica(r) for r in range(n_rep)]
    progress(f"{n_rep} replicas of {wls[0].shape[::-1]}, chains "
             f"{sorted(set(int(w.beads_R.shape[0]) for w in wls))}")
    # the persistent kernel extrapolates linearly (it has no quadratic start)
    start = ek.EK_WS_PREV if args.start == "previous" else ek.EK_WS_EXTRAP
    start_name = "previous" if args.start == "previous" else "extrapolated"
    ens = ek.ensemble_from_workloads(wls, precision=ek.EK_FP32, poisson_tol=1e-8,
                                     warm_start=start)
    progress("ensemble ready")
    tune = ens.autotune(steps=max(2, args.warmup // 3))
    progress(f"autotuned: {tune}")
    ens.step(1)
    torch.cuda.synchronize()
    ph0 = [ens.phase_times(r) for r in range(n_rep)]
    t0 = time.perf_counter()
    ens.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    progress(f"timed {steps} steps in {dt:.3f} s")
    ph1 = [ens.phase_times(r) for r in range(n_rep)]
    # per-step phase times of each replica's team (the kernel's own clock)
    phase = {k: [(ph1[r][k] - ph0[r][k]) / steps for r in range(n_rep)]
             for k in ("charge", "poisson", "chain", "lb")}
    sites = n_rep * wls[0].sites
    cycles = [ens.stats(r)["poisson_iters"] for r in range(n_rep)]
    # release the ensemble while the runtime is fully up, not from a finaliser
    # at interpreter exit
    torch.cuda.synchronize()
    ens.close()
    torch.cuda.synchronize()
    fluid = sum(w.fluid_sites for w in wls)
    lb_bytes = fluid * (2 * 57 * 4 + 8) + sites * 4
    # the teams run their collide-and-stream phases side by side: the
    # ensemble's lattice bytes of a step over the slowest team's phase time
    lb_max = max(phase["lb"])
    lb_gbs = lb_bytes / (lb_max * 1e-3) / 1e9
    return {
        "value": round(3 * sites * steps / dt / 1e6, 1),
        "ms_per_step": round(dt / steps * 1e3, 4),
        "dtype": "f32",
        "config": {
            "workload": f"ensemble of {n_rep} pore replicas 48x48x96 (E_z ~ U[0.01, 0.1], "
                        f"chains of 16-64 beads), one persistent launch per call",
            "sites": sites,
            "threads_per_workgroup": tune["threads"],
            "workgroups_per_replica": tune["group"],
            "poisson": f"mg to 1e-8 per replica from the {start_name} start, "
                       f"last solve {min(cycles)}-{max(cycles)} cycles",
            "lb_bytes_per_step_gb": round(lb_bytes / 1e9, 3),
            "phase_ms_per_step": {k: round(float(np.mean(v)), 4) for k, v in phase.items()},
            "phase_ms_per_step_max": {k: round(float(np.max(v)), 4) for k, v in phase.items()},
        },
        "lb_phase_roofline": {
            "phase": "fused collide-and-stream of all replicas (per-team clock in the kernel)",
            "bound": "hbm", "achieved": round(lb_gbs, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(lb_gbs / 8000.0, 4), "bytes_per_step": int(lb_bytes),
            "ms_per_step": round(lb_max, 4),
        },
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large",
                    choices=["large", "single-pore", "ensemble", "plain", "single-pore-open"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--poisson", default="mg", choices=["sor", "mg"])
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--start", default="quadratic",
                    choices=["previous", "extrapolated", "quadratic", "cubic"],
                    help="start of each step's Poisson solve: the previous solution, the "
                         "linear extrapolation of the two previous ones, the quadratic one "
                         "of the three previous ones or the cubic one of the four previous "
                         "ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="measure only the named workload (no single-pore and ensemble keys)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-warm-start comparison")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="after the main workload, copy this many GiB device-to-device three "
                         "times (a kernel of known traffic for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the data-parallel step runs on a single MI355X; "
              "runs on several GPUs are not supported.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ensemble":
        main_leg = measure_ensemble(args, args.steps)
        wl = None
    else:
        wl = build_workload(args.workload)
        main_leg = measure_context(wl, args, args.steps, args.warmup)
    line = {
        "metric": "MLUPS per species-step",
        "value": main_leg["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_leg["dtype"],
        "data": "synthetic",
        "config": main_leg["config"],
    }
    if "roofline" in main_leg:
        line["roofline"] = main_leg["roofline"]
        if wl is not None:
            cb = copy_bandwidth()
            line["roofline"]["copy_kernel"] = {
                "what": "device-to-device copy of 2 GiB (torch copy_), bytes read + written",
                "achieved": cb, "unit": "GB/s",
                "frac_of_copy": round(line["roofline"]["achieved"] / cb, 4)}
    if args.copy_probe_gib > 0:
        import torch
        n = int(args.copy_probe_gib * 2 ** 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_extra and args.workload == "large":
        sp = build_workload("single-pore")
        leg = measure_context(sp, args, args.steps, args.warmup)
        line["single_pore_64x64x128"] = leg
        if not args.no_learned:
            line["single_pore_64x64x128"]["learned_vs_plain_poisson"] = learned_comparison()
        line["ensemble_64x48x48x96"] = measure_ensemble(args, args.steps)
    elif args.workload == "single-pore" and not args.no_learned:
        line["learned_vs_plain_poisson"] = learned_comparison()
    if not args.no_cpu_baseline and wl is not None:
        progress("timing the oracle on the host")
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
