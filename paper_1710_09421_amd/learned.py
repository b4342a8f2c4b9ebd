"""Learned warm start of the Poisson solve: training pairs, training loop,
evaluation.

Every number here comes from the library's own kernels: the pairs
(right-hand side, solid mask) -> potential are the method's Poisson solves read
back with ek_get_poisson_system after lattice steps of pore systems, the
network is trained with the ek_unet forward / backward / Adam entry points,
and the evaluation times ek_poisson_solve with a zero, previous-step or learned
start finished by multigrid to the same tolerance.  torch only holds device
memory.

    python -m paper_1710_09421_amd.learned train --out model.npz
    python -m paper_1710_09421_amd.learned evaluate --model model.npz
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import ek, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "unet_pore_128x64x64.npz")
SHAPE = (128, 64, 64)                 # (z, y, x)
INV_EPS = 4.0 * math.pi * 0.7 / 3.0   # 1 / eps for l_B = 0.7, kT = 1/3

# Layer table of the network (taps, c_in, c_out) in parameter order.
LAYERS = [(27, 2, 16), (27, 16, 32), (27, 32, 64), (1, 64, 32), (1, 32, 16), (27, 16, 1)]


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, in ABI order."""
    rng = np.random.default_rng(seed)
    parts = []
    for taps, cin, cout in LAYERS:
        parts.append(rng.normal(scale=math.sqrt(2.0 / (taps * cin)), size=taps * cin * cout))
        parts.append(np.zeros(cout))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == ek.UNET_PARAMS
    return p


def draw_system(rng, shape=SHAPE):
    """One pore system for the training distribution: salt c0 ~ U[0.001, 0.05],
    wall charge ~ U[-0.02, 0], pore radius 3..7, slab 8..12 thick, field
    E_z ~ U[0, 0.05], and every other system a 32-bead chain."""
    c0 = float(rng.uniform(0.001, 0.05))
    wq = float(rng.uniform(-0.02, 0.0))
    radius = int(rng.integers(3, 8))
    slab = int(rng.choice([8, 10, 12]))
    ez = float(rng.uniform(0.0, 0.05))
    chain = 32 if rng.uniform() < 0.5 else 0
    seed = int(rng.integers(1 << 30))
    wl = workloads.pore_system(shape, slab, radius, c0, ez, wq, chain, seed)
    return wl, dict(c0=c0, wall_charge=wq, radius=radius, slab=slab, E_z=ez, beads=chain, seed=seed)


def generate(n_traj, per_traj, every, seed, shape=SHAPE, first=1, tol=1e-10, log=print):
    """Pairs from n_traj trajectories: after `first` steps, then every `every`
    steps, the solved system (rhs with its mean removed, potential) is copied
    out.  Returns device tensors rhs, psi [N, z, y, x] float64, solid [N, z, y,
    x] uint8 and the per-trajectory draws."""
    import torch
    rng = np.random.default_rng(seed)
    n = n_traj * per_traj
    rhs = torch.empty((n,) + shape, dtype=torch.float64, device="cuda")
    psi = torch.empty_like(rhs)
    solid = torch.empty((n,) + shape, dtype=torch.uint8, device="cuda")
    meta = []
    t0 = time.time()
    for i in range(n_traj):
        wl, m = draw_system(rng, shape)
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                               poisson_tol=tol, poisson_max_iter=400)
        sol = torch.from_numpy(wl.solid.astype(np.uint8)).to("cuda")
        for k in range(per_traj):
            ctx.step(first if k == 0 else every)
            j = i * per_traj + k
            ctx.poisson_system(rhs[j], psi[j])
            solid[j].copy_(sol)
        ctx.close()
        meta.append(m)
        if (i + 1) % max(1, n_traj // 10) == 0:
            log(f"generated {i + 1}/{n_traj} trajectories ({(i + 1) * per_traj} pairs, "
                f"{time.time() - t0:.1f} s)")
    return dict(rhs=rhs, psi=psi, solid=solid, meta=meta, per_traj=per_traj, every=every)


def generate_workload(wl, per_traj, first=20, every=1, tol=1e-10, log=print):
    """Held-out pairs from one trajectory of a given workload (its own
    geometry and size): after `first` steps, then every `every` steps."""
    import torch
    shape = wl.shape
    rhs = torch.empty((per_traj,) + shape, dtype=torch.float64, device="cuda")
    psi = torch.empty_like(rhs)
    solid = torch.empty((per_traj,) + shape, dtype=torch.uint8, device="cuda")
    ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                           poisson_tol=tol, poisson_max_iter=400)
    sol = torch.from_numpy(wl.solid.astype(np.uint8)).to("cuda")
    for k in range(per_traj):
        ctx.step(first if k == 0 else every)
        ctx.poisson_system(rhs[k], psi[k])
        solid[k].copy_(sol)
    ctx.close()
    log(f"generated {per_traj} pairs of {wl.name}")
    return dict(rhs=rhs, psi=psi, solid=solid, meta=[dict(workload=wl.name)], per_traj=per_traj,
                every=every)


def output_scale(data):
    """RMS of psi over RMS of rhs, averaged over the pairs: the network then
    predicts values of order one."""
    import torch
    r = torch.sqrt((data["rhs"] ** 2).mean(dim=(1, 2, 3)))
    p = torch.sqrt((data["psi"] ** 2).mean(dim=(1, 2, 3)))
    return float((p / r).mean())


def train(data, epochs=12, batch=8, lr=2e-3, lr_min=1e-4, seed=0, log=print):
    """Adam on the mean squared error of the normalised potential; the
    learning rate follows a cosine from lr to lr_min.  Returns (params,
    out_scale, history)."""
    n = data["rhs"].shape[0]
    shape = tuple(data["rhs"].shape[1:])
    scale = output_scale(data)
    net = ek.UNet(shape, training=True)
    net.set_params(init_params(seed), scale)
    rng = np.random.default_rng(seed)
    steps_per_epoch = (n + batch - 1) // batch
    total = epochs * steps_per_epoch
    hist = []
    t0 = time.time()
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            for i in idx:
                net.accumulate(data["rhs"][i], data["solid"][i], data["psi"][i])
            frac = step / max(1, total - 1)
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * frac))
            net.adam_step(lr_t, grad_scale=1.0 / len(idx))
            step += 1
        loss, cnt = net.read_loss()
        hist.append(dict(epoch=ep + 1, loss=loss, samples=cnt, seconds=time.time() - t0))
        log(f"epoch {ep + 1}/{epochs}: mean loss {loss:.4e} over {cnt} samples, "
            f"{time.time() - t0:.1f} s")
    params, sc = net.params()
    net.close()
    return params, sc, hist


def save_model(path, params, out_scale, info):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(params, dtype=np.float32),
             out_scale=np.float32(out_scale), info=np.array(json.dumps(info)))


def load_model(path=DEFAULT_MODEL):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), float(z["out_scale"]), json.loads(str(z["info"]))


def _timed(fn, sync):
    sync()
    t = time.perf_counter()
    r = fn()
    return r, (time.perf_counter() - t) * 1e3


def evaluate(params, out_scale, data, tol=1e-8, repeats=3, log=print, method=None):
    """Poisson solves of every held-out pair to `tol` from a zero start, from
    the network's guess, and (for consecutive pairs of one trajectory) from
    the previous pair's solution with and without the network; the finisher
    is multigrid (method None or EK_POISSON_MG) or the paper's red-black SOR
    with the Chebyshev schedule (EK_POISSON_SOR, residual tested every 4
    iterations).  Wall time per solve is the median over `repeats` (host
    clock around the call, which ends synchronised), network included."""
    import torch
    n = data["rhs"].shape[0]
    shape = tuple(data["rhs"].shape[1:])
    method = ek.EK_POISSON_MG if method is None else method
    sor = method == ek.EK_POISSON_SOR
    p = ek.make_params((shape[0], shape[1], shape[2]), poisson_method=method,
                       poisson_tol=tol, poisson_max_iter=100000 if sor else 400,
                       poisson_check_every=4 if sor else 1, warm_start=ek.EK_WS_LEARNED)
    ctx = ek.Context(p)
    ctx.set_model(params, out_scale)
    # the network on its own, for starts that take its guess whatever its
    # residual ("learned, kept"): the gate compares residuals, which suits
    # multigrid; SOR's slow modes are the smooth ones a guess can supply even
    # when its residual is large
    net = ek.UNet(shape, training=False)
    net.set_params(params, out_scale)
    sync = torch.cuda.synchronize
    psi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    rows = []
    cur_solid = None
    per = data.get("per_traj", 1)
    for i in range(n):
        sol = data["solid"][i]
        if cur_solid is None or not torch.equal(sol, cur_solid):
            ctx.set_geometry(sol.cpu().numpy())
            cur_solid = sol.clone()
        rho = -data["rhs"][i] / INV_EPS
        row = dict(index=i)
        for name, ws in (("zero", ek.EK_WS_ZERO), ("learned", ek.EK_WS_LEARNED)):
            ts = []
            for _ in range(repeats):
                psi.zero_()
                rep, ms = _timed(lambda: ctx.poisson_solve(rho, psi, ws), sync)
                ts.append(ms)
            row[name] = dict(cycles=rep["iterations"], residual=rep["residual"],
                             initial=rep["initial_residual"], ms=float(np.median(ts)),
                             fallback=ctx.stats()["fallback"] if ws == ek.EK_WS_LEARNED else 0,
                             consulted=ctx.stats()["consulted"] if ws == ek.EK_WS_LEARNED else 0)
            if name == "zero":
                err_ref = psi.clone()
        row["learned"]["max_diff_vs_zero_start"] = float((psi - err_ref).abs().max() /
                                                         err_ref.abs().max())
        solid_u8 = sol.to(torch.uint8)
        ts = []
        for _ in range(repeats):
            def kept():
                net.forward(data["rhs"][i], solid_u8, psi)
                return ctx.poisson_solve(rho, psi, ek.EK_WS_PREV)
            rep, ms = _timed(kept, sync)
            ts.append(ms)
        row["learned, kept"] = dict(cycles=rep["iterations"], residual=rep["residual"],
                                    initial=rep["initial_residual"], ms=float(np.median(ts)),
                                    fallback=0, consulted=1)
        if i % per > 0:
            for name, ws in (("previous", ek.EK_WS_PREV), ("previous+learned", ek.EK_WS_LEARNED)):
                ts = []
                for _ in range(repeats):
                    psi.copy_(data["psi"][i - 1])
                    rep, ms = _timed(lambda: ctx.poisson_solve(rho, psi, ws), sync)
                    ts.append(ms)
                row[name] = dict(cycles=rep["iterations"], residual=rep["residual"],
                                 initial=rep["initial_residual"], ms=float(np.median(ts)),
                                 fallback=ctx.stats()["fallback"] if ws == ek.EK_WS_LEARNED else 0,
                                 consulted=ctx.stats()["consulted"] if ws == ek.EK_WS_LEARNED else 0)
        rows.append(row)
    ctx.close()
    net.close()
    summary = {}
    for name in ("zero", "learned", "learned, kept", "previous", "previous+learned"):
        rs = [r[name] for r in rows if name in r]
        if not rs:
            continue
        summary[name] = dict(n=len(rs), cycles=float(np.mean([r["cycles"] for r in rs])),
                             ms=float(np.mean([r["ms"] for r in rs])),
                             initial_residual=float(np.exp(np.mean(np.log(
                                 [max(r["initial"], 1e-300) for r in rs])))),
                             max_residual=float(max(r["residual"] for r in rs)),
                             consulted=int(sum(r["consulted"] for r in rs)),
                             fallbacks=int(sum(r["fallback"] for r in rs)))
    log(json.dumps(summary))
    return summary, rows


def simulate(params, out_scale, steps=200, warmup=20, wl=None, log=print):
    """Single-pore time loop with the previous-step start, the extrapolated
    start (2 psi(t-1) - psi(t-2)) and the learned start (previous step kept
    as the fallback): Poisson milliseconds and cycles per step from the
    context's phase timers."""
    wl = wl or workloads.single_pore()
    out = {}
    for name, ws in (("previous", ek.EK_WS_PREV), ("extrapolated", ek.EK_WS_EXTRAP),
                     ("learned", ek.EK_WS_LEARNED)):
        ctx = ek.from_workload(wl, precision=ek.EK_FP32, poisson_method=ek.EK_POISSON_MG,
                               poisson_tol=1e-8, poisson_max_iter=200, warm_start=ws)
        if ws == ek.EK_WS_LEARNED:
            ctx.set_model(params, out_scale)
        ctx.step(warmup)
        ctx.set_timing(True)
        fb = con = 0
        for _ in range(steps):
            ctx.step(1)
            st = ctx.stats()
            fb += st["fallback"]
            con += st["consulted"]
        t = ctx.timing()
        out[name] = dict(ms_poisson_per_step=t["ms_poisson"] / t["n_steps"],
                         cycles_per_step=t["poisson_iters"] / t["n_steps"],
                         consulted_steps=con, fallback_steps=fb, steps=steps)
        ctx.close()
    log(json.dumps(out))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_MODEL)
    t.add_argument("--n-traj", type=int, default=40)
    t.add_argument("--per-traj", type=int, default=50)
    t.add_argument("--every", type=int, default=4)
    t.add_argument("--epochs", type=int, default=12)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--eval-traj", type=int, default=4)
    t.add_argument("--report", default=None, help="write the evaluation summary as JSON here")
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--n-traj", type=int, default=4)
    e.add_argument("--per-traj", type=int, default=6)
    e.add_argument("--seed", type=int, default=777)
    e.add_argument("--simulate", type=int, default=0, help="single-pore steps per start")
    e.add_argument("--workload", default="training", choices=["training", "large"],
                   help="held-out fields: systems of the training distribution at 64x64x128, "
                        "or one trajectory of the 256x256x512 pore (the model applied at that size)")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    if a.cmd == "train":
        data = generate(a.n_traj, a.per_traj, a.every, a.seed, log=log)
        params, sc, hist = train(data, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
        del data
        info = dict(shape=list(SHAPE), n_traj=a.n_traj, per_traj=a.per_traj, every=a.every,
                    epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, history=hist)
        save_model(a.out, params, sc, info)
        log(f"saved {a.out}")
        held = generate(a.eval_traj, 6, 1, a.seed + 100000, first=20, log=log)
        summary, _ = evaluate(params, sc, held, log=log)
        if a.report:
            with open(a.report, "w") as f:
                json.dump(dict(train=info, evaluation=summary), f, indent=1)
    else:
        params, sc, info = load_model(a.model)
        if a.workload == "large":
            held = generate_workload(workloads.large_system(), a.per_traj, log=log)
        else:
            held = generate(a.n_traj, a.per_traj, 1, a.seed, first=20, log=log)
        evaluate(params, sc, held, log=log)
        if a.simulate:
            simulate(params, sc, steps=a.simulate, log=log)
    return 0


if __name__ == "__main__":
    sys.exit(main())
