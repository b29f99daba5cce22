"""Learned collision closure: training-data generation, training and evaluation.

The coarse lattice (2x coarser in space and time, acoustic scaling) runs the plain forced
BGK step plus a learned correction of its non-conserved moments (the closure of the C ABI:
lbm_set_closure).  The network is trained to reproduce one coarse step of the restricted
fine-lattice flow:

  data     fine channel 256x128x128 (tau_f = 1.0) with 16 platelets of 2562 nodes, top wall
           speed U ~ U(0.02, 0.05) per seed; after a spin-up, snapshot pairs
           (f_f(t), f_f(t + 2 dt_f)) every `every` fine steps, restricted to the coarse
           lattice (lbm_restrict) and turned into (features, target moments) by
           closure_targets -- all on the GPU;
  training mean-square loss on the 15 target moments, Adam, minibatches of contiguous
           coarse cells from random snapshots (mlp_grad / mlp_adam on the matrix cores);
           validation on held-out seeds;
  eval     the same suspension on the fine lattice (reference), on the plain coarse lattice
           and on the learned coarse lattice; errors of the bottom-wall shear stress and of
           the platelet centroid velocities against the (restricted) fine reference, and the
           throughput of each run.

Every computation runs in the library's kernels; this module only sequences the calls,
holds the tensors and draws the random minibatch positions.

    python -m paper_1312_2234_amd.closure --out results.json [--quick]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, lbm

TAU_F = 1.0
TAU_C = 0.75


def _nodes_setup(lat, ch, dev):
    import torch

    b = ch.bodies
    lat.set_nodes(b.n)
    mem = lbm.Membrane(b, device=dev)
    X = torch.from_numpy(b.X.copy()).to(dev)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=dev)
    U = torch.zeros_like(F)
    return mem, X, F, U


def generate(seeds, u_range=(0.02, 0.05), spinup=400, snapshots=25, every=80, dev="cuda:0", count=16,
             fine=(256, 128, 128), log=print):
    """Training pairs of the given seeds: returns (feat [S, Nc, 16], target [S, Nc, 16]) as
    device tensors (S = len(seeds) * snapshots)."""
    import torch

    feats, tgts = None, None
    k = 0
    for seed in seeds:
        u_top = float(np.random.default_rng(10_000 + seed).uniform(*u_range))
        chf, chc = inputs.coarse_fine_pair(seed, u_top=u_top, count=count, fine=fine, tau_f=TAU_F)
        lat = lbm.Lattice([chf], max_nodes=chf.bodies.n, device=dev)
        lat.init()
        mem, X, F, U = _nodes_setup(lat, chf, dev)
        lat.coupled_steps(mem, spinup, X, F, U)
        nc = chc.nx * chc.ny * chc.nz
        if feats is None:
            S = len(seeds) * snapshots
            feats = torch.empty((S, nc, 16), dtype=torch.float32, device=dev)
            tgts = torch.empty((S, nc, 16), dtype=torch.float32, device=dev)
        for s in range(snapshots):
            # time t: the force of step t is spread, the state is f(t)
            mem.forces(X, F)
            lat.spread(X, F)
            g0, Fc = lat.restrict(TAU_C)
            lat.step(1)
            lat.interp(X, U)
            lat.advance(X, U)
            lat.coupled_steps(mem, 1, X, F, U)
            g1, _ = lat.restrict(TAU_C)
            lbm.closure_targets(chc, g0, Fc, g1, out=(feats[k], tgts[k]))
            k += 1
            lat.coupled_steps(mem, every - 2, X, F, U)
        flags = lat.error_flags()
        log("seed %d: U = %.4f, %d snapshot pairs, flags %d" % (seed, u_top, snapshots, flags))
        del lat
    return feats, tgts


def init_params(rng, dev):
    """He-normal hidden layers, small output layer, zero biases (flat MLP_PARAMS layout)."""
    import torch

    W1 = rng.normal(0, np.sqrt(2.0 / 16), (16, 64))
    W2 = rng.normal(0, np.sqrt(2.0 / 64), (64, 64))
    W3 = rng.normal(0, 0.01, (64, 16))
    th = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.zeros(16)])
    return torch.from_numpy(th.astype(np.float32)).to(dev)


# Output lanes of the network and the moment rows they correct: lanes 0-5 are the second-
# order rows 4-9 (normal and shear stresses, which set the viscosity), lanes 6-14 the third-
# and fourth-order rows 10-18.
HYDRO_LANES = range(0, 6)


def train(feat, tgt, vfeat, vtgt, steps=3000, batch=65536, lr=1e-3, seed=0, log=print, log_every=500,
          higher_only=False):
    """Adam on minibatches of `batch` contiguous coarse cells of random training snapshots.
    With higher_only the second-order moments are left to the BGK relaxation: their targets
    are scaled away in training (out_scale -> huge, so the standardised target is ~0) and
    their output scale is 0 at inference.  Returns (params, norm, history, seconds)."""
    import torch

    dev = feat.device
    S, nc, _ = feat.shape
    flat_f = feat.view(-1, 16)
    flat_t = tgt.view(-1, 16)
    norm = lbm.mlp_norm(flat_f, flat_t)
    if higher_only:
        for k in HYDRO_LANES:
            norm[32 + k] = 1e30
    params = init_params(np.random.default_rng(seed), dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    rng = np.random.default_rng(seed + 1)
    work = torch.empty(lbm.lib().mlp_grad_workspace_bytes(batch), dtype=torch.uint8, device=dev)
    hist = []
    vf, vt = vfeat.view(-1, 16), vtgt.view(-1, 16)
    vwork = torch.empty(lbm.lib().mlp_grad_workspace_bytes(vf.shape[0]), dtype=torch.uint8, device=dev)

    def val_loss():
        P = lbm.mlp_pack(params, norm)
        return float(lbm.mlp_grad(P, vf, vt, vwork)[1].item())

    hist.append((0, None, val_loss()))
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        s = int(rng.integers(S))
        o = int(rng.integers(nc - batch + 1))
        P = lbm.mlp_pack(params, norm)
        grad, loss = lbm.mlp_grad(P, feat[s, o:o + batch], tgt[s, o:o + batch], work)
        lbm.mlp_adam(params, grad, m, v, step, lr=lr)
        if step % log_every == 0 or step == steps:
            tl = float(loss.item())
            vl = val_loss()
            hist.append((step, tl, vl))
            log("step %d: train loss %.4f, validation loss %.4f (%.1f s)" % (step, tl, vl, time.perf_counter() - t0))
    torch.cuda.synchronize()
    if higher_only:
        for k in HYDRO_LANES:
            norm[32 + k] = 0.0
    return params, norm, hist, time.perf_counter() - t0


def _centroid_velocity(U, offsets):
    Un = U.detach().cpu().numpy().astype(np.float64)
    return np.stack([Un[:, a:b].mean(axis=1) for a, b in zip(offsets[:-1], offsets[1:])])


def _run(lat, mem, X, F, U, steps, sample_every, wall_shape):
    """Coupled steps with the wall stress and platelet centroid velocities sampled over the
    last quarter of the run; returns (mean bottom-wall sigma_xy [nz, nx], mean centroid
    velocities [bodies, 3], seconds of the timed stepping)."""
    import torch

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wss, vel, ns = 0.0, 0.0, 0
    elapsed = 0.0
    done = 0
    start_sampling = steps - steps // 4
    while done < steps:
        k = min(sample_every, steps - done)
        torch.cuda.synchronize()
        ev0.record(lat.stream)
        lat.coupled_steps(mem, k, X, F, U)
        ev1.record(lat.stream)
        torch.cuda.synchronize()
        elapsed += ev0.elapsed_time(ev1) * 1e-3
        done += k
        if done > start_sampling:
            lo, _ = lat.wall_stress()
            nz, nx = wall_shape
            wss = wss + lo[: nz * nx].view(nz, nx).double().cpu().numpy()
            vel = vel + _centroid_velocity(U, mem.offsets)
            ns += 1
    return wss / ns, vel / ns, elapsed


def evaluate(params, norm, seeds, u_top=0.05, coarse_steps=2000, sample_every=50, dev="cuda:0", count=16,
             fine=(256, 128, 128), c_guard=1.0, log=print):
    """Fine reference vs plain coarse vs learned coarse on held-out seeds."""
    out = []
    for seed in seeds:
        chf, chc = inputs.coarse_fine_pair(seed, u_top=u_top, count=count, fine=fine, tau_f=TAU_F)
        res = {"seed": seed, "u_top": u_top}
        runs = {}
        for name, ch, steps, closure in (("fine", chf, 2 * coarse_steps, False), ("plain", chc, coarse_steps, False),
                                         ("learned", chc, coarse_steps, True)):
            lat = lbm.Lattice([ch], max_nodes=ch.bodies.n, device=dev)
            lat.init()
            mem, X, F, U = _nodes_setup(lat, ch, dev)
            mem.offsets = ch.bodies.body_offsets
            if closure:
                lat.set_closure(params, norm, c_guard)
            every = sample_every * (2 if name == "fine" else 1)
            wss, vel, secs = _run(lat, mem, X, F, U, steps, every, (ch.nz, ch.nx))
            runs[name] = (wss, vel)
            res[name + "_mlups"] = ch.cells * steps / secs / 1e6
            res[name + "_flags"] = lat.error_flags()
            if closure:
                res["guarded_updates"] = lat.closure_guarded()
            del lat
        wf, vf = runs["fine"]
        wf_c = wf.reshape(chc.nz, 2, chc.nx, 2).mean(axis=(1, 3))  # fine wall stress on coarse cells
        base = float(np.mean(wf_c))  # the mean (Couette) part
        for name in ("plain", "learned"):
            w, v = runs[name]
            res[name + "_wss_rel_l2"] = float(np.linalg.norm(w - wf_c) / np.linalg.norm(wf_c))
            res[name + "_wss_dev_rel_l2"] = float(np.linalg.norm((w - np.mean(w)) - (wf_c - base)) /
                                                  max(np.linalg.norm(wf_c - base), 1e-300))
            res[name + "_wss_mean_rel"] = float(abs(np.mean(w) - base) / abs(base))
            res[name + "_vel_rel_l2"] = float(np.linalg.norm(v - vf) / np.linalg.norm(vf))
        log("seed %d: " % seed + ", ".join("%s %.4g" % (k, v) for k, v in res.items() if isinstance(v, float)))
        out.append(res)
    return out


def _patch_mean(w, patches=(16, 32)):
    """Wall-stress field [nz, nx] averaged over a fixed grid of wall patches (z, x), the same
    physical areas at every resolution."""
    nz, nx = w.shape
    pz, px = patches
    return w.reshape(pz, nz // pz, px, nx // px).mean(axis=(1, 3))


def _graph_rate(lat, mem, X, F, U, steps=200, warmup=10):
    """Coupled steps per second of the HIP graph replay (the benchmark's schedule)."""
    import torch

    from . import tune

    G = tune.graph_steps(lat.get_launch())
    lat.graph_capture(mem, G, X, F, U)
    lat.graph_launch(max(1, warmup // G))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, steps // G)
    ev0.record(lat.stream)
    lat.graph_launch(reps)
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    return reps * G / (ev0.elapsed_time(ev1) * 1e-3)


def _interp_log(xs, ys, y):
    """x at which the piecewise log-log line through (xs, ys) (ys decreasing) reaches y, or
    None outside the measured range."""
    for (x0, y0), (x1, y1) in zip(zip(xs, ys), zip(xs[1:], ys[1:])):
        if min(y0, y1) <= y <= max(y0, y1) and y0 != y1:
            t = (np.log(y) - np.log(y0)) / (np.log(y1) - np.log(y0))
            return float(np.exp(np.log(x0) + t * (np.log(x1) - np.log(x0))))
    return None


def ladder(params, norm, seeds, sizes=(128, 160, 192, 224, 256), storages=("f16", "bf16"), fine_steps=4000,
           fine_every=80, c_guard=1.0, dev="cuda:0", fine=(256, 128, 128), count=16, log=print):
    """Throughput at a fixed wall-stress error.  Plain float32 runs of the same suspension at
    several resolutions (acoustic scaling, equal physical time: fine_steps * r steps), the
    learned closure at the coarsest, and the 16-bit storage forms at the finest; every error
    against the finest float32 run.  The bottom-wall shear stress, averaged over the last
    quarter of the run at the same physical times, is compared on a 16 x 32 grid of wall
    patches (8 x 8 cells at the finest resolution); centroid velocities of the platelets likewise.  Throughput is the HIP-graph
    coupled-step rate, also as fine-equivalent cell updates (cells / r^3 per step, 1 / r fine
    steps per step: MLUPS / r^4).  The plain error-vs-resolution curve, interpolated in
    log-log, gives the plain resolution (and its throughput) that matches each other run's
    error."""
    import torch

    sizes = sorted(sizes)
    top = sizes[-1]
    if top != fine[0]:
        raise ValueError("the finest rung must be the fine lattice")
    patches = (fine[2] // 8, fine[0] // 8)
    per_seed = []
    for seed in seeds:
        rungs = inputs.resolution_ladder(seed, sizes, count=count, fine=fine)
        specs = [("plain%d" % n, n, "f32", False) for n in sizes]
        if params is not None:
            specs.append(("learned%d" % sizes[0], sizes[0], "f32", True))
        specs += [("%s%d" % (st, top), top, st, False) for st in storages]
        res = {}
        for name, n, st, closure in specs:
            ch, r = rungs[n]
            lat = lbm.Lattice([ch], storage=st, max_nodes=ch.bodies.n, device=dev)
            from . import tune

            cfg = tune.load(lat)
            if cfg is not None:
                lat.set_launch(**dict(tune.DEFAULT, **cfg))
            lat.init()
            mem, X, F, U = _nodes_setup(lat, ch, dev)
            mem.offsets = ch.bodies.body_offsets
            if closure:
                lat.set_closure(params, norm, c_guard)
            steps, every = int(round(fine_steps * r)), int(round(fine_every * r))
            wss, vel, _ = _run(lat, mem, X, F, U, steps, every, (ch.nz, ch.nx))
            flags = lat.error_flags()
            rate = _graph_rate(lat, mem, X, F, U)
            torch.cuda.synchronize()
            res[name] = {"nx": n, "r": r, "storage": st, "closure": closure, "steps": steps, "tau": ch.tau,
                         "nodes": ch.bodies.n, "wss": _patch_mean(wss, patches), "vel": vel,
                         "mlups": ch.cells * rate / 1e6, "fine_eq_mlups": ch.cells * rate / 1e6 / r ** 4,
                         "flags": flags}
            del lat
        ref = res["plain%d" % top]
        base = float(np.mean(ref["wss"]))
        for name, v in res.items():
            v["wss_rel_l2"] = float(np.linalg.norm(v["wss"] - ref["wss"]) / np.linalg.norm(ref["wss"]))
            v["wss_mean_rel"] = float(abs(np.mean(v["wss"]) - base) / abs(base))
            v["vel_rel_l2"] = float(np.linalg.norm(v["vel"] - ref["vel"]) / np.linalg.norm(ref["vel"]))
        for name, v in res.items():
            v["wss_patches"] = v.pop("wss").tolist()
            del v["vel"]
            log("seed %d %-10s nx %3d tau %.4f steps %4d: wss %.4g mean %.4g vel %.4g, %.0f MLUPS, %.0f fine-eq" % (
                seed, name, v["nx"], v["tau"], v["steps"], v["wss_rel_l2"], v["wss_mean_rel"], v["vel_rel_l2"],
                v["mlups"], v["fine_eq_mlups"]))
        per_seed.append({"seed": seed, "runs": res})
    # seed-averaged errors and rates, and the plain resolution matching each run's error
    names = list(per_seed[0]["runs"])
    avg = {}
    for name in names:
        rs = [p["runs"][name] for p in per_seed]
        avg[name] = {k: (float(np.mean([x[k] for x in rs])) if isinstance(rs[0][k], float) else rs[0][k])
                     for k in rs[0] if k != "wss_patches"}
    plain = [avg["plain%d" % n] for n in sizes[:-1]]
    xs = [p["nx"] for p in plain]
    for name, v in avg.items():
        if name.startswith("plain"):
            continue
        n_eq = _interp_log(xs, [p["wss_rel_l2"] for p in plain], v["wss_rel_l2"])
        v["plain_nx_at_same_wss_error"] = n_eq
        if n_eq is not None:
            feq = _interp_log_value(xs, [p["fine_eq_mlups"] for p in plain], n_eq)
            v["plain_fine_eq_mlups_at_same_wss_error"] = feq
            v["speedup_at_same_wss_error"] = v["fine_eq_mlups"] / feq
        log("%-10s wss %.4g -> plain nx %s; %s" % (name, v["wss_rel_l2"], n_eq,
                                                   v.get("speedup_at_same_wss_error")))
    return {"seeds": list(seeds), "sizes": sizes, "fine_steps": fine_steps, "per_seed": per_seed, "mean": avg}


def _interp_log_value(xs, ys, x):
    """Value at x of the piecewise log-log line through (xs, ys)."""
    lx = np.log(xs)
    return float(np.exp(np.interp(np.log(x), lx, np.log(ys))))


def train_throughput(steps, snapshots=8, cells=524288, batch=65536, dev="cuda:0"):
    """Training rate on seeded synthetic data of the production shape (no fine runs): features
    ~ N(0, 1e-4^2), targets ~ N(0, 1e-6^2), `snapshots` x `cells` samples, one validation
    batch.  Prints one JSON line."""
    import torch

    g = torch.Generator(device=dev).manual_seed(0)
    feat = torch.randn(snapshots, cells, 16, device=dev, generator=g) * 1e-4
    tgt = torch.randn(snapshots, cells, 16, device=dev, generator=g) * 1e-6
    vf, vt = feat[:1, :batch].clone(), tgt[:1, :batch].clone()
    torch.cuda.synchronize()
    _, _, _, secs = train(feat, tgt, vf, vt, steps=steps, batch=batch, log_every=10 ** 9, log=lambda m: None)
    rep = {"adam_steps": steps, "batch": batch, "seconds": round(secs, 4),
           "samples_per_s": round(steps * batch / secs, 1), "us_per_step": round(secs / steps * 1e6, 2)}
    print(json.dumps(rep), flush=True)
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="small run (smoke size)")
    ap.add_argument("--train-seeds", type=int, default=8)
    ap.add_argument("--val-seeds", type=int, default=1)
    ap.add_argument("--eval-seeds", type=int, default=2)
    ap.add_argument("--snapshots", type=int, default=25)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--coarse-steps", type=int, default=2000)
    ap.add_argument("--higher-only", action="store_true", help="correct only moments above second order")
    ap.add_argument("--weights", default=None, help="evaluate saved weights (a *_weights.pt of a run) only")
    ap.add_argument("--alpha", type=float, nargs="*", default=[1.0],
                    help="evaluate with the correction scaled by these factors")
    ap.add_argument("--select-alpha", action="store_true",
                    help="run the --alpha candidates on the validation seeds, keep the one with the lowest "
                         "wall-stress error, and evaluate only that one on the held-out seeds")
    ap.add_argument("--c-guard", type=float, default=1.0)
    ap.add_argument("--ladder", action="store_true",
                    help="with --weights and one --alpha: plain float32 at a ladder of resolutions, the learned "
                         "closure and the 16-bit storage forms, compared at the same wall-stress error")
    ap.add_argument("--ladder-sizes", type=int, nargs="*", default=[128, 160, 192, 224, 256])
    ap.add_argument("--train-throughput", type=int, default=0, metavar="STEPS",
                    help="time STEPS Adam steps on seeded synthetic data (8 snapshots of 524,288 cells) and "
                         "print the training rate")
    args = ap.parse_args(argv)

    import torch

    def log(msg):
        print(msg, flush=True)

    if args.train_throughput:
        return train_throughput(args.train_throughput)
    kw = {}
    if args.quick:
        kw = dict(fine=(64, 48, 32), count=2)
        args.train_seeds, args.val_seeds, args.eval_seeds = 2, 1, 1
        args.snapshots, args.steps, args.coarse_steps = 4, 200, 200
    t0 = time.perf_counter()
    train_seeds = list(range(args.train_seeds))
    val_seeds = list(range(100, 100 + args.val_seeds))
    eval_seeds = list(range(200, 200 + args.eval_seeds))
    if args.ladder:
        params = norm = None
        if args.weights:
            w = torch.load(args.weights, weights_only=True)
            params, norm = w["params"].to("cuda:0"), w["norm"].to("cuda:0").clone()
            norm[32:48] *= args.alpha[0]
        sizes = args.ladder_sizes
        if args.quick:
            sizes = [kw["fine"][0] * k // 8 for k in (4, 6, 8)]
        rep = ladder(params, norm, eval_seeds, sizes=sizes, c_guard=args.c_guard,
                     fine_steps=2 * args.coarse_steps, log=log, **kw)
        rep["alpha"] = args.alpha[0] if args.weights else None
        if args.out:
            with open(args.out, "w") as f:
                json.dump(rep, f, indent=1)
        return rep
    if args.weights:
        w = torch.load(args.weights, weights_only=True)
        params, norm = w["params"].to("cuda:0"), w["norm"].to("cuda:0")
        hist, t_train, t_data, nsamp = [], 0.0, 0.0, 0
    else:
        feat, tgt = generate(train_seeds, snapshots=args.snapshots, log=log, **kw)
        vfeat, vtgt = generate(val_seeds, snapshots=max(2, args.snapshots // 5), log=log, **kw)
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        log("data: %d training samples, %d validation samples, %.1f s" % (feat.shape[0] * feat.shape[1],
                                                                           vfeat.shape[0] * vfeat.shape[1], t_data))
        params, norm, hist, t_train = train(feat, tgt, vfeat, vtgt, steps=args.steps,
                                            batch=min(65536, feat.shape[1]), log=log,
                                            log_every=max(1, args.steps // 6), higher_only=args.higher_only)
        nsamp = args.steps * min(65536, feat.shape[1])
        log("training: %d steps, %.1f s, %.1f M samples/s" % (args.steps, t_train, nsamp / t_train / 1e6))
        del feat, tgt
    alphas = list(args.alpha)
    selection = None
    if args.select_alpha:
        scores = []
        for alpha in alphas:
            na = norm.clone()
            na[32:48] *= alpha
            log("validation, alpha %.3g:" % alpha)
            rs = evaluate(params, na, val_seeds, coarse_steps=args.coarse_steps, log=log, c_guard=args.c_guard, **kw)
            scores.append((float(np.mean([r["learned_wss_rel_l2"] for r in rs])), alpha, rs))
        best = min(scores, key=lambda t: t[0])
        selection = {"candidates": [(a, sc) for sc, a, _ in scores], "chosen": best[1],
                     "plain_wss_rel_l2": float(np.mean([r["plain_wss_rel_l2"] for r in best[2]]))}
        log("selected alpha %.3g on the validation seeds" % best[1])
        alphas = [best[1]]
    ev = []
    for alpha in alphas:
        na = norm.clone()
        na[32:48] *= alpha  # output scale: the correction times alpha
        log("alpha %.3g:" % alpha)
        for r in evaluate(params, na, eval_seeds, coarse_steps=args.coarse_steps, log=log, c_guard=args.c_guard, **kw):
            r["alpha"] = alpha
            ev.append(r)
    rep = {"train_seeds": train_seeds, "val_seeds": val_seeds, "eval_seeds": eval_seeds,
           "snapshots_per_seed": args.snapshots, "adam_steps": args.steps, "history": hist,
           "train_seconds": t_train, "data_seconds": t_data,
           "train_samples_per_s": nsamp / t_train if t_train else None,
           "eval": ev, "alpha_selection": selection, "norm": norm.cpu().numpy().tolist(),
           "higher_only": args.higher_only,
           "c_guard": args.c_guard}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)
        if not args.weights:
            torch.save({"params": params.cpu(), "norm": norm.cpu()}, args.out.rsplit(".", 1)[0] + "_weights.pt")
    return rep


if __name__ == "__main__":
    main()
