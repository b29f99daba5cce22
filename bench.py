"""Throughput of the coupled D3Q19 LBM + immersed-boundary step on one MI355X.

One step = the whole hot path of Fig. 1 on the GPU: membrane forces -> IB spreading ->
lattice-Boltzmann step -> IB interpolation -> node update, for the production shear
workload (256x128x128 lattice, moving top wall u = 0.05, tau = 1.0, 16 oblate platelets of
2562 nodes with spring network and bending, cosine delta kernel, weight-shifted float32
populations).  The step sequence is replayed from a captured HIP graph; inputs are resident
in HBM before the timed region starts.

Prints ONE JSON line.  Besides the contract fields it carries:
  roofline      the coupled step's lattice-update launch (which moves >97% of the bytes: in the
                single-channel schedule the body-force update of every cell, in the same launch
                as the IB spread): algorithmic bytes per launch (152 B per cell in float32, 76 B
                in 16-bit) over its mean duration, timed with HIP events recorded by the library
                around that launch on its own stream, against the 8 TB/s HBM peak; `step_frac`
                is the same bytes over the whole step time, i.e. the step's own fraction of peak;
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LBM+IB MLUPS, % HBM peak; FP16-store/learned vs plain FP32 at fixed error"
HBM_PEAK = 8.0e12
BYTES_PER_CELL = {"f32": 152, "f16": 76, "bf16": 76}
DTYPE = {"f32": "f32", "f16": "f16-store/f32", "bf16": "bf16-store/f32"}


def make_workload(name):
    import dataclasses

    from paper_1312_2234_amd import inputs

    if name == "shear":
        ch = inputs.shear_platelets(seed=0)
        desc = ("shear channel 256x128x128, top wall u=0.05, tau=1.0, 16 oblate platelets "
                "(6,2,6) x 2562 IB nodes, spring k=0.005 + bending 1e-4")
        return [ch], desc
    if name == "shear_large":
        ch = inputs.shear_platelets(seed=0, nx=512, ny=256, nz=128, count=64)
        desc = ("shear channel 512x256x128 (populations too large for the 256 MB Infinity Cache in every storage "
                "form), top wall u=0.05, tau=1.0, 64 oblate platelets (6,2,6) x 2562 IB nodes, spring k=0.005 + "
                "bending 1e-4")
        return [ch], desc
    if name == "shear_onsite":
        ch = dataclasses.replace(inputs.shear_platelets(seed=0), walls="onsite")
        desc = ("shear channel 256x128x128 with on-site velocity walls (Eq. 23-30) on rows 0 and 127, "
                "top wall u=0.05, tau=1.0, 16 oblate platelets (6,2,6) x 2562 IB nodes, spring k=0.005 + "
                "bending 1e-4")
        return [ch], desc
    if name == "shear_constrained":
        ks, kt, kv = inputs.table2_constraint_coefficients()
        ch = inputs.shear_platelets(seed=0)
        ch = dataclasses.replace(ch, bodies=inputs.with_constraints(ch.bodies, ks, kt, kv))
        desc = ("shear channel 256x128x128, top wall u=0.05, tau=1.0, 16 oblate platelets (6,2,6) x 2562 IB "
                "nodes, spring k=0.005 + bending 1e-4 + area/volume constraints of Eq. 4-5 (Table 2: "
                "k_s=k_t=%.4f, k_v=%.4f lattice units)" % (ks, kv))
        return [ch], desc
    if name == "shear_fe":
        k0 = inputs.table2_bending_modulus()
        ch = inputs.shear_platelets(seed=0)
        ch = dataclasses.replace(ch, bodies=inputs.with_fe_bending(ch.bodies, k0))
        desc = ("shear channel 256x128x128, top wall u=0.05, tau=1.0, 16 oblate platelets (6,2,6) x 2562 IB "
                "nodes, spring k=0.005 + finite-element bending of Eq. 6-10 on six-node triangles (Table 2: "
                "k_0 = 200 k_BT = %.3e lattice units) in place of the dihedral stand-in" % k0)
        return [ch], desc
    if name == "shear_adhesion":
        ch = inputs.shear_platelets(seed=0, y_band=(2.3, 2.6))
        desc = ("shear channel 256x128x128, top wall u=0.05, tau=1.0, 16 oblate platelets (6,2,6) x 2562 IB nodes "
                "resting 0.1-0.6 lattice units above the lower wall, spring k=0.005 + bending 1e-4, with the "
                "adhesion of section 3.2: 5344 receptor points per platelet, vWF ligands at 25 per um^2 on the "
                "wall, Table 2's k_on0 and k_off0 (sigma = 1e-3 N/m, gamma = 0.7 nm assumed, l_b = 128 nm)")
        return [ch], desc
    if name == "batched":
        chans = inputs.batched_channels(seed=0)
        desc = ("64 independent shear channels, sizes uniform over {48x32x32, 64x48x48, 96x64x64, 128x64x64}, "
                "1-8 platelets of 642/2562 IB nodes, u_top U(0.01,0.05), tau U(0.7,1.2)")
        return chans, desc
    if name == "coarse":
        _, ch = inputs.coarse_fine_pair(seed=200, u_top=0.05)
        desc = ("coarse twin of the shear channel (2x coarser in space and time): 128x64x64, tau=0.75, "
                "16 platelets (3,1,3) x 1282 IB nodes; one update stands for 16 fine cell-updates")
        return [ch], desc
    if name == "sphere":
        ch = inputs.poiseuille_sphere(seed=0)
        return [ch], "32^3 body-force channel, tau=0.8, tethered 642-node sphere"
    raise SystemExit("unknown workload " + name)


# Sources of the lattice kernels: a counter summary under profiles/ applies only while they are
# unchanged (their SHA-256 is recorded in the summary).
KERNEL_SOURCES = ("paper_1312_2234_amd/csrc/lattice.hip", "paper_1312_2234_amd/csrc/ib.hip",
                  "paper_1312_2234_amd/csrc/lbm_device.h", "paper_1312_2234_amd/csrc/lbm_internal.h")
# the launch the library's timer brackets, by the kind it reports
TIMED_KERNEL = {0: "k_step", 1: "k_spread_far", 2: "k_step_cl"}
TIMED_KERNEL_DESC = {0: "k_step (fused lattice step with the IB force)",
                     1: "k_spread_far (body-force lattice update of every cell + the IB spread, one launch)",
                     2: "k_step_cl (lattice step + learned closure)"}


def kernel_sources_sha256():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, storage, workload):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE summary for
    this storage form and workload (counter readings scaled by the same counters' reading of a
    plain copy of known size), or None if there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_hbm_counters.md" % (kernel, storage, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = re.search(r"^sources_sha256:\s*([0-9a-f]{64})", text, re.M)
    val = re.search(r"^traffic_bytes_per_launch:\s*(\d+)", text, re.M)
    if not sha or not val or sha.group(1) != kernel_sources_sha256():
        return None
    return int(val.group(1))


# Closure network cost per cell (16 -> 64 -> 64 -> 16 on the matrix cores)
MLP_FLOP_PER_CELL = 2 * (16 * 64 + 64 * 64 + 64 * 16)
MFMA_BF16_PEAK = 2.5e15


def closure_weights(torch, dev):
    """Seeded network for throughput runs: He-normal layers; inputs scaled to unit size and a
    small output scale, so that every correction passes the guard."""
    import numpy as np

    rng = np.random.default_rng(0)
    th = np.concatenate([rng.normal(0, 0.35, 1024), np.zeros(64), rng.normal(0, 0.18, 4096), np.zeros(64),
                         rng.normal(0, 0.01, 1024), np.zeros(16)])
    norm = np.concatenate([np.zeros(16), np.full(16, 1e4), np.full(16, 1e-7)])
    return (torch.from_numpy(th.astype(np.float32)).to(dev), torch.from_numpy(norm.astype(np.float32)).to(dev))


def adhesion_of(workload, channels):
    """The adhesion description of the shear_adhesion workload (None for the others)."""
    if workload != "shear_adhesion":
        return None
    from paper_1312_2234_amd import inputs

    ch = channels[0]
    p = inputs.table2_adhesion()
    rt, rb = inputs.receptor_points(ch.bodies, per_body=p["receptors_per_body"], seed=0)
    lig = inputs.wall_ligands(ch.nx, ch.nz, density=p["ligand_density"], seed=1)
    return dict(rec_tri=rt, rec_bary=rb, ligands=lig, wall_y=-0.5, nx=float(ch.nx), nz=float(ch.nz),
                capture=p["capture"], sigma=p["sigma"], l_b=p["l_b"], gamma=p["gamma"], kT=p["kT"],
                k_on0=p["k_on0"], k_off0=p["k_off0"], seed=0)


def cpu_baseline(channels, kernel, steps, single_steps=4, adhesion=None):
    """The FP64 oracle (as it stands) on `steps` coupled steps of the first channel."""
    import numpy as np

    from oracle import oracle

    ch = channels[0]
    b = ch.bodies
    o = oracle.Lattice(ch.nx, ch.ny, ch.nz, ch.tau, walls=ch.walls, body=ch.body, u_wall_lo=ch.u_wall_lo,
                       u_wall_hi=ch.u_wall_hi, kernel=kernel)
    o.init(u=o.shear_profile()) if ch.init == "shear" else o.init()
    mem = oracle.Membrane(b.X_rest, b.edges, k_spring=b.k_spring, hinges=b.hinges, k_bend=b.k_bend,
                          anchors=b.anchors, k_tether=b.k_tether, triangles=b.triangles,
                          body_tri=b.tri_offsets if b.triangles is not None else None,
                          k_area_global=b.k_area_global, k_area_local=b.k_area_local, k_volume=b.k_volume,
                          elements6=b.elements6, k_fe=b.k_fe)
    adh = None
    if adhesion is not None:
        from oracle import dam_oracle

        a = adhesion
        adh = dam_oracle.Adhesion(a["rec_tri"], a["rec_bary"], a["ligands"], a["wall_y"], a["nx"], a["nz"],
                                  a["capture"], a["sigma"], a["l_b"], a["gamma"], a["kT"], a["k_on0"],
                                  a["k_off0"], a["seed"])
    X = b.X.copy()
    oracle.coupled_step(o, mem, X, adhesion=adh)  # first touch of the arrays, not timed
    cores = oracle.threads()
    t0 = time.perf_counter()
    for s in range(steps):
        oracle.coupled_step(o, mem, X, adhesion=adh, step=s + 1)
    dt = time.perf_counter() - t0
    out = {"value": round(ch.cells * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": "%d coupled steps (forces, spread, LBM, interpolation, move) of the full %dx%dx%d "
                     "workload, FP64, %.1f s" % (steps, ch.nx, ch.ny, ch.nz, dt),
           "host": {"cpu": cpu_model(), "nproc": os.cpu_count()}}
    if single_steps > 0:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        for s in range(single_steps):
            oracle.coupled_step(o, mem, X, adhesion=adh, step=steps + 1 + s)
        d1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        out["single_core"] = {"value": round(ch.cells * single_steps / d1 / 1e6, 4), "unit": "MLUPS", "cores": 1,
                              "sample": "%d coupled steps, %.1f s" % (single_steps, d1)}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="shear")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--kernel", default="cos", choices=["cos", "peskin4"])
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--cpu-single-steps", type=int, default=4, help="steps of the one-thread oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lbm-only-steps", type=int, default=200)
    ap.add_argument("--timer-steps", type=int, default=60,
                    help="eager coupled steps over which the lattice-update launch is timed")
    ap.add_argument("--tune", action="store_true",
                    help="re-time the coupled step over the lattice launch shapes and schedules")
    ap.add_argument("--launch", default=None,
                    help="lattice launch shape as JSON, e.g. '{\"block\": 256, \"xcd_remap\": 0}' (skips the tuner cache)")
    ap.add_argument("--closure", action="store_true",
                    help="run the step with the learned closure (seeded weights; throughput only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run plain device copies of the lattice kernel's byte count (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1312_2234_amd import lbm

    dev = "cuda:0"
    channels, desc = make_workload(args.workload)
    nodes = sum(c.bodies.n for c in channels)
    cells = sum(c.cells for c in channels)
    lat = lbm.Lattice(channels, storage=args.storage, kernel=args.kernel, max_nodes=nodes, device=dev)
    lat.init()
    from paper_1312_2234_amd import inputs, tune

    b, offs = inputs.concat_bodies(channels)
    lat.set_nodes(b.n, offs if len(channels) > 1 else None)
    mem = lbm.Membrane(b, device=dev, adhesion=adhesion_of(args.workload, channels))
    X = torch.from_numpy(b.X.copy()).to(dev)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=dev)
    U = torch.zeros_like(F)
    if args.closure:
        lat.set_closure(*closure_weights(torch, dev), 1.0)
    if args.launch:
        cfg = dict(tune.DEFAULT, **json.loads(args.launch))
        lat.set_launch(**cfg)
    else:
        # the cached launch and schedule of this size class (tuned on the graph-replayed
        # coupled step), or a tuning run now, which advances the state: start again after it
        tune.apply_cached_or_tune(lat, retune=args.tune, coupled=(mem, X, F, U))
    lat.init()
    X.copy_(torch.from_numpy(b.X))
    F.zero_()
    U.zero_()
    # the graph replays G steps (2, or 2 rebin when the nodes are binned every `rebin` steps)
    # from the buffer parities and binning phase current at capture: the warm-up steps beyond a
    # multiple of G run eagerly before the capture, the timed ones after the last replay
    G = tune.graph_steps(lat.get_launch())
    if args.warmup % G:
        lat.coupled_steps(mem, args.warmup % G, X, F, U)
    lat.graph_capture(mem, G, X, F, U)
    stream = lat.stream  # the library's stream: events are recorded on it
    if args.warmup // G:
        lat.graph_launch(args.warmup // G)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    if args.steps // G:
        lat.graph_launch(args.steps // G)
    if args.steps % G:
        lat.coupled_steps(mem, args.steps % G, X, F, U)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    flags = lat.error_flags()

    # the coupled step's lattice-update launch, timed by the library's event pairs around it
    lat.launch_timer(True)
    lat.coupled_steps(mem, args.timer_steps, X, F, U)
    n_timed, us_update, kind = lat.launch_timer_read()
    lat.launch_timer(False)
    flags |= lat.error_flags()

    # lattice kernel alone: back-to-back launches on the same stream
    lat.step(10)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(args.lbm_only_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_lbm = e0.elapsed_time(e1) / args.lbm_only_steps
    bytes_launch = BYTES_PER_CELL[args.storage] * cells
    achieved = bytes_launch / (us_update * 1e-6)
    achieved_lbm = bytes_launch / (ms_lbm * 1e-3)
    achieved_step = bytes_launch / (ms * 1e-3)
    ceiling, ceiling_cfg = tune.copy_ceiling(torch, lat.device, bytes_launch // 2)
    kernel = TIMED_KERNEL[kind]
    out = {
        "metric": METRIC,
        "value": round(cells / (ms * 1e-3) / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage] + ("+bf16-mlp" if args.closure else ""),
        "data": "synthetic",
        "config": {"workload": desc, "cells": cells, "ib_nodes": nodes, "storage": args.storage,
                   "delta_kernel": args.kernel, "launch": lat.get_launch(), "graph": "%d-step HIP graph replay" % G,
                   "closure": "seeded 16-64-64-16 network (throughput run)" if args.closure else None},
        "ib_nodes_per_s": round(nodes / (ms * 1e-3), 1),
        "mlups_fine_equivalent": round(16 * cells / (ms * 1e-3) / 1e6, 2) if args.workload == "coarse" else None,
        "lbm_only_mlups": round(cells / (ms_lbm * 1e-3) / 1e6, 2),
        "error_flags": flags,
        "roofline": {"bound": "hbm", "kernel": TIMED_KERNEL_DESC[kind], "achieved": round(achieved / 1e9, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4),
                     "traffic": measured_traffic(kernel, args.storage, args.workload),
                     "bytes_per_launch": bytes_launch, "avg_launch_us": round(us_update, 2),
                     "timed_launches": n_timed,
                     "step_frac": round(achieved_step / HBM_PEAK, 4),
                     "copy_ceiling_GBps": round(ceiling / 1e9, 1),
                     "frac_of_copy_ceiling": round(achieved / ceiling, 4),
                     "lattice_only": {"kernel": "k_step_cl" if args.closure else "k_step",
                                      "avg_launch_us": round(ms_lbm * 1e3, 2),
                                      "achieved": round(achieved_lbm / 1e9, 1),
                                      "frac": round(achieved_lbm / HBM_PEAK, 4),
                                      "note": "back-to-back lbm_step launches, outside the timed step"}},
    }
    if args.closure:
        fl = MLP_FLOP_PER_CELL * cells / (us_update * 1e-6)
        out["roofline"]["mfma"] = {"achieved": round(fl / 1e12, 2), "peak": MFMA_BF16_PEAK / 1e12, "unit": "TFLOP/s",
                                   "frac": round(fl / MFMA_BF16_PEAK, 4), "flop_per_cell": MLP_FLOP_PER_CELL}
        out["closure_guarded"] = lat.closure_guarded()
        out["roofline"]["traffic"] = None
    if args.copy_probe:
        half = bytes_launch // 2  # read half, write half: the same bytes as one lattice launch
        src = torch.empty(half // 16 * 16, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            lbm.stream_copy(src, dst, 0, 0)
        torch.cuda.synchronize()
        out["copy_probe_bytes_read"] = src.numel()
        del src, dst
    if not args.no_cpu_baseline and args.cpu_steps > 0 and len(channels) == 1:
        del lat
        out["cpu_baseline"] = cpu_baseline(channels, args.kernel, args.cpu_steps, args.cpu_single_steps,
                                           adhesion_of(args.workload, channels))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
