"""Autotuner for the launch shape and schedule of the coupled step.

Times each candidate `lbm_launch` on the caller's own context with HIP events and keeps the
fastest.  With the Lagrangian nodes and membrane of a workload it times what the benchmark
runs: the whole coupled step (forces -> spread -> lattice update -> interpolation -> move),
replayed from a captured HIP graph, over the lattice kernel's launch shapes (workgroup
size, XCD-aware order, persistent grid, non-temporal stores, cells per lane), the two
coupled-step schedules (one fused update after the spread, or the body-force update in the
spread's launch followed by the flagged tiles) and the binning interval (every step, or every
2, 4 or 8 steps with a margin).  Without nodes it times back-to-back lattice
steps.  Results are cached in a JSON file keyed by GPU architecture, storage form, size class
(total cells rounded to a power of two, number of channels) and what was timed, so later runs
reuse them without re-timing.
"""
from __future__ import annotations

import json
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_HERE, "tuned_launch.json")

DEFAULT = dict(block=256, xcd_remap=1, persistent=0, nontemporal=1, vec=0, overlap=0, split=-1, rebin=1)


def graph_steps(cfg):
    """Steps of a captured coupled-step graph for the launch cfg (a multiple of 2 rebin)."""
    return 2 * max(1, int(cfg.get("rebin", 1)))


def lattice_candidates(n_cu=256):
    """Launch shapes of the lattice kernel."""
    out = []
    for vec in (0, 2, 4):
        for nt in (0, 1):
            for remap in (1, 0):
                blocks = (64, 128, 256, 512, 1024) if vec == 0 else (256,)
                for block in blocks:
                    out.append(dict(block=block, xcd_remap=remap, persistent=0, nontemporal=nt, vec=vec))
    for vec in (0, 2):
        for per_cu in (4, 8, 16):
            out.append(dict(block=256, xcd_remap=1, persistent=per_cu * n_cu, nontemporal=0, vec=vec))
    return out


def coupled_candidates(n_cu=256):
    """Coupled-step schedules: the fused update over every lattice launch shape, and the split
    update (its body-force launch has a fixed shape; only the store kind and the flagged-tile
    launch vary)."""
    out = [dict(c, split=0) for c in lattice_candidates(n_cu)]
    # binning every 2, 4 or 8 steps: 8 keeps the half-cell margin for nodes up to 1/16 cell per step
    for nt in (0, 1):
        for rebin in (1, 2, 4, 8):
            out.append(dict(block=256, xcd_remap=1, persistent=0, nontemporal=nt, vec=0, split=1, rebin=rebin))
    for rebin in (2, 4, 8):
        out.append(dict(block=128, xcd_remap=0, persistent=0, nontemporal=1, vec=0, split=0, rebin=rebin))
    return out


def size_class(lat, what):
    return "%s|cells~2^%d|nch=%d|%s" % (lat.storage, int(round(math.log2(max(lat.total_cells, 1)))), lat.nch, what)


def arch_name(torch, device):
    try:
        return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_launch(lat, cfg, steps=20, warmup=3):
    """Average time (ms) of one lattice step with launch shape `cfg` (the state advances)."""
    torch = lat.torch
    lat.set_launch(**dict(DEFAULT, **cfg))
    lat.step(warmup)
    e0, e1 = _events(torch)
    torch.cuda.synchronize()
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_coupled(lat, cfg, coupled, steps=20, warmup=4):
    """Average time (ms) of one coupled step with launch `cfg`, replayed from a captured graph of
    graph_steps(cfg) steps (the state and the nodes advance).  coupled = (membrane, X, F, U)."""
    torch = lat.torch
    mem, X, F, U = coupled
    full = dict(DEFAULT, **cfg)
    lat.set_launch(**full)
    G = graph_steps(full)
    lat.graph_capture(mem, G, X, F, U)
    lat.graph_launch(max(1, warmup // G))
    reps = max(1, steps // G)
    e0, e1 = _events(torch)
    torch.cuda.synchronize()
    e0.record(lat.stream)
    lat.graph_launch(reps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (G * reps)


def tune(lat, steps=20, cands=None, verbose=False, coupled=None):
    """Time every candidate on `lat` (coupled steps when `coupled` = (membrane, X, F, U) is
    given, else lattice steps); set and return (best_cfg, table)."""
    table = []
    if cands is None:
        cands = coupled_candidates() if coupled is not None else lattice_candidates()
    for cfg in cands:
        ms = time_coupled(lat, cfg, coupled, steps=steps) if coupled is not None else time_launch(lat, cfg, steps=steps)
        table.append((ms, cfg))
        if verbose:
            print("%.4f ms  %s" % (ms, cfg), flush=True)
    table.sort(key=lambda t: t[0])
    best = dict(DEFAULT, **table[0][1])
    lat.set_launch(**best)
    return best, table


def _key(lat, what):
    return arch_name(lat.torch, lat.device) + "|" + size_class(lat, what)


def load(lat, what="coupled"):
    """Cached best launch for this context's size class, or None."""
    if not os.path.exists(CACHE):
        return None
    try:
        data = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    return data.get(_key(lat, what), {}).get("launch")


def save(lat, best, ms, what="coupled"):
    data = {}
    if os.path.exists(CACHE):
        try:
            data = json.load(open(CACHE))
        except (OSError, ValueError):
            data = {}
    timed = ("coupled step, HIP graph replay" if what == "coupled" else "lattice step, back-to-back launches")
    data[_key(lat, what)] = {"launch": best, "ms_per_step": ms, "timed": timed}
    tmp = CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def apply_cached_or_tune(lat, steps=20, verbose=False, retune=False, coupled=None):
    """Use the cached launch for this size class if there is one, else tune and cache.  With
    `coupled` = (membrane, X, F, U) the coupled step is what is timed (the lattice state and X
    advance: re-initialise them afterwards)."""
    what = "coupled" if coupled is not None else "lattice"
    cfg = None if retune else load(lat, what)
    if cfg is not None:
        cfg = dict(DEFAULT, **cfg)
        lat.set_launch(**cfg)
        return cfg, None
    best, table = tune(lat, steps=steps, verbose=verbose, coupled=coupled)
    save(lat, best, table[0][0], what)
    return best, table


def copy_ceiling(torch, device, nbytes, reps=10):
    """Best copy rate (bytes read + written per second) of the library's STREAM-style copy
    over a few grid shapes and store variants, for `nbytes` read and `nbytes` written."""
    from . import lbm

    src = torch.empty(nbytes // 16 * 16, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    best = None
    for variant in (0, 1):
        for grid in (0, 256 * 8, 256 * 16, 256 * 32):
            lbm.stream_copy(src, dst, variant, grid)
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record()
            for _ in range(reps):
                lbm.stream_copy(src, dst, variant, grid)
            e1.record()
            torch.cuda.synchronize()
            rate = 2 * src.numel() * reps / (e0.elapsed_time(e1) * 1e-3)
            if best is None or rate > best[0]:
                best = (rate, dict(variant=variant, grid=grid))
    return best


def workload_context(channels, storage="f32", device="cuda:0"):
    """A context of `channels` with their nodes declared, their membrane and X, F, U."""
    import torch

    from . import inputs, lbm

    b, offs = inputs.concat_bodies(channels)
    lat = lbm.Lattice(channels, storage=storage, kernel="cos", max_nodes=b.n, device=device)
    lat.init()
    lat.set_nodes(b.n, offs if len(channels) > 1 else None)
    mem = lbm.Membrane(b, device=device)
    X = torch.from_numpy(b.X.copy()).to(device)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=device)
    U = torch.zeros_like(F)
    return lat, (mem, X, F, U)


def main(argv=None):
    """python -m paper_1312_2234_amd.tune [--storage f32] [--workload shear|batched|coarse]
    [--lattice]: tune the coupled step (or, with --lattice, the lattice kernel alone) for a
    benchmark workload and cache the result."""
    import argparse

    import torch

    from . import inputs

    ap = argparse.ArgumentParser()
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--workload", default="shear", choices=["shear", "batched", "coarse"])
    ap.add_argument("--lattice", action="store_true", help="time back-to-back lattice steps only")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--copy", action="store_true", help="also measure the copy ceiling")
    args = ap.parse_args(argv)
    if args.workload == "batched":
        chans = inputs.batched_channels(seed=0)
    elif args.workload == "coarse":
        chans = [inputs.coarse_fine_pair(seed=200, u_top=0.05)[1]]
    else:
        chans = [inputs.shear_platelets(seed=0)]
    lat, coupled = workload_context(chans, storage=args.storage)
    what = "lattice" if args.lattice else "coupled"
    best, table = tune(lat, steps=args.steps, verbose=True, coupled=None if args.lattice else coupled)
    save(lat, best, table[0][0], what)
    bpc = 152 if args.storage == "f32" else 76
    for ms, cfg in table[:5]:
        print("best: %.4f ms  %.1f GB/s (algorithmic, whole %s step)  %s"
              % (ms, bpc * lat.total_cells / (ms * 1e-3) / 1e9, what, cfg), flush=True)
    if args.copy:
        rate, cfg = copy_ceiling(torch, lat.device, bpc * lat.total_cells // 2)
        print("copy ceiling: %.1f GB/s %s" % (rate / 1e9, cfg), flush=True)


if __name__ == "__main__":
    main()
