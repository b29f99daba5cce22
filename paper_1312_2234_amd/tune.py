"""Autotuner for the lattice kernel's launch shape.

Times each candidate `lbm_launch` (workgroup size, XCD-aware order, persistent grid,
non-temporal stores, cells per lane) on the caller's own context with HIP events around
back-to-back launches on the library's stream, and keeps the fastest.  Results are cached
in a JSON file keyed by GPU architecture, storage form and size class (total cells rounded
to a power of two, number of channels), so later runs reuse them without re-timing.
"""
from __future__ import annotations

import json
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_HERE, "tuned_launch.json")

DEFAULT = dict(block=256, xcd_remap=1, persistent=0, nontemporal=1, vec=0, overlap=0, split=-1)


def candidates(n_cu=256):
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


def size_class(lat):
    return "%s|cells~2^%d|nch=%d" % (lat.storage, int(round(math.log2(max(lat.total_cells, 1)))), lat.nch)


def arch_name(torch, device):
    try:
        return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def time_launch(lat, cfg, steps=20, warmup=3):
    """Average time (ms) of one lattice step with launch shape `cfg` (the state advances)."""
    torch = lat.torch
    lat.set_launch(**dict(DEFAULT, **cfg))
    lat.step(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(lat, steps=20, cands=None, verbose=False):
    """Time every candidate on `lat`; set and return (best_cfg, table)."""
    table = []
    for cfg in cands or candidates():
        ms = time_launch(lat, cfg, steps=steps)
        table.append((ms, cfg))
        if verbose:
            print("%.4f ms  %s" % (ms, cfg), flush=True)
    table.sort(key=lambda t: t[0])
    best = dict(DEFAULT, **table[0][1])
    lat.set_launch(**best)
    return best, table


def load(lat):
    """Cached best launch for this context's size class, or None."""
    if not os.path.exists(CACHE):
        return None
    try:
        data = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    key = arch_name(lat.torch, lat.device) + "|" + size_class(lat)
    return data.get(key, {}).get("launch")


def save(lat, best, ms):
    data = {}
    if os.path.exists(CACHE):
        try:
            data = json.load(open(CACHE))
        except (OSError, ValueError):
            data = {}
    key = arch_name(lat.torch, lat.device) + "|" + size_class(lat)
    data[key] = {"launch": best, "ms_per_step": ms}
    tmp = CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def apply_cached_or_tune(lat, steps=20, verbose=False, retune=False):
    """Use the cached launch for this size class if there is one, else tune and cache."""
    cfg = None if retune else load(lat)
    if cfg is not None:
        cfg = dict(DEFAULT, **cfg)
        lat.set_launch(**cfg)
        return cfg, None
    best, table = tune(lat, steps=steps, verbose=verbose)
    save(lat, best, table[0][0])
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
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                lbm.stream_copy(src, dst, variant, grid)
            e1.record()
            torch.cuda.synchronize()
            rate = 2 * src.numel() * reps / (e0.elapsed_time(e1) * 1e-3)
            if best is None or rate > best[0]:
                best = (rate, dict(variant=variant, grid=grid))
    return best


def main(argv=None):
    """python -m paper_1312_2234_amd.tune [--storage f32] [--batched]: tune the lattice
    kernel for the production shear lattice (or the batched channel set) and cache the result."""
    import argparse

    import torch

    from . import inputs, lbm

    ap = argparse.ArgumentParser()
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--batched", action="store_true")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--copy", action="store_true", help="also measure the copy ceiling")
    args = ap.parse_args(argv)
    chans = inputs.batched_channels(seed=0) if args.batched else [inputs.shear_platelets(seed=0)]
    lat = lbm.Lattice(chans, storage=args.storage, device="cuda:0")
    lat.init()
    best, table = tune(lat, steps=args.steps, verbose=True)
    save(lat, best, table[0][0])
    bpc = 152 if args.storage == "f32" else 76
    for ms, cfg in table[:5]:
        print("best: %.4f ms  %.1f GB/s  %s" % (ms, bpc * lat.total_cells / (ms * 1e-3) / 1e9, cfg), flush=True)
    if args.copy:
        rate, cfg = copy_ceiling(torch, lat.device, bpc * lat.total_cells // 2)
        print("copy ceiling: %.1f GB/s %s" % (rate / 1e9, cfg), flush=True)


if __name__ == "__main__":
    main()
