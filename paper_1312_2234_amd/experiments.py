"""Jeffery-orbit workload (section 4.1): one oblate platelet tumbling in the middle of a
shear channel, run on the GPU through the C ABI, its rotation period against Jeffery's
rigid-spheroid period T = 2 pi (r + 1/r) / shear_rate (Jeffery 1922; the paper states no
formula).

The platelet's symmetry axis is the short axis of the gyration tensor of its nodes.  Shear
u_x(y) turns it in the x-y plane (vorticity along z).  The axis is a director, so its angle
advances by pi in half a period; the run stops after `half_turns` such advances and reports
the mean time per half turn.

    python -m paper_1312_2234_amd.experiments --jeffery [--n 64] [--nodes 642] [--u-top 0.05]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs


def jeffery_period(r: float, shear_rate: float) -> float:
    """Jeffery's period of a rigid spheroid of aspect ratio r in unbounded Stokes shear."""
    return 2.0 * math.pi * (r + 1.0 / r) / shear_rate


def symmetry_axis(X: np.ndarray) -> np.ndarray:
    """Unit short axis of the gyration tensor of the points X [3, n]."""
    d = X - X.mean(axis=1, keepdims=True)
    w, v = np.linalg.eigh(d @ d.T)
    return v[:, 0]


class DirectorTracker:
    """Unwrapped turning angle of a director (a sign-less axis) in the x-y plane, counted
    positive clockwise seen from +z (the sense in which u_x growing with y turns it), and the
    steps at which it passes each multiple of pi (linear interpolation within a sample)."""

    def __init__(self, axis0):
        self.prev = np.asarray(axis0, float)
        self.angle = 0.0
        self.marks = []

    def update(self, axis, steps, chunk):
        a = np.asarray(axis, float)
        if a @ self.prev < 0:  # director: keep the sign continuous
            a = -a
        d = math.atan2(self.prev[0] * a[1] - self.prev[1] * a[0], self.prev[0] * a[0] + self.prev[1] * a[1])
        new = self.angle - d
        k_old, k_new = math.floor(self.angle / math.pi), math.floor(new / math.pi)
        for k in range(k_old + 1, k_new + 1):
            target = k * math.pi
            self.marks.append(steps - chunk + chunk * (target - self.angle) / (new - self.angle))
        self.angle, self.prev = new, a


def jeffery(n=64, nodes=642, semi_axes=(6.0, 2.0, 6.0), u_top=0.05, tau=1.0, chunk=200, half_turns=2,
            max_steps=200000, seed=0, device="cuda:0", log=print):
    """Run the tumbling platelet until its axis has advanced by half_turns * pi.  Returns the
    measured time per half turn and Jeffery's, for the nominal aspect ratio."""
    import torch

    from . import lbm

    ch = inputs.jeffery_platelet(n=n, nodes=nodes, semi_axes=semi_axes, u_top=u_top, tau=tau, seed=seed)
    b = ch.bodies
    lat = lbm.Lattice([ch], kernel="cos", max_nodes=b.n, device=device)
    lat.init()
    lat.set_nodes(b.n)
    mem = lbm.Membrane(b, device=device)
    X = torch.from_numpy(b.X.copy()).to(device)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=device)
    U = torch.zeros_like(F)
    lat.graph_capture(mem, 2, X, F, U)
    shear_rate = u_top / ch.ny  # halfway walls at y = -1/2 and ny - 1/2
    tr = DirectorTracker(symmetry_axis(b.X))
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps and len(tr.marks) < half_turns + 1:
        lat.graph_launch(chunk // 2)
        steps += chunk
        tr.update(symmetry_axis(X.cpu().numpy()), steps, chunk)
    marks = tr.marks
    secs = time.perf_counter() - t0
    flags = lat.error_flags()
    r = semi_axes[1] / semi_axes[0]
    # the first crossing comes after the start-up (flow and shape settle); time per half turn
    # between the first and the last crossing
    per_half = (marks[-1] - marks[0]) / (len(marks) - 1) if len(marks) > 1 else float("nan")
    res = {
        "lattice": [ch.nx, ch.ny, ch.nz], "nodes": b.n, "semi_axes": list(semi_axes), "tau": tau,
        "shear_rate": shear_rate, "steps": steps, "seconds": round(secs, 2), "flags": flags,
        "half_turn_steps": marks, "measured_half_period": per_half,
        "jeffery_half_period_nominal": jeffery_period(r, shear_rate) / 2,
        "ratio_to_nominal": per_half / (jeffery_period(r, shear_rate) / 2),
    }
    log(json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jeffery", action="store_true")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nodes", type=int, default=642)
    ap.add_argument("--u-top", type=float, default=0.05)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--half-turns", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=200)
    args = ap.parse_args()
    if args.jeffery:
        jeffery(n=args.n, nodes=args.nodes, u_top=args.u_top, tau=args.tau, half_turns=args.half_turns,
                chunk=args.chunk)


if __name__ == "__main__":
    main()
