"""Jeffery-orbit workload (section 4.1): one oblate platelet tumbling in the middle of a
shear channel, run on the GPU through the C ABI, its rotation period against Jeffery's
rigid-spheroid period T = 2 pi (r + 1/r) / shear_rate (Jeffery 1922; the paper states no
formula).

The platelet's symmetry axis is the short axis of the gyration tensor of its nodes.  Shear
u_x(y) turns it in the x-y plane (vorticity along z).  The axis is a director, so its angle
advances by pi in half a period; the run stops after `half_turns` such advances and reports
the mean time per half turn.

    python -m paper_1312_2234_amd.experiments --jeffery [--n 64] [--nodes 642] [--u-top 0.05]

The effective thickness of the immersed interface is measured on its own: the drag of a
tethered IB sphere in a periodic box gives the radius of the rigid sphere with the same drag
(`hydrodynamic_radius`, `--radius`).

    python -m paper_1312_2234_amd.experiments --radius [--n 96]
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


def periodic_array_drag_factor(c: float) -> float:
    """Drag of a sphere in a simple cubic array at volume fraction c relative to Stokes' drag
    (Hasimoto 1959; Sangani & Acrivos 1982): 1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2)."""
    return 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)


def hydrodynamic_radius(radius=6.0, nodes=2562, n=96, tau=1.0, g=2e-8, k_tether=0.05, chunk=1000,
                        max_steps=40000, tol=2e-4, device="cuda:0", log=print):
    """Effective radius of an immersed-boundary sphere mesh, from its drag: the sphere is held by
    tethers at the centre of a periodic n^3 box whose fluid a body force g along x accelerates.
    The mean flow U (over the box; the enclosed fluid stays with the shell) takes ~n^3/(6 pi mu a)
    steps to settle, but the flow around the sphere follows it within a few box diffusion times,
    so the drag is quasi-steady: the tethers' total force F(t) = 6 pi mu a U(t) K(4/3 pi a^3 / n^3)
    (Hasimoto's K for a periodic array) gives the radius a of the rigid sphere with that drag
    (fixed-point iteration) at every sample.  The run stops when a changes by less than `tol`
    between samples.  Returns the measured radius and the steps run."""
    import torch

    from . import lbm

    rng = np.random.default_rng(0)
    c0 = (n - 1) / 2.0
    b = inputs.tethered_sphere(rng, (c0, c0, c0), radius, nodes, k_tether, 0.0)
    ch = inputs.Channel(n, n, n, tau, body=(g, 0.0, 0.0), walls=False, bodies=b)
    lat = lbm.Lattice([ch], kernel="cos", max_nodes=b.n, device=device)
    lat.init()
    lat.set_nodes(b.n)
    mem = lbm.Membrane(b, device=device)
    X = torch.from_numpy(b.X.copy()).to(device)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=device)
    U = torch.zeros_like(F)
    mu = (tau - 0.5) / 3.0
    steps, prev, a, Um, Fx = 0, None, float("nan"), float("nan"), float("nan")
    while steps < max_steps:
        lat.coupled_steps(mem, chunk, X, F, U)
        steps += chunk
        _, v = lat.moments_channel(0)
        Um = float(v[0].double().mean().item())
        Fx = -float(F[0].double().sum().item())  # the tethers hold the sphere against the flow
        a = radius
        for _ in range(50):
            c = 4.0 / 3.0 * math.pi * a ** 3 / n ** 3
            a = Fx / (6.0 * math.pi * mu * Um * periodic_array_drag_factor(c))
        if prev is not None and abs(a - prev) <= tol * a:
            break
        prev = a
    res = {"radius": radius, "nodes": nodes, "box": n, "tau": tau, "steps": steps, "mean_velocity": Um,
           "tether_force": Fx, "reynolds": Um * 2 * radius / mu, "hydrodynamic_radius": a, "delta": a - radius,
           "flags": lat.error_flags()}
    log(json.dumps(res))
    return res


def rotational_radius(radius=6.0, nodes=2562, n=96, tau=1.0, u_top=0.05, k_tether=0.05, chunk=1000,
                      max_steps=30000, tol=2e-4, device="cuda:0", log=print):
    """Effective radius of an immersed-boundary sphere mesh for rotation: the sphere is held by
    tethers at the centre of an n^3 shear channel started on its linear profile (shear rate
    g = u_top / n).  The fluid turns at -g/2 about z; the torque on a sphere that does not turn is
    4 pi mu a^3 g (Stokes), read off the tethers: T_z = -sum (X - c) x F.  Solved for a; the run
    stops when a changes by less than `tol` between samples."""
    import torch

    from . import lbm

    rng = np.random.default_rng(0)
    c0 = (n - 1) / 2.0
    b = inputs.tethered_sphere(rng, (c0, c0, c0), radius, nodes, k_tether, 0.0)
    ch = inputs.Channel(n, n, n, tau, u_wall_hi=(u_top, 0.0, 0.0), init="shear", bodies=b)
    lat = lbm.Lattice([ch], kernel="cos", max_nodes=b.n, device=device)
    lat.init()
    lat.set_nodes(b.n)
    mem = lbm.Membrane(b, device=device)
    X = torch.from_numpy(b.X.copy()).to(device)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=device)
    U = torch.zeros_like(F)
    mu = (tau - 0.5) / 3.0
    g = u_top / n  # halfway walls at y = -1/2 and n - 1/2
    steps, prev, a, Tz = 0, None, float("nan"), float("nan")
    while steps < max_steps:
        lat.coupled_steps(mem, chunk, X, F, U)
        steps += chunk
        Xn = X.double().cpu().numpy()
        Fn = F.double().cpu().numpy()
        d = Xn - Xn.mean(axis=1, keepdims=True)
        Tz = -float(np.sum(d[0] * Fn[1] - d[1] * Fn[0]))  # torque of the fluid on the sphere
        a = (abs(Tz) / (4.0 * math.pi * mu * g)) ** (1.0 / 3.0)
        if prev is not None and abs(a - prev) <= tol * a:
            break
        prev = a
    res = {"radius": radius, "nodes": nodes, "box": n, "tau": tau, "shear_rate": g, "steps": steps, "torque": Tz,
           "rotational_radius": a, "delta": a - radius, "flags": lat.error_flags()}
    log(json.dumps(res))
    return res


def jeffery_ratio_with_thickness(semi_axes=(6.0, 2.0, 6.0), delta=0.0) -> float:
    """Jeffery half-period of the spheroid thickened by delta on every side, relative to the
    nominal one (only the aspect ratio enters)."""
    r0 = semi_axes[1] / semi_axes[0]
    r = (semi_axes[1] + delta) / (semi_axes[0] + delta)
    return (r + 1.0 / r) / (r0 + 1.0 / r0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jeffery", action="store_true")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nodes", type=int, default=642)
    ap.add_argument("--u-top", type=float, default=0.05)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--half-turns", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--radius", action="store_true", help="effective radius of an IB sphere from its drag")
    args = ap.parse_args()
    if args.radius:
        hydrodynamic_radius(n=args.n)
        rotational_radius(n=args.n)
    if args.jeffery:
        jeffery(n=args.n, nodes=args.nodes, u_top=args.u_top, tau=args.tau, half_turns=args.half_turns,
                chunk=args.chunk)


if __name__ == "__main__":
    main()
