"""Parity at the benchmark's full sizes, in the launch configuration the benchmark times
(launch shape from the tuned cache, steps replayed from a 2-step HIP graph), against the
FP64 oracle on every cell: the 256x128x128 shear channel with 16 platelets of 2562 nodes
(with halfway walls, with the on-site walls of Eq. 23-30, with the area and volume
constraints of Eq. 4-5 at Table 2's coefficients, and with the FE bending of Eq. 6-10 at Table 2's
modulus in place of the dihedral stand-in) over 100 coupled steps, and the 64-channel
batch (18.2 M cells, 0.50 M nodes) over 20.  Tolerances as in test_gpu_parity: velocity
e_max <= 1e-5, interpolated velocities likewise, wall stress 1e-4."""
import dataclasses

import numpy as np
import pytest

from paper_1312_2234_amd import inputs
from test_gpu_parity import DEV, N, T, TOL32, emax, run_oracle_coupled

pytestmark = pytest.mark.gpu


def gpu_bench_config(gpu, channels, steps):
    """The benchmark's launch configuration: tuned launch shape, schedule and binning interval,
    graph replay (the steps beyond a multiple of the graph's length eagerly)."""
    import torch

    from paper_1312_2234_amd import tune

    b, offs = inputs.concat_bodies(channels)
    g = gpu.Lattice(channels, kernel="cos", max_nodes=b.n, device=DEV)
    g.init()
    g.set_nodes(b.n, offs if len(channels) > 1 else None)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    tune.apply_cached_or_tune(g, coupled=(mem, X, F, U))
    g.init()
    X.copy_(T(b.X))
    G = tune.graph_steps(g.get_launch())
    g.graph_capture(mem, G, X, F, U)
    g.graph_launch(steps // G)
    if steps % G:
        g.coupled_steps(mem, steps % G, X, F, U)
    torch.cuda.synchronize()
    return g, N(X), N(U), offs


def shear_workload(variant):
    ch = inputs.shear_platelets(seed=0)
    if variant == "onsite":
        ch = dataclasses.replace(ch, walls="onsite")
    if variant == "constrained":
        ch = dataclasses.replace(ch, bodies=inputs.with_constraints(ch.bodies, *inputs.table2_constraint_coefficients()))
    if variant == "fe_bending":
        ch = dataclasses.replace(ch, bodies=inputs.with_fe_bending(ch.bodies, inputs.table2_bending_modulus()))
    return ch


@pytest.mark.parametrize("variant", ["halfway", "onsite", "constrained", "fe_bending"])
def test_full_shear_workload_against_oracle(orc, gpu, variant):
    ch = shear_workload(variant)
    steps = 100
    g, Xg, Ug, _ = gpu_bench_config(gpu, [ch], steps)
    o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", steps)
    drho, v = g.moments_channel(0)
    e = emax(N(v), o.moments()[1])
    eu = emax(Ug, Uo)
    print("full shear (%s), %d steps: velocity e_max %.3e, node velocity %.3e" % (variant, steps, e, eu))
    assert e <= TOL32 and eu <= TOL32
    assert np.abs(Xg - Xo).max() <= TOL32 * np.abs(Uo).max() * steps
    lo_g, _ = g.wall_stress()
    lo_o, _ = o.wall_stress()
    assert emax(N(lo_g).reshape(lo_o.shape), lo_o) <= 1e-4
    assert g.error_flags() == 0


def test_full_batched_workload_against_oracle(orc, gpu):
    chans = inputs.batched_channels(seed=0)
    steps = 20
    g, Xg, Ug, offs = gpu_bench_config(gpu, chans, steps)
    worst = 0.0
    for c, ch in enumerate(chans):
        o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", steps)
        _, v = g.moments_channel(c)
        e = emax(N(v), o.moments()[1])
        eu = emax(Ug[:, offs[c]:offs[c + 1]], Uo)
        worst = max(worst, e, eu)
        assert e <= TOL32 and eu <= TOL32, "channel %d" % c
    print("full batch (%d channels), %d steps: worst e_max %.3e" % (len(chans), steps, worst))
    assert g.error_flags() == 0
