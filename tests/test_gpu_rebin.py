"""Binning every `rebin` coupled steps with a half-cell margin (lbm_launch.rebin): the spread sums
exact integers over each tile's cells, so a superset of listed nodes changes nothing and the
results must be bitwise those of binning every step, in both coupled-step schedules, with the
FE bending and the constraints, in eager and graph-replayed runs; a node moved beyond the
margin between binnings is reported (LBM_FLAG_REBIN_MARGIN)."""
import dataclasses

import numpy as np
import pytest

from paper_1312_2234_amd import inputs
from test_gpu_parity import DEV, N, T

pytestmark = pytest.mark.gpu


def channel(seed=3, nodes=642, count=2, fe=False, cons=False):
    ch = inputs.shear_platelets(seed=seed, nx=64, ny=48, nz=48, count=count, nodes=nodes, y_band=(8.0, 14.0))
    b = ch.bodies
    if fe:
        b = inputs.with_fe_bending(b, inputs.table2_bending_modulus())
    if cons:
        b = inputs.with_constraints(b, 0.05, 0.02, 0.1)
    return dataclasses.replace(ch, bodies=b)


def run(gpu, ch, steps, rebin, split, graph=False):
    import torch

    b = ch.bodies
    g = gpu.Lattice([ch], kernel="cos", max_nodes=b.n, device=DEV)
    g.set_launch(block=256, xcd_remap=1, nontemporal=1, split=split, rebin=rebin)
    g.init()
    g.set_nodes(b.n)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    if graph:
        G = 2 * rebin
        g.graph_capture(mem, G, X, F, U)
        g.graph_launch(steps // G)
        if steps % G:
            g.coupled_steps(mem, steps % G, X, F, U)
    else:
        g.coupled_steps(mem, steps, X, F, U)
    torch.cuda.synchronize()
    return g, N(X), N(U), N(g.get_state())


@pytest.mark.parametrize("split", [1, 0])
@pytest.mark.parametrize("rebin", [2, 4, 8])
def test_rebin_is_bitwise_binning_every_step(gpu, split, rebin):
    ch = channel()
    g1, X1, U1, S1 = run(gpu, ch, 36, 1, split)
    g2, X2, U2, S2 = run(gpu, ch, 36, rebin, split)
    assert np.array_equal(X1, X2) and np.array_equal(U1, U2) and np.array_equal(S1, S2)
    assert g1.error_flags() == 0 and g2.error_flags() == 0


def test_rebin_with_fe_bending_and_constraints(gpu):
    ch = channel(seed=5, fe=True, cons=True)
    g1, X1, U1, S1 = run(gpu, ch, 24, 1, 1)
    g2, X2, U2, S2 = run(gpu, ch, 24, 4, 1)
    assert np.array_equal(X1, X2) and np.array_equal(U1, U2) and np.array_equal(S1, S2)
    assert g2.error_flags() == 0


def test_rebin_graph_replay_equals_eager(gpu):
    ch = channel(seed=7)
    g1, X1, U1, S1 = run(gpu, ch, 35, 4, 1)
    g2, X2, U2, S2 = run(gpu, ch, 35, 4, 1, graph=True)
    assert np.array_equal(X1, X2) and np.array_equal(U1, U2) and np.array_equal(S1, S2)
    # a capture must hold a multiple of 2 rebin steps
    import torch

    b = ch.bodies
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    with pytest.raises(gpu.LbmError):
        g2.graph_capture(mem, 4, X, F, torch.zeros_like(F))


def test_node_moved_beyond_the_margin_is_reported(gpu):
    """The caller shifts the nodes by a whole cell between binnings (without telling the context):
    the next step between binnings reports it."""
    import torch

    ch = channel(seed=9, count=1)
    b = ch.bodies
    g = gpu.Lattice([ch], kernel="cos", max_nodes=b.n, device=DEV)
    g.set_launch(block=256, xcd_remap=1, nontemporal=1, split=1, rebin=4)
    g.init()
    g.set_nodes(b.n)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    g.coupled_steps(mem, 2, X, F, U)
    assert g.error_flags() == 0
    X[0] += 1.0
    g.coupled_steps(mem, 1, X, F, U)
    assert g.error_flags() & gpu.FLAG_REBIN_MARGIN
    # declaring the nodes again makes the next step bin afresh
    g.set_nodes(b.n)
    g.coupled_steps(mem, 3, X, F, U)
    assert g.error_flags() == 0
