"""On-site velocity walls (Eq. 23-30 turned to a y-normal wall, lbm_params.walls = 2) on the
GPU, through the C ABI, against the FP64 oracle and against closed forms.

Same bar as the halfway-wall parity tests: float32 velocities within e_max <= 1e-5 of the
oracle, populations within a few float32 ulps, launch shapes and coupled-step schedules
bitwise equal to each other.  Sizes are ragged (not multiples of the 64-cell segment or the
8-cell tile) and platelets sit near the lower wall, so IB stencils reach the wall rows.
"""
import dataclasses
import types

import numpy as np
import pytest

from paper_1312_2234_amd import inputs
from test_gpu_parity import DEV, TOL32, N, T, emax, gpu_fields, pair, run_gpu_coupled, run_oracle_coupled

pytestmark = pytest.mark.gpu


def onsite(ch):
    return dataclasses.replace(ch, walls="onsite")


def channel(dims, **kw):
    d = dict(tau=0.8, body=(1e-5, 0.0, 2e-6), u_wall_lo=(0.01, 0.0, -0.02), u_wall_hi=(0.05, 0.0, 0.01),
             init="shear", walls="onsite")
    d.update(kw)
    return inputs.Channel(*dims, **d)


def platelet_near_wall(seed=31, nx=48, ny=24, nz=40):
    """One 642-node platelet whose lower stencil rows reach the wall row y = 0."""
    ch = inputs.shear_platelets(seed=seed, nx=nx, ny=ny, nz=nz, count=1, nodes=642, tau=0.9, u_top=0.03,
                                y_band=(3.5, 4.5))
    y = ch.bodies.X[1]
    assert y.min() - 1 < 1.0  # the 4-wide stencil of the lowest node covers row 0
    return onsite(ch)


@pytest.mark.parametrize("dims", [(45, 21, 29), (48, 20, 16)])
def test_onsite_lattice_matches_oracle(orc, gpu, dims):
    ch = channel(dims)
    o, g = pair(orc, gpu, ch)
    assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32  # on-site shear start pulls back to f_eq
    o.step(150)
    g.step(150)
    rho_o, v_o = o.moments()
    drho_g, v_g = gpu_fields(g)
    assert emax(v_g, v_o) <= TOL32
    assert np.abs(drho_g - (rho_o - 1)).max() < 1e-6
    # the wall rows move with their walls (float32 rounding only)
    v_g = v_g.reshape(3, dims[2], dims[1], dims[0])
    assert np.abs(v_g[:, :, 0, :] - np.array(ch.u_wall_lo)[:, None, None]).max() < 1e-6
    assert np.abs(v_g[:, :, -1, :] - np.array(ch.u_wall_hi)[:, None, None]).max() < 1e-6
    lo_g, hi_g = g.wall_stress()
    lo_o, hi_o = o.wall_stress()
    assert emax(N(lo_g).reshape(lo_o.shape), lo_o) <= 1e-4
    assert emax(N(hi_g).reshape(hi_o.shape), hi_o) <= 1e-4


def test_onsite_poiseuille_closed_form(gpu):
    """Steady body-force channel with walls on the rows: u_x = g/(2 nu) y (H - y), H = ny - 1,
    at every tau (no slip term), from the GPU alone."""
    ny, gx, tau = 12, 1e-5, 0.8
    nu = (tau - 0.5) / 3
    ch = inputs.Channel(8, ny, 8, tau, body=(gx, 0.0, 0.0), walls="onsite")
    g = gpu.Lattice([ch], device=DEV)
    g.init()
    g.step(int(60 * ny * ny / nu))
    v = gpu_fields(g)[1].reshape(3, 8, ny, 8)
    y = np.arange(ny)
    ex = gx / (2 * nu) * y * (ny - 1 - y)
    assert np.abs(v[0] - ex[None, :, None]).max() <= TOL32 * ex.max()
    assert np.abs(v[1:]).max() <= TOL32 * ex.max()


def test_onsite_populations_roundtrip(orc, gpu):
    ch = channel((33, 20, 17))
    o, g = pair(orc, gpu, ch)
    o.step(7)
    g.step(7)
    ref = o.populations()  # wall rows' entering populations set by Eq. (23)-(30)
    f_g = N(g.populations()).reshape(ref.shape)
    ulp = 2.0 ** -25
    assert np.abs(f_g - ref).max() < 4 * ulp
    # the stored placeholders of the entering populations are ignored on the way in
    g.set_populations(T(o.f.reshape(-1), np.float32))
    assert np.abs(N(g.populations()).reshape(ref.shape) - ref).max() < 4 * ulp


def test_onsite_coupled_platelet_near_wall(orc, gpu):
    ch = platelet_near_wall()
    o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", 20)
    g, Xg, Ug = run_gpu_coupled(gpu, ch, "cos", 20)
    assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32
    assert emax(N(Ug), Uo) <= TOL32
    assert np.abs(N(Xg) - Xo).max() <= TOL32 * np.abs(Xo - ch.bodies.X).max()
    lo_g, _ = g.wall_stress()
    lo_o, _ = o.wall_stress()
    assert emax(N(lo_g).reshape(lo_o.shape), lo_o) <= 1e-4
    assert g.error_flags() == 0


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_onsite_coupled_schedules_bitwise(gpu, storage):
    """Split (body-force update + flagged-tile update), fused and overlapped schedules of the
    coupled step give bitwise the same state with on-site walls."""
    import torch

    ch = platelet_near_wall(seed=32, nx=40, ny=22, nz=36)
    b = ch.bodies
    out = []
    for launch in (dict(split=1), dict(split=0), dict(overlap=1)):
        g = gpu.Lattice([ch], storage=storage, kernel="cos", max_nodes=b.n, device=DEV)
        g.set_launch(**launch)
        g.init()
        g.set_nodes(b.n)
        mem = gpu.Membrane(b, device=DEV)
        X = T(b.X)
        F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
        U = torch.zeros_like(F)
        g.coupled_steps(mem, 12, X, F, U)
        torch.cuda.synchronize()
        out.append((N(g.get_state()), N(X), N(U)))
    for st, X, U in out[1:]:
        assert np.array_equal(st, out[0][0]) and np.array_equal(X, out[0][1]) and np.array_equal(U, out[0][2])


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_onsite_launch_shapes_bitwise(gpu, storage):
    """Scalar and vector steps, persistent and XCD-remapped grids agree bitwise with on-site
    walls and an IB force field that reaches the wall rows."""
    rng = np.random.default_rng(41)
    ch = channel((48, 20, 16))
    X = np.stack([rng.uniform(0, 48, 300), rng.uniform(-0.5, 19.5, 300), rng.uniform(0, 16, 300)])
    F = 1e-3 * rng.standard_normal((3, 300))
    out = []
    for launch in (dict(), dict(vec=2), dict(vec=4, nontemporal=1), dict(block=64, persistent=37),
                   dict(block=1024, xcd_remap=1)):
        g = gpu.Lattice([ch], storage=storage, max_nodes=300, device=DEV)
        g.set_launch(**launch)
        g.init()
        g.set_nodes(300)
        g.spread(T(X), T(F, np.float32))
        g.step(12)
        out.append(N(g.populations()))
    for o in out[1:]:
        assert np.array_equal(o, out[0])


@pytest.mark.parametrize("storage,bound", [("f16", 5e-3), ("bf16", 5e-2)])
def test_onsite_half_storage_error_bounded(orc, gpu, storage, bound):
    """16-bit storage with on-site walls against the FP64 oracle (both walls moving in x and z,
    body force): reported, with the same loose bounds as the halfway-wall storage report; it
    catches a broken wall rule in the 16-bit paths, the float32 tests carry parity."""
    ch = channel((40, 24, 20), body=(1e-6, 0.0, 0.0))
    o, g = pair(orc, gpu, ch, storage=storage)
    o.step(100)
    g.step(100)
    e = emax(gpu_fields(g)[1], o.moments()[1])
    print("%s on-site e_max %.3e" % (storage, e))
    assert e <= bound


def test_onsite_closure_matches_oracle(orc, gpu):
    """Learned-closure step with on-site walls against the closure oracle (whose features are
    taken from the completed wall-row populations), 10 steps, e_max <= 1e-4 as for halfway
    walls; a zero last layer is bitwise the plain step."""
    import oracle.closure_oracle as co
    from test_gpu_closure import norm_for, theta_bf16

    ch = inputs.Channel(40, 24, 20, 0.75, body=(2e-6, 0, 0), u_wall_hi=(0.04, 0, 0.01), walls="onsite")
    rng = np.random.default_rng(5)
    o = orc.Lattice(ch.nx, ch.ny, ch.nz, ch.tau, walls="onsite", body=ch.body, u_wall_hi=ch.u_wall_hi)
    o.init(u=rng.normal(0, 0.02, (3, ch.nz, ch.ny, ch.nx)))
    o.step(6)
    o.f[...] = o.f.astype(np.float32).astype(np.float64)
    # feature scaling from the populations the step reads (the stored wall-row placeholders
    # of the entering populations are not part of the state)
    nrm, flat = norm_for(types.SimpleNamespace(f=o.populations(), g=o.g, p=o.p), 0.2)

    def fresh():
        g = gpu.Lattice([ch], device=DEV)
        g.set_populations(T(o.f.reshape(-1), np.float32))
        return g

    a, b = fresh(), fresh()
    b.set_closure(T(theta_bf16(np.random.default_rng(6), zero_last=True), np.float32), T(flat, np.float32), 1.0)
    a.step(3)
    b.step(3)
    assert np.array_equal(N(a.get_state()), N(b.get_state()))

    th = theta_bf16(np.random.default_rng(7))
    g = fresh()
    g.set_closure(T(th, np.float32), T(flat, np.float32), 1e30)
    for _ in range(10):
        co.closure_step(o, th, nrm, c_guard=1e30, bf16=True)
    g.step(10)
    _, v = g.moments_channel(0)
    _, vr = o.moments()
    e = np.abs(N(v) - vr).max() / np.abs(vr).max()
    print("10 on-site closure steps: e_max %.3e" % e)
    assert e <= 1e-4
    assert g.error_flags() == 0


def test_onsite_rejected_where_unsupported(gpu):
    import paper_1312_2234_amd.lbm as L

    with pytest.raises(L.LbmError):  # two wall rows need a fluid row between them
        gpu.Lattice([inputs.Channel(8, 2, 8, 0.8, walls="onsite")], device=DEV)
    g = gpu.Lattice([channel((16, 8, 8))], device=DEV)
    g.init()
    with pytest.raises(L.LbmError):  # 2x2x2 restriction blocks align with halfway walls only
        g.restrict(0.75)
    import torch

    z = torch.zeros((19, 4 * 4 * 4), dtype=torch.float32, device=DEV)
    with pytest.raises(L.LbmError):
        L.closure_targets(inputs.Channel(4, 4, 4, 0.75, walls="onsite"), z, z[:3].contiguous(), z)
