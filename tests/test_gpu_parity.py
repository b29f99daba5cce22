"""GPU (gfx950 HIP, through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerance for float32 (weight-shifted storage, float32 arithmetic): the maximum relative
velocity error e_max = max|v_gpu - v_ref| / max|v_ref| <= 1e-5; positions and
interpolated velocities likewise relative to their own scale.  Lattice sizes include
ragged ones (not multiples of the 64-cell segment or the 8-cell IB tile).
"""
import numpy as np
import pytest

from paper_1312_2234_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL32 = 1e-5


def emax(a, ref):
    a, ref = np.asarray(a, float), np.asarray(ref, float)
    return np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300)


def T(x, dtype=None):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def N(t):
    return t.detach().cpu().numpy()


def pair(orc, gpu, ch, kernel="cos", storage="f32", max_nodes=0):
    o = orc.Lattice(ch.nx, ch.ny, ch.nz, ch.tau, walls=ch.walls, body=ch.body, u_wall_lo=ch.u_wall_lo,
                    u_wall_hi=ch.u_wall_hi, kernel=kernel)
    g = gpu.Lattice([ch], storage=storage, kernel=kernel, max_nodes=max_nodes, device=DEV)
    if ch.init == "shear":
        o.init(u=o.shear_profile())
    else:
        o.init()
    g.init()
    return o, g


def gpu_fields(g, c=0):
    drho, v = g.moments_channel(c)
    return N(drho), N(v)


# ----------------------------------------------------------------------------- lattice only
@pytest.mark.parametrize("dims", [(32, 32, 32), (45, 37, 29)])
def test_lbm_poiseuille_box(orc, gpu, dims):
    ch = inputs.Channel(*dims, 0.8, body=(1e-6, 0.0, 0.0))
    o, g = pair(orc, gpu, ch)
    o.step(100)
    g.step(100)
    rho_o, v_o = o.moments()
    drho_g, v_g = gpu_fields(g)
    assert emax(v_g, v_o) <= TOL32
    assert np.abs(drho_g - (rho_o - 1)).max() < 1e-9


def test_lbm_couette_shear_init(orc, gpu):
    ch = inputs.Channel(40, 24, 16, 1.0, u_wall_hi=(0.05, 0.0, 0.02), u_wall_lo=(-0.01, 0.0, 0.0), init="shear")
    o, g = pair(orc, gpu, ch)
    _, v0 = gpu_fields(g)
    _, vo0 = o.moments()
    assert emax(v0, vo0) <= TOL32      # the un-streamed initial state pulls back to f_eq(u0)
    o.step(200)
    g.step(200)
    assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32
    lo_g, hi_g = g.wall_stress()
    lo_o, hi_o = o.wall_stress()
    assert emax(N(lo_g).reshape(lo_o.shape), lo_o) <= 1e-4
    assert emax(N(hi_g).reshape(hi_o.shape), hi_o) <= 1e-4


def test_lbm_periodic_random_velocity(orc, gpu):
    rng = np.random.default_rng(11)
    ch = inputs.Channel(24, 20, 18, 0.7, walls=False, body=(1e-5, -2e-6, 0.0))
    o, g = pair(orc, gpu, ch)
    u = 0.02 * rng.standard_normal((3, 18, 20, 24))
    rho = 1 + 0.01 * rng.standard_normal((18, 20, 24))
    o.init(rho=rho, u=u)
    g.init(rho=T(rho.reshape(-1), np.float32), u=T(u.reshape(-1), np.float32))
    o.step(50)
    g.step(50)
    rho_o, v_o = o.moments()
    drho_g, v_g = gpu_fields(g)
    assert emax(v_g, v_o) <= TOL32
    assert np.abs(drho_g - (rho_o - 1)).max() < 1e-6   # input rho rounded to float32


def test_mass_conservation_float32(gpu):
    """Mass changes only by float32 rounding of the stored populations: at most 19 half-ulps
    of max|g| (~1e-2 here) per cell and step.  A mass source such as the '+ c_s^2 I' reading of
    Eq. (19) would add 6 (1 - 1/2tau) v.F per cell and step, ~10x more than this bound."""
    ch = inputs.Channel(64, 48, 40, 0.9, u_wall_hi=(0.05, 0, 0), init="shear", body=(1e-6, 0, 0))
    g = gpu.Lattice([ch], device=DEV)
    g.init()
    m0 = float(N(g.moments()[0]).astype(np.float64).sum())
    steps = 300
    g.step(steps)
    m1 = float(N(g.moments()[0]).astype(np.float64).sum())
    bound = 19 * 2.0 ** -24 * 1e-2 * ch.cells * steps
    print("mass drift %.3e (bound %.3e)" % (m1 - m0, bound))
    assert abs(m1 - m0) < bound


# ----------------------------------------------------------------------------- IB in isolation
@pytest.mark.parametrize("kernel", ["cos", "peskin4"])
@pytest.mark.parametrize("dims", [(32, 32, 32), (45, 37, 29)])
def test_spread_matches_oracle(orc, gpu, kernel, dims):
    """At rest with no body force v = g/2, so the moments expose the spread force field."""
    rng = np.random.default_rng(12)
    nx, ny, nz = dims
    ch = inputs.Channel(nx, ny, nz, 0.8)
    o, g = pair(orc, gpu, ch, kernel=kernel, max_nodes=500)
    n = 500
    X = np.stack([rng.uniform(-3, nx + 3, n), rng.uniform(-0.5, ny - 0.5, n), rng.uniform(-3, nz + 3, n)])
    X[:, :40] = np.round(X[:, :40])      # nodes exactly on lattice points
    F = 1e-3 * rng.standard_normal((3, n))
    F32 = F.astype(np.float32)
    o.spread(X, F32.astype(np.float64))
    g.set_nodes(n)
    g.spread(T(X), T(F32))
    _, v_g = gpu_fields(g)
    assert emax(2 * v_g, o.g) <= 2e-6
    assert g.error_flags() == 0


@pytest.mark.parametrize("kernel", ["cos", "peskin4"])
def test_interp_matches_oracle(orc, gpu, kernel):
    rng = np.random.default_rng(13)
    nx, ny, nz = 45, 37, 29
    ch = inputs.Channel(nx, ny, nz, 0.8, u_wall_lo=(0.01, 0, 0), u_wall_hi=(-0.02, 0, 0.03))
    o, g = pair(orc, gpu, ch, kernel=kernel, max_nodes=400)
    u = 0.01 * rng.standard_normal((3, nz, ny, nx))
    o.init(u=u)
    g.init(u=T(u.reshape(-1), np.float32))
    n = 400
    X = np.stack([rng.uniform(0, nx, n), rng.uniform(-0.5, ny - 0.5, n), rng.uniform(0, nz, n)])
    F = np.zeros((3, n), np.float32)
    o.spread(X, F.astype(np.float64))
    g.set_nodes(n)
    g.spread(T(X), T(F))
    U_o = o.interp(X)
    U_g = N(g.interp(T(X)))
    assert emax(U_g, U_o) <= TOL32
    # nodes that moved off the spread footprint are evaluated on the fly
    X2 = X.copy()
    X2[0] += 7.3
    U2_o = o.interp(X2)
    U2_g = N(g.interp(T(X2)))
    assert emax(U2_g, U2_o) <= TOL32


def test_spread_is_deterministic_and_empty_ok(gpu):
    rng = np.random.default_rng(14)
    ch = inputs.Channel(64, 40, 48, 0.8)
    g = gpu.Lattice([ch], max_nodes=20000, device=DEV)
    g.init()
    n = 20000
    X = T(np.stack([rng.uniform(0, 64, n), rng.uniform(0, 39, n), rng.uniform(0, 48, n)]))
    F = T(rng.standard_normal((3, n)), np.float32)
    g.set_nodes(n)
    g.spread(X, F)
    a = N(g.moments()[1])
    g.spread(X, F)
    b = N(g.moments()[1])
    assert np.array_equal(a, b)
    g.set_nodes(0)
    g.spread(None, None)
    _, v = g.moments()
    assert float(N(v).__abs__().max()) == 0.0


def tile_pairs(X, dims, walls):
    """Node-tile pairs of the 8^3 tiles the 4^3 stencils touch (rows inside a wall dropped)."""
    tot = np.ones(X.shape[1], np.int64)
    for d, n in enumerate(dims):
        cells = np.floor(X[d]).astype(np.int64)[:, None] - 1 + np.arange(4)[None, :]
        if d == 1 and walls:
            cells = np.where((cells >= 0) & (cells < n), cells, -1)
            t = np.where(cells >= 0, cells // 8, -1)
            first = np.max(np.where(t >= 0, t, -1), axis=1)
            lo = np.min(np.where(t >= 0, t, 1 << 30), axis=1)
            tot *= np.where(first < 0, 0, first - lo + 1)
        else:
            t = (cells % n) // 8
            tot *= 1 + (t[:, 3] != t[:, 0])
    return int(tot.sum())


def test_spread_partial_capacity_exhausted(orc, gpu):
    """More 256-entry chunks than partial force blocks (16384): the tiles beyond the capacity are
    spread by a single work item over their whole list.  Both kinds must agree with the oracle."""
    rng = np.random.default_rng(15)
    dims = (64, 48, 64)
    ch = inputs.Channel(*dims, 0.8)
    n = 2_000_000
    X = np.stack([rng.uniform(0, 64, n), rng.uniform(-0.5, 47.5, n), rng.uniform(0, 64, n)])
    pairs = tile_pairs(X, dims, True)
    assert pairs / 256 > 1.1 * 16384, pairs      # the capacity is exceeded
    F32 = (1e-3 * rng.standard_normal((3, n))).astype(np.float32)
    o, g = pair(orc, gpu, ch, max_nodes=n)
    o.spread(X, F32.astype(np.float64))
    g.set_nodes(n)
    g.spread(T(X), T(F32))
    _, v_g = gpu_fields(g)
    e = emax(2 * v_g, o.g)
    print("%d nodes, %d node-tile pairs: e_max %.3e" % (n, pairs, e))
    assert e <= 2e-6
    assert g.error_flags() == 0


def test_spread_full_batch_of_coincident_nodes(orc, gpu):
    """256 nodes on one lattice point (a whole staged batch on one cell, weight 1/8 there), each
    with the largest force below a power of two: at the scale of that power of two every
    contribution would round to 2^23 and the 32-bit batch sum would wrap; the scale must keep
    the sum below 2^31."""
    ch = inputs.Channel(16, 16, 16, 0.8)
    n = 256
    X = np.tile(np.array([[5.0], [6.0], [7.0]]), (1, n))
    F32 = np.zeros((3, n), np.float32)
    F32[0] = np.nextafter(np.float32(1.0), np.float32(0.0))
    F32[1] = -F32[0]
    F32[2] = np.float32(0.5)
    o, g = pair(orc, gpu, ch, max_nodes=n)
    o.spread(X, F32.astype(np.float64))
    g.set_nodes(n)
    g.spread(T(X), T(F32))
    _, v_g = gpu_fields(g)
    assert abs(o.g[0, 7, 6, 5] - 32 * float(F32[0, 0])) < 1e-12
    assert emax(2 * v_g, o.g) <= 2e-6
    assert g.error_flags() == 0


def _scattered_nodes(rng, n, dims):
    nx, ny, nz = dims
    return np.stack([rng.uniform(0, nx, n), rng.uniform(-0.5, ny - 0.5, n), rng.uniform(0, nz, n)])


def test_spread_scattered_nodes_fill_the_bin_hash(orc, gpu):
    """4096 nodes scattered over the 256x128x128 lattice: a block of 256 nodes touches ~670
    distinct tiles, more than its 512-entry LDS table, so the binning's direct-count branch
    runs; the field must still match the oracle."""
    rng = np.random.default_rng(16)
    dims = (256, 128, 128)
    n = 4096
    X = _scattered_nodes(rng, n, dims)
    blocks = [X[:, k:k + 256] for k in range(0, n, 256)]
    distinct = [len({tuple(t) for t in _node_tiles(B, dims)}) for B in blocks]
    assert min(distinct) > 512, distinct          # every bin block overflows its table
    F32 = (1e-3 * rng.standard_normal((3, n))).astype(np.float32)
    ch = inputs.Channel(*dims, 0.8)
    o, g = pair(orc, gpu, ch, max_nodes=n)
    o.spread(X, F32.astype(np.float64))
    g.set_nodes(n)
    g.spread(T(X), T(F32))
    _, v_g = gpu_fields(g)
    assert emax(2 * v_g, o.g) <= 2e-6
    assert g.error_flags() == 0


def test_coupled_scattered_tethered_nodes_fill_the_bin_hash(orc, gpu):
    """The coupled step's binning (beside the membrane forces) with 4096 scattered tethered
    nodes on the 256x128x128 shear channel: the direct-count branch of every bin block runs
    in the split schedule; 3 coupled steps against the oracle."""
    rng = np.random.default_rng(17)
    dims = (256, 128, 128)
    n = 4096
    X0 = _scattered_nodes(rng, n, dims)
    X0[1] = np.clip(X0[1], 1.0, dims[1] - 2.0)
    assert min(len(set(_node_tiles(X0[:, k:k + 256], dims))) for k in range(0, n, 256)) > 512
    anchors = X0 + 0.3 * rng.standard_normal(X0.shape)
    anchors[1] = np.clip(anchors[1], 1.0, dims[1] - 2.0)
    bodies = inputs.Bodies(X=X0, X_rest=X0.copy(), edges=np.zeros((0, 2), np.int32), hinges=np.zeros((0, 4), np.int32),
                           anchors=anchors, k_tether=0.01, body_offsets=[0, n])
    ch = inputs.Channel(*dims, 1.0, u_wall_hi=(0.05, 0.0, 0.0), init="shear", bodies=bodies)
    o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", 3)
    g, Xg, Ug = run_gpu_coupled(gpu, ch, "cos", 3)
    assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32
    assert emax(N(Ug), Uo) <= TOL32
    assert g.error_flags() == 0


def _node_tiles(X, dims):
    """(tx, ty, tz) of every 8^3 tile any node's 4^3 stencil touches (walls in y)."""
    out = []
    for m in range(X.shape[1]):
        ax = []
        for d, n in enumerate(dims):
            cells = int(np.floor(X[d, m])) - 1 + np.arange(4)
            if d == 1:
                cells = cells[(cells >= 0) & (cells < n)]
            else:
                cells = cells % n
            ax.append(sorted({int(c) // 8 for c in cells}))
        out += [(a, b, c) for a in ax[0] for b in ax[1] for c in ax[2]]
    return out


def test_error_flags(gpu):
    ch = inputs.Channel(16, 16, 16, 0.8)
    g = gpu.Lattice([ch], max_nodes=2, device=DEV)
    g.init()
    g.set_nodes(2)
    X = T(np.array([[4.0, 5.0], [40.0, 3.0], [4.0, 5.0]]))
    F = T(np.array([[1.0, np.inf], [0, 0], [0, 0]]), np.float32)
    g.spread(X, F)
    fl = g.error_flags()
    assert fl & gpu.FLAG_NODE_OUTSIDE and fl & gpu.FLAG_FORCE_NONFINITE
    assert g.error_flags() == 0


# ----------------------------------------------------------------------------- membrane forces
def test_membrane_forces_match_oracle(orc, gpu):
    rng = np.random.default_rng(15)
    b = inputs.platelets(rng, 64, 48, 64, 2, (6.0, 2.0, 6.0), 2562, (8.0, 20.0), 0.005, 1e-4)
    X = b.X + 0.05 * rng.standard_normal(b.X.shape)
    om = orc.Membrane(b.X_rest, b.edges, k_spring=b.k_spring, hinges=b.hinges, k_bend=b.k_bend)
    gm = gpu.Membrane(b, device=DEV)
    F_o = om.forces(X)
    F_g = N(gm.forces(T(X)))
    assert emax(F_g, F_o) <= 1e-6
    t = inputs.tethered_sphere(rng, (16, 10, 16), 4.0, 642, 0.01, 0.1)
    om = orc.Membrane(t.X_rest, t.edges, anchors=t.anchors, k_tether=t.k_tether)
    gm = gpu.Membrane(t, device=DEV)
    assert emax(N(gm.forces(T(t.X))), om.forces(t.X)) <= 1e-6


# ----------------------------------------------------------------------------- coupled steps
def run_oracle_coupled(orc, ch, kernel, steps):
    b = ch.bodies
    o = orc.Lattice(ch.nx, ch.ny, ch.nz, ch.tau, walls=ch.walls, body=ch.body, u_wall_lo=ch.u_wall_lo,
                    u_wall_hi=ch.u_wall_hi, kernel=kernel)
    o.init(u=o.shear_profile()) if ch.init == "shear" else o.init()
    mem = orc.Membrane(b.X_rest, b.edges, k_spring=b.k_spring, hinges=b.hinges, k_bend=b.k_bend,
                       anchors=b.anchors, k_tether=b.k_tether, triangles=b.triangles,
                       body_tri=b.tri_offsets if b.triangles is not None else None,
                       k_area_global=b.k_area_global, k_area_local=b.k_area_local, k_volume=b.k_volume,
                       elements6=b.elements6, k_fe=b.k_fe)
    X = b.X.copy()
    for _ in range(steps):
        F, U = orc.coupled_step(o, mem, X)
    return o, X, U


def run_gpu_coupled(gpu, ch, kernel, steps, graph=False, storage="f32"):
    import torch

    b = ch.bodies
    g = gpu.Lattice([ch], storage=storage, kernel=kernel, max_nodes=b.n, device=DEV)
    g.init()
    g.set_nodes(b.n)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    if graph:
        g.graph_capture(mem, 2, X, F, U)
        g.graph_launch(steps // 2)
    else:
        g.coupled_steps(mem, steps, X, F, U)
    torch.cuda.synchronize()
    return g, X, U


@pytest.mark.parametrize("kernel", ["peskin4", "cos"])
def test_coupled_poiseuille_sphere_100_steps(orc, gpu, kernel):
    """32^3 box, body force 1e-6, tethered 642-node sphere (k = 0.01, N(0, 0.1^2) start), 100 steps."""
    for seed in range(5):
        ch = inputs.poiseuille_sphere(seed=seed)
        o, Xo, Uo = run_oracle_coupled(orc, ch, kernel, 100)
        g, Xg, Ug = run_gpu_coupled(gpu, ch, kernel, 100)
        assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32
        assert emax(N(Ug), Uo) <= TOL32
        assert np.abs(N(Xg) - Xo).max() <= TOL32 * np.abs(Xo - ch.bodies.X).max()
        assert g.error_flags() == 0


def test_graph_replay_matches_eager(gpu):
    ch = inputs.poiseuille_sphere(seed=2)
    g1, X1, U1 = run_gpu_coupled(gpu, ch, "peskin4", 20)
    g2, X2, U2 = run_gpu_coupled(gpu, ch, "peskin4", 20, graph=True)
    assert np.array_equal(N(X1), N(X2)) and np.array_equal(N(U1), N(U2))
    assert np.array_equal(N(g1.moments()[1]), N(g2.moments()[1]))


def test_graph_launch_checks_buffer_parity(gpu):
    """A captured 2-step graph replays from the population buffer and tile set current at
    capture: after an odd number of eager steps (or a lone lbm_step) the replay is refused;
    even interleaves of eager steps and replays equal eager execution bit for bit."""
    import torch

    ch = inputs.poiseuille_sphere(seed=3)
    g1, X1, U1 = run_gpu_coupled(gpu, ch, "peskin4", 10)
    b = ch.bodies
    g = gpu.Lattice([ch], kernel="peskin4", max_nodes=b.n, device=DEV)
    g.init()
    g.set_nodes(b.n)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    g.graph_capture(mem, 2, X, F, U)
    g.graph_launch(2)                  # 4 steps
    g.coupled_steps(mem, 2, X, F, U)   # 6
    g.graph_launch(1)                  # 8
    g.coupled_steps(mem, 1, X, F, U)   # 9: odd, a replay would read the stale buffer
    with pytest.raises(gpu.LbmError):
        g.graph_launch(1)
    g.coupled_steps(mem, 1, X, F, U)   # 10
    torch.cuda.synchronize()
    assert np.array_equal(N(X1), N(X)) and np.array_equal(N(U1), N(U))
    assert np.array_equal(N(g1.moments()[1]), N(g.moments()[1]))
    g.step(1)                          # a lone lattice step flips the buffer only
    with pytest.raises(gpu.LbmError):
        g.graph_launch(1)


def test_launch_timer_brackets_the_lattice_update(gpu):
    """The measurement helper times the lattice-update launch of eager coupled steps only."""
    import torch

    ch = inputs.poiseuille_sphere(seed=4)
    b = ch.bodies
    g = gpu.Lattice([ch], kernel="cos", max_nodes=b.n, device=DEV)
    g.init()
    g.set_nodes(b.n)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    g.launch_timer(True)
    g.coupled_steps(mem, 3, X, F, U)
    n, us, kind = g.launch_timer_read()
    assert n == 3 and 0.0 < us < 1e5 and kind == 1   # one channel: split schedule
    g.graph_capture(mem, 2, X, F, U)
    g.graph_launch(1)
    assert g.launch_timer_read()[0] == 0             # graph replays are not timed
    g.set_launch(split=0)
    g.coupled_steps(mem, 2, X, F, U)
    n, us, kind = g.launch_timer_read()
    assert n == 2 and us > 0.0 and kind == 0
    g.launch_timer(False)
    g.coupled_steps(mem, 2, X, F, U)
    assert g.launch_timer_read()[0] == 0


def test_coupled_shear_platelets_crop(orc, gpu):
    """Production-shear setup at reduced size: 96x48x64, 3 platelets of 642 nodes, 30 steps."""
    ch = inputs.shear_platelets(seed=5, nx=96, ny=48, nz=64, count=3, nodes=642)
    o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", 30)
    g, Xg, Ug = run_gpu_coupled(gpu, ch, "cos", 30)
    assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32
    assert emax(N(Ug), Uo) <= TOL32
    lo_g, _ = g.wall_stress()
    lo_o, _ = o.wall_stress()
    assert emax(N(lo_g).reshape(lo_o.shape), lo_o) <= 1e-4


# ----------------------------------------------------------------------------- state, channels
def test_populations_roundtrip_and_resume(orc, gpu):
    import torch

    ch = inputs.Channel(33, 20, 17, 0.85, u_wall_hi=(0.03, 0, 0), init="shear")
    o, g = pair(orc, gpu, ch)
    o.step(7)
    g.step(7)
    f_g = N(g.populations()).reshape(19, 17, 20, 33)
    ulp = 2.0 ** -25  # float32 ulp of f near 1/3 is 2^-25 * 2 = 3e-8
    assert np.abs(f_g - o.f).max() < 2 * ulp * 2
    g.set_populations(T(o.f.reshape(-1), np.float32))
    assert np.abs(N(g.populations()).reshape(o.f.shape) - o.f).max() < 2 * ulp * 2
    st = g.get_state().clone()
    g.step(5)
    a = N(g.moments()[1])
    g.set_state(st)
    g.step(5)
    torch.cuda.synchronize()
    assert np.array_equal(a, N(g.moments()[1]))


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_vector_step_matches_scalar_all_storages(gpu, storage):
    rng = np.random.default_rng(21)
    ch = inputs.Channel(64, 24, 16, 0.9, u_wall_hi=(0.04, 0, 0), init="shear")
    out = []
    for vec in (0, 2, 4):
        g = gpu.Lattice([ch], storage=storage, max_nodes=300, device=DEV)
        g.set_launch(vec=vec)
        g.init()
        X = T(np.stack([rng.uniform(0, 64, 300), rng.uniform(2, 20, 300), rng.uniform(0, 16, 300)]))
        F = T(1e-3 * rng.standard_normal((3, 300)), np.float32)
        rng = np.random.default_rng(21)
        g.set_nodes(300)
        g.spread(X, F)
        g.step(12)
        out.append(N(g.populations()))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_stream_copy(gpu):
    import torch

    src = torch.arange(1 << 20, dtype=torch.float32, device=DEV)
    for variant in (0, 1):
        dst = torch.zeros_like(src)
        gpu.stream_copy(src, dst, variant, 0 if variant == 0 else 512)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)


def test_multichannel_batch(orc, gpu):
    chans = [inputs.Channel(48, 32, 32, 0.75, u_wall_hi=(0.02, 0, 0), init="shear"),
             inputs.Channel(37, 21, 19, 1.1, body=(2e-6, 0, 0)),
             inputs.Channel(64, 48, 48, 0.95, u_wall_hi=(0.04, 0, 0.01), init="shear")]
    g = gpu.Lattice(chans, device=DEV)
    g.init()
    g.step(40)
    for c, ch in enumerate(chans):
        o = orc.Lattice(ch.nx, ch.ny, ch.nz, ch.tau, walls=ch.walls, body=ch.body, u_wall_lo=ch.u_wall_lo,
                        u_wall_hi=ch.u_wall_hi)
        o.init(u=o.shear_profile()) if ch.init == "shear" else o.init()
        o.step(40)
        assert emax(gpu_fields(g, c)[1], o.moments()[1]) <= TOL32


def test_multichannel_coupled_ib(orc, gpu):
    """Several channels of different size, tau, wall speed and platelet count in one context
    (one launch per kernel for all of them) against an independent oracle per channel."""
    import torch

    chans = [inputs.shear_platelets(seed=7, nx=48, ny=32, nz=32, count=1, nodes=642, tau=0.75, u_top=0.02,
                                    y_band=(8.0, 12.0)),
             inputs.shear_platelets(seed=8, nx=64, ny=48, nz=48, count=2, nodes=642, tau=1.1, u_top=0.04),
             inputs.shear_platelets(seed=9, nx=40, ny=24, nz=36, count=1, nodes=642, tau=0.9, u_top=0.03,
                                    y_band=(6.0, 10.0))]
    b, offs = inputs.concat_bodies(chans)
    g = gpu.Lattice(chans, kernel="cos", max_nodes=b.n, device=DEV)
    g.init()
    g.set_nodes(b.n, offs)
    mem = gpu.Membrane(b, device=DEV)
    X = T(b.X)
    F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
    U = torch.zeros_like(F)
    g.coupled_steps(mem, 20, X, F, U)
    torch.cuda.synchronize()
    Xg, Ug = N(X), N(U)
    for c, ch in enumerate(chans):
        o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", 20)
        assert emax(gpu_fields(g, c)[1], o.moments()[1]) <= TOL32
        assert emax(Ug[:, offs[c]:offs[c + 1]], Uo) <= TOL32
    assert g.error_flags() == 0


@pytest.mark.parametrize("dims", [(45, 37, 29), (48, 20, 16)])
@pytest.mark.parametrize("launch", [dict(block=64, xcd_remap=0), dict(block=1024, xcd_remap=1),
                                    dict(block=256, persistent=97), dict(block=512, nontemporal=1),
                                    dict(vec=2), dict(vec=4, nontemporal=1), dict(vec=2, persistent=33),
                                    dict(vec=4, xcd_remap=0)])
def test_launch_shapes_agree(gpu, launch, dims):
    """Every launch shape (scalar and vector steps) gives bitwise the same state; (48,20,16)
    is eligible for the vector step, (45,37,29) falls back to the scalar one."""
    ch = inputs.Channel(*dims, 0.8, u_wall_hi=(0.05, 0, 0.01), u_wall_lo=(0, 0, -0.02), init="shear",
                        body=(1e-5, 0, 0))
    ref = gpu.Lattice([ch], device=DEV)
    ref.init()
    ref.step(10)
    g = gpu.Lattice([ch], device=DEV)
    g.set_launch(**{**dict(block=256, xcd_remap=1, persistent=0, nontemporal=0, vec=0), **launch})
    g.init()
    g.step(10)
    assert np.array_equal(N(ref.populations()), N(g.populations()))


# ----------------------------------------------------------------------------- 16-bit storage
def bf16_rne32(x):
    """float32 -> nearest bfloat16 (ties to even), as float32: the integer rounding rule."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_rounding_is_nearest_even(gpu, storage):
    """The stored 16-bit value of a population is g = f - w_i rounded to nearest, ties to
    even (float32 arithmetic, then one conversion).  Exact ties, their neighbours and random
    values go in through lbm_set_populations (periodic box: the state round-trips through
    streaming exactly) and must come back as w_i + round(f - w_i), bit for bit."""
    rng = np.random.default_rng(21)
    ch = inputs.Channel(16, 8, 8, 0.8, walls=False)
    w = np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3], np.float32)
    n = ch.cells
    mag = rng.uniform(1e-4, 1e-2, (19, n)) * rng.choice([-1.0, 1.0], (19, n))
    g = mag.astype(np.float32)
    u = g.view(np.uint32).copy()
    if storage == "bf16":
        half = n // 3   # exact ties of bfloat16, and one float32 step either side
        u[:, :half] = (u[:, :half] & 0xFFFF0000) | 0x8000
        u[:, half:2 * half] = (u[:, half:2 * half] & 0xFFFF0000) | 0x8000
        u[:, half:2 * half] += rng.choice([-1, 1], (19, half)).astype(np.uint32)
    else:
        half = n // 3   # exact ties of float16 (13 dropped bits: tie at bit 12)
        u[:, :half] = (u[:, :half] & 0xFFFFE000) | 0x1000
        u[:, half:2 * half] = (u[:, half:2 * half] & 0xFFFFE000) | 0x1000
        u[:, half:2 * half] += rng.choice([-1, 1], (19, half)).astype(np.uint32)
    g = u.view(np.float32)
    f = (w[:, None] + g).astype(np.float32)
    gg = (f - w[:, None]).astype(np.float32)            # what the device rounds
    if storage == "bf16":
        stored = bf16_rne32(gg)
    else:
        stored = gg.astype(np.float16).astype(np.float32)
    expect = (w[:, None] + stored).astype(np.float32)
    lat = gpu.Lattice([ch], storage=storage, device=DEV)
    lat.set_populations(T(f.reshape(-1)))
    got = lat.populations().cpu().numpy().reshape(19, n)
    assert np.array_equal(got.view(np.uint32), expect.view(np.uint32))
    # the ties really were ties: some of them rounded down, some up
    tie = gg[:, :half]
    assert np.any(stored[:, :half] > tie) and np.any(stored[:, :half] < tie)


@pytest.mark.parametrize("storage,bound", [("f16", 2e-3), ("bf16", 2e-2)])
def test_half_storage_error_bounded(orc, gpu, storage, bound):
    """Weight-shifted 16-bit storage, float32 arithmetic: error against the FP64 oracle on a
    sheared channel (reported, loosely bounded)."""
    ch = inputs.Channel(64, 32, 32, 1.0, u_wall_hi=(0.05, 0, 0), init="shear")
    o, g = pair(orc, gpu, ch, storage=storage)
    o.step(200)
    g.step(200)
    e = emax(gpu_fields(g)[1], o.moments()[1])
    print("%s e_max after 200 steps: %.3e" % (storage, e))
    assert e <= bound


def test_storage_precision_report_with_platelet(orc, gpu):
    """Weight-shifted float32 / float16 / bfloat16 storage (float32 arithmetic) against the
    FP64 oracle on a standalone 64x32x32 sheared channel (top wall u = 0.05, tau = 1) with one
    oblate platelet of 2562 nodes, 200 coupled steps: velocity e_max and relative L2 error,
    bottom-wall shear-stress error, platelet centroid displacement error.  The 16-bit forms
    are reported with loose bounds; float32 is held to the 1e-5 bar."""
    ch = inputs.shear_platelets(seed=3, nx=64, ny=32, nz=32, count=1)
    steps = 200
    o, Xo, _ = run_oracle_coupled(orc, ch, "cos", steps)
    _, vref = o.moments()
    wref = o.wall_stress()[0][0]
    b = ch.bodies
    disp_ref = (Xo - b.X).mean(axis=1)
    rows = []
    for storage, bound in (("f32", 1e-5), ("f16", 5e-3), ("bf16", 5e-2)):
        g, X, _ = run_gpu_coupled(gpu, ch, "cos", steps, storage=storage)
        _, v = gpu_fields(g)
        lo, _ = g.wall_stress()
        w = N(lo)[: ch.nz * ch.nx].reshape(ch.nz, ch.nx)
        e = emax(v, vref)
        l2 = np.linalg.norm(v - vref) / np.linalg.norm(vref)
        ew = np.abs(w - wref).max() / np.abs(wref).max()
        disp = (N(X) - b.X).mean(axis=1)
        ed = np.linalg.norm(disp - disp_ref) / np.linalg.norm(disp_ref)
        rows.append((storage, e, l2, ew, ed))
        print("%-4s e_max %.3e  L2 %.3e  wall stress %.3e  platelet displacement %.3e" % (storage, e, l2, ew, ed))
        assert e <= bound and ew <= 10 * bound
        assert g.error_flags() == 0


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_overlapped_schedule_is_bitwise_sequential(gpu, storage):
    """The split coupled steps give the same bits as the fused update, eagerly and replayed
    from a graph:
    - overlap: the body-force-only update on a second stream, then the flagged IB tiles
      updated again with their force;
    - split: the body-force-only update in the spread's launch, then the flagged tiles
      updated with their force, merging split tiles' partial sums on the way."""
    import torch

    ch = inputs.shear_platelets(seed=2, nx=96, ny=48, nz=64, count=3)
    b = ch.bodies
    out = []
    for overlap, split in ((1, 0), (0, 1), (0, 0)):
        g = gpu.Lattice([ch], storage=storage, max_nodes=b.n, device=DEV)
        g.set_launch(block=128, xcd_remap=0, nontemporal=1, overlap=overlap, split=split)
        g.init()
        g.set_nodes(b.n)
        mem = gpu.Membrane(b, device=DEV)
        X = T(b.X)
        F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
        U = torch.zeros_like(F)
        g.coupled_steps(mem, 7, X, F, U)
        g.graph_capture(mem, 4, X, F, U)
        g.graph_launch(3)
        g.coupled_steps(mem, 1, X, F, U)
        torch.cuda.synchronize()
        out.append((N(g.get_state()), N(X), g.error_flags()))
    assert all(o[2] == 0 for o in out)
    for o in out[:2]:
        assert np.array_equal(o[0], out[2][0])
        assert np.array_equal(o[1], out[2][1])


def test_split_update_multichannel_is_bitwise_fused(gpu):
    """Several channels (uneven sizes and platelet counts): the split coupled step, forced on,
    gives the fused update's bits; the default for several channels is the fused update."""
    import torch

    chans = inputs.batched_channels(seed=3, nch=5)
    b, offs = inputs.concat_bodies(chans)
    out = []
    for split in (1, 0, -1):
        g = gpu.Lattice(chans, max_nodes=b.n, device=DEV)
        g.set_launch(block=256, xcd_remap=0, nontemporal=1, split=split)
        g.init()
        g.set_nodes(b.n, offs)
        mem = gpu.Membrane(b, device=DEV)
        X = T(b.X)
        F = torch.zeros((3, b.n), dtype=torch.float32, device=DEV)
        U = torch.zeros_like(F)
        g.coupled_steps(mem, 5, X, F, U)
        g.graph_capture(mem, 2, X, F, U)
        g.graph_launch(2)
        torch.cuda.synchronize()
        out.append((N(g.get_state()), N(X), g.error_flags(), g.get_launch()["split"]))
    assert all(o[2] == 0 for o in out)
    assert out[2][3] == -1
    for o in out[:2]:
        assert np.array_equal(o[0], out[2][0]) and np.array_equal(o[1], out[2][1])
