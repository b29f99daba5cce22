"""Seeded workload generators: mesh sizes, topology, placement rules, determinism."""
import numpy as np
import pytest

from paper_1312_2234_amd import inputs


def test_icosphere_counts_and_closed_mesh():
    for lev, nv in [(3, 642), (4, 2562)]:
        V, T = inputs.icosphere(lev)
        assert len(V) == nv and len(T) == 2 * nv - 4
        E, H = inputs.mesh_edges(T), inputs.mesh_hinges(T)
        assert len(E) == len(H) == 3 * nv - 6           # closed triangulation: every edge a hinge
        assert np.allclose(np.linalg.norm(V, axis=1), 1.0)


def test_fibonacci_sphere_1282():
    V, T = inputs.fibonacci_sphere(1282)
    assert len(V) == 1282 and len(T) == 2 * 1282 - 4
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    assert np.all(np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0)  # outward


def test_hinge_convention():
    V, T = inputs.icosphere(1)
    tri = {tuple(t) for t in T} | {tuple(np.roll(t, 1)) for t in T} | {tuple(np.roll(t, 2)) for t in T}
    for x0, x1, x2, x3 in inputs.mesh_hinges(T):
        assert (x0, x1, x2) in tri and (x3, x2, x1) in tri


def test_csr_roundtrip():
    V, T = inputs.icosphere(2)
    E = inputs.mesh_edges(T)
    ptr, idx = inputs.csr_neighbours(len(V), E)
    pairs = {(i, j) for i in range(len(V)) for j in idx[ptr[i]:ptr[i + 1]]}
    assert pairs == {(a, b) for a, b in E} | {(b, a) for a, b in E}
    H = inputs.mesh_hinges(T)
    hp, hi = inputs.csr_hinges(len(V), H)
    for i in range(len(V)):
        for code in hi[hp[i]:hp[i + 1]]:
            assert H[code >> 2][code & 3] == i


def test_shear_platelets_placement():
    ch = inputs.shear_platelets(seed=0)
    b = ch.bodies
    assert b.n == 16 * 2562 and len(b.body_offsets) == 17
    cen = np.array([b.X[:, b.body_offsets[k]:b.body_offsets[k + 1]].mean(axis=1) for k in range(16)])
    assert np.all(cen[:, 1] >= 7.5 - 1e-9) and np.all(cen[:, 1] <= 19.5 + 1e-9)
    for i in range(16):
        for j in range(i):
            d = np.abs(cen[i] - cen[j])
            d[0] = min(d[0], 256 - d[0])
            d[2] = min(d[2], 128 - d[2])
            assert np.linalg.norm(d) >= 16 - 1e-9
    again = inputs.shear_platelets(seed=0)
    assert np.array_equal(again.bodies.X, b.X)
    assert not np.array_equal(inputs.shear_platelets(seed=1).bodies.X, b.X)


def test_poiseuille_sphere():
    ch = inputs.poiseuille_sphere(seed=3)
    b = ch.bodies
    assert b.n == 642 and ch.tau == 0.8 and ch.body == (1e-6, 0.0, 0.0)
    r = np.linalg.norm(b.X_rest - np.array([[16], [10], [16]]), axis=0)
    assert np.allclose(r, 4.0)
    assert 0.08 < np.std(b.X - b.X_rest) < 0.12


def test_resolution_ladder_acoustic_scaling():
    """Each rung is the fine suspension under acoustic scaling: wall planes map onto each other,
    platelet centroids sit at (x_f + 1/2) r - 1/2, semi-axes scale by r, the viscosity
    (tau - 1/2) by r, spring stiffness by r and bending by r^3; the finest and half rungs are
    the two channels of coarse_fine_pair."""
    lad = inputs.resolution_ladder(seed=5, sizes=(128, 160, 192, 256))
    fine, coarse = inputs.coarse_fine_pair(seed=5)
    assert np.array_equal(lad[256][0].bodies.X, fine.bodies.X)
    assert np.array_equal(lad[128][0].bodies.X, coarse.bodies.X)
    bf = fine.bodies
    cen_f = np.array([bf.X[:, a:b].mean(axis=1) for a, b in zip(bf.body_offsets[:-1], bf.body_offsets[1:])])
    ext_f = np.array([np.ptp(bf.X[:, a:b], axis=1) for a, b in zip(bf.body_offsets[:-1], bf.body_offsets[1:])])
    for n, (ch, r) in lad.items():
        assert r == n / 256 and (ch.nx, ch.ny, ch.nz) == (n, n // 2, n // 2)
        assert abs((ch.tau - 0.5) - 0.5 * r) < 1e-15
        b = ch.bodies
        assert abs(b.k_spring - 0.005 * r) < 1e-15 and abs(b.k_bend - 1e-4 * r ** 3) < 1e-18
        cen = np.array([b.X[:, a:c].mean(axis=1) for a, c in zip(b.body_offsets[:-1], b.body_offsets[1:])])
        ext = np.array([np.ptp(b.X[:, a:c], axis=1) for a, c in zip(b.body_offsets[:-1], b.body_offsets[1:])])
        assert np.allclose(cen, (cen_f + 0.5) * r - 0.5, atol=2e-3)  # node means: the 1282-point set is not exactly centred
        assert np.allclose(ext, ext_f * r, rtol=0.02)        # sphere point sets differ below 3/4
        # wall planes: y = -1/2 and y = ny - 1/2 are the images of the fine planes
        assert (-0.5 + 0.5) * r - 0.5 == -0.5 and (127.5 + 0.5) * r - 0.5 == ch.ny - 0.5
        assert b.n == 16 * (2562 if r >= 0.75 else 1282)
    try:
        inputs.resolution_ladder(seed=5, sizes=(99,))
    except ValueError:
        pass
    else:
        raise AssertionError("a rung that does not scale to whole cells must be rejected")


def test_log_log_interpolation():
    from paper_1312_2234_amd.closure import _interp_log, _interp_log_value, _patch_mean

    xs, ys = [128, 160, 192], [0.02, 0.01, 0.004]
    assert abs(_interp_log(xs, ys, 0.01) - 160) < 1e-9
    # on a power law the log-log line is exact
    x = 150.0
    p = np.log(0.02 / 0.01) / np.log(160 / 128)
    assert abs(_interp_log(xs, ys, 0.02 * (x / 128) ** -p) - x) < 1e-9
    assert _interp_log(xs, ys, 0.03) is None and _interp_log(xs, ys, 0.001) is None
    assert abs(_interp_log_value(xs, [1e5, 5e4, 2e4], 160) - 5e4) < 1e-6
    w = np.arange(4 * 6, dtype=float).reshape(4, 6)
    assert np.array_equal(_patch_mean(w, (2, 3)), np.array([[3.5, 5.5, 7.5], [15.5, 17.5, 19.5]]))


def test_table2_constraint_coefficients_in_lattice_units():
    """Table 2's k_s = k_t = 6000 k_B T / l_0^2 and k_v = 6000 k_B T / l_0^3 taken to SI (N/m and
    N/m^2 at 300 K, l_0 = 75 nm) and divided by the lattice units of stiffness rho h^3 / dt^2 and
    rho h^2 / dt^2 (h = 0.2 um, dt = 1e-8 s, rho = 1023.9 kg/m^3)."""
    ks, kt, kv = inputs.table2_constraint_coefficients()
    kT = 1.380649e-23 * 300
    ks_si, kv_si = 6000 * kT / 75e-9 ** 2, 6000 * kT / 75e-9 ** 3
    assert abs(ks - ks_si / (1023.9 * 0.2e-6 ** 3 / 1e-16)) < 1e-12 * ks
    assert ks == kt
    assert abs(kv - kv_si / (1023.9 * 0.2e-6 ** 2 / 1e-16)) < 1e-12 * kv
    assert abs(kv / ks - 0.2e-6 / 75e-9) < 1e-12


def test_with_constraints_triangles_are_outward_and_complete():
    """Every body's triangles close its surface (each edge in exactly two triangles, opposite
    directions) with positive volume, and the offsets partition the triangle list."""
    ch = inputs.shear_platelets(seed=1, nx=64, ny=32, nz=48, count=2, nodes=642)
    b = inputs.with_constraints(ch.bodies, 0.1, 0.1, 0.1)
    assert b.tri_offsets[0] == 0 and b.tri_offsets[-1] == len(b.triangles)
    X = b.X.T
    for (lo, hi), (n0, n1) in zip(zip(b.tri_offsets[:-1], b.tri_offsets[1:]), zip(b.body_offsets[:-1], b.body_offsets[1:])):
        T = b.triangles[lo:hi]
        assert T.min() >= n0 and T.max() < n1
        directed = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
        assert len({tuple(e) for e in directed}) == len(directed)            # each directed edge once
        assert {tuple(e) for e in directed} == {tuple(e[::-1]) for e in directed}  # and its reverse too
        a, c, d = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
        assert np.einsum("ij,ij->i", a, np.cross(c, d)).sum() > 0


def test_director_tracker_counts_half_turns():
    """A director turning clockwise (seen from +z) at a varying rate, sampled coarsely and
    with random sign flips: the tracker's pi-crossings match the analytic crossing times."""
    import math

    from paper_1312_2234_amd.experiments import DirectorTracker, jeffery_period

    rng = np.random.default_rng(5)
    r, g = 1 / 3, 1e-3
    T = jeffery_period(r, g)
    # Jeffery's orbit of the director: tan(phi) = r tan(w t) with w = 2 pi / T (clockwise phi)
    def axis(t):
        phi = math.atan2(r * math.sin(2 * math.pi * t / T), math.cos(2 * math.pi * t / T))
        v = np.array([math.sin(phi), math.cos(phi), 0.0])   # starts along +y, turns clockwise
        return v if rng.random() < 0.5 else -v
    tr = DirectorTracker(axis(0.0))
    chunk = 50
    for k in range(1, int(1.6 * T / chunk)):
        tr.update(axis(k * chunk), k * chunk, chunk)
    # the director passes phi = pi/2 + m pi at t = T/4 + m T/2 ... and phi = m pi at t = m T/2
    assert len(tr.marks) == 3
    for m, t in enumerate(tr.marks, start=1):
        assert abs(t - m * T / 2) < 0.02 * T


def test_with_constraints_rejects_bodies_of_other_meshes():
    rng = np.random.default_rng(0)
    t = inputs.tethered_sphere(rng, (16, 10, 16), 4.0, 642, 0.01, 0.1)
    with pytest.raises(ValueError):
        inputs.with_constraints(t, 0.1, 0.1, 0.1)
