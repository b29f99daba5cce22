"""Seeded workload generators: mesh sizes, topology, placement rules, determinism."""
import numpy as np

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
