"""Pins of the FE bending oracle (section 3.1, Eq. (6)-(10) and the bending force stated after
Eq. (10)) against closed forms and exact identities: the curvatures of spheres and ellipsoids,
the Laplace-Beltrami eigenfunctions of the sphere, the sphere's energy 2 pi k0 at any radius, the
vanishing work of the force on a dilating sphere (and the printed force's nonzero work), the
energy's directional derivatives, and the exact invariances under rotation, translation and
scaling.  Discretisation errors are checked to shrink about fourfold per mesh level (second
order in the node spacing)."""
import numpy as np
import pytest

from oracle import bending_oracle as bo
from paper_1312_2234_amd import inputs

LEVELS = (3, 4, 5)


@pytest.fixture(scope="module")
def meshes():
    return {lev: inputs.icosphere_quadratic(lev) for lev in LEVELS}


def ellipsoid_curvatures(X, a, b, c):
    """Mean (outward normal: positive) and Gaussian curvature of x^2/a^2 + y^2/b^2 + z^2/c^2 = 1."""
    x, y, z = X
    q = x * x / a ** 4 + y * y / b ** 4 + z * z / c ** 4
    H = (a * a + b * b + c * c - x * x - y * y - z * z) / (2 * (a * b * c) ** 2 * q ** 1.5)
    G = 1.0 / ((a * b * c) ** 2 * q * q)
    return H, G


def test_six_node_mesh_structure(meshes):
    for lev, (V, E6) in meshes.items():
        assert E6.shape == (20 * 4 ** (lev - 1), 6)
        assert len(np.unique(E6)) == len(V) == 10 * 4 ** lev + 2
        # midpoints lie between their corners (on the unit sphere, along the bisector)
        for m, (p, q) in ((3, (0, 1)), (4, (1, 2)), (5, (2, 0))):
            mid = V[E6[:, p]] + V[E6[:, q]]
            mid /= np.linalg.norm(mid, axis=1)[:, None]
            assert np.abs(V[E6[:, m]] - mid).max() < 1e-14
        # corners outward
        a, b, c = (V[E6[:, k]] for k in range(3))
        assert (np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0).all()


def test_sphere_curvatures_converge(meshes):
    errK, errG = [], []
    for lev in LEVELS:
        V, E6 = meshes[lev]
        R = 2.5
        c = bo.curvatures(V.T * R, E6)
        errK.append(np.abs(c["K"] * R - 1).max())
        errG.append(np.abs(c["G"] * R * R - 1).max())
        # the averaged normal is the radial direction
        assert np.abs(c["n"] - V).max() < 5 * errK[-1]
    assert errK[-1] < 4e-3 and errG[-1] < 8e-3
    for e in (errK, errG):
        assert e[0] / e[1] > 3.3 and e[1] / e[2] > 3.3, e


def test_ellipsoid_curvatures_match_closed_form(meshes):
    errK, errG = [], []
    for lev in LEVELS:
        V, E6 = meshes[lev]
        X = (V * np.array([2.0, 1.5, 1.0])).T
        c = bo.curvatures(X, E6)
        H, G = ellipsoid_curvatures(X, 2.0, 1.5, 1.0)
        errK.append(np.abs(c["K"] / H - 1).max())
        errG.append(np.abs(c["G"] / G - 1).max())
    assert errK[-1] < 4e-3 and errG[-1] < 8e-3
    for e in (errK, errG):
        assert e[0] / e[1] > 3.3 and e[1] / e[2] > 3.3, e


def test_laplace_beltrami_spherical_harmonics(meshes):
    """Lap Y_l = -l(l+1) Y_l / R^2 on a sphere of radius R (l = 1: z; l = 2: x^2 - y^2)."""
    err1, err2 = [], []
    for lev in LEVELS:
        V, E6 = meshes[lev]
        R = 2.0
        X = V.T * R
        x, y, z = X
        l1 = bo.laplace_beltrami(X, E6, z)
        l2 = bo.laplace_beltrami(X, E6, x * x - y * y)
        err1.append(np.abs(l1 + 2 * z / R ** 2).max() / (2 / R))
        err2.append(np.abs(l2 + 6 * (x * x - y * y) / R ** 2).max() / 6)
    assert err1[-1] < 3e-3 and err2[-1] < 6e-3
    assert err1[0] / err1[1] > 3.0 and err1[1] / err1[2] > 3.0, err1
    assert err2[0] > err2[1] > err2[2], err2


@pytest.mark.parametrize("R", [0.5, 3.0, 40.0])
def test_sphere_energy_is_2pi_k0_at_any_radius(meshes, R):
    k0 = 2.5e-4
    E = {lev: bo.energy(meshes[lev][0].T * R, meshes[lev][1], k0) for lev in LEVELS}
    assert abs(E[5] / (2 * np.pi * k0) - 1) < 5e-3
    assert abs(E[3] - 2 * np.pi * k0) > 3.0 * abs(E[4] - 2 * np.pi * k0) > 9.0 * abs(E[5] - 2 * np.pi * k0)
    # scale invariance of the discrete energy (K^2 dS is dimensionless)
    E1 = bo.energy(meshes[4][0].T, meshes[4][1], k0)
    assert abs(E[4] - E1) <= 1e-12 * E1


def test_sphere_force_does_no_work_on_dilation(meshes):
    """With the Gaussian-curvature term the force on a sphere does no work on a uniform dilation
    (the energy is scale invariant); the force as printed after Eq. (10) would do k0/2 * 8 pi."""
    k0 = 1.0
    w, w0 = [], []
    for lev in LEVELS:
        V, E6 = meshes[lev]
        X = V.T * 3.0 + np.array([[4.0], [5.0], [6.0]])
        c = X.mean(axis=1, keepdims=True)
        w.append(np.sum(bo.forces(X, E6, k0) * (X - c)))
        w0.append(np.sum(bo.forces(X, E6, k0, gaussian=False) * (X - c)))
    assert abs(w0[-1] / (4 * np.pi * k0) - 1) < 1e-2      # the printed force's work, k0/2 * 2K^3 * 4 pi R^3
    assert abs(w[-1]) < 1e-3 * 4 * np.pi * k0
    assert abs(w[0]) > abs(w[2])


def test_force_is_minus_energy_gradient(meshes):
    """Directional derivative of the energy along smooth deformations of an ellipsoid against the
    force's work: -dE/de = sum_i F_i . v_i up to discretisation, shrinking with the mesh."""
    rel = {}
    for lev in (4, 5):
        V, E6 = meshes[lev]
        X = (V * np.array([2.0, 1.5, 1.0])).T
        F = bo.forces(X, E6, 1.0)
        rel[lev] = []
        for v in (np.stack([0.1 * X[1] * X[2], 0.05 * X[0] ** 2, -0.07 * X[0] * X[1] + 0.03 * X[2]]),
                  np.stack([0.2 * X[0] ** 3, 0.0 * X[1], 0.1 * X[2] * X[0]]),
                  np.stack([0.3 * X[0] * X[1] ** 2, 0.2 * X[1] ** 3, 0.1 * X[2] * X[0] ** 2])):
            h = 1e-5
            dE = (bo.energy(X + h * v, E6, 1.0) - bo.energy(X - h * v, E6, 1.0)) / (2 * h)
            assert abs(dE) > 0.1
            rel[lev].append(abs(-dE - np.sum(F * v)) / abs(dE))
    print(rel)
    assert max(rel[5]) < 2e-2
    assert all(a / b > 2.5 for a, b in zip(rel[4], rel[5])), rel


def test_force_invariances(meshes):
    V, E6 = meshes[4]
    X = (V * np.array([2.0, 1.5, 1.0])).T
    F = bo.forces(X, E6, 1.0)
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    Rm = Rx @ Rz
    Fr = bo.forces(Rm @ X + np.array([[1.0], [2.0], [3.0]]), E6, 1.0)
    assert np.abs(Rm @ F - Fr).max() <= 1e-9 * np.abs(F).max()
    # F(lambda X) = F(X) / lambda: force density ~ lambda^-3, nodal area ~ lambda^2
    assert np.abs(3.0 * bo.forces(3.0 * X, E6, 1.0) - F).max() <= 1e-9 * np.abs(F).max()
    # linear in k0
    assert np.abs(bo.forces(X, E6, 2.5) - 2.5 * F).max() <= 1e-14 * np.abs(F).max()


def test_nodal_areas_sum_to_the_flat_mesh_area(meshes):
    V, E6 = meshes[4]
    A = bo.nodal_areas(V.T, E6)
    T = inputs.icosphere(4)[1]
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    flat = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()
    assert abs(A.sum() - flat) <= 1e-12 * flat
    assert abs(flat / (4 * np.pi) - 1) < 3e-3
