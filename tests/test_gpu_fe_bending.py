"""Finite-element bending of Eq. (6)-(10) (six-node triangles, force (k0/2)(Lap K + 2K(K^2 - G)) n A)
on the GPU, through the C ABI, against the FP64 oracle: forces alone on deformed platelets
(1e-6 relative to the largest force, as the other membrane terms), alone and with springs and
the area and volume constraints; inside the coupled step (float32 bar e_max <= 1e-5); bitwise
deterministic, and graph replay equal to eager execution."""
import dataclasses

import numpy as np
import pytest

from paper_1312_2234_amd import inputs
from test_gpu_parity import DEV, TOL32, N, T, emax, gpu_fields, run_gpu_coupled, run_oracle_coupled

pytestmark = pytest.mark.gpu
K0 = inputs.table2_bending_modulus()


def deformed(seed=3, count=2, nodes=642, sigma=0.1, k0=K0, springs=True, constraints=False):
    """Platelets with FE bending whose nodes start N(0, sigma^2) off their rest shape."""
    ch = inputs.shear_platelets(seed=seed, nx=64, ny=32, nz=48, count=count, nodes=nodes)
    b = inputs.with_fe_bending(ch.bodies, k0)
    if not springs:
        b = dataclasses.replace(b, k_spring=0.0)
    if constraints:
        b = inputs.with_constraints(b, 0.05, 0.02, 0.1)
    rng = np.random.default_rng(seed)
    X = b.X_rest + sigma * rng.standard_normal(b.X_rest.shape)
    return dataclasses.replace(ch, bodies=dataclasses.replace(b, X=np.ascontiguousarray(X)))


def oracle_membrane(orc, b):
    return orc.Membrane(b.X_rest, b.edges, k_spring=b.k_spring, hinges=b.hinges, k_bend=b.k_bend,
                        triangles=b.triangles, body_tri=b.tri_offsets if b.triangles is not None else None,
                        k_area_global=b.k_area_global, k_area_local=b.k_area_local, k_volume=b.k_volume,
                        elements6=b.elements6, k_fe=b.k_fe)


@pytest.mark.parametrize("nodes,springs,constraints", [(642, False, False), (2562, False, False),
                                                       (642, True, False), (2562, True, True)])
def test_fe_forces_match_oracle(orc, gpu, nodes, springs, constraints):
    ch = deformed(nodes=nodes, springs=springs, constraints=constraints)
    b = ch.bodies
    F_o = oracle_membrane(orc, b).forces(b.X)
    gm = gpu.Membrane(b, device=DEV)
    F_g = N(gm.forces(T(b.X)))
    e = emax(F_g, F_o)
    print("%d nodes, springs %s, constraints %s: e_max %.3e" % (nodes, springs, constraints, e))
    assert e <= 1e-6
    # the bending part is resolved, not hidden under the other terms
    no_fe = dataclasses.replace(b, elements6=None, k_fe=0.0)
    dF = F_o - oracle_membrane(orc, no_fe).forces(b.X)
    assert np.abs(dF).max() > 1e-2 * np.abs(F_o).max()
    dF_g = F_g - N(gpu.Membrane(no_fe, device=DEV).forces(T(b.X)))
    assert emax(dF_g, dF) <= 1e-5
    # deterministic: every sum has a fixed order
    assert np.array_equal(F_g, N(gm.forces(T(b.X))))


def test_fe_forces_on_a_sphere_are_small(orc, gpu):
    """A tethered-free sphere of radius 4: the FE force is the discretisation residual only, small
    against the force the printed formula (without the Gaussian term) would give, on the GPU too."""
    from oracle import bending_oracle as bo

    E6 = inputs._quadratic(2562)
    V0 = inputs._topology(2562)[0]
    X = np.ascontiguousarray((V0 * 4.0 + 20.0).T)
    b = inputs.Bodies(X=X, X_rest=X.copy(), edges=inputs._topology(2562)[2], hinges=np.zeros((0, 4), np.int32),
                      anchors=None, body_offsets=[0, 2562], elements6=E6, k_fe=1.0)
    F_g = N(gpu.Membrane(b, device=DEV).forces(T(X)))
    c = X.mean(axis=1, keepdims=True)
    w = np.sum(F_g.astype(np.float64) * (X - c))
    w0 = np.sum(bo.forces(X, E6, 1.0, gaussian=False) * (X - c))
    assert abs(w0 / (4 * np.pi) - 1) < 3e-2     # the printed force's dilation work (level 4 mesh)
    assert abs(w) < 2e-3 * abs(w0)


def test_coupled_with_fe_bending_matches_oracle(orc, gpu):
    ch = deformed(seed=4, count=1, sigma=0.05)
    o, Xo, Uo = run_oracle_coupled(orc, ch, "cos", 20)
    g, Xg, Ug = run_gpu_coupled(gpu, ch, "cos", 20)
    assert emax(gpu_fields(g)[1], o.moments()[1]) <= TOL32
    assert emax(N(Ug), Uo) <= TOL32
    assert np.abs(N(Xg) - Xo).max() <= TOL32 * np.abs(Xo - ch.bodies.X).max()
    assert g.error_flags() == 0


def test_coupled_with_fe_bending_graph_equals_eager(gpu):
    ch = deformed(seed=5, count=2, sigma=0.05, constraints=True)
    g1, X1, U1 = run_gpu_coupled(gpu, ch, "cos", 12)
    g2, X2, U2 = run_gpu_coupled(gpu, ch, "cos", 12, graph=True)
    assert np.array_equal(N(X1), N(X2)) and np.array_equal(N(U1), N(U2))
    assert np.array_equal(N(g1.get_state()), N(g2.get_state()))
