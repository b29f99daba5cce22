"""Pins of the FP64 learned-closure reference against facts fixed by the mathematics:
orthonormality and the closed forms of the moment basis, exact conservation of the
correction, the zero-network special case, finite-difference gradients, the permutation
structure of streaming, recovery of a known correction by the target pipeline and the
exact Couette solution under restriction."""
import numpy as np
import pytest

from oracle import closure_oracle as co
from oracle import oracle


def _theta(rng, scale=0.3, zero_last=False):
    W1 = rng.normal(0, scale, (16, 64))
    b1 = rng.normal(0, 0.1, 64)
    W2 = rng.normal(0, scale / 2, (64, 64))
    b2 = rng.normal(0, 0.1, 64)
    W3 = np.zeros((64, 16)) if zero_last else rng.normal(0, scale / 4, (64, 16))
    b3 = np.zeros(16) if zero_last else rng.normal(0, 0.05, 16)
    return np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)])


def _norm(scale_in=1e3, scale_out=1e-4):
    return dict(in_mean=np.zeros(16), in_scale=np.full(16, scale_in), out_scale=np.full(16, scale_out))


def _random_lattice(rng, nx=6, ny=8, nz=4, tau=0.75, walls=True, u_hi=(0.04, 0, 0.01)):
    lat = oracle.Lattice(nx, ny, nz, tau, walls=walls, body=(1e-5, 0, 0), u_wall_hi=u_hi)
    lat.init(u=rng.normal(0, 0.02, (3, nz, ny, nx)))
    lat.f += rng.normal(0, 1e-3, lat.f.shape) * np.asarray(oracle.tables()[1])[:, None, None, None]
    lat.g[...] = rng.normal(0, 1e-4, lat.g.shape)
    return lat


def test_basis_orthonormal():
    M = co.moment_basis()
    assert np.abs(M @ M.T - np.eye(19)).max() < 1e-14


def test_basis_closed_form_rows():
    # sum over D3Q19 of 1 = 19, of c_x^2 = 10 (2 axis + 8 diagonal velocities)
    c, _ = co.velocities()
    M = co.moment_basis()
    assert np.allclose(M[0], np.full(19, 1 / np.sqrt(19)), atol=1e-15)
    for a in range(3):
        e = c[:, a] / np.sqrt(10)
        assert np.allclose(M[1 + a], e, atol=1e-15)
    r4 = c[:, 0] ** 2 - 10.0 / 19.0
    assert np.allclose(M[4], r4 / np.linalg.norm(r4), atol=1e-15)
    # xy row: c_x c_y is already orthogonal to every earlier monomial; 4 velocities, norm 2
    assert np.allclose(M[7], c[:, 0] * c[:, 1] / 2.0, atol=1e-15)


def test_non_conserved_rows_orthogonal_to_mass_and_momentum():
    c, _ = co.velocities()
    M = co.moment_basis()
    assert np.abs(M[4:].sum(axis=1)).max() < 1e-15
    assert np.abs(M[4:] @ c).max() < 1e-15
    # rows 0-3 span exactly {1, c_x, c_y, c_z}
    P = M[:4].T @ M[:4]
    for v in (np.ones(19), c[:, 0], c[:, 1], c[:, 2]):
        assert np.abs(P @ v - v).max() < 1e-14


def test_correction_conserves_mass_and_momentum():
    rng = np.random.default_rng(1)
    lat = _random_lattice(rng)
    c, _ = co.velocities()
    dF, nrej = co.correction(lat.f, lat.g, np.array(lat.p.body[:]), _theta(rng), _norm(), c_guard=1e30)
    assert nrej == 0 and np.abs(dF).max() > 1e-7
    assert np.abs(dF.sum(axis=0)).max() < 1e-15 * 1e3 * np.abs(dF).max()
    assert np.abs(c.T @ dF).max() < 1e-15 * 1e3 * np.abs(dF).max()


def test_zero_last_layer_is_plain_step():
    rng = np.random.default_rng(2)
    lat = _random_lattice(rng)
    ref = oracle.Lattice(6, 8, 4, 0.75, walls=True, body=(1e-5, 0, 0), u_wall_hi=(0.04, 0, 0.01))
    ref.f[...] = lat.f
    ref.g[...] = lat.g
    theta = _theta(rng, zero_last=True)
    for _ in range(3):
        assert co.closure_step(lat, theta, _norm()) == 0
        ref.step(1)
        assert np.array_equal(lat.f, ref.f)


def test_guard_rejects_large_corrections():
    rng = np.random.default_rng(3)
    lat = _random_lattice(rng)
    ref_f = lat.f.copy()
    theta = _theta(rng)
    big = dict(in_mean=np.zeros(16), in_scale=np.full(16, 1e3), out_scale=np.full(16, 1e6))
    N = lat.N
    nrej = co.closure_step(lat, theta, big)
    assert nrej == N
    ref = oracle.Lattice(6, 8, 4, 0.75, walls=True, body=(1e-5, 0, 0), u_wall_hi=(0.04, 0, 0.01))
    ref.f[...] = ref_f
    ref.g[...] = lat.g
    ref.step(1)
    assert np.array_equal(lat.f, ref.f)
    # non-finite corrections are rejected too
    theta_nan = theta.copy()
    theta_nan[-2] = np.nan  # b3[14]; lane 15 is unused and may hold anything
    lat.f[...] = ref_f
    assert co.closure_step(lat, theta_nan, _norm()) == N


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    theta = _theta(rng)
    x = rng.normal(0, 1, (6, 16))
    t = rng.normal(0, 0.3, (6, 16))
    y, cache = co.mlp_forward(x, theta)
    # keep clear of the ReLU kinks so the finite difference is smooth
    assert np.abs(cache[1]).min() > 1e-3 and np.abs(cache[3]).min() > 1e-3
    g = co.mlp_backward(y, t, cache, theta)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (co.loss(co.mlp_forward(x, tp)[0], t) - co.loss(co.mlp_forward(x, tm)[0], t)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(g).max()
    # unused output lane 15 gets no gradient
    W3g = co.unpack(g)[4]
    assert np.all(W3g[:, 15] == 0)


def test_adam_first_step_is_signed_lr():
    # with bias correction the first step is -lr * g / (|g| + eps) per parameter
    g = np.array([1e-3, -2.0, 0.5])
    th, m, v = co.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -3.14159, 1e-30])
    r = co.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0  # halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert r[2] == 1.0 + 2 ** -6  # halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert r[3] == 1.0
    assert abs(r[4] + 3.14159) <= 2 ** -8 * 4
    assert abs(r[5] - 1e-30) <= 1e-30 * 2 ** -8


@pytest.mark.parametrize("u_hi", [(0.0, 0.0, 0.0), (0.05, 0.0, 0.02)])
def test_unstream_inverts_stream(u_hi):
    rng = np.random.default_rng(5)
    lat = _random_lattice(rng, u_hi=u_hi)
    fs = lat.collide()
    lat.stream_from(fs)
    back = lat.unstream(lat.f)
    if u_hi == (0.0, 0.0, 0.0):
        assert np.array_equal(back, fs)
    else:
        assert np.abs(back - fs).max() <= 4 * np.finfo(float).eps * np.abs(fs).max()
    f1 = lat.f.copy()
    lat.stream_from(back)
    assert np.abs(lat.f - f1).max() <= 4 * np.finfo(float).eps * np.abs(f1).max()


def test_targets_recover_a_known_correction():
    rng = np.random.default_rng(6)
    lat = _random_lattice(rng)
    theta, norm = _theta(rng), _norm()
    f0, g0 = lat.f.copy(), lat.g.copy()
    body = np.array(lat.p.body[:])
    dF, nrej = co.correction(f0, g0, body, theta, norm, c_guard=1e30)
    assert nrej == 0
    co.closure_step(lat, theta, norm, c_guard=1e30)
    f1 = lat.f.copy()
    M = co.moment_basis()
    dm_applied = (M[4:] @ dF).T
    raw, dm = co.targets(lat, f0, g0, f1)
    # f* + dF is rounded once per population: the recovered moments carry that rounding
    bound = 19 * np.finfo(float).eps * np.abs(f1).max()
    assert np.abs(dm - dm_applied).max() <= bound < 1e-8 * np.abs(dm_applied).max()
    assert np.allclose(raw, co.raw_features(f0, g0, body), rtol=0, atol=1e-18)


def test_targets_vanish_for_a_plain_coarse_step():
    rng = np.random.default_rng(7)
    lat = _random_lattice(rng)
    f0, g0 = lat.f.copy(), lat.g.copy()
    lat.step(1)
    _, dm = co.targets(lat, f0, g0, lat.f.copy())
    assert np.abs(dm).max() <= 19 * np.finfo(float).eps * np.abs(f0).max()


def test_restriction_block_means():
    rng = np.random.default_rng(8)
    lat = _random_lattice(rng, nx=8, ny=8, nz=4)
    f_c, g_c, body_c = co.restrict(lat.f, lat.g, lat.p.body[:], 1.0, 0.75)
    c, _ = co.velocities()
    rho = lat.f.sum(0).reshape(2, 2, 4, 2, 4, 2).mean(axis=(1, 3, 5))
    j = np.tensordot(c.T, lat.f, axes=(1, 0)).reshape(3, 2, 2, 4, 2, 4, 2).mean(axis=(2, 4, 6))
    assert np.allclose(f_c.sum(0), rho, rtol=0, atol=1e-15)
    assert np.allclose(np.tensordot(c.T, f_c, axes=(1, 0)), j, rtol=0, atol=1e-16)
    assert np.allclose(g_c, 2 * lat.g.reshape(3, 2, 2, 4, 2, 4, 2).mean(axis=(2, 4, 6)), rtol=0, atol=1e-18)
    assert np.allclose(body_c, 2e-5 * np.array([1, 0, 0]))


def _couette_restriction_residual(U):
    fine = oracle.Lattice(4, 32, 4, 1.0, u_wall_hi=(U, 0, 0))
    fine.init(u=fine.shear_profile())
    fine.step(3000)
    coarse = oracle.Lattice(2, 16, 2, 0.75, u_wall_hi=(U, 0, 0))
    coarse.init(u=coarse.shear_profile())
    coarse.step(3000)
    f_c, _, _ = co.restrict(fine.f, fine.g, (0, 0, 0), 1.0, 0.75)
    return f_c - coarse.f


def test_restriction_of_fine_couette_is_coarse_couette_to_first_order():
    """Steady Couette is exact on both lattices.  Under acoustic scaling (tau_c = 0.75 for
    tau_f = 1) the rescaled restriction of the fine steady state equals the coarse steady
    state in every term linear in the wall speed: the residual is purely quadratic in U
    (the second-order non-equilibrium part does not follow the tau * gradient rescaling;
    that part is what the closure is trained on)."""
    d1 = _couette_restriction_residual(0.05)
    d2 = _couette_restriction_residual(0.025)
    assert np.abs(d1 - 4 * d2).max() <= 1e-12
    assert 1e-7 < np.abs(d1).max() <= 0.05 ** 2 / 500
