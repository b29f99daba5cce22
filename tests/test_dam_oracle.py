"""Pins of the adhesion oracle (section 3.2, Eq. (12)-(14)): the published known-answer vectors of
Philox4x32-10, the exact conversion of two words to a uniform, statistics of the Monte-Carlo
machinery against closed forms (mean bond lifetime at constant force = 1/P_r steps, i.e. 1/k_off
for small rates, and its Bell dependence on force; the stationary bound fraction P_f/(P_f + P_r)
of an isolated pair; the per-step formation fraction), and exact invariants (one bond per
receptor, at most four per ligand with the lowest receptor ids accepted first, the nearest free
ligand chosen, periodic minimum image, capture radius), and the bond force as minus the gradient of
the spring energy."""
import numpy as np
import pytest

from oracle import dam_oracle as dam


def test_philox_known_answers():
    """Known-answer vectors published with Philox4x32-10 (Random123)."""
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = tuple(int(w) for w in dam.philox4x32(ctr, key))
        assert got == want, [hex(w) for w in got]


def test_uniform53_is_exact_and_in_range():
    assert dam.uniform53(0, 0) == 0.0
    assert dam.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert dam.uniform53(1 << 5, 0) == 2.0 ** -27
    assert dam.uniform53(0, 1 << 6) == 2.0 ** -53
    ub, uf = dam.uniforms(12345, 7, np.arange(200000))
    for u in (ub, uf):
        assert u.min() >= 0.0 and u.max() < 1.0
        assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
        assert abs(np.mean(u < 0.01) - 0.01) < 4 * np.sqrt(0.01 * 0.99 / len(u))
    assert abs(np.corrcoef(ub, uf)[0, 1]) < 4 / np.sqrt(len(ub))
    # different steps and seeds give different streams
    assert not np.array_equal(dam.uniforms(12345, 8, np.arange(10))[0], ub[:10])
    assert not np.array_equal(dam.uniforms(12346, 7, np.arange(10))[0], ub[:10])


def pairs(nr, heights, spacing=4.0, nx=None, nz=8.0):
    """nr receptors, each alone above its own ligand (spacing apart in x, so no receptor reaches
    another's ligand): each receptor sits on its own triangle (weights 1/3 each) whose centroid is
    at height `heights` above the wall plane y = 0 and above the ligand."""
    h = np.broadcast_to(np.asarray(heights, float), (nr,))
    xs = spacing * (np.arange(nr) + 0.5)
    X = np.zeros((3, 3 * nr))
    for k, off in enumerate(((0.3, 0.0, 0.0), (-0.15, 0.0, 0.26), (-0.15, 0.0, -0.26))):
        X[0, k::3] = xs + off[0]
        X[1, k::3] = h
        X[2, k::3] = nz / 2 + off[2]
    tri = np.arange(3 * nr).reshape(nr, 3)
    bary = np.full((nr, 3), 1.0 / 3.0)
    lig = np.stack([xs, np.full(nr, nz / 2)], axis=1)
    return X, tri, bary, lig, (nx or spacing * nr), nz


def model(tri, bary, lig, nx, nz, **kw):
    p = dict(capture=0.64, sigma=0.05, l_b=0.2, gamma=0.5, kT=0.01, k_on0=0.0, k_off0=0.0, seed=99)
    p.update(kw)
    return dam.Adhesion(tri, bary, lig, 0.0, nx, nz, **p)


@pytest.mark.parametrize("stretch", [0.0, 0.1])
def test_mean_bond_lifetime_is_one_over_the_off_rate(stretch):
    """Bonds held at a constant length l_b + stretch, no re-forming: lifetimes are geometric with
    mean 1/P_r steps, P_r = 1 - exp(-k_off0 exp(gamma sigma stretch / kT)) (Eq. (12))."""
    nr = 4000
    X, tri, bary, lig, nx, nz = pairs(nr, 0.2 + stretch)
    m = model(tri, bary, lig, nx, nz, k_off0=0.05)
    m.bond[:] = np.arange(nr)
    m.count[:] = 1
    life = np.zeros(nr)
    alive = np.ones(nr, bool)
    for s in range(1, 1000):
        m.step(X, s)
        ended = alive & (m.bond < 0)
        life[ended] = s
        alive &= ~ended
        if not alive.any():
            break
    assert not alive.any()
    kon = 0.05 * np.exp(0.5 * 0.05 * stretch / 0.01)
    Pr = 1 - np.exp(-kon)
    mean = 1 / Pr
    se = np.sqrt((1 - Pr) / Pr ** 2 / nr)
    print("stretch %.2f: mean lifetime %.2f steps, 1/P_r %.2f, 1/k_off %.2f" % (stretch, life.mean(), mean, 1 / kon))
    assert abs(life.mean() - mean) < 4 * se
    assert abs(mean - 1 / kon) < 0.6 * kon * mean    # 1/k_off up to O(k_off dt) for small per-step rates
    assert (m.count == 0).all()


def test_stationary_bound_fraction_of_isolated_pairs():
    """A pair switches bound -> free with P_r and free -> bound with P_f (a bond broken in a step
    does not re-form in that step), so the time-averaged bound fraction is P_f / (P_f + P_r)."""
    nr = 3000
    height = 0.35
    X, tri, bary, lig, nx, nz = pairs(nr, height)
    kw = dict(k_on0=0.03, k_off0=0.05)
    m = model(tri, bary, lig, nx, nz, **kw)
    frac = []
    for s in range(1, 301):
        m.step(X, s)
        if s > 100:
            frac.append(np.mean(m.bond >= 0))
    s_ = abs(height - 0.2)
    Pf = 1 - np.exp(-0.03 * np.exp(0.05 * s_ * (0.5 - 0.5 * s_) / 0.01))
    Pr = 1 - np.exp(-0.05 * np.exp(0.5 * 0.05 * s_ / 0.01))
    want = Pf / (Pf + Pr)
    got = float(np.mean(frac))
    print("bound fraction %.4f, P_f/(P_f+P_r) %.4f" % (got, want))
    assert abs(got - want) < 0.01
    assert (m.count == (m.bond[:, None] == np.arange(len(lig))[None, :]).sum(axis=0)).all()


def test_formation_fraction_follows_the_on_rate_with_distance():
    nr = 20000
    heights = np.where(np.arange(nr) % 2 == 0, 0.1, 0.5)
    X, tri, bary, lig, nx, nz = pairs(nr, heights)
    m = model(tri, bary, lig, nx, nz, k_on0=0.2)
    m.step(X, 1)
    for h in (0.1, 0.5):
        sel = heights == h
        s_ = abs(h - 0.2)
        Pf = 1 - np.exp(-0.2 * np.exp(0.05 * s_ * (0.5 - 0.5 * s_) / 0.01))
        got = np.mean(m.bond[sel] >= 0)
        assert abs(got - Pf) < 4 * np.sqrt(Pf * (1 - Pf) / sel.sum()), (h, got, Pf)


def crowd(nr, nl=1, lig_x=(2.0,), y=0.3):
    """nr receptors in a small cluster above ligand(s) at x = lig_x (z = 2), all within reach."""
    rng = np.random.default_rng(5)
    c = np.stack([2.0 + 0.05 * rng.standard_normal(nr), np.full(nr, y), 2.0 + 0.05 * rng.standard_normal(nr)])
    X = np.zeros((3, 3 * nr))
    for k, off in enumerate(((0.01, 0, 0), (-0.005, 0, 0.009), (-0.005, 0, -0.009))):
        X[:, k::3] = c + np.array(off)[:, None]
    tri = np.arange(3 * nr).reshape(nr, 3)
    bary = np.full((nr, 3), 1.0 / 3.0)
    lig = np.stack([np.asarray(lig_x, float), np.full(nl, 2.0)], axis=1)
    return X, tri, bary, lig


def test_ligand_takes_at_most_four_lowest_receptor_ids_first():
    X, tri, bary, lig = crowd(7)
    m = model(tri, bary, lig, 16.0, 16.0, k_on0=1e6)  # P_f = 1
    perm = np.array([5, 2, 6, 0, 3, 1, 4])             # receptor ids shuffled against positions
    m.rec_tri = tri[perm]
    m.step(X, 1)
    assert sorted(np.nonzero(m.bond >= 0)[0].tolist()) == [0, 1, 2, 3]
    assert m.count[0] == 4
    m.step(X, 2)                                        # full: nothing changes
    assert sorted(np.nonzero(m.bond >= 0)[0].tolist()) == [0, 1, 2, 3] and m.count[0] == 4


def test_ligand_with_three_bonds_takes_one_more():
    X, tri, bary, lig = crowd(5)
    m = model(tri, bary, lig, 16.0, 16.0, k_on0=1e6)
    m.bond[[0, 2, 4]] = 0                               # three bonds already there, none breaks
    m.count[0] = 3
    m.step(X, 1)
    assert m.count[0] == 4 and m.bond[1] == 0 and m.bond[3] == -1


def test_nearest_free_ligand_is_chosen():
    X, tri, bary, lig = crowd(6, nl=2, lig_x=(2.1, 1.6))
    m = model(tri, bary, lig, 16.0, 16.0, k_on0=1e6)
    m.step(X, 1)
    # every receptor is nearer ligand 0 (x = 2.1) than ligand 1 (x = 1.6): four go to 0; the
    # other two found 0 free at the start of the step but lost to lower ids, so stay unbound
    assert m.count.tolist() == [4, 0] and (m.bond[:4] == 0).all() and (m.bond[4:] < 0).all()
    m.step(X, 2)                                        # 0 is now full: the rest go to 1
    assert m.count.tolist() == [4, 2] and (m.bond[4:] == 1).all()


def test_periodic_minimum_image_and_capture_radius():
    X, tri, bary, lig, nx, nz = pairs(1, 0.3)
    X[0] -= X[0].mean() - 0.1                          # receptor at x = 0.1
    lig[0, 0] = 4.0 - 0.2                              # ligand at x = nx - 0.2: 0.3 away through the seam
    m = model(tri, bary, lig, nx, nz, k_on0=1e6)
    m.step(X, 1)
    assert m.bond[0] == 0
    d = m.separation(m.receptor_positions(X), m.bond)
    assert abs(np.linalg.norm(d[:, 0]) - np.hypot(0.3, 0.3)) < 1e-12
    X2, tri, bary, lig, nx, nz = pairs(1, 0.65)        # just outside the capture radius
    m = model(tri, bary, lig, nx, nz, k_on0=1e6)
    m.step(X2, 1)
    assert m.bond[0] == -1


def test_invariants_under_random_motion():
    rng = np.random.default_rng(11)
    nr, nl, nx, nz = 600, 120, 12.0, 10.0
    c = np.stack([rng.uniform(0, nx, nr), rng.uniform(0.0, 0.8, nr), rng.uniform(0, nz, nr)])
    X = np.zeros((3, 3 * nr))
    for k in range(3):
        X[:, k::3] = c + 0.02 * rng.standard_normal((3, nr))
    tri = np.arange(3 * nr).reshape(nr, 3)
    bary = rng.dirichlet(np.ones(3), nr)
    lig = np.stack([rng.uniform(0, nx, nl), rng.uniform(0, nz, nl)], axis=1)
    m = model(tri, bary, lig, nx, nz, k_on0=0.3, k_off0=0.05)
    for s in range(1, 41):
        before = m.bond.copy()
        m.step(X, s)
        assert (m.count == np.bincount(m.bond[m.bond >= 0], minlength=nl)).all()
        assert m.count.max() <= 4
        new = np.nonzero((before < 0) & (m.bond >= 0))[0]
        if len(new):
            d = m.separation(m.receptor_positions(X)[:, new], m.bond[new])
            assert (np.linalg.norm(d, axis=0) < m.capture).all()
        # a bond present before the step either persists unchanged or is gone
        kept = before >= 0
        assert ((m.bond[kept] == before[kept]) | (m.bond[kept] < 0)).all()
        X[1] += 0.01 * rng.standard_normal(X.shape[1])
    assert m.count.sum() > 20


def test_bond_force_is_minus_the_spring_energy_gradient():
    rng = np.random.default_rng(3)
    nr, nx, nz = 40, 10.0, 10.0
    X = np.stack([rng.uniform(0, nx, 3 * nr), rng.uniform(0.1, 0.6, 3 * nr), rng.uniform(0, nz, 3 * nr)])
    tri = np.arange(3 * nr).reshape(nr, 3)
    bary = rng.dirichlet(np.ones(3), nr)
    lig = np.stack([rng.uniform(0, nx, nr), rng.uniform(0, nz, nr)], axis=1)
    m = model(tri, bary, lig, nx, nz)
    m.bond[:] = np.arange(nr)
    m.count[:] = 1
    F = m.forces(X)
    h = 1e-6
    for i in rng.choice(3 * nr, 12, replace=False):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[c, i] += h
            Xm[c, i] -= h
            g = (m.energy(Xp) - m.energy(Xm)) / (2 * h)
            assert abs(F[c, i] + g) < 1e-7 * max(1.0, abs(g))
    # per receptor the node forces add up to the spring force, zero at the rest length
    d = m.separation(m.receptor_positions(X), m.bond)
    L = np.linalg.norm(d, axis=0)
    assert abs(F.sum(axis=1) - (-m.sigma * (L - m.l_b) * d / L).sum(axis=1)).max() < 1e-12
