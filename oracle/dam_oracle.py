"""FP64 reference of the stochastic dynamic adhesion submodel (DAM) of section 3.2, Eq. (12)-(14)
(test infrastructure).

TEST INFRASTRUCTURE ONLY: the independent reference the GPU library is checked against.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the GPU library.

Model (lattice units; the per-step rates are rate times the time step):

* Receptor points sit on the membrane: receptor r lies in triangle (a, b, c) at barycentric
  weights (w_a, w_b, w_c), so its position is w_a X_a + w_b X_b + w_c X_c.  Ligands (the
  immobilised vWF) are points (x, z) on the lower wall plane y = y_w (x and z periodic).
* A bond joins one receptor to one ligand: a receptor holds at most one bond (rule 1 of
  section 3.2, steric blocking) and a ligand at most four (rule 2).
* Bond force (Eq. (14) as a linear spring of rest length l_b along the bond): with
  d = X_r - L, F_r = -sigma (|d| - l_b) d / |d|, shared among the triangle's nodes by the
  barycentric weights (the gradient of sigma/2 (|d| - l_b)^2 with respect to the nodes).
* One Monte-Carlo step at the positions after the move (the last box of Fig. 1):
  1. every bond present at the start of the step breaks with probability
     P_r = 1 - exp(-k_off dt), k_off = k_off0 exp(gamma F_b / kT) (Eq. (12), Bell), F_b = sigma
     | |d| - l_b |;
  2. every receptor unbound at the start of the step picks the nearest ligand (the lower id on a
     tie) closer than the capture radius (128 nm in the paper) among those with fewer than four
     bonds at the start of the step, and proposes a bond with probability P_f = 1 - exp(-k_on dt),
     k_on = k_on0 exp(sigma |x_b - l_b| (gamma - |x_b - l_b| / 2) / kT) (Eq. (13) as printed),
     x_b = |d|;
  3. every ligand accepts the proposals it received in ascending receptor id while its bonds
     after this step's breaks plus those accepted stay at most four.
* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011), key (seed mod 2^32,
  seed div 2^32), counter (receptor, step mod 2^32, step div 2^32, 0); words 0-1 give the
  breaking uniform and words 2-3 the forming uniform, each as (w_a >> 5) 2^-27 + (w_b >> 6) 2^-53
  in [0, 1); an event happens when the uniform is below its probability.
"""
from __future__ import annotations

import numpy as np

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key, rounds=10):
    """Philox4x32 on arrays of counters: counter = 4 arrays (or ints), key = 2; returns 4 uint64
    arrays holding 32-bit words."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in counter]
    k0, k1 = (np.asarray(x, dtype=np.uint64) & _MASK for x in key)
    m0, m1 = np.uint64(PHILOX_M[0]), np.uint64(PHILOX_M[1])
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W[0])) & _MASK
            k1 = (k1 + np.uint64(PHILOX_W[1])) & _MASK
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniform53(wa, wb):
    """A double in [0, 1) from two 32-bit words: 27 bits of wa and 26 of wb."""
    hi = (np.asarray(wa, dtype=np.uint64) >> np.uint64(5)).astype(np.float64)
    lo = (np.asarray(wb, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    return hi * 2.0 ** -27 + lo * 2.0 ** -53


def uniforms(seed, step, receptors):
    """(breaking, forming) uniforms of the given receptors at `step`."""
    r = np.asarray(receptors, dtype=np.uint64)
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    ctr = (r, np.full_like(r, step & 0xFFFFFFFF), np.full_like(r, (step >> 32) & 0xFFFFFFFF), np.zeros_like(r))
    w = philox4x32(ctr, key)
    return uniform53(w[0], w[1]), uniform53(w[2], w[3])


def off_rate(Fb, k_off0, gamma, kT):
    """Eq. (12)."""
    return k_off0 * np.exp(gamma * Fb / kT)


def on_rate(xb, k_on0, sigma, l_b, gamma, kT):
    """Eq. (13) as printed."""
    s = np.abs(xb - l_b)
    return k_on0 * np.exp(sigma * s * (gamma - 0.5 * s) / kT)


class Adhesion:
    """Receptors, ligands and bonds of one wall; see the module docstring."""

    def __init__(self, rec_tri, rec_bary, ligands, wall_y, nx, nz, capture, sigma, l_b, gamma, kT, k_on0,
                 k_off0, seed):
        self.rec_tri = np.asarray(rec_tri, dtype=np.int64).reshape(-1, 3)
        self.rec_bary = np.asarray(rec_bary, dtype=np.float64).reshape(-1, 3)
        self.lig = np.asarray(ligands, dtype=np.float64).reshape(-1, 2)   # (x, z)
        self.wall_y, self.nx, self.nz = float(wall_y), float(nx), float(nz)
        self.capture, self.sigma, self.l_b, self.gamma, self.kT = map(float, (capture, sigma, l_b, gamma, kT))
        self.k_on0, self.k_off0 = float(k_on0), float(k_off0)
        self.seed = int(seed)
        self.bond = np.full(len(self.rec_tri), -1, dtype=np.int64)
        self.count = np.zeros(len(self.lig), dtype=np.int64)

    # ---------------------------------------------------------------- geometry
    def receptor_positions(self, X):
        X = np.asarray(X, dtype=np.float64)
        return np.einsum("rk,crk->cr", self.rec_bary, X[:, self.rec_tri])

    def separation(self, Xr, lig):
        """d = X_r - L for receptor positions Xr [3, m] and ligand ids lig [m] (x, z minimum image)."""
        d = np.empty_like(Xr)
        dx = Xr[0] - self.lig[lig, 0]
        dz = Xr[2] - self.lig[lig, 1]
        d[0] = dx - self.nx * np.round(dx / self.nx)
        d[1] = Xr[1] - self.wall_y
        d[2] = dz - self.nz * np.round(dz / self.nz)
        return d

    # ---------------------------------------------------------------- forces (Eq. (14))
    def energy(self, X):
        on = np.nonzero(self.bond >= 0)[0]
        if len(on) == 0:
            return 0.0
        d = self.separation(self.receptor_positions(X)[:, on], self.bond[on])
        return float(np.sum(0.5 * self.sigma * (np.linalg.norm(d, axis=0) - self.l_b) ** 2))

    def forces(self, X):
        X = np.asarray(X, dtype=np.float64)
        F = np.zeros_like(X)
        on = np.nonzero(self.bond >= 0)[0]
        if len(on) == 0:
            return F
        d = self.separation(self.receptor_positions(X)[:, on], self.bond[on])
        L = np.linalg.norm(d, axis=0)
        Fr = -self.sigma * (L - self.l_b) * d / L
        for k in range(3):
            for c in range(3):
                np.add.at(F[c], self.rec_tri[on, k], self.rec_bary[on, k] * Fr[c])
        return F

    # ---------------------------------------------------------------- Monte-Carlo step
    def nearest_free_ligand(self, Xr, count0):
        """Per receptor position (columns of Xr): the nearest ligand with fewer than four bonds
        closer than the capture radius (lower id on a tie), or -1; and that distance.  Ligands are
        looked up in a table of wall cells at least one capture radius wide (the 3 x 3 cells
        around a receptor hold every ligand in reach)."""
        m = Xr.shape[1]
        best = np.full(m, -1, dtype=np.int64)
        bestd = np.full(m, np.inf)
        near = np.nonzero(np.abs(Xr[1] - self.wall_y) < self.capture)[0]
        free = np.nonzero(count0 < 4)[0]
        if len(near) == 0 or len(free) == 0:
            return best, bestd
        cx = max(1, int(self.nx // self.capture))
        cz = max(1, int(self.nz // self.capture))
        lx = np.minimum((self.lig[free, 0] / self.nx * cx).astype(np.int64), cx - 1)
        lz = np.minimum((self.lig[free, 1] / self.nz * cz).astype(np.int64), cz - 1)
        cell = lz * cx + lx
        order = np.argsort(cell, kind="stable")
        start = np.searchsorted(cell[order], np.arange(cx * cz + 1))
        occ = int(np.diff(start).max())
        table = np.full((cx * cz, occ), -1, dtype=np.int64)      # free ligand ids per cell
        for c in np.nonzero(np.diff(start))[0]:
            table[c, :start[c + 1] - start[c]] = free[order[start[c]:start[c + 1]]]
        rx = np.floor(np.mod(Xr[0, near], self.nx) / self.nx * cx).astype(np.int64) % cx
        rz = np.floor(np.mod(Xr[2, near], self.nz) / self.nz * cz).astype(np.int64) % cz
        cand = np.concatenate([table[((rz + dz) % cz) * cx + (rx + dx) % cx]
                               for dz in (-1, 0, 1) for dx in (-1, 0, 1)], axis=1)   # [near, 9 occ]
        ok = cand >= 0
        safe = np.where(ok, cand, 0)
        dx = Xr[0, near][:, None] - self.lig[safe, 0]
        dz = Xr[2, near][:, None] - self.lig[safe, 1]
        dx -= self.nx * np.round(dx / self.nx)
        dz -= self.nz * np.round(dz / self.nz)
        dy = (Xr[1, near] - self.wall_y)[:, None]
        dist = np.sqrt(dx * dx + dy * dy + dz * dz)
        dist = np.where(ok & (dist < self.capture), dist, np.inf)
        dmin = dist.min(axis=1)
        hit = np.isfinite(dmin)
        # the lowest id among the candidates at the minimum distance (a small grid lists a ligand
        # in several of the nine cells; the duplicates agree)
        ids = np.where(dist == dmin[:, None], cand, np.iinfo(np.int64).max)
        best[near[hit]] = ids[hit].min(axis=1)
        bestd[near[hit]] = dmin[hit]
        return best, bestd

    def step(self, X, step):
        """One Monte-Carlo step at positions X; returns (breaks, new bonds)."""
        Xr = self.receptor_positions(X)
        nr = Xr.shape[1]
        ub, uf = uniforms(self.seed, int(step), np.arange(nr))
        count0 = self.count.copy()
        bound0 = self.bond >= 0
        # 1. breaks
        on = np.nonzero(bound0)[0]
        broken = np.zeros(nr, dtype=bool)
        if len(on):
            d = self.separation(Xr[:, on], self.bond[on])
            Fb = self.sigma * np.abs(np.linalg.norm(d, axis=0) - self.l_b)
            Pr = 1.0 - np.exp(-off_rate(Fb, self.k_off0, self.gamma, self.kT))
            broken[on] = ub[on] < Pr
        after = count0.copy()
        for r in np.nonzero(broken)[0]:
            after[self.bond[r]] -= 1
            self.bond[r] = -1
        # 2. proposals by the receptors unbound at the start
        cand, dist = self.nearest_free_ligand(Xr, count0)
        proposals = []
        for r in np.nonzero((~bound0) & (cand >= 0))[0]:
            Pf = 1.0 - np.exp(-on_rate(dist[r], self.k_on0, self.sigma, self.l_b, self.gamma, self.kT))
            if uf[r] < Pf:
                proposals.append((cand[r], r))
        # 3. acceptance in ascending receptor id per ligand
        formed = 0
        for lig, r in sorted(proposals):
            if after[lig] < 4:
                after[lig] += 1
                self.bond[r] = lig
                formed += 1
        self.count = after
        return int(broken.sum()), formed
