"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module holds no arithmetic of the method (no lattice-Boltzmann, delta kernel
or force law): only the workload geometry that both sides receive as plain arrays.

* Platelet shape: an oblate ellipsoid (section 3.1, the shape equation with aspect
  ratio lambda), meshed as a subdivided icosahedron (642 / 2562 nodes) or as a
  Fibonacci point set triangulated by its convex hull (any node count, e.g. 1282).
* Mesh topology: undirected edges (the cytoskeleton springs of Eq. (2)-(3)) and
  hinges (pairs of triangles sharing an edge, used by the bending term).
* Placement: uniform in x and z, centroid height uniform in a band above the lower
  wall (plane y = -1/2), bounding spheres kept apart by rejection (periodic
  minimum-image distance in x and z).
* Random draws: numpy PCG64 seeded per workload.

Positions are returned as float64 arrays of shape [3, n] (SoA, as the library takes
them); connectivity as int32.
"""
from __future__ import annotations

import dataclasses
import functools
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------- meshes


def icosphere(level: int):
    """Unit icosphere: 10*4**level + 2 vertices; triangles oriented outward."""
    V, T, _ = _icosphere(level)
    return V, T


def icosphere_quadratic(level: int):
    """The icosphere of `level` >= 1 as six-node triangles: each triangle of level - 1 with its
    three edge midpoints, rows (a, b, c, m_ab, m_bc, m_ca), corners outward.  Returns (V, E6)."""
    if level < 1:
        raise ValueError("six-node triangles need level >= 1")
    V, _, E6 = _icosphere(level)
    return V, E6


def _icosphere(level):
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    T = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        T2, E6 = [], []
        for a, b, c in T:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            T2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
            E6.append((a, b, c, ab, bc, ca))
        T = T2
    V = np.array(V)
    T = np.array(T, dtype=np.int32)
    E6 = np.array(E6 if level > 0 else [], dtype=np.int32).reshape(-1, 6)
    if len(E6):
        # outward corners; reversing (a, b, c) to (a, c, b) renames the midpoints to (ca, bc, ab)
        flip = _orient_outward(V, E6[:, :3])[:, 1] != E6[:, 1]
        E6[flip] = E6[flip][:, [0, 2, 1, 5, 4, 3]]
    return V, _orient_outward(V, T), E6


def fibonacci_sphere(n: int):
    """n points on the unit sphere (golden-angle spiral), triangulated by the convex hull."""
    from scipy.spatial import ConvexHull

    i = np.arange(n) + 0.5
    yv = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - yv * yv)
    ang = np.pi * (3.0 - 5.0 ** 0.5) * np.arange(n)
    V = np.stack([r * np.cos(ang), yv, r * np.sin(ang)], axis=1)
    T = ConvexHull(V).simplices.astype(np.int32)
    return V, _orient_outward(V, T)


def unit_sphere(nodes: int):
    for lev in range(7):
        if 10 * 4 ** lev + 2 == nodes:
            return icosphere(lev)
    return fibonacci_sphere(nodes)


def _orient_outward(V, T):
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cen = (a + b + c) / 3.0
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), cen) < 0
    T = T.copy()
    T[flip, 1], T[flip, 2] = T[flip, 2], T[flip, 1].copy()
    return T


def mesh_edges(T):
    """Unique undirected edges (i < j) of a triangle mesh."""
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0).astype(np.int32)


def mesh_hinges(T):
    """Hinges (x0, x1, x2, x3): triangle (x0,x1,x2) and triangle (x3,x2,x1) share edge x1-x2.
    One hinge per interior edge of a consistently oriented closed mesh."""
    directed = {}
    for t in T:
        for k in range(3):
            a, b, c = int(t[k]), int(t[(k + 1) % 3]), int(t[(k + 2) % 3])
            directed[(b, c)] = a  # directed edge b->c, opposite vertex a
    H = []
    for (b, c), a in directed.items():
        if b < c and (c, b) in directed:
            H.append((a, b, c, directed[(c, b)]))
    return np.array(H, dtype=np.int32).reshape(-1, 4)


def csr_neighbours(n, edges):
    """CSR adjacency (both directions) of an undirected edge list: ptr[n+1], idx[nnz]."""
    src = np.concatenate([edges[:, 0], edges[:, 1]])
    dst = np.concatenate([edges[:, 1], edges[:, 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, src + 1, 1)
    return np.cumsum(ptr).astype(np.int32), dst.astype(np.int32)


def csr_hinges(n, hinges):
    """CSR incidence node -> (hinge << 2 | role), role 0..3 = position in the hinge tuple."""
    nh = len(hinges)
    node = hinges.reshape(-1).astype(np.int64)
    code = (np.repeat(np.arange(nh, dtype=np.int64), 4) << 2) | np.tile(np.arange(4), nh)
    order = np.lexsort((code, node))
    node, code = node[order], code[order]
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, node + 1, 1)
    return np.cumsum(ptr).astype(np.int32), code.astype(np.int32)


def csr_elements(n, E6):
    """CSR incidence node -> (element << 3 | local node), local node 0..5; per node in element
    order."""
    ne = len(E6)
    node = np.asarray(E6, np.int64).reshape(-1)
    code = (np.repeat(np.arange(ne, dtype=np.int64), 6) << 3) | np.tile(np.arange(6), ne)
    order = np.lexsort((code, node))
    node, code = node[order], code[order]
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, node + 1, 1)
    return np.cumsum(ptr).astype(np.int32), code.astype(np.int32)


def csr_receptors(n, rec_tri):
    """CSR incidence node -> (receptor << 2 | corner), corner 0..2; per node in receptor order."""
    nr = len(rec_tri)
    node = np.asarray(rec_tri, np.int64).reshape(-1)
    code = (np.repeat(np.arange(nr, dtype=np.int64), 3) << 2) | np.tile(np.arange(3), nr)
    order = np.lexsort((code, node))
    node, code = node[order], code[order]
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, node + 1, 1)
    return np.cumsum(ptr).astype(np.int32), code.astype(np.int32)


def csr_triangles(n, tri):
    """CSR incidence node -> (triangle << 2 | corner), corner 0..2 = position in the triangle."""
    nt = len(tri)
    node = np.asarray(tri).reshape(-1).astype(np.int64)
    code = (np.repeat(np.arange(nt, dtype=np.int64), 3) << 2) | np.tile(np.arange(3), nt)
    order = np.lexsort((code, node))
    node, code = node[order], code[order]
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, node + 1, 1)
    return np.cumsum(ptr).astype(np.int32), code.astype(np.int32)


# ----------------------------------------------------------------------------- bodies


@dataclass
class Bodies:
    """Lagrangian nodes of all immersed bodies of one channel (global node numbering)."""
    X: np.ndarray                 # [3, n] float64 initial positions
    X_rest: np.ndarray            # [3, n] float64 rest shape (springs / hinges measured on it)
    edges: np.ndarray             # [ne, 2] int32 spring edges
    hinges: np.ndarray            # [nh, 4] int32 bending hinges
    anchors: np.ndarray | None    # [3, n] tether anchors or None
    k_spring: float = 0.0
    k_bend: float = 0.0
    k_tether: float = 0.0
    body_offsets: list = field(default_factory=list)   # node offset of each body, plus n
    # area and volume constraints of Eq. (4)-(5) (off unless triangles are set; with_constraints)
    triangles: np.ndarray | None = None   # [nt, 3] int32, outward, each body's contiguous
    tri_offsets: list = field(default_factory=list)    # triangle offset of each body, plus nt
    k_area_global: float = 0.0
    k_area_local: float = 0.0
    k_volume: float = 0.0
    # finite-element bending of Eq. (6)-(10) (off unless elements are set; with_fe_bending)
    elements6: np.ndarray | None = None   # [ne, 6] int32 six-node triangles, corners outward
    k_fe: float = 0.0                      # k_0 of Eq. (6)

    @property
    def n(self):
        return self.X.shape[1]


def with_constraints(b, k_area_global=0.0, k_area_local=0.0, k_volume=0.0):
    """The same bodies with the area and volume constraints of Eq. (4)-(5): the outward
    triangles of each body's sphere mesh (the mesh its nodes were made from), with the given
    coefficients.  Rest areas and volumes are measured on X_rest by the library and the oracle."""
    T, offs = [], [0]
    for lo, hi in zip(b.body_offsets[:-1], b.body_offsets[1:]):
        Tb = _topology(hi - lo)[1] + lo
        T.append(Tb)
        offs.append(offs[-1] + len(Tb))
    # the triangles must be those of the bodies' own meshes: their edges are the spring edges
    tri_edges = mesh_edges(np.concatenate(T))
    springs = np.unique(np.sort(np.asarray(b.edges, np.int64), axis=1), axis=0)
    if len(b.edges) == 0 or not np.array_equal(tri_edges.astype(np.int64), springs):
        raise ValueError("with_constraints needs bodies built from the sphere meshes (platelets)")
    return dataclasses.replace(b, triangles=np.concatenate(T).astype(np.int32), tri_offsets=offs,
                               k_area_global=float(k_area_global), k_area_local=float(k_area_local),
                               k_volume=float(k_volume))


def with_fe_bending(b, k0):
    """The same bodies with the finite-element bending of Eq. (6)-(10) (modulus k0) in place of
    the dihedral stand-in: each body's icosphere mesh as six-node triangles (its nodes are the
    corners and edge midpoints of the icosphere one level down)."""
    E, off = [], 0
    for lo, hi in zip(b.body_offsets[:-1], b.body_offsets[1:]):
        E.append(_quadratic(hi - lo) + lo)
    E = np.concatenate(E).astype(np.int32)
    # the six-node triangles must be the bodies' own meshes: their half-edges are spring edges
    half = np.concatenate([E[:, [0, 3]], E[:, [3, 1]], E[:, [1, 4]], E[:, [4, 2]], E[:, [2, 5]], E[:, [5, 0]]])
    springs = {tuple(e) for e in np.sort(np.asarray(b.edges, np.int64), axis=1).tolist()}
    if len(b.edges) == 0 or any(tuple(e) not in springs for e in np.sort(half, axis=1).tolist()):
        raise ValueError("with_fe_bending needs bodies built from icosphere meshes (642, 2562, ... nodes)")
    return dataclasses.replace(b, elements6=E, k_fe=float(k0), k_bend=0.0)


def table2_bending_modulus():
    """k_0 of Table 2 (200 k_B T at 300 K) in lattice units (energy unit rho h^5 / dt^2 with
    h = 0.2 um, dt = 1e-8 s, plasma density 1.0239 g/cm^3)."""
    h, dt, rho = 0.2e-6, 1e-8, 1023.9
    return 200.0 * 1.380649e-23 * 300.0 / (rho * h ** 5 / dt ** 2)


def receptor_points(b, per_body=5344, seed=0):
    """Receptor points of the adhesion model (section 3.2: 5344 per platelet, each standing for two
    GPIb-alpha receptors), uniform over each body's rest surface: a triangle of the body's sphere
    mesh drawn with probability proportional to its rest area, then uniform barycentric weights.
    Returns (rec_tri [nr, 3] int32 node ids, rec_bary [nr, 3] float64)."""
    rng = np.random.default_rng(seed)
    T_all, W_all = [], []
    for lo, hi in zip(b.body_offsets[:-1], b.body_offsets[1:]):
        T = _topology(hi - lo)[1] + lo
        P = b.X_rest.T[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        t = rng.choice(len(T), size=per_body, p=area / area.sum())
        u1, u2 = rng.uniform(size=per_body), rng.uniform(size=per_body)
        s1 = np.sqrt(u1)
        W_all.append(np.stack([1.0 - s1, s1 * (1.0 - u2), s1 * u2], axis=1))
        T_all.append(T[t])
    return np.concatenate(T_all).astype(np.int32), np.concatenate(W_all)


def wall_ligands(nx, nz, density=1.0, seed=0):
    """Immobilised ligand (vWF) points on the lower wall, uniform over the nx x nz plane:
    round(density nx nz) of them, as (x, z) [nl, 2] float64 (25 per um^2 is 1.0 per lattice
    unit^2 at h = 0.2 um)."""
    rng = np.random.default_rng(seed)
    nl = int(round(density * nx * nz))
    return np.stack([rng.uniform(0.0, nx, nl), rng.uniform(0.0, nz, nl)], axis=1)


def table2_adhesion(sigma_si=1e-3, l_b_si=128e-9, gamma_si=0.7e-9):
    """Adhesion parameters in lattice units (h = 0.2 um, dt = 1e-8 s, plasma density
    1.0239 g/cm^3): per-step rates k_on0 dt and k_off0 dt of Table 2 (1e-5 and 3.45 per s), kT at
    300 K, the capture radius (the 128 nm bond length of section 3.2) and the receptor and ligand
    densities of section 3.2.  The spring constant sigma (N/m), the rest length l_b (m) and the
    reactive compliance gamma (m) are not in Table 2: the caller supplies them (the default rest
    length is the bond length of section 3.2; sigma and gamma default to assumptions of this
    workload, not values of the paper)."""
    h, dt, rho = 0.2e-6, 1e-8, 1023.9
    force = rho * h ** 4 / dt ** 2
    energy = rho * h ** 5 / dt ** 2
    return dict(k_on0=1e-5 * dt, k_off0=3.45 * dt, kT=1.380649e-23 * 300.0 / energy, capture=128e-9 / h,
                sigma=sigma_si / (force / h), l_b=l_b_si / h, gamma=gamma_si / h, receptors_per_body=5344,
                ligand_density=25e12 * h * h)


def table2_constraint_coefficients():
    """k_s, k_t, k_v of Table 2 (6000 k_B T / l_0^2, 6000 k_B T / l_0^2, 6000 k_B T / l_0^3) in
    lattice units: spacing h = 0.2 um and step dt = 1e-8 s (section 3.3), plasma density
    1.0239 g/cm^3, T = 300 K and l_0 = 75 nm (Table 2).  Energy unit rho h^5 / dt^2."""
    h, dt, rho = 0.2e-6, 1e-8, 1023.9
    kT = 1.380649e-23 * 300.0 / (rho * h ** 5 / dt ** 2)
    l0 = 75e-9 / h
    return 6000.0 * kT / l0 ** 2, 6000.0 * kT / l0 ** 2, 6000.0 * kT / l0 ** 3


def morton_order(V, bits=10):
    """Permutation that numbers points along a Morton (Z-order) curve of their position, so
    that nodes with nearby numbers are nearby in space."""
    lo, hi = V.min(axis=0), V.max(axis=0)
    q = ((V - lo) / np.maximum(hi - lo, 1e-30) * ((1 << bits) - 1)).astype(np.int64)
    code = np.zeros(len(V), np.int64)
    for b in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def renumber(V, T, order):
    """Renumber vertices so that new vertex k is old vertex order[k]."""
    inv = np.empty(len(order), np.int64)
    inv[order] = np.arange(len(order))
    return V[order], inv[T].astype(np.int32)


@functools.lru_cache(maxsize=None)
def _topology(nodes):
    V0, T = unit_sphere(nodes)
    V0, T = renumber(V0, T, morton_order(V0))
    return V0, T, mesh_edges(T), mesh_hinges(T)


@functools.lru_cache(maxsize=None)
def _quadratic(nodes):
    """Six-node triangles of the icosphere mesh of `nodes` nodes, in _topology's numbering."""
    for lev in range(1, 7):
        if 10 * 4 ** lev + 2 == nodes:
            V0, E6 = icosphere_quadratic(lev)
            order = morton_order(V0)
            inv = np.empty(len(order), np.int64)
            inv[order] = np.arange(len(order))
            return inv[E6].astype(np.int32)
    raise ValueError("six-node triangles exist for icosphere node counts only, not %d" % nodes)


def _concat(parts):
    Xs, edges, hinges, offs, off = [], [], [], [0], 0
    for V, nodes in parts:
        _, _, E, H = _topology(nodes)
        Xs.append(V)
        edges.append(E + off)
        hinges.append(H + off)
        off += len(V)
        offs.append(off)
    X = np.ascontiguousarray(np.concatenate(Xs).T)
    return X, np.concatenate(edges).astype(np.int32), np.concatenate(hinges).astype(np.int32), offs


def place_bodies(rng, nx, nz, count, radius, y_lo, y_hi, max_tries=4000):
    """Centres uniform in x,z and in [y_lo, y_hi]; bounding spheres of `radius` kept apart
    (periodic minimum image in x and z).  Returns fewer centres if the box is full."""
    C = []
    tries = 0
    while len(C) < count and tries < max_tries * count:
        tries += 1
        c = np.array([rng.uniform(0, nx), rng.uniform(y_lo, y_hi), rng.uniform(0, nz)])
        ok = True
        for d in C:
            dx = abs(c[0] - d[0]); dx = min(dx, nx - dx)
            dz = abs(c[2] - d[2]); dz = min(dz, nz - dz)
            if dx * dx + (c[1] - d[1]) ** 2 + dz * dz < (2 * radius) ** 2:
                ok = False
                break
        if ok:
            C.append(c)
    return np.array(C).reshape(-1, 3)


def platelets(rng, nx, ny, nz, count, semi_axes, nodes, y_band, k_spring, k_bend, margin=2.0):
    """Oblate platelets: unit sphere mesh scaled by semi_axes (x, y, z) (short axis along the
    wall normal y), centres from place_bodies.  Rest shape = initial shape."""
    a = np.asarray(semi_axes, float)
    V0 = _topology(nodes)[0]
    y_lo = -0.5 + y_band[0]
    y_hi = min(-0.5 + y_band[1], ny - 0.5 - a[1] - 2.0)
    cen = place_bodies(rng, nx, nz, count, float(a.max()) + margin, y_lo, y_hi)
    parts = [(V0 * a[None, :] + c[None, :], nodes) for c in cen]
    X, edges, hinges, offs = _concat(parts)
    return Bodies(X=X, X_rest=X.copy(), edges=edges, hinges=hinges, anchors=None,
                  k_spring=k_spring, k_bend=k_bend, body_offsets=offs)


def tethered_sphere(rng, centre, radius, nodes, k_tether, sigma):
    """Sphere whose nodes are tied to their rest positions; initial positions perturbed by
    N(0, sigma^2) per component."""
    V0, T = unit_sphere(nodes)
    X_rest = np.ascontiguousarray((V0 * radius + np.asarray(centre, float)[None, :]).T)
    X = X_rest + rng.normal(0.0, sigma, size=X_rest.shape)
    return Bodies(X=np.ascontiguousarray(X), X_rest=X_rest, edges=np.zeros((0, 2), np.int32),
                  hinges=np.zeros((0, 4), np.int32), anchors=X_rest.copy(), k_tether=k_tether,
                  body_offsets=[0, X.shape[1]])


# ----------------------------------------------------------------------------- workloads


@dataclass
class Channel:
    nx: int
    ny: int
    nz: int
    tau: float
    body: tuple = (0.0, 0.0, 0.0)
    u_wall_lo: tuple = (0.0, 0.0, 0.0)
    u_wall_hi: tuple = (0.0, 0.0, 0.0)
    walls: bool | str = True      # False, True (halfway bounce-back) or "onsite" (Eq. 23-30)
    init: str = "rest"            # "rest" (u = 0) or "shear" (linear wall-driven profile)
    bodies: Bodies | None = None

    @property
    def cells(self):
        return self.nx * self.ny * self.nz


def poiseuille_sphere(seed=0, n=32):
    """Plain method: 32^3 box, tau = 0.8, walls normal to y, body force 1e-6 along x;
    one tethered sphere of 642 nodes, radius 4, centred at (16, 10, 16), k = 0.01,
    rest positions perturbed by N(0, 0.1^2)."""
    rng = np.random.default_rng(seed)
    b = tethered_sphere(rng, (n / 2, 10.0, n / 2), 4.0, 642, 0.01, 0.1)
    return Channel(n, n, n, 0.8, body=(1e-6, 0.0, 0.0), bodies=b)


def shear_platelets(seed=0, nx=256, ny=128, nz=128, count=16, nodes=2562, semi_axes=(6.0, 2.0, 6.0),
                    tau=1.0, u_top=0.05, k_spring=0.005, k_bend=1e-4, y_band=(8.0, 20.0)):
    """Production shear: moving top wall (u_top along x), resting bottom wall, linear Couette
    start; `count` oblate platelets with spring network + bending, centroids 8-20 lattice
    units above the bottom wall."""
    rng = np.random.default_rng(seed)
    b = platelets(rng, nx, ny, nz, count, semi_axes, nodes, y_band, k_spring, k_bend)
    return Channel(nx, ny, nz, tau, u_wall_hi=(u_top, 0.0, 0.0), init="shear", bodies=b)


def jeffery_platelet(n=64, nodes=642, semi_axes=(6.0, 2.0, 6.0), u_top=0.05, tau=1.0, seed=0,
                     k_spring=0.005, k_bend=1e-4):
    """Jeffery-orbit workload (section 4.1): an n x n x n shear channel (moving top wall,
    resting bottom wall, linear Couette start) with one oblate platelet, short axis along y,
    at its centre, as far from the walls as the box allows."""
    a = np.asarray(semi_axes, float)
    V = _topology(nodes)[0]
    c = np.array([(n - 1) / 2.0, (n - 1) / 2.0, (n - 1) / 2.0])
    X, E, H, O = _concat([(V * a[None, :] + c[None, :], nodes)])
    b = Bodies(X=X, X_rest=X.copy(), edges=E, hinges=H, anchors=None, k_spring=k_spring, k_bend=k_bend,
               body_offsets=O)
    return Channel(n, n, n, tau, u_wall_hi=(u_top, 0.0, 0.0), init="shear", bodies=b)


def _suspension_centres(seed, count, fine, semi_axes, y_band):
    rng = np.random.default_rng(seed)
    nx, ny, nz = fine
    a = np.asarray(semi_axes, float)
    y_lo = -0.5 + y_band[0]
    y_hi = min(-0.5 + y_band[1], ny - 0.5 - a[1] - 2.0)
    return place_bodies(rng, nx, nz, count, float(a.max()) + 2.0, y_lo, y_hi)


def _scaled_channel(cen, r, nodes, fine, tau_f, u_top, semi_axes, k_spring, k_bend):
    """The suspension with fine-lattice centres `cen` on the lattice r times as fine (acoustic
    scaling: dx and dt both grow by 1/r, lattice velocities are unchanged).  A fine point x_f
    sits at x = (x_f + 1/2) r - 1/2, so the wall planes y = -1/2 and y = ny - 1/2 map onto each
    other; semi-axes scale by r; tau = 1/2 + (tau_f - 1/2) r keeps the physical viscosity;
    the membrane stiffness k dt^2/(rho dx^3) scales by r and the bending energy
    k_b dt^2/(rho dx^5) by r^3."""
    nx, ny, nz = (int(round(d * r)) for d in fine)
    a = np.asarray(semi_axes, float) * r
    V = _topology(nodes)[0]
    X, E, H, O = _concat([(V * a[None, :] + (c * r + (r - 1.0) / 2)[None, :], nodes) for c in cen])
    b = Bodies(X=X, X_rest=X.copy(), edges=E, hinges=H, anchors=None, k_spring=k_spring * r,
               k_bend=k_bend * r ** 3, body_offsets=O)
    return Channel(nx, ny, nz, 0.5 + (tau_f - 0.5) * r, u_wall_hi=(u_top, 0.0, 0.0), init="shear", bodies=b)


def coarse_fine_pair(seed=0, u_top=0.05, count=16, fine=(256, 128, 128), tau_f=1.0, nodes_f=2562,
                     nodes_c=1282, semi_axes=(6.0, 2.0, 6.0), k_spring=0.005, k_bend=1e-4, y_band=(8.0, 20.0)):
    """The same platelet suspension on a fine lattice and on the 2x coarser one (acoustic
    scaling: dx_c = 2 dx_f, dt_c = 2 dt_f, so lattice velocities are equal and
    tau_c = 1/2 + (tau_f - 1/2)/2).  Platelet centres are drawn once in fine units; a fine
    point x_f sits at x_c = (x_f - 1/2)/2 on the coarse lattice (cell centres at integers on
    both).  Coarse platelets have half the semi-axes and `nodes_c` nodes; their spring and
    bending constants follow the same scaling (membrane stiffness k dt^2/(rho dx^3) halves,
    bending energy k_b dt^2/(rho dx^5) drops by 8).  Returns (fine Channel, coarse Channel)."""
    cen = _suspension_centres(seed, count, fine, semi_axes, y_band)
    kw = dict(fine=fine, tau_f=tau_f, u_top=u_top, semi_axes=semi_axes, k_spring=k_spring, k_bend=k_bend)
    return _scaled_channel(cen, 1.0, nodes_f, **kw), _scaled_channel(cen, 0.5, nodes_c, **kw)


def resolution_ladder(seed=0, sizes=(128, 160, 192, 224, 256), u_top=0.05, count=16, fine=(256, 128, 128),
                      tau_f=1.0, semi_axes=(6.0, 2.0, 6.0), k_spring=0.005, k_bend=1e-4, y_band=(8.0, 20.0)):
    """The suspension of coarse_fine_pair(seed) at several resolutions (lattice length in x
    from `sizes`; the other dimensions in proportion), all acoustically scaled from the fine
    one: returns {nx: (Channel, r)} with r = nx / fine nx.  Platelets of r < 3/4 carry 1282
    nodes, finer ones 2562 (node spacing below one lattice unit on every rung).  The rungs
    nx = fine and nx = fine / 2 are exactly the two channels of coarse_fine_pair."""
    cen = _suspension_centres(seed, count, fine, semi_axes, y_band)
    kw = dict(fine=fine, tau_f=tau_f, u_top=u_top, semi_axes=semi_axes, k_spring=k_spring, k_bend=k_bend)
    out = {}
    for n in sizes:
        r = n / fine[0]
        if any(abs(d * r - round(d * r)) > 1e-9 for d in fine):
            raise ValueError("rung %d does not scale the lattice %s to whole cells" % (n, fine))
        out[n] = (_scaled_channel(cen, r, 2562 if r >= 0.75 else 1282, **kw), r)
    return out


BATCH_SIZES = [(48, 32, 32), (64, 48, 48), (96, 64, 64), (128, 64, 64)]


def batched_channels(seed=0, nch=64, sizes=BATCH_SIZES):
    """Independent channels of uneven size: dims uniform over `sizes`, 1-8 platelets of 642 or
    2562 nodes, top-wall speed U(0.01, 0.05), tau U(0.7, 1.2)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nch):
        nx, ny, nz = sizes[rng.integers(len(sizes))]
        count = int(rng.integers(1, 9))
        nodes = int(rng.choice([642, 2562]))
        u = float(rng.uniform(0.01, 0.05))
        tau = float(rng.uniform(0.7, 1.2))
        band = (8.0, min(20.0, ny - 10.0))
        b = platelets(rng, nx, ny, nz, count, (6.0, 2.0, 6.0), nodes, band, 0.005, 1e-4)
        out.append(Channel(nx, ny, nz, tau, u_wall_hi=(u, 0.0, 0.0), init="shear", bodies=b))
    return out


def concat_bodies(channels):
    """Bodies of several channels in one global node numbering (channel order), and the
    node offsets of the channels (len(channels) + 1 entries)."""
    Xs, Xr, E, H, A, offs = [], [], [], [], [], [0]
    T, TO, E6, kf = [], [0], [], set()
    off = 0
    ks, kc = set(), set()
    for ch in channels:
        b = ch.bodies
        if b.triangles is not None:
            T.append(b.triangles + off)
            TO += [o + TO[-1] for o in b.tri_offsets[1:]]
        kc.add((b.k_area_global, b.k_area_local, b.k_volume))
        if b.elements6 is not None:
            E6.append(b.elements6 + off)
        kf.add(b.k_fe)
        Xs.append(b.X)
        Xr.append(b.X_rest)
        E.append(b.edges + off)
        H.append(b.hinges + off)
        if b.anchors is not None:
            A.append(b.anchors)
        ks.add((b.k_spring, b.k_bend, b.k_tether))
        off += b.n
        offs.append(off)
    if len(ks) != 1 or len(kc) != 1 or len(kf) != 1 or len(T) not in (0, len(channels)) or \
            len(E6) not in (0, len(channels)):
        raise ValueError("channels must share the membrane constants")
    k_spring, k_bend, k_tether = ks.pop()
    k_area_global, k_area_local, k_volume = kc.pop()
    anchors = np.ascontiguousarray(np.concatenate(A, axis=1)) if A and len(A) == len(channels) else None
    b = Bodies(X=np.ascontiguousarray(np.concatenate(Xs, axis=1)), X_rest=np.ascontiguousarray(np.concatenate(Xr, axis=1)),
               edges=np.concatenate(E).astype(np.int32), hinges=np.concatenate(H).astype(np.int32), anchors=anchors,
               k_spring=k_spring, k_bend=k_bend, k_tether=k_tether, body_offsets=offs,
               triangles=np.concatenate(T).astype(np.int32) if T else None, tri_offsets=TO if T else [],
               k_area_global=k_area_global, k_area_local=k_area_local, k_volume=k_volume,
               elements6=np.concatenate(E6).astype(np.int32) if E6 else None, k_fe=kf.pop())
    return b, offs
