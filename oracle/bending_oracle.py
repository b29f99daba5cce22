"""FP64 reference of the finite-element bending of the lipid bilayer, section 3.1, Eq. (6)-(10)
and the bending force stated after Eq. (10) (test infrastructure).

TEST INFRASTRUCTURE ONLY: the independent reference the GPU library is checked against.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the GPU library.

What is computed (numpy, float64), on a mesh of quadratic six-node triangles (corners 1-3 and
edge midpoints 4 = m12, 5 = m23, 6 = m31 at the parametric points (0,0), (1,0), (0,1), (1/2,0),
(1/2,1/2), (0,1/2)), with the position interpolated as in Eq. (7):

* At every node k of every element, the tangents a_xi, a_eta, the unit normal n = a_xi x a_eta /
  |.| of the interpolated surface, and its derivatives d n / d xi, d n / d eta (from the second
  derivatives of the interpolated position).  The curvature tensor kappa solves Eq. (9):
  a_xi . kappa = dn/dxi, a_eta . kappa = dn/deta, n . kappa = 0, i.e. kappa = a^xi (x) dn/dxi +
  a^eta (x) dn/deta with a^xi, a^eta the dual tangents.  kappa is averaged over the elements
  sharing the node (and so is n, then normalised).
* K = tr(kappa) / 2 (Eq. 10; K = 1/R on a sphere with outward normals) and the Gaussian
  curvature G = ((tr kappa)^2 - tr(kappa kappa)) / 2.
* The Laplace-Beltrami operator of K the same way: the surface gradient grad K = a^xi dK/dxi +
  a^eta dK/deta of the quadratically interpolated nodal K at every element node, averaged at the
  node; then the surface divergence a^xi . d(grad K)/dxi + a^eta . d(grad K)/deta, averaged.
* Nodal areas A_i: a third of the area of each flat triangle of the element's four
  (1,4,6), (4,2,5), (6,5,3), (4,5,6) that touches the node.
* Energy of Eq. (6): H = k0 sum_i K_i^2 / 2 * A_i.
* Force: the normal force density of the energy's variational derivative,
  f = (k0 / 2) (Lap K + 2 K (K^2 - G)) n, times A_i.  The force printed after Eq. (10) has
  neither the factor k0/2 nor the Gaussian-curvature term -2KG; without that term a sphere would
  feel a force, while with it the force vanishes on any sphere (reading recorded in the design
  notes).  Eq. (8) (the deformation gradient of the in-plane strain) plays no part in the
  curvature and is not used.
"""
from __future__ import annotations

import numpy as np

# parametric coordinates of the six nodes of the quadratic triangle
NODE_XI = np.array([0.0, 1.0, 0.0, 0.5, 0.5, 0.0])
NODE_ETA = np.array([0.0, 0.0, 1.0, 0.0, 0.5, 0.5])
# the four flat sub-triangles (local node numbers) used for the nodal areas
SUBTRI = np.array([[0, 3, 5], [3, 1, 4], [5, 4, 2], [3, 4, 5]])


def shape_derivatives(xi, eta):
    """First derivatives d N_j / d xi, d N_j / d eta of the six quadratic basis functions at
    (xi, eta): N = (z(2z-1), xi(2xi-1), eta(2eta-1), 4 xi z, 4 xi eta, 4 eta z), z = 1-xi-eta."""
    z = 1.0 - xi - eta
    dxi = np.array([-(4 * z - 1), 4 * xi - 1, 0.0, 4 * (z - xi), 4 * eta, -4 * eta])
    deta = np.array([-(4 * z - 1), 0.0, 4 * eta - 1, -4 * xi, 4 * xi, 4 * (z - eta)])
    return dxi, deta


# second derivatives of the basis (constant over the element): d2/dxi2, d2/dxi deta, d2/deta2
D2_XIXI = np.array([4.0, 4.0, 0.0, -8.0, 0.0, 0.0])
D2_XIETA = np.array([4.0, 0.0, 0.0, -4.0, 4.0, -4.0])
D2_ETAETA = np.array([4.0, 0.0, 4.0, 0.0, 0.0, -8.0])

DN = [shape_derivatives(NODE_XI[k], NODE_ETA[k]) for k in range(6)]


def _element_frames(P):
    """For element node positions P [ne, 6, 3]: per element node k, the tangents, dual tangents,
    unit normal and its derivatives.  Returns dicts of arrays [ne, 6, 3]."""
    a11 = np.einsum("j,ejc->ec", D2_XIXI, P)
    a12 = np.einsum("j,ejc->ec", D2_XIETA, P)
    a22 = np.einsum("j,ejc->ec", D2_ETAETA, P)
    out = {k: np.empty(P.shape) for k in ("a1", "a2", "d1", "d2", "n", "dn1", "dn2")}
    for k in range(6):
        dxi, deta = DN[k]
        a1 = np.einsum("j,ejc->ec", dxi, P)
        a2 = np.einsum("j,ejc->ec", deta, P)
        m = np.cross(a1, a2)
        mn = np.linalg.norm(m, axis=1)[:, None]
        n = m / mn
        dm1 = np.cross(a11, a2) + np.cross(a1, a12)
        dm2 = np.cross(a12, a2) + np.cross(a1, a22)
        dn1 = (dm1 - n * np.einsum("ec,ec->e", n, dm1)[:, None]) / mn
        dn2 = (dm2 - n * np.einsum("ec,ec->e", n, dm2)[:, None]) / mn
        g11 = np.einsum("ec,ec->e", a1, a1)
        g12 = np.einsum("ec,ec->e", a1, a2)
        g22 = np.einsum("ec,ec->e", a2, a2)
        det = g11 * g22 - g12 * g12
        d1 = (g22[:, None] * a1 - g12[:, None] * a2) / det[:, None]   # dual tangents a^xi, a^eta
        d2 = (g11[:, None] * a2 - g12[:, None] * a1) / det[:, None]
        for name, v in (("a1", a1), ("a2", a2), ("d1", d1), ("d2", d2), ("n", n), ("dn1", dn1), ("dn2", dn2)):
            out[name][:, k] = v
    return out


def _node_average(E6, vals, n):
    """Mean over the element nodes (e, k) with E6[e, k] = i of vals[e, k, ...]."""
    flat = E6.ravel()
    v = vals.reshape((flat.size,) + vals.shape[2:])
    tot = np.zeros((n,) + vals.shape[2:])
    np.add.at(tot, flat, v)
    cnt = np.bincount(flat, minlength=n).astype(float)
    return tot / cnt.reshape((n,) + (1,) * (vals.ndim - 2))


def _surface_gradient(E6, fr, u):
    """Gradient of the nodal field u [n] (quadratic interpolation) at every element node: [ne, 6, 3]."""
    U = u[E6]
    g = np.empty(E6.shape + (3,))
    for k in range(6):
        dxi, deta = DN[k]
        g[:, k] = fr["d1"][:, k] * (U @ dxi)[:, None] + fr["d2"][:, k] * (U @ deta)[:, None]
    return g


def _surface_divergence(E6, fr, w):
    """Divergence of the nodal vector field w [n, 3] at every element node: [ne, 6]."""
    W = w[E6]                          # [ne, 6, 3]
    d = np.empty(E6.shape)
    for k in range(6):
        dxi, deta = DN[k]
        dW1 = np.einsum("j,ejc->ec", dxi, W)
        dW2 = np.einsum("j,ejc->ec", deta, W)
        d[:, k] = np.einsum("ec,ec->e", fr["d1"][:, k], dW1) + np.einsum("ec,ec->e", fr["d2"][:, k], dW2)
    return d


def nodal_areas(X, E6):
    """A_i: a third of each flat sub-triangle's area at each of its corners ([n])."""
    P = X.T[E6]
    A = np.zeros(X.shape[1])
    for s in SUBTRI:
        a, b, c = P[:, s[0]], P[:, s[1]], P[:, s[2]]
        ar = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
        for j in s:
            np.add.at(A, E6[:, j], ar / 3.0)
    return A


def curvatures(X, E6):
    """Per node: mean curvature K, Gaussian curvature G, unit normal n [n, 3], the averaged
    curvature tensor kappa [n, 3, 3], Lap K and the nodal area A (X: [3, n])."""
    X = np.asarray(X, float)
    n = X.shape[1]
    fr = _element_frames(X.T[E6])
    kap_e = np.einsum("eka,ekb->ekab", fr["d1"], fr["dn1"]) + np.einsum("eka,ekb->ekab", fr["d2"], fr["dn2"])
    kap = _node_average(E6, kap_e, n)
    nrm = _node_average(E6, fr["n"], n)
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    tr = np.einsum("iaa->i", kap)
    K = 0.5 * tr
    G = 0.5 * (tr * tr - np.einsum("iab,iba->i", kap, kap))
    return {"K": K, "G": G, "n": nrm, "kappa": kap, "lapK": _laplace_beltrami(E6, fr, K, n),
            "A": nodal_areas(X, E6)}


def _laplace_beltrami(E6, fr, u, n):
    grad = _node_average(E6, _surface_gradient(E6, fr, u), n)
    return _node_average(E6, _surface_divergence(E6, fr, grad), n)


def laplace_beltrami(X, E6, u):
    """Lap u of a nodal field u [n] by the same node-averaged gradient and divergence that give
    Lap K."""
    X = np.asarray(X, float)
    return _laplace_beltrami(E6, _element_frames(X.T[E6]), np.asarray(u, float), X.shape[1])


def energy(X, E6, k0):
    """Eq. (6) on the mesh: k0 sum_i K_i^2 / 2 A_i."""
    c = curvatures(X, E6)
    return float(k0 * np.sum(0.5 * c["K"] ** 2 * c["A"]))


def forces(X, E6, k0, gaussian=True):
    """Nodal bending forces [3, n]: (k0/2)(Lap K + 2K(K^2 - G)) n A.  gaussian=False drops the
    -2KG term (the force as printed after Eq. (10), scaled by k0/2)."""
    c = curvatures(X, E6)
    K = c["K"]
    cubic = 2.0 * K * (K * K - (c["G"] if gaussian else 0.0))
    f = 0.5 * k0 * (c["lapK"] + cubic) * c["A"]
    return np.ascontiguousarray((f[:, None] * c["n"]).T)
