"""FP64 reference of the learned collision closure (test infrastructure).

TEST INFRASTRUCTURE ONLY: the independent reference that the GPU closure kernels are
checked against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; it shares no code with the GPU library.

The paper has no learned closure; this is the extension built on its collision step
(Eq. 16 with the forcing of Eq. 19 and the equilibrium of Eq. 20).  Everything here is
written out in plain numpy, double precision, one definition per function:

  moment_basis   orthonormal D3Q19 moment basis M (19 x 19) by Gram-Schmidt of the
                 monomials 1, x, y, z, x^2, y^2, z^2, xy, xz, yz, x^2y, x^2z, y^2x, y^2z,
                 z^2x, z^2y, x^2y^2, x^2z^2, y^2z^2 of the lattice velocities (in this
                 order); rows 0-3 span {1, c_x, c_y, c_z}, rows 4-18 are the
                 non-conserved moments.  M is orthogonal, so M^-1 = M^T.
  features       15 standardised non-equilibrium moments M_nc (f - f^eq(rho, v)) of
                 the pre-collision state plus one lane |g_IB| scaled (16 lanes).
  mlp_forward    16 -> 64 -> 64 -> 16 with ReLU; output lanes 0-14 (times out_scale)
                 are the corrections dm of the post-collision non-conserved moments,
                 lane 15 is unused.
  apply          f* = f*_BGK + M_nc^T dm, guarded: a node keeps the plain step unless
                 dm is finite and |dm| <= c |m_neq| (c = 1).
  mlp_backward   gradients of the masked mean-square loss, by the chain rule.
  adam           Adam update (Kingma & Ba 2015) with bias correction.
  restrict       2x coarsening of a fine pre-collision state under acoustic scaling:
                 block means of rho and j, equilibrium of those plus the block mean of the
                 fine non-equilibrium part times 2 tau_c / tau_f (Dupuis & Chopard 2003);
                 force density 2 x block mean.
  targets        dm the closure should add: M_nc (unstream(R f(t+2)) - collide(R f(t))).

Precision emulation for comparing with the BF16 matrix-core path: with ``bf16=True``
the network inputs and both hidden activations are rounded to bfloat16 (round to
nearest even) at the points where the GPU path rounds them; the weights passed in are
taken as given (the caller rounds them once).
"""
from __future__ import annotations

import numpy as np

from . import oracle

NIN, NH, NOUT, NNC = 16, 64, 16, 15
NPARAM = NIN * NH + NH + NH * NH + NH + NH * NOUT + NOUT  # 6288

MONOMIALS = ("1", "x", "y", "z", "xx", "yy", "zz", "xy", "xz", "yz",
             "xxy", "xxz", "yyx", "yyz", "zzx", "zzy", "xxyy", "xxzz", "yyzz")


def velocities():
    c, w, opp = oracle.tables()
    return np.asarray(c, dtype=np.float64), np.asarray(w, dtype=np.float64)


def moment_basis():
    """Gram-Schmidt (with one re-orthogonalisation pass) of the monomials in MONOMIALS
    evaluated on the 19 lattice velocities; rows normalised to unit length."""
    c, _ = velocities()
    comp = {"x": c[:, 0], "y": c[:, 1], "z": c[:, 2]}
    rows = []
    for mono in MONOMIALS:
        v = np.ones(19)
        for ch in mono:
            if ch != "1":
                v = v * comp[ch]
        for _ in range(2):
            for r in rows:
                v = v - np.dot(r, v) * r
        nrm = np.linalg.norm(v)
        if nrm < 1e-9:
            raise ValueError("monomial %s is dependent on the previous ones" % mono)
        rows.append(v / nrm)
    return np.array(rows)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.  The value is
    first rounded to float32, as the GPU path holds it in a float32 register."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------- lattice quantities
def macro(f, g, body):
    """rho = sum f, v = (sum c f + F/2) / rho with F = body + g (Eq. 17-18, shift under
    Eq. 19).  f: [19, ...], g: [3, ...] or None."""
    c, _ = velocities()
    rho = f.sum(axis=0)
    j = np.tensordot(c.T, f, axes=(1, 0))
    F = np.asarray(body, dtype=np.float64).reshape((3,) + (1,) * (f.ndim - 1)) + (0.0 if g is None else g)
    v = (j + 0.5 * F) / rho
    return rho, v, F


def equilibrium(rho, v):
    """Eq. 20: w_i rho (1 + 3 c.v + 9/2 (c.v)^2 - 3/2 v.v)."""
    c, w = velocities()
    cv = np.tensordot(c, v, axes=(1, 0))
    vv = (v * v).sum(axis=0)
    return w.reshape((19,) + (1,) * rho.ndim) * rho * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv)


def raw_features(f, g, body):
    """15 non-equilibrium non-conserved moments of the pre-collision state and |g_IB|.
    Returns [N, 16] for f of shape [19, ...]."""
    M = moment_basis()
    rho, v, _ = macro(f, g, body)
    fneq = (f - equilibrium(rho, v)).reshape(19, -1)
    m = M[4:] @ fneq
    gmag = np.zeros(fneq.shape[1]) if g is None else np.sqrt((g.reshape(3, -1) ** 2).sum(axis=0))
    return np.concatenate([m, gmag[None, :]], axis=0).T


def standardise(raw, norm):
    """(raw - in_mean) * in_scale per lane; norm = dict(in_mean[16], in_scale[16], out_scale[16])."""
    return (raw - norm["in_mean"][None, :]) * norm["in_scale"][None, :]


# ----------------------------------------------------------------- network
def unpack(theta):
    """Flat parameter vector -> (W1[16,64], b1, W2[64,64], b2, W3[64,16], b3)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for shape in ((NIN, NH), (NH,), (NH, NH), (NH,), (NH, NOUT), (NOUT,)):
        n = int(np.prod(shape))
        out.append(theta[o:o + n].reshape(shape))
        o += n
    assert o == NPARAM
    return out


def mlp_forward(x, theta, bf16=False):
    """x: [B, 16] standardised inputs -> (y [B, 16], cache for the backward pass)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    r = bf16_round if bf16 else (lambda a: a)
    x = r(x)
    a1 = x @ W1 + b1
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ W2 + b2
    h2 = r(np.maximum(a2, 0.0))
    y = h2 @ W3 + b3
    return y, (x, a1, h1, a2, h2)


def loss(y, t):
    """Mean square error over the 15 used output lanes: sum_b sum_{k<15} (y-t)^2 / (15 B)."""
    d = (y - t)[:, :NNC]
    return float((d * d).sum() / (NNC * y.shape[0]))


def mlp_backward(y, t, cache, theta):
    """Gradient of loss(y, t) with respect to the flat parameters (chain rule)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    x, a1, h1, a2, h2 = cache
    B = y.shape[0]
    dy = np.zeros_like(y)
    dy[:, :NNC] = 2.0 * (y - t)[:, :NNC] / (NNC * B)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (a2 > 0)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (a1 > 0)
    dW1 = x.T @ dh1
    db1 = dh1.sum(axis=0)
    return np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])


def adam(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ----------------------------------------------------------------- closure step
def correction(f, g, body, theta, norm, c_guard=1.0, bf16=False):
    """Per-node correction of the post-collision populations, dF [19, N], and the
    number of nodes whose correction the guard rejected."""
    M = moment_basis()
    raw = raw_features(f, g, body)
    y, _ = mlp_forward(standardise(raw, norm), theta, bf16=bf16)
    dm = y[:, :NNC] * norm["out_scale"][None, :NNC]
    mneq = raw[:, :NNC]
    ok = np.all(np.isfinite(dm), axis=1) & (np.sqrt((dm * dm).sum(axis=1)) <= c_guard * np.sqrt((mneq * mneq).sum(axis=1)))
    dm = np.where(ok[:, None], dm, 0.0)
    return M[4:].T @ dm.T, int((~ok).sum())


def closure_step(lat, theta, norm, c_guard=1.0, bf16=False):
    """One step of the coarse lattice with the learned closure: collide (Eq. 16, 19, 20),
    add the guarded correction, stream.  Returns the number of guarded nodes.  The
    features are those of the populations the step reads (with on-site walls, the wall
    rows' entering populations set by Eq. (23)-(30))."""
    fs = lat.collide()
    body = np.array(lat.p.body[:])
    dF, nrej = correction(lat.populations(), lat.g, body, theta, norm, c_guard, bf16)
    lat.stream_from(fs + dF.reshape(fs.shape))
    return nrej


# ----------------------------------------------------------------- training data
def restrict(f, g, body_f, tau_f, tau_c):
    """2x restriction of the fine pre-collision state f [19, NZ, NY, NX] and force g
    [3, NZ, NY, NX] (acoustic scaling, dt_c = 2 dt_f).  Returns (f_c, g_c, body_c)."""
    c, _ = velocities()
    q, NZ, NY, NX = f.shape

    def avg(a):
        k = a.shape[0]
        return a.reshape(k, NZ // 2, 2, NY // 2, 2, NX // 2, 2).mean(axis=(2, 4, 6))

    rho = f.sum(axis=0)
    j = np.tensordot(c.T, f, axes=(1, 0))
    fneq = f - equilibrium(rho, j / rho)
    rho_c = avg(rho[None])[0]
    j_c = avg(j)
    f_c = equilibrium(rho_c, j_c / rho_c) + (2.0 * tau_c / tau_f) * avg(fneq)
    g_c = 2.0 * avg(g)
    return f_c, g_c, 2.0 * np.asarray(body_f, dtype=np.float64)


def targets(lat_c, f_c0, g_c, f_c1):
    """Features and moment targets for one snapshot pair on the coarse lattice `lat_c`:
    f_c0 = R f(t), f_c1 = R f(t + 2 dt_f), g_c the restricted force.  Returns
    (raw features [N, 16], dm_target [N, 15])."""
    M = moment_basis()
    lat_c.f[...] = f_c0
    lat_c.g[...] = g_c
    fs_bgk = lat_c.collide()
    fs_target = lat_c.unstream(f_c1)
    dm = M[4:] @ (fs_target - fs_bgk).reshape(19, -1)
    return raw_features(f_c0, g_c, np.array(lat_c.p.body[:])), dm.T
