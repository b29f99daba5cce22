"""FP64 CPU oracle of the coupled LBM + immersed-boundary step (test infrastructure).

TEST INFRASTRUCTURE ONLY: the independent reference the GPU library is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library: the lattice and
IB arithmetic live in ``lbm_oracle.c`` (plain loops, double precision), this module
only marshals numpy arrays into it and strings the calls together in the order of
the paper's Fig. 1.  The learned-closure reference (numpy, FP64) is in
``closure_oracle.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import bending_oracle

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A prebuilt variant of the same source (the sanitizer build of the tests) may be named here;
# it is then loaded as is, never rebuilt.
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")
_lib = None

KERNELS = {"cos": 0, "peskin4": 1}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_int32),
                ("tau", C.c_double), ("body", C.c_double * 3),
                ("uw_lo", C.c_double * 3), ("uw_hi", C.c_double * 3)]


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
        dp, ip, pp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(_Params)
        L.orc_feq.argtypes = [C.c_double, dp, dp]
        L.orc_source.argtypes = [C.c_double, dp, dp, dp]
        L.orc_phi.argtypes = [C.c_int32, C.c_double]
        L.orc_phi.restype = C.c_double
        L.orc_tables.argtypes = [ip, dp, ip]
        L.orc_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_init.argtypes = [pp, dp, dp, dp]
        L.orc_moments.argtypes = [pp, dp, dp, dp, dp]
        L.orc_complete.argtypes = [pp, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, dp, dp]
        L.orc_collide.argtypes = [pp, dp, dp, dp]
        L.orc_stream.argtypes = [pp, dp, dp]
        L.orc_unstream.argtypes = [pp, dp, dp]
        L.orc_spread.argtypes = [pp, C.c_int32, C.c_int64, dp, dp, dp]
        L.orc_interp.argtypes = [pp, C.c_int32, C.c_int64, dp, dp, dp]
        L.orc_advance.argtypes = [C.c_int64, dp, dp]
        L.orc_wall_stress.argtypes = [pp, dp, dp, dp, dp]
        L.orc_hinge_angles.argtypes = [C.c_int64, dp, C.c_int64, ip, dp]
        L.orc_edge_lengths.argtypes = [C.c_int64, dp, C.c_int64, ip, dp]
        L.orc_membrane_energy.argtypes = [C.c_int64, dp, C.c_int64, ip, dp, C.c_double, C.c_int64, ip, dp,
                                          C.c_double, dp, C.c_double]
        L.orc_membrane_energy.restype = C.c_double
        L.orc_membrane_forces.argtypes = [C.c_int64, dp, C.c_int64, ip, dp, C.c_double, C.c_int64, ip, dp,
                                          C.c_double, dp, C.c_double, dp]
        L.orc_triangle_rest.argtypes = [C.c_int64, dp, ip, C.c_int64, ip, dp, dp]
        L.orc_constraint_energy.argtypes = [C.c_int64, dp, ip, C.c_int64, ip, dp, dp, C.c_double, C.c_double,
                                            C.c_double]
        L.orc_constraint_energy.restype = C.c_double
        L.orc_constraint_forces.argtypes = [C.c_int64, dp, ip, C.c_int64, ip, dp, dp, C.c_double, C.c_double,
                                            C.c_double, dp]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------- point functions
def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def set_threads(n):
    """Threads for later parallel loops (timing only)."""
    lib().orc_set_threads(int(n))


def tables():
    """D3Q19 velocities c[19,3], weights w[19], opposite index opp[19] (paper order)."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    o = np.zeros(19, np.int32)
    lib().orc_tables(_i(c), _d(w), _i(o))
    return c, w, o


def feq(rho, v):
    out = np.zeros(19)
    lib().orc_feq(float(rho), _d(_f64(v)), _d(out))
    return out


def source(tau, v, F):
    out = np.zeros(19)
    lib().orc_source(float(tau), _d(_f64(v)), _d(_f64(F)), _d(out))
    return out


def phi(r, kernel="cos"):
    k = KERNELS[kernel]
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda x: lib().orc_phi(k, float(x)))(r)


def lattice_timestep(tau, h, mu, rho):
    """Physical time step from the relaxation time: dt = (tau - 1/2) h^2 / (3 nu), nu = mu/rho
    (section 3.3, the parameter choice after Eq. (22)).  SI units in and out."""
    nu = mu / rho
    return (tau - 0.5) * h * h / (3.0 * nu)


# ----------------------------------------------------------------- lattice object
def wall_mode(walls) -> int:
    """0 = periodic in y, 1 = halfway bounce-back walls (R4), 2 = on-site walls on the
    rows y = 0 and ny-1 (Eq. 23-30, R22).  True means 1; "onsite" means 2."""
    if walls == "onsite":
        return 2
    if walls is True or walls is False:
        return int(walls)
    if walls in (0, 1, 2):
        return int(walls)
    raise ValueError(f"walls must be False, True, 'onsite' or 0/1/2, not {walls!r}")


class Lattice:
    """One channel: populations f[19][nz][ny][nx] (paper order) and the IB force field
    g[3][nz][ny][nx], both FP64.  Methods follow the per-step order of Fig. 1.  With
    on-site walls the populations entering at a wall row are not stored (they read as 0
    in ``f``); ``populations()`` gives the state with them set by Eq. (23)-(30)."""

    def __init__(self, nx, ny, nz, tau, walls=True, body=(0, 0, 0), u_wall_lo=(0, 0, 0),
                 u_wall_hi=(0, 0, 0), kernel="cos"):
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.walls = wall_mode(walls)
        self.p = _Params(nx, ny, nz, self.walls, float(tau), (C.c_double * 3)(*body),
                         (C.c_double * 3)(*u_wall_lo), (C.c_double * 3)(*u_wall_hi))
        self.kernel = KERNELS[kernel]
        self.f = np.zeros((19, nz, ny, nx))
        self.g = np.zeros((3, nz, ny, nx))

    @property
    def tau(self):
        return self.p.tau

    def init(self, rho=None, u=None):
        lib().orc_init(C.byref(self.p), _d(self.f), _d(_f64(rho)), _d(_f64(u)))

    def shear_profile(self):
        """Linear profile between the two walls (planes y=-1/2 and y=ny-1/2; rows 0 and
        ny-1 with on-site walls)."""
        nz, ny, nx = self.shape
        s = np.arange(ny) / (ny - 1) if self.walls == 2 else (np.arange(ny) + 0.5) / ny
        lo, hi = np.array(self.p.uw_lo[:]), np.array(self.p.uw_hi[:])
        u = lo[:, None] + (hi - lo)[:, None] * s[None, :]
        return np.ascontiguousarray(np.broadcast_to(u[:, None, :, None], (3, nz, ny, nx)))

    def step(self, nsteps=1):
        out = np.empty_like(self.f)
        for _ in range(nsteps):
            lib().orc_step(C.byref(self.p), _d(self.f), _d(self.g), _d(out))
            self.f, out = out, self.f

    def collide(self):
        """Post-collision populations f* of the current state (Eq. 16, 19, 20); no update."""
        fs = np.empty_like(self.f)
        lib().orc_collide(C.byref(self.p), _d(self.f), _d(self.g), _d(fs))
        return fs

    def stream_from(self, fs):
        """Set the state to the streamed post-collision populations `fs` (with bounce-back)."""
        fs = np.ascontiguousarray(fs, dtype=np.float64)
        lib().orc_stream(C.byref(self.p), _d(fs), _d(self.f))

    def unstream(self, f):
        """Post-collision populations that streaming maps onto `f` (inverse of stream_from)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        fs = np.empty_like(f)
        lib().orc_unstream(C.byref(self.p), _d(f), _d(fs))
        return fs

    def populations(self):
        """The pre-collision populations the next step reads: ``f`` with the on-site wall
        rule applied at the wall rows (a copy of ``f`` otherwise)."""
        fc = np.empty_like(self.f)
        lib().orc_complete(C.byref(self.p), _d(self.f), _d(self.g), _d(fc))
        return fc

    def moments(self):
        rho = np.empty(self.shape)
        v = np.empty((3,) + self.shape)
        lib().orc_moments(C.byref(self.p), _d(self.f), _d(self.g), _d(rho), _d(v))
        return rho, v

    def spread(self, X, F):
        X, F = _f64(X), _f64(F)
        lib().orc_spread(C.byref(self.p), self.kernel, X.shape[1], _d(X), _d(F), _d(self.g))

    def interp_field(self, X, v):
        X, v = _f64(X), _f64(v)
        U = np.empty_like(X)
        lib().orc_interp(C.byref(self.p), self.kernel, X.shape[1], _d(X), _d(v), _d(U))
        return U

    def interp(self, X):
        _, v = self.moments()
        return self.interp_field(X, v)

    def wall_stress(self):
        nz, ny, nx = self.shape
        lo = np.empty((2, nz, nx))
        hi = np.empty((2, nz, nx))
        lib().orc_wall_stress(C.byref(self.p), _d(self.f), _d(self.g), _d(lo), _d(hi))
        return lo, hi


# ----------------------------------------------------------------- membrane forces
class Membrane:
    """Spring network (Eq. 2-3), tethers, the dihedral bending stand-in and the area and
    volume constraints of Eq. (4)-(5) (``triangles`` [nt, 3], outward by the right-hand rule,
    each body's triangles contiguous: ``body_tri`` = [0, ..., nt]; one body if omitted).
    Rest lengths, angles, areas and volumes are measured on ``X_rest`` by the oracle itself."""

    def __init__(self, X_rest, edges, k_spring=0.0, hinges=None, k_bend=0.0, anchors=None,
                 k_tether=0.0, triangles=None, body_tri=None, k_area_global=0.0, k_area_local=0.0,
                 k_volume=0.0, elements6=None, k_fe=0.0):
        X_rest = _f64(X_rest)
        self.n = X_rest.shape[1]
        self.edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        self.hinges = (np.zeros((0, 4), np.int32) if hinges is None
                       else np.ascontiguousarray(hinges, dtype=np.int32).reshape(-1, 4))
        self.k_spring, self.k_bend, self.k_tether = float(k_spring), float(k_bend), float(k_tether)
        self.anchors = _f64(anchors)
        self.rest_len = np.zeros(len(self.edges))
        lib().orc_edge_lengths(self.n, _d(X_rest), len(self.edges), _i(self.edges), _d(self.rest_len))
        self.rest_theta = np.zeros(len(self.hinges))
        lib().orc_hinge_angles(self.n, _d(X_rest), len(self.hinges), _i(self.hinges), _d(self.rest_theta))
        # finite-element bending of Eq. (6)-(10) (bending_oracle.py)
        self.elements6 = None if elements6 is None else np.asarray(elements6, dtype=np.int64).reshape(-1, 6)
        self.k_fe = float(k_fe)
        self.tri = (None if triangles is None
                    else np.ascontiguousarray(triangles, dtype=np.int32).reshape(-1, 3))
        self.k_area_global, self.k_area_local, self.k_volume = float(k_area_global), float(k_area_local), float(k_volume)
        if self.tri is not None:
            nt = len(self.tri)
            self.body_tri = np.ascontiguousarray([0, nt] if body_tri is None else body_tri, dtype=np.int32)
            self.nb = len(self.body_tri) - 1
            self.rest_area = np.zeros(nt)
            self.rest_body = np.zeros((self.nb, 2))
            lib().orc_triangle_rest(self.n, _d(X_rest), _i(self.tri), self.nb, _i(self.body_tri),
                                    _d(self.rest_area), _d(self.rest_body))

    def measures(self, X):
        """(area, volume) of each body for the shape X (Eq. 4-5's S^total and V)."""
        X = _f64(X)
        a0, b = np.zeros(len(self.tri)), np.zeros((self.nb, 2))
        lib().orc_triangle_rest(self.n, _d(X), _i(self.tri), self.nb, _i(self.body_tri), _d(a0), _d(b))
        return b[:, 0], b[:, 1]

    def _constraint_args(self):
        return (_i(self.tri), self.nb, _i(self.body_tri), _d(self.rest_area), _d(self.rest_body),
                self.k_area_global, self.k_area_local, self.k_volume)

    def energy(self, X):
        X = _f64(X)
        E = lib().orc_membrane_energy(self.n, _d(X), len(self.edges), _i(self.edges), _d(self.rest_len),
                                      self.k_spring, len(self.hinges), _i(self.hinges),
                                      _d(self.rest_theta), self.k_bend, _d(self.anchors), self.k_tether)
        if self.tri is not None:
            E += lib().orc_constraint_energy(self.n, _d(X), *self._constraint_args())
        if self.elements6 is not None and self.k_fe != 0.0:
            E += bending_oracle.energy(X, self.elements6, self.k_fe)
        return E

    def forces(self, X):
        X = _f64(X)
        F = np.empty_like(X)
        lib().orc_membrane_forces(self.n, _d(X), len(self.edges), _i(self.edges), _d(self.rest_len),
                                  self.k_spring, len(self.hinges), _i(self.hinges), _d(self.rest_theta),
                                  self.k_bend, _d(self.anchors), self.k_tether, _d(F))
        if self.tri is not None:
            Fc = np.empty_like(X)
            lib().orc_constraint_forces(self.n, _d(X), *self._constraint_args(), _d(Fc))
            F += Fc
        if self.elements6 is not None and self.k_fe != 0.0:
            F += bending_oracle.forces(X, self.elements6, self.k_fe)
        return F


def coupled_step(lat: Lattice, mem: Membrane | None, X: np.ndarray, adhesion=None, step=0):
    """One step of Fig. 1: membrane forces F(X^n) (with the bonds of `adhesion`, a
    dam_oracle.Adhesion) -> spread g^n -> LBM step -> interpolate v^{n+1} at X^n ->
    X^{n+1} = X^n + U -> the adhesion's Monte-Carlo step `step` at X^{n+1}.  Returns (F, U); X is
    updated in place."""
    F = mem.forces(X) if mem is not None else np.zeros_like(X)
    if adhesion is not None:
        F = F + adhesion.forces(X)
    lat.spread(X, F)
    lat.step(1)
    U = lat.interp(X)
    lib().orc_advance(X.shape[1], _d(X), _d(U))
    if adhesion is not None:
        adhesion.step(X, step)
    return F, U
