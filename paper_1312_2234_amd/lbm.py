"""ctypes binding of the gfx950 C-ABI library (include/lbm.h).

Argument marshalling only: every computation runs in the library's HIP kernels.  PyTorch
provides the device memory (the workspace and the caller-owned arrays) and the stream.
The library must be built (``python -m paper_1312_2234_amd.build``); loading fails
loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmib.so")

STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
KERNEL = {"cos": 0, "peskin4": 1}
FLAG_NODE_OUTSIDE, FLAG_LIST_OVERFLOW, FLAG_FORCE_NONFINITE, FLAG_CLOSURE_FALLBACK = 1, 2, 4, 8
FLAG_ADHESION_BIDS = 16
FLAG_REBIN_MARGIN = 32

EXPORTS = [
    "lbm_workspace_bytes", "lbm_create", "lbm_destroy", "lbm_init", "lbm_step", "ib_set_nodes",
    "ib_spread", "ib_interp", "ib_advance", "lbm_moments", "lbm_get_populations",
    "lbm_set_populations", "lbm_state_bytes", "lbm_get_state", "lbm_set_state", "lbm_wall_stress",
    "lbm_error_flags", "lbm_status_string", "ib_membrane_rest", "ib_membrane_forces",
    "lbm_coupled_steps", "lbm_graph_capture", "lbm_graph_launch", "lbm_set_launch", "lbm_get_launch",
    "lbm_stream_copy", "mlp_pack", "lbm_set_closure", "lbm_closure_guarded", "mlp_forward",
    "mlp_grad_workspace_bytes", "mlp_grad", "mlp_adam", "mlp_norm_workspace_bytes", "mlp_norm",
    "lbm_restrict", "closure_targets", "lbm_launch_timer", "lbm_launch_timer_read", "mlp_grad_noalloc",
    "ib_adhesion_step", "ib_adhesion_work_ints",
]

MLP_PARAMS, MLP_NORM, MLP_PACKED_BYTES = 6288, 48, 23360
_SIZE_FNS = ("lbm_workspace_bytes", "lbm_state_bytes", "lbm_status_string", "mlp_grad_workspace_bytes",
             "mlp_norm_workspace_bytes", "ib_adhesion_work_ints")


class LbmParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_int32),
                ("tau", C.c_float), ("body_force", C.c_float * 3), ("u_wall_lo", C.c_float * 3),
                ("u_wall_hi", C.c_float * 3)]


class LbmLaunch(C.Structure):
    _fields_ = [("block", C.c_int32), ("xcd_remap", C.c_int32), ("persistent", C.c_int32),
                ("nontemporal", C.c_int32), ("vec", C.c_int32), ("overlap", C.c_int32), ("split", C.c_int32),
                ("rebin", C.c_int32)]


class IbMembrane(C.Structure):
    _fields_ = [("n", C.c_int64), ("nbr_ptr", C.c_void_p), ("nbr_idx", C.c_void_p), ("rest_len", C.c_void_p),
                ("k_spring", C.c_double), ("hinge_ptr", C.c_void_p), ("hinge_inc", C.c_void_p),
                ("hinges", C.c_void_p), ("rest_cs", C.c_void_p),
                ("nh", C.c_int64), ("k_bend", C.c_double),
                ("anchors", C.c_void_p), ("k_tether", C.c_double),
                ("tri", C.c_void_p), ("nt", C.c_int64), ("tri_ptr", C.c_void_p), ("tri_inc", C.c_void_p),
                ("tri_body", C.c_void_p), ("body_tri", C.c_void_p), ("nb", C.c_int64),
                ("rest_area", C.c_void_p), ("rest_body", C.c_void_p), ("body_now", C.c_void_p),
                ("k_area_global", C.c_double), ("k_area_local", C.c_double), ("k_volume", C.c_double),
                ("elem6", C.c_void_p), ("ne", C.c_int64), ("elem_ptr", C.c_void_p), ("elem_inc", C.c_void_p),
                ("elem_slot", C.c_void_p), ("fe_work", C.c_void_p), ("k_fe", C.c_double),
                ("adh_nr", C.c_int64), ("rec_tri", C.c_void_p), ("rec_bary", C.c_void_p), ("rec_ptr", C.c_void_p),
                ("rec_inc", C.c_void_p), ("adh_nl", C.c_int64), ("lig_xz", C.c_void_p), ("bond", C.c_void_p),
                ("lig_count", C.c_void_p), ("adh_work", C.c_void_p), ("adh_wall_y", C.c_double),
                ("adh_nx", C.c_double), ("adh_nz", C.c_double), ("adh_capture", C.c_double),
                ("adh_sigma", C.c_double), ("adh_lb", C.c_double), ("adh_gamma", C.c_double), ("adh_kT", C.c_double),
                ("adh_kon0", C.c_double), ("adh_koff0", C.c_double), ("adh_seed", C.c_uint64)]


ADH_MAX_BIDS = 32


_lib = None


def lib():
    """Load liblbmib.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbmib.so is not built: run `python -m paper_1312_2234_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f32p = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
        P = C.POINTER(LbmParams)
        L.lbm_workspace_bytes.argtypes = [P, i32, i32, i64]
        L.lbm_workspace_bytes.restype = C.c_size_t
        L.lbm_create.argtypes = [P, i32, i32, i32, i64, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_init.argtypes = [vp, vp, vp]
        L.lbm_step.argtypes = [vp, i32]
        L.ib_set_nodes.argtypes = [vp, i64, C.POINTER(C.c_int64)]
        L.ib_spread.argtypes = [vp, i64, vp, vp]
        L.ib_interp.argtypes = [vp, i64, vp, vp]
        L.ib_advance.argtypes = [vp, i64, vp, vp]
        L.lbm_moments.argtypes = [vp, vp, vp]
        L.lbm_get_populations.argtypes = [vp, vp]
        L.lbm_set_populations.argtypes = [vp, vp]
        L.lbm_state_bytes.argtypes = [vp]
        L.lbm_state_bytes.restype = C.c_size_t
        L.lbm_get_state.argtypes = [vp, vp]
        L.lbm_set_state.argtypes = [vp, vp]
        L.lbm_wall_stress.argtypes = [vp, vp, vp]
        L.lbm_error_flags.argtypes = [vp, C.POINTER(C.c_uint32)]
        L.lbm_status_string.argtypes = [i32]
        L.lbm_status_string.restype = C.c_char_p
        M = C.POINTER(IbMembrane)
        L.ib_membrane_rest.argtypes = [M, vp, vp]
        L.ib_membrane_forces.argtypes = [M, vp, vp, vp]
        L.ib_adhesion_step.argtypes = [M, vp, vp]
        L.ib_adhesion_work_ints.argtypes = [i64, C.c_double, C.c_double, C.c_double]
        L.ib_adhesion_work_ints.restype = C.c_int64
        L.lbm_coupled_steps.argtypes = [vp, M, i32, vp, vp, vp]
        L.lbm_graph_capture.argtypes = [vp, M, i32, vp, vp, vp]
        L.lbm_graph_launch.argtypes = [vp, i32]
        L.lbm_set_launch.argtypes = [vp, C.POINTER(LbmLaunch)]
        L.lbm_get_launch.argtypes = [vp, C.POINTER(LbmLaunch)]
        L.lbm_stream_copy.argtypes = [vp, vp, C.c_size_t, i32, i64, vp]
        f32 = C.c_float
        L.mlp_pack.argtypes = [vp, vp, f32, vp, vp]
        L.lbm_set_closure.argtypes = [vp, vp, vp, f32, i32]
        L.lbm_closure_guarded.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.mlp_grad_workspace_bytes.argtypes = [i64]
        L.mlp_grad_workspace_bytes.restype = C.c_size_t
        L.mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, C.c_size_t, vp]
        L.mlp_grad_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.mlp_adam.argtypes = [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp]
        L.mlp_norm_workspace_bytes.argtypes = [i64]
        L.mlp_norm_workspace_bytes.restype = C.c_size_t
        L.mlp_norm.argtypes = [vp, vp, i64, vp, vp, C.c_size_t, vp]
        L.lbm_restrict.argtypes = [vp, f32, vp, vp]
        L.closure_targets.argtypes = [P, vp, vp, vp, vp, vp, vp]
        L.lbm_launch_timer.argtypes = [vp, i32]
        L.lbm_launch_timer_read.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        for name in EXPORTS:
            if name not in _SIZE_FNS:
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


class LbmError(RuntimeError):
    pass


def _check(status, what):
    if status != 0:
        msg = lib().lbm_status_string(status).decode()
        raise LbmError("%s failed: %s (%d)" % (what, msg, status))


def _ptr(t):
    if t is None:
        return None
    assert t.is_contiguous(), "arrays passed to the library must be contiguous"
    return C.c_void_p(t.data_ptr())


def wall_code(walls) -> int:
    """lbm_params.walls: False/0 periodic, True/1 halfway bounce-back, "onsite"/2 on-site walls."""
    if walls == "onsite":
        return 2
    if walls is True or walls is False or walls in (0, 1, 2):
        return int(walls)
    raise ValueError(f"walls must be False, True, 'onsite' or 0/1/2, not {walls!r}")


def params_of(ch) -> LbmParams:
    """lbm_params from an inputs.Channel (or any object with the same fields)."""
    return LbmParams(ch.nx, ch.ny, ch.nz, wall_code(ch.walls), float(ch.tau), (C.c_float * 3)(*ch.body),
                     (C.c_float * 3)(*ch.u_wall_lo), (C.c_float * 3)(*ch.u_wall_hi))


def _stream_ptr(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class _Ordered:
    """Order the context's stream after torch's current stream on entry and torch's current
    stream after the context's stream on exit (event waits, no host synchronisation)."""

    def __init__(self, lat):
        self.lat = lat

    def __enter__(self):
        self.lat.stream.wait_stream(self.lat.torch.cuda.current_stream(self.lat.device))

    def __exit__(self, *exc):
        self.lat.torch.cuda.current_stream(self.lat.device).wait_stream(self.lat.stream)
        return False


class Lattice:
    """One context over `channels` (list of inputs.Channel-like objects).

    The context owns a torch stream of default priority (a non-default stream, so that its
    work can be captured into a HIP graph); every call is ordered after torch's current
    stream and torch's current stream after it."""

    def __init__(self, channels, storage="f32", kernel="cos", max_nodes=0, device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.ordered = _Ordered(self)
        self.channels = list(channels)
        self.nch = len(self.channels)
        arr = (LbmParams * self.nch)(*[params_of(c) for c in self.channels])
        self._params = arr
        self.storage = storage
        nbytes = lib().lbm_workspace_bytes(arr, self.nch, STORAGE[storage], int(max_nodes))
        if nbytes == 0:
            raise LbmError("invalid lattice parameters")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        with self.ordered:
            _check(lib().lbm_create(arr, self.nch, STORAGE[storage], KERNEL[kernel], int(max_nodes),
                                    C.c_void_p(base + off), nbytes, C.c_void_p(self.stream.cuda_stream),
                                    C.byref(h)), "lbm_create")
        self.h = h
        self.cells = [c.nx * c.ny * c.nz for c in self.channels]
        self.total_cells = sum(self.cells)
        self.n_nodes = 0

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- lattice
    def init(self, rho=None, u=None):
        with self.ordered:
            _check(lib().lbm_init(self.h, _ptr(rho), _ptr(u)), "lbm_init")

    def step(self, nsteps=1):
        with self.ordered:
            _check(lib().lbm_step(self.h, int(nsteps)), "lbm_step")

    def moments(self):
        t = self.torch
        drho = t.empty(self.total_cells, dtype=t.float32, device=self.device)
        v = t.empty(3 * self.total_cells, dtype=t.float32, device=self.device)
        with self.ordered:
            _check(lib().lbm_moments(self.h, _ptr(drho), _ptr(v)), "lbm_moments")
        return drho, v

    def moments_channel(self, c=0):
        """(drho[nz,ny,nx], v[3,nz,ny,nx]) of channel c as torch tensors."""
        drho, v = self.moments()
        ch = self.channels[c]
        off = sum(self.cells[:c])
        n = self.cells[c]
        shp = (ch.nz, ch.ny, ch.nx)
        return drho[off:off + n].view(shp), v[3 * off:3 * off + 3 * n].view((3,) + shp)

    def populations(self):
        t = self.torch
        f = t.empty(19 * self.total_cells, dtype=t.float32, device=self.device)
        with self.ordered:
            _check(lib().lbm_get_populations(self.h, _ptr(f)), "lbm_get_populations")
        return f

    def set_populations(self, f):
        with self.ordered:
            _check(lib().lbm_set_populations(self.h, _ptr(f)), "lbm_set_populations")

    def state_bytes(self):
        return lib().lbm_state_bytes(self.h)

    def get_state(self):
        t = self.torch
        buf = t.empty(self.state_bytes(), dtype=t.uint8, device=self.device)
        with self.ordered:
            _check(lib().lbm_get_state(self.h, _ptr(buf)), "lbm_get_state")
        return buf

    def set_state(self, buf):
        with self.ordered:
            _check(lib().lbm_set_state(self.h, _ptr(buf)), "lbm_set_state")

    def wall_stress(self):
        t = self.torch
        tot = sum(2 * c.nx * c.nz for c in self.channels)
        lo = t.empty(tot, dtype=t.float32, device=self.device)
        hi = t.empty(tot, dtype=t.float32, device=self.device)
        with self.ordered:
            _check(lib().lbm_wall_stress(self.h, _ptr(lo), _ptr(hi)), "lbm_wall_stress")
        return lo, hi

    def error_flags(self):
        f = C.c_uint32()
        _check(lib().lbm_error_flags(self.h, C.byref(f)), "lbm_error_flags")
        return f.value

    # -- immersed boundary
    def set_nodes(self, n, offsets=None):
        if offsets is not None:
            arr = (C.c_int64 * len(offsets))(*[int(o) for o in offsets])
            _check(lib().ib_set_nodes(self.h, int(n), arr), "ib_set_nodes")
        else:
            _check(lib().ib_set_nodes(self.h, int(n), None), "ib_set_nodes")
        self.n_nodes = int(n)

    def spread(self, X, F):
        with self.ordered:
            _check(lib().ib_spread(self.h, self.n_nodes, _ptr(X), _ptr(F)), "ib_spread")

    def interp(self, X, U=None):
        t = self.torch
        if U is None:
            U = t.empty((3, self.n_nodes), dtype=t.float32, device=self.device)
        with self.ordered:
            _check(lib().ib_interp(self.h, self.n_nodes, _ptr(X), _ptr(U)), "ib_interp")
        return U

    def advance(self, X, U):
        with self.ordered:
            _check(lib().ib_advance(self.h, self.n_nodes, _ptr(X), _ptr(U)), "ib_advance")

    def coupled_steps(self, membrane, nsteps, X, F, U):
        m = C.byref(membrane.struct) if membrane is not None else None
        with self.ordered:
            _check(lib().lbm_coupled_steps(self.h, m, int(nsteps), _ptr(X), _ptr(F), _ptr(U)), "lbm_coupled_steps")

    def graph_capture(self, membrane, nsteps, X, F, U):
        m = C.byref(membrane.struct) if membrane is not None else None
        with self.ordered:
            _check(lib().lbm_graph_capture(self.h, m, int(nsteps), _ptr(X), _ptr(F), _ptr(U)), "lbm_graph_capture")

    def graph_launch(self, repeats=1):
        with self.ordered:
            _check(lib().lbm_graph_launch(self.h, int(repeats)), "lbm_graph_launch")

    # -- learned closure
    def set_closure(self, params=None, norm=None, c_guard=1.0, enable=True):
        """Enable the learned closure with float32 device tensors params[6288], norm[48]
        (or disable it with enable=False)."""
        with self.ordered:
            _check(lib().lbm_set_closure(self.h, _ptr(params) if enable else None, _ptr(norm) if enable else None,
                                         float(c_guard), 1 if enable else 0), "lbm_set_closure")

    def closure_guarded(self):
        n = C.c_uint64()
        with self.ordered:
            _check(lib().lbm_closure_guarded(self.h, C.byref(n)), "lbm_closure_guarded")
        return n.value

    def restrict(self, tau_coarse):
        """2x restriction of the current state: (shifted populations [19, Nc], force [3, Nc])."""
        t = self.torch
        ch = self.channels[0]
        nc = (ch.nx // 2) * (ch.ny // 2) * (ch.nz // 2)
        g = t.empty((19, nc), dtype=t.float32, device=self.device)
        F = t.empty((3, nc), dtype=t.float32, device=self.device)
        with self.ordered:
            _check(lib().lbm_restrict(self.h, float(tau_coarse), _ptr(g), _ptr(F)), "lbm_restrict")
        return g, F

    def launch_timer(self, enable=True):
        """Time the lattice-update launch of later eager coupled steps (measurement helper)."""
        _check(lib().lbm_launch_timer(self.h, 1 if enable else 0), "lbm_launch_timer")

    def launch_timer_read(self):
        """(count, mean microseconds, kind) of the timed launches since the last read; kind 0 =
        fused lattice step, 1 = body-force update with the spread (split schedule), 2 = closure step."""
        n, us, kind = C.c_int64(), C.c_double(), C.c_int32()
        with self.ordered:
            _check(lib().lbm_launch_timer_read(self.h, C.byref(n), C.byref(us), C.byref(kind)),
                   "lbm_launch_timer_read")
        return n.value, us.value, kind.value

    def set_launch(self, block=256, xcd_remap=1, persistent=0, nontemporal=0, vec=0, overlap=0, split=-1, rebin=1):
        cfg = LbmLaunch(block, xcd_remap, persistent, nontemporal, vec, overlap, split, rebin)
        _check(lib().lbm_set_launch(self.h, C.byref(cfg)), "lbm_set_launch")

    def get_launch(self):
        cfg = LbmLaunch()
        _check(lib().lbm_get_launch(self.h, C.byref(cfg)), "lbm_get_launch")
        return dict(block=cfg.block, xcd_remap=cfg.xcd_remap, persistent=cfg.persistent,
                    nontemporal=cfg.nontemporal, vec=cfg.vec, overlap=cfg.overlap, split=cfg.split,
                    rebin=cfg.rebin)


def stream_copy(src, dst, variant=0, grid=0):
    """Device copy with the library's STREAM-style kernel (measurement helper); ordered on
    torch's current stream."""
    import torch

    assert src.numel() * src.element_size() == dst.numel() * dst.element_size()
    _check(lib().lbm_stream_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), int(variant), int(grid),
                                 _stream_ptr(torch, src.device)), "lbm_stream_copy")


# ----------------------------------------------------------------- network (training side)
def _cur(torch, t):
    return _stream_ptr(torch, t.device)


def mlp_pack(params, norm, c_guard=1.0):
    """Packed network (uint8 device tensor of MLP_PACKED_BYTES) for mlp_forward / mlp_grad."""
    import torch

    P = torch.empty(MLP_PACKED_BYTES, dtype=torch.uint8, device=params.device)
    _check(lib().mlp_pack(_ptr(params), _ptr(norm), float(c_guard), _ptr(P), _cur(torch, params)), "mlp_pack")
    return P


def mlp_forward(packed, raw):
    """dm[B, 16] = network(raw[B, 16]) * out_scale (no guard)."""
    import torch

    dm = torch.empty_like(raw)
    _check(lib().mlp_forward(_ptr(packed), _ptr(raw), raw.shape[0], _ptr(dm), _cur(torch, raw)), "mlp_forward")
    return dm


def mlp_grad(packed, raw, target, work=None):
    """(grad[6288], loss[1]) of the masked mean-square loss on B samples."""
    import torch

    B = raw.shape[0]
    nbytes = lib().mlp_grad_workspace_bytes(B)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device=raw.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=raw.device)
    loss = torch.empty(1, dtype=torch.float32, device=raw.device)
    _check(lib().mlp_grad(_ptr(packed), _ptr(raw), _ptr(target), B, _ptr(grad), _ptr(loss), _ptr(work), nbytes,
                          _cur(torch, raw)), "mlp_grad")
    return grad, loss


def mlp_grad_noalloc(packed, raw, target, grad=None, loss=None):
    """mlp_grad with the library's own per-GPU scratch: allocates no device memory when the caller
    passes grad[6288] and loss[1]."""
    import torch

    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=raw.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=raw.device)
    _check(lib().mlp_grad_noalloc(_ptr(packed), _ptr(raw), _ptr(target), raw.shape[0], _ptr(grad), _ptr(loss),
                                  _cur(torch, raw)), "mlp_grad_noalloc")
    return grad, loss


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    import torch

    _check(lib().mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(step), float(lr),
                          float(beta1), float(beta2), float(eps), _cur(torch, params)), "mlp_adam")


def mlp_norm(raw, target):
    """norm[48] = (in_mean, in_scale, out_scale) of a training set."""
    import torch

    B = raw.shape[0]
    nbytes = lib().mlp_norm_workspace_bytes(B)
    work = torch.empty(nbytes, dtype=torch.uint8, device=raw.device)
    norm = torch.empty(MLP_NORM, dtype=torch.float32, device=raw.device)
    _check(lib().mlp_norm(_ptr(raw), _ptr(target), B, _ptr(norm), _ptr(work), nbytes, _cur(torch, raw)), "mlp_norm")
    return norm


def closure_targets(coarse, g0, F, g1, out=None):
    """(feat[N, 16], target[N, 16]) of one coarse step; coarse is an inputs.Channel-like;
    `out` optionally gives the two (contiguous) output tensors."""
    import torch

    N = coarse.nx * coarse.ny * coarse.nz
    if out is None:
        feat = torch.empty((N, 16), dtype=torch.float32, device=g0.device)
        tgt = torch.empty((N, 16), dtype=torch.float32, device=g0.device)
    else:
        feat, tgt = out
        assert feat.shape == (N, 16) and tgt.shape == (N, 16)
    p = params_of(coarse)
    _check(lib().closure_targets(C.byref(p), _ptr(g0), _ptr(F), _ptr(g1), _ptr(feat), _ptr(tgt), _cur(torch, g0)),
           "closure_targets")
    return feat, tgt


class Membrane:
    """Device copy of a spring / hinge / tether network (inputs.Bodies) for
    ib_membrane_rest / ib_membrane_forces (run on torch's current stream).  `adhesion`: a dict
    with rec_tri [nr, 3], rec_bary [nr, 3], ligands [nl, 2] and the scalars wall_y, nx, nz,
    capture, sigma, l_b, gamma, kT, k_on0, k_off0, seed (and optionally bond [nr], lig_count [nl]
    as the initial state) turns on the adhesion of section 3.2."""

    def __init__(self, bodies, device="cuda:0", stream=None, adhesion=None):
        import torch

        from . import inputs

        dev = torch.device(device)
        n = bodies.n
        self._keep = []

        def dev_i32(a):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
            self._keep.append(t)
            return t

        s = IbMembrane()
        s.n = n
        if len(bodies.edges):
            ptr, idx = inputs.csr_neighbours(n, bodies.edges)
            p, i = dev_i32(ptr), dev_i32(idx)
            rl = torch.zeros(len(idx), dtype=torch.float64, device=dev)
            self._keep.append(rl)
            s.nbr_ptr, s.nbr_idx, s.rest_len = p.data_ptr(), i.data_ptr(), rl.data_ptr()
        s.k_spring = float(bodies.k_spring)
        if len(bodies.hinges) and bodies.k_bend != 0.0:
            hp, hi = inputs.csr_hinges(n, bodies.hinges)
            hpt, hit, ht = dev_i32(hp), dev_i32(hi), dev_i32(bodies.hinges.reshape(-1))
            rt = torch.zeros(2 * len(bodies.hinges), dtype=torch.float64, device=dev)
            self._keep += [rt]
            s.hinge_ptr, s.hinge_inc, s.hinges, s.rest_cs = hpt.data_ptr(), hit.data_ptr(), ht.data_ptr(), rt.data_ptr()
            s.nh = len(bodies.hinges)
        s.k_bend = float(bodies.k_bend)
        if bodies.anchors is not None:
            a = torch.from_numpy(np.ascontiguousarray(bodies.anchors, dtype=np.float64)).to(dev)
            self._keep.append(a)
            s.anchors = a.data_ptr()
        s.k_tether = float(bodies.k_tether)
        tri = getattr(bodies, "triangles", None)
        ks = (float(getattr(bodies, "k_area_global", 0.0)), float(getattr(bodies, "k_area_local", 0.0)),
              float(getattr(bodies, "k_volume", 0.0)))
        if tri is not None and len(tri) and any(ks):
            tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
            toff = np.asarray(bodies.tri_offsets, dtype=np.int64)
            tp, tinc = inputs.csr_triangles(n, tri)
            tb = np.repeat(np.arange(len(toff) - 1, dtype=np.int32), np.diff(toff))
            t_d, tp_d, ti_d, tb_d, bt_d = dev_i32(tri.reshape(-1)), dev_i32(tp), dev_i32(tinc), dev_i32(tb), dev_i32(toff)
            nb = len(toff) - 1
            ra = torch.zeros(len(tri), dtype=torch.float64, device=dev)
            rb = torch.zeros(2 * nb, dtype=torch.float64, device=dev)
            bn = torch.zeros(4 * nb, dtype=torch.float64, device=dev)
            self._keep += [ra, rb, bn]
            s.tri, s.nt, s.tri_ptr, s.tri_inc = t_d.data_ptr(), len(tri), tp_d.data_ptr(), ti_d.data_ptr()
            s.tri_body, s.body_tri, s.nb = tb_d.data_ptr(), bt_d.data_ptr(), nb
            s.rest_area, s.rest_body, s.body_now = ra.data_ptr(), rb.data_ptr(), bn.data_ptr()
            s.k_area_global, s.k_area_local, s.k_volume = ks
        e6 = getattr(bodies, "elements6", None)
        if e6 is not None and len(e6) and float(getattr(bodies, "k_fe", 0.0)) != 0.0:
            e6 = np.ascontiguousarray(e6, dtype=np.int32).reshape(-1, 6)
            ep, einc = inputs.csr_elements(n, e6)
            e_d, ep_d, ei_d = dev_i32(e6.reshape(-1)), dev_i32(ep), dev_i32(einc)
            es = torch.zeros(6 * len(e6), dtype=torch.int32, device=dev)
            fw = torch.zeros(84 * len(e6) + 6 * n, dtype=torch.float64, device=dev)
            self._keep += [es, fw]
            s.elem6, s.ne, s.elem_ptr, s.elem_inc = e_d.data_ptr(), len(e6), ep_d.data_ptr(), ei_d.data_ptr()
            s.elem_slot, s.fe_work, s.k_fe = es.data_ptr(), fw.data_ptr(), float(bodies.k_fe)
            self.fe_work = fw
        if adhesion is not None:
            a = adhesion
            rt = np.ascontiguousarray(a["rec_tri"], dtype=np.int32).reshape(-1, 3)
            nr = len(rt)
            rp, rinc = inputs.csr_receptors(n, rt)
            lig = np.ascontiguousarray(a["ligands"], dtype=np.float64).reshape(-1, 2)
            nl = len(lig)
            rt_d, rp_d, ri_d = dev_i32(rt.reshape(-1)), dev_i32(rp), dev_i32(rinc)
            rb_d = torch.from_numpy(np.ascontiguousarray(a["rec_bary"], dtype=np.float64).reshape(-1)).to(dev)
            lg_d = torch.from_numpy(lig.reshape(-1)).to(dev)
            bond0 = a.get("bond")
            self.bond = (torch.full((nr,), -1, dtype=torch.int32, device=dev) if bond0 is None
                         else torch.from_numpy(np.ascontiguousarray(bond0, dtype=np.int32)).to(dev))
            cnt0 = a.get("lig_count")
            self.lig_count = (torch.zeros(nl, dtype=torch.int32, device=dev) if cnt0 is None
                              else torch.from_numpy(np.ascontiguousarray(cnt0, dtype=np.int32)).to(dev))
            words = lib().ib_adhesion_work_ints(nl, float(a["nx"]), float(a["nz"]), float(a["capture"]))
            if words <= 0:
                raise LbmError("ib_adhesion_work_ints: invalid adhesion geometry")
            self.adh_work = torch.zeros(words, dtype=torch.int32, device=dev)
            self._keep += [rb_d, lg_d, self.bond, self.lig_count, self.adh_work]
            s.adh_nr, s.rec_tri, s.rec_bary, s.rec_ptr, s.rec_inc = nr, rt_d.data_ptr(), rb_d.data_ptr(), \
                rp_d.data_ptr(), ri_d.data_ptr()
            s.adh_nl, s.lig_xz, s.bond, s.lig_count = nl, lg_d.data_ptr(), self.bond.data_ptr(), \
                self.lig_count.data_ptr()
            s.adh_work = self.adh_work.data_ptr()
            for k in ("wall_y", "nx", "nz", "capture", "sigma", "gamma", "kT", "kon0", "koff0"):
                setattr(s, "adh_" + k, float(a[{"kon0": "k_on0", "koff0": "k_off0"}.get(k, k)]))
            s.adh_lb = float(a["l_b"])
            s.adh_seed = int(a["seed"])
        self.struct = s
        self.n = n
        st = stream if stream is not None else _stream_ptr(torch, dev)
        Xr = torch.from_numpy(np.ascontiguousarray(bodies.X_rest, dtype=np.float64)).to(dev)
        _check(lib().ib_membrane_rest(C.byref(s), _ptr(Xr), st), "ib_membrane_rest")
        self._keep.append(Xr)
        self.stream = st

    def forces(self, X, F=None):
        import torch

        if F is None:
            F = torch.empty((3, self.n), dtype=torch.float32, device=X.device)
        _check(lib().ib_membrane_forces(C.byref(self.struct), _ptr(X), _ptr(F), self.stream), "ib_membrane_forces")
        return F

    def adhesion_step(self, X):
        """One Monte-Carlo step of the adhesion at positions X (device [3, n] float64)."""
        _check(lib().ib_adhesion_step(C.byref(self.struct), _ptr(X), self.stream), "ib_adhesion_step")
