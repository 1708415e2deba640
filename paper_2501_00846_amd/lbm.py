"""Thin ctypes binding of liblbm.so (the C ABI declared in include/lbm.h).

Every function of the ABI is exposed under its C name with argument
marshalling only; all computation happens in the HIP library.  PyTorch
supplies the device memory (through the allocator callbacks) and the stream.
There is no fallback: if liblbm.so is missing or fails to load, every call
raises.

The Context class bundles the calls for one set of boxes.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK = 0
STATUS = {0: "LBM_OK", -1: "LBM_ERR_ARG", -2: "LBM_ERR_UNSUPPORTED", -3: "LBM_ERR_OOM",
          -4: "LBM_ERR_DEVICE", -5: "LBM_ERR_UNSTABLE", -6: "LBM_ERR_STATE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16_os": 2, "bf16_os": 3}
PERIODIC, WALL = 0, 1
LITERAL_ADVECTION = 1
GRADIENT_CLOSURE = 2
HIGH_ORDER_AC = 4
FINE_PHASE = 8
FIELDS = ("phi", "P", "Jx", "Jy", "Jz", "Qxx", "Qyy", "Qzz", "Qxy", "Qxz", "Qyz")


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, message))
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lattice", ctypes.c_int32), ("bc", ctypes.c_int32 * 3),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
                ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double),
                ("sigma", ctypes.c_double), ("mobility", ctypes.c_double),
                ("width", ctypes.c_double), ("gravity", ctypes.c_double * 3),
                ("rho_ref", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class lbm_device(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("user", ctypes.c_void_p)]


class lbm_diag(ctypes.Structure):
    _fields_ = [("phase_mass", ctypes.c_double), ("pstar_sum", ctypes.c_double),
                ("momentum", ctypes.c_double * 3), ("kinetic", ctypes.c_double),
                ("umax", ctypes.c_double), ("centroid_l", ctypes.c_double * 3),
                ("velocity_l", ctypes.c_double * 3), ("centroid_g", ctypes.c_double * 3),
                ("velocity_g", ctypes.c_double * 3), ("p_l", ctypes.c_double),
                ("p_g", ctypes.c_double), ("n_l", ctypes.c_double), ("n_g", ctypes.c_double),
                ("nonfinite", ctypes.c_int32)]


class lbm_tuning(ctypes.Structure):
    _fields_ = [("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("z_chunk", ctypes.c_int32), ("persistent", ctypes.c_int32)]


_lib = None

_SIGS = {
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.c_int32,
                                  ctypes.POINTER(lbm_device), ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_init_phase": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_step_unbatched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_get_fields": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(lbm_diag)]),
    "lbm_diagnostics_all": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(lbm_diag)]),
    "lbm_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "lbm_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "lbm_get_fine_phase": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "lbm_set_fine_phase": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "lbm_get_state_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_get_fine_phase_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                                 ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_set_encoding": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "lbm_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(lbm_tuning)]),
    "lbm_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(lbm_tuning)]),
    "lbm_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(lbm_tuning)]),
    "lbm_set_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_bytes_per_update": (ctypes.c_double, [ctypes.c_void_p]),
    "lbm_total_nodes": (ctypes.c_int64, [ctypes.c_void_p]),
    "lbm_step_noalloc": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.POINTER(lbm_tuning),
                                        ctypes.c_void_p * 2, ctypes.c_void_p * 2, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "lbm_destroy": (None, [ctypes.c_void_p]),
    "lbm_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}


def load_library():
    """Load liblbm.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbm.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_2501_00846_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, ctx=None):
    if status != LBM_OK:
        msg = load_library().lbm_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")


def _f64(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_params(prob, precision="fp64"):
    """lbm_params from a workloads.Problem-like object."""
    p = lbm_params()
    p.nx, p.ny, p.nz = int(prob.nx), int(prob.ny), int(prob.nz)
    p.lattice = 0
    for a in range(3):
        p.bc[a] = int(prob.bc[a])
        p.gravity[a] = float(prob.gravity[a])
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.flags = (LITERAL_ADVECTION if getattr(prob, "literal_advection", False) else 0) | \
        (GRADIENT_CLOSURE if getattr(prob, "gradient_closure", False) else 0) | \
        (HIGH_ORDER_AC if getattr(prob, "high_order_ac", False) else 0) | \
        (FINE_PHASE if getattr(prob, "fine_phase", False) else 0)
    p.rho_l, p.rho_g = float(prob.rho_l), float(prob.rho_g)
    p.nu_l, p.nu_g = float(prob.nu_l), float(prob.nu_g)
    p.sigma, p.mobility, p.width = float(prob.sigma), float(prob.mobility), float(prob.width)
    p.rho_ref = float(prob.rho_ref)
    return p


# ---------------------------------------------------------------------------
# Functions with the C names (marshalling only)
# ---------------------------------------------------------------------------

def lbm_create(params: Sequence[lbm_params], device: Optional[lbm_device] = None):
    lib = load_library()
    arr = (lbm_params * len(params))(*params)
    out = ctypes.c_void_p()
    _check(lib.lbm_create(arr, len(params), ctypes.byref(device) if device is not None else None,
                          ctypes.byref(out)))
    return out


def lbm_init_phase(ctx, box, n, phi, u=None, pstar=None):
    phi = _f64(phi, n)
    u = None if u is None else _f64(u, 3 * n)
    pstar = None if pstar is None else _f64(pstar, n)
    _check(load_library().lbm_init_phase(ctx, box, _ptr(phi), _ptr(u), _ptr(pstar)), ctx)


def lbm_step(ctx, nsteps):
    _check(load_library().lbm_step(ctx, int(nsteps)), ctx)


def lbm_step_unbatched(ctx, nsteps):
    _check(load_library().lbm_step_unbatched(ctx, int(nsteps)), ctx)


def lbm_get_fields(ctx, box, n, rho=True, u=True, phi=True, p=True):
    outs = dict(rho=np.empty(n) if rho else None, u=np.empty(3 * n) if u else None,
                phi=np.empty(n) if phi else None, p=np.empty(n) if p else None)
    _check(load_library().lbm_get_fields(ctx, box, _ptr(outs["rho"]), _ptr(outs["u"]),
                                         _ptr(outs["phi"]), _ptr(outs["p"])), ctx)
    return outs


def lbm_diagnostics(ctx, box):
    d = lbm_diag()
    st = load_library().lbm_diagnostics(ctx, box, ctypes.byref(d))
    out = {name: (list(getattr(d, name)) if isinstance(getattr(d, name), ctypes.Array)
                  else getattr(d, name)) for name, _ in lbm_diag._fields_}
    _check(st, ctx)
    return out


def _diag_dict(d):
    return {name: (list(getattr(d, name)) if isinstance(getattr(d, name), ctypes.Array)
                   else getattr(d, name)) for name, _ in lbm_diag._fields_}


def lbm_diagnostics_all(ctx, n_boxes):
    arr = (lbm_diag * n_boxes)()
    st = load_library().lbm_diagnostics_all(ctx, arr)
    out = [_diag_dict(d) for d in arr]
    _check(st, ctx)
    return out


def lbm_get_state(ctx, box, n):
    st = np.empty(11 * n)
    _check(load_library().lbm_get_state(ctx, box, _ptr(st)), ctx)
    return st


def lbm_get_fine_phase(ctx, box, n):
    out = np.empty(8 * n)
    _check(load_library().lbm_get_fine_phase(ctx, box, _ptr(out)), ctx)
    return out


def lbm_set_fine_phase(ctx, box, n, phif):
    _check(load_library().lbm_set_fine_phase(ctx, box, _ptr(_f64(phif, 8 * n))), ctx)


def lbm_get_fine_phase_points(ctx, box, nodes):
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty(nodes.size)
    _check(load_library().lbm_get_fine_phase_points(ctx, box, nodes.size, _ptr(nodes), _ptr(out)), ctx)
    return out


def lbm_get_state_points(ctx, box, nodes):
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty(11 * nodes.size)
    _check(load_library().lbm_get_state_points(ctx, box, nodes.size, _ptr(nodes), _ptr(out)), ctx)
    return out.reshape(11, nodes.size)


def lbm_set_state(ctx, box, n, state):
    state = _f64(state, 11 * n)
    _check(load_library().lbm_set_state(ctx, box, _ptr(state)), ctx)


def lbm_set_encoding(ctx, box, offset, scale):
    off = _f64(offset, 10)
    sc = _f64(scale, 10)
    _check(load_library().lbm_set_encoding(ctx, box, _ptr(off), _ptr(sc)), ctx)


def lbm_set_tuning(ctx, block_x, block_y, z_chunk, persistent=0):
    t = lbm_tuning(block_x, block_y, z_chunk, persistent)
    _check(load_library().lbm_set_tuning(ctx, ctypes.byref(t)), ctx)


def lbm_get_tuning(ctx):
    t = lbm_tuning()
    _check(load_library().lbm_get_tuning(ctx, ctypes.byref(t)), ctx)
    return dict(block_x=t.block_x, block_y=t.block_y, z_chunk=t.z_chunk, persistent=t.persistent)


def lbm_autotune(ctx, steps):
    t = lbm_tuning()
    _check(load_library().lbm_autotune(ctx, int(steps), ctypes.byref(t)), ctx)
    return dict(block_x=t.block_x, block_y=t.block_y, z_chunk=t.z_chunk, persistent=t.persistent)


def lbm_set_graphs(ctx, enabled):
    _check(load_library().lbm_set_graphs(ctx, 1 if enabled else 0), ctx)


def lbm_synchronize(ctx):
    _check(load_library().lbm_synchronize(ctx), ctx)


def lbm_bytes_per_update(ctx):
    return load_library().lbm_bytes_per_update(ctx)


def lbm_total_nodes(ctx):
    return load_library().lbm_total_nodes(ctx)


def lbm_step_noalloc(params, tuning, phi, mom, enc_offset=None, enc_scale=None, parity=0, nsteps=1,
                     stream=None):
    """params: lbm_params; tuning: lbm_tuning or None; phi, mom: two device
    addresses each (the caller's ping-pong buffers); stream: a hipStream_t
    handle (int) or None."""
    off = None if enc_offset is None else _f64(enc_offset, 10)
    sc = None if enc_scale is None else _f64(enc_scale, 10)
    ph = (ctypes.c_void_p * 2)(*[int(v) for v in phi])
    mo = (ctypes.c_void_p * 2)(*[int(v) for v in mom])
    _check(load_library().lbm_step_noalloc(ctypes.byref(params), None if tuning is None else ctypes.byref(tuning),
                                           ph, mo, _ptr(off), _ptr(sc), int(parity), int(nsteps),
                                           None if stream is None else ctypes.c_void_p(int(stream))))


def row_pitch(precision, nx):
    """Stored row length (elements) of the device layout: nx rounded up so that
    rows of phi and of every moment field start on 64-byte boundaries (the
    layout lbm_step_noalloc documents)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    e = 8 if prec == 0 else (4 if prec == 1 else 2)
    q = 64 // e
    return (nx + q - 1) // q * q


def lbm_destroy(ctx):
    load_library().lbm_destroy(ctx)


def lbm_last_error(ctx=None):
    msg = load_library().lbm_last_error(ctx)
    return msg.decode() if msg else ""


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------

class Context:
    """A set of boxes stepped together on one GPU.

    problems: objects with the fields of workloads.Problem.  Device memory is
    allocated through PyTorch's caching allocator and all work runs on a
    dedicated torch stream (self.stream).
    """

    def __init__(self, problems, precision="fp64", device=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP GPU; none is visible")
        load_library()
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.precision = precision
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        self._blocks = {}

        def _alloc(nbytes, user):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except RuntimeError:
                return None
            ptr = t.data_ptr()
            self._blocks[ptr] = t
            return ptr

        def _free(ptr, user):
            self._blocks.pop(ptr, None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        dev = lbm_device(ctypes.c_void_p(self.stream.cuda_stream), self._alloc_cb, self._free_cb, None)
        self.params = [make_params(p, precision) for p in self.problems]
        self.ctx = lbm_create(self.params, dev)
        self.sizes = [p.nx * p.ny * p.nz for p in self.problems]

    # state -------------------------------------------------------------------
    def init_phase(self, box, phi, u=None, pstar=None):
        lbm_init_phase(self.ctx, box, self.sizes[box], phi, u, pstar)

    def init_case(self, box, case):
        self.init_phase(box, case.phi, case.u, case.pstar)

    def set_state(self, box, state):
        lbm_set_state(self.ctx, box, self.sizes[box], state)

    def get_state(self, box):
        p = self.problems[box]
        return lbm_get_state(self.ctx, box, self.sizes[box]).reshape(11, p.nz, p.ny, p.nx)

    def get_fine_phase(self, box):
        """The fine phase field (LBM_FINE_PHASE) as (2nz, 2ny, 2nx)."""
        p = self.problems[box]
        return lbm_get_fine_phase(self.ctx, box, self.sizes[box]).reshape(2 * p.nz, 2 * p.ny, 2 * p.nx)

    def fine_phase_at(self, box, points):
        """Fine phi at fine nodes (X, Y, Z) -> (n,)."""
        p = self.problems[box]
        pts = np.asarray(points, dtype=np.int64).reshape(-1, 3)
        nodes = pts[:, 0] + 2 * p.nx * (pts[:, 1] + 2 * p.ny * pts[:, 2])
        return lbm_get_fine_phase_points(self.ctx, box, nodes)

    def set_fine_phase(self, box, phif):
        lbm_set_fine_phase(self.ctx, box, self.sizes[box], phif)

    def state_at(self, box, points):
        """11 decoded state values at (x, y, z) points -> (11, n)."""
        p = self.problems[box]
        pts = np.asarray(points, dtype=np.int64).reshape(-1, 3)
        nodes = pts[:, 0] + p.nx * (pts[:, 1] + p.ny * pts[:, 2])
        return lbm_get_state_points(self.ctx, box, nodes)

    def fields(self, box):
        p = self.problems[box]
        out = lbm_get_fields(self.ctx, box, self.sizes[box])
        shape = (p.nz, p.ny, p.nx)
        return dict(rho=out["rho"].reshape(shape), u=out["u"].reshape((3,) + shape),
                    phi=out["phi"].reshape(shape), p=out["p"].reshape(shape))

    def diagnostics(self, box):
        return lbm_diagnostics(self.ctx, box)

    def diagnostics_all(self):
        return lbm_diagnostics_all(self.ctx, len(self.problems))

    # stepping ----------------------------------------------------------------
    def step(self, n=1):
        lbm_step(self.ctx, n)

    def step_unbatched(self, n=1):
        lbm_step_unbatched(self.ctx, n)

    def synchronize(self):
        lbm_synchronize(self.ctx)

    def set_graphs(self, enabled):
        lbm_set_graphs(self.ctx, enabled)

    def set_encoding(self, box, offset, scale):
        lbm_set_encoding(self.ctx, box, offset, scale)

    def set_tuning(self, block_x, block_y, z_chunk, persistent=0):
        lbm_set_tuning(self.ctx, block_x, block_y, z_chunk, persistent)

    def tuning(self):
        return lbm_get_tuning(self.ctx)

    def autotune(self, steps=4):
        return lbm_autotune(self.ctx, steps)

    @property
    def bytes_per_update(self):
        return lbm_bytes_per_update(self.ctx)

    @property
    def total_nodes(self):
        return lbm_total_nodes(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_destroy(self.ctx)
            self.ctx = None
            self._blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
