"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/lbm.h, and rejects bad arguments with the documented
status codes before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2501_00846_amd import lbm
from paper_2501_00846_amd.workloads import Problem, PERIODIC, WALL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load_library()
    names = declared_functions()
    assert "lbm_create" in names and "lbm_step" in names and len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in lbm._SIGS, "binding lacks " + name


def _params(**kw):
    prob = Problem(8, 8, 8)
    p = lbm.make_params(prob)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _create(params, n=None):
    lib = lbm.load_library()
    out = ctypes.c_void_p()
    arr = (lbm.lbm_params * len(params))(*params)
    st = lib.lbm_create(arr, len(params) if n is None else n, None, ctypes.byref(out))
    return st, out, lbm.lbm_last_error(None)


@pytest.mark.parametrize("kw,code,frag", [
    (dict(nx=0), -1, "dims"),
    (dict(nz=-3), -1, "dims"),
    (dict(lattice=1), -2, "lattice"),
    (dict(width=0.0), -1, "width"),
    (dict(width=float("nan")), -1, "width"),
    (dict(nu_l=0.0), -1, "viscosit"),
    (dict(nu_g=-1.0), -1, "viscosit"),
    (dict(rho_g=0.0), -1, "densit"),
    (dict(sigma=-1.0), -1, "sigma"),
    (dict(mobility=-0.1), -1, "mobility"),
    (dict(precision=7), -1, "precision"),
    (dict(flags=16), -1, "flags"),
])
def test_create_rejects_bad_parameters(kw, code, frag):
    st, out, msg = _create([_params(**kw)])
    assert st == code
    assert out.value is None
    assert frag in msg


def test_create_rejects_wall_axis_of_one_node():
    p = _params(nz=1)
    p.bc[2] = WALL
    st, _, msg = _create([p])
    assert st == -1 and "wall" in msg


def test_create_rejects_mixed_precisions():
    st, _, msg = _create([_params(precision=0), _params(precision=1)])
    assert st == -2 and "precision" in msg


def test_create_rejects_null_and_counts():
    lib = lbm.load_library()
    out = ctypes.c_void_p()
    assert lib.lbm_create(None, 1, None, ctypes.byref(out)) == -1
    st, _, _ = _create([_params()], n=0)
    assert st == -1
    arr = (lbm.lbm_params * 1)(_params())
    assert lib.lbm_create(arr, 1, None, None) == -1


def test_null_context_calls_fail_cleanly():
    lib = lbm.load_library()
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_synchronize(None) == -1
    assert lib.lbm_get_fields(None, 0, None, None, None, None) == -1
    assert lib.lbm_get_fine_phase(None, 0, None) == -1
    assert lib.lbm_set_fine_phase(None, 0, None) == -1
    assert lib.lbm_get_fine_phase_points(None, 0, 0, None, None) == -1
    assert lib.lbm_bytes_per_update(None) == 0.0
    assert lib.lbm_total_nodes(None) == 0
    lib.lbm_destroy(None)


def test_python_binding_raises_lbm_error():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create([_params(nx=0)])
    assert ei.value.status == -1


def test_create_rejects_oversized_boxes():
    """Edges are at most 2^20, and a stored plane (rows padded to a multiple of
    32 elements) at most 2^28 elements, so per-lane byte offsets stay 32-bit."""
    st, _, msg = _create([_params(nx=(1 << 20) + 1)])
    assert st == -1 and "2^20" in msg
    st, _, msg = _create([_params(nx=16385, ny=16384, nz=1)])
    assert st == -1 and "2^28" in msg


def _noalloc(params, tuning=None, phi=(0x10000, 0x20000), mom=(0x30000, 0x40000), off=None, sc=None,
             parity=0, nsteps=0):
    lib = lbm.load_library()
    ph = (ctypes.c_void_p * 2)(*phi)
    mo = (ctypes.c_void_p * 2)(*mom)
    offa = None if off is None else (ctypes.c_double * 10)(*off)
    sca = None if sc is None else (ctypes.c_double * 10)(*sc)
    st = lib.lbm_step_noalloc(ctypes.byref(params) if params is not None else None,
                              ctypes.byref(tuning) if tuning is not None else None,
                              ph, mo, ctypes.cast(offa, ctypes.c_void_p) if offa else None,
                              ctypes.cast(sca, ctypes.c_void_p) if sca else None, parity, nsteps, None)
    return st, lbm.lbm_last_error(None)


def test_noalloc_step_checks_arguments_before_any_device_call():
    """The entry point that allocates nothing validates everything on the
    host: with valid arguments and nsteps = 0 it returns LBM_OK without a
    device (none exists here); every bad argument is rejected with its code."""
    assert _noalloc(_params())[0] == 0
    assert _noalloc(_params(precision=2), off=[0.0] * 10, sc=[1024.0] * 10)[0] == 0
    st, msg = _noalloc(None)
    assert st == -1 and "NULL" in msg
    st, msg = _noalloc(_params(nx=0))
    assert st == -1 and "dims" in msg
    st, msg = _noalloc(_params(), phi=(0x10000, 0))
    assert st == -1 and "NULL" in msg
    st, msg = _noalloc(_params(), mom=(0x30004, 0x40000))  # FP64 moments need 8-byte alignment
    assert st == -1 and "aligned" in msg
    st, msg = _noalloc(_params(), parity=2)
    assert st == -1 and "parity" in msg
    st, msg = _noalloc(_params(), nsteps=-1)
    assert st == -1 and "nsteps" in msg
    st, msg = _noalloc(_params(precision=2), off=[0.0] * 10)
    assert st == -1 and "together" in msg
    st, msg = _noalloc(_params(precision=2), off=[0.0] * 10, sc=[1000.0] * 10)
    assert st == -1 and "power of two" in msg
    st, msg = _noalloc(_params(precision=2), off=[float("inf")] + [0.0] * 9, sc=[1024.0] * 10)
    assert st == -1 and "finite" in msg
    # the scale and its reciprocal must be normal FP32 numbers, the offset finite in FP32
    st, msg = _noalloc(_params(precision=2), off=[0.0] * 10, sc=[1024.0] * 9 + [2.0 ** 127])
    assert st == -1 and "enc_scale[9]" in msg
    st, msg = _noalloc(_params(precision=3), off=[0.0] * 10, sc=[2.0 ** -127] + [1024.0] * 9)
    assert st == -1 and "enc_scale[0]" in msg
    st, msg = _noalloc(_params(precision=2), off=[0.0, 1e39] + [0.0] * 8, sc=[1024.0] * 10)
    assert st == -1 and "enc_offset[1]" in msg and "finite" in msg
    st, msg = _noalloc(_params(), tuning=lbm.lbm_tuning(33, 8, 4, 0))
    assert st == -2 and "unsupported" in msg
    st, msg = _noalloc(_params(), tuning=lbm.lbm_tuning(34, 8, 0, 0))
    assert st == -1 and "z_chunk" in msg


def test_noalloc_step_rejects_tile_lists_beyond_its_static_scratch():
    """1 MiB of scratch holds 32,736 tiles: a 512^3 box with 32 x 13 output
    columns per tile (640 tiles per z-chunk) fits from z-chunk 11 up."""
    big = _params(nx=512, ny=512, nz=512)
    assert _noalloc(big, tuning=lbm.lbm_tuning(34, 15, 11, 0))[0] == 0
    st, msg = _noalloc(big, tuning=lbm.lbm_tuning(34, 15, 10, 0))
    assert st == -1 and "scratch" in msg and "33280" in msg
    assert _noalloc(big)[0] == 0  # the default z-chunk fits


def test_high_order_variant_needs_four_nodes_on_wall_axes():
    p = _params(nz=3, flags=4)
    p.bc[2] = WALL
    st, _, msg = _create([p])
    assert st == -1 and ">= 4" in msg
    p2 = _params(nz=3, flags=4)  # periodic axes take any size
    p3 = _params(flags=4)
    p3.bc[0] = WALL
    st, _, msg = _create([p2, _params()])
    assert st == -2 and "LBM_HIGH_ORDER_AC" in msg
    assert _noalloc(p3)[0] == -2
    st, _, msg = _create([_params(flags=4), _params(flags=5)])  # printed advection in one box only
    assert st == -2 and "LBM_LITERAL_ADVECTION" in msg


def test_fine_phase_variant_checks():
    """LBM_FINE_PHASE (8): shared by every box of a context, not combined with
    the fourth-order update or the printed advection, not through
    lbm_step_noalloc (all checked before any device call)."""
    st, _, msg = _create([_params(flags=8), _params()])
    assert st == -2 and "LBM_FINE_PHASE" in msg
    st, _, msg = _create([_params(flags=8 | 4)])
    assert st == -2 and "LBM_FINE_PHASE" in msg
    st, _, msg = _create([_params(flags=8 | 1)])
    assert st == -2 and "LBM_FINE_PHASE" in msg
    st, msg = _noalloc(_params(flags=8))
    assert st == -2 and "LBM_FINE_PHASE" in msg
    p = _params(flags=8)
    p.mobility = 0.09  # 4 M * 5.78 > 2: the fine grid's FTCS diffusion would be unstable
    st, _, msg = _create([p])
    assert st == -1 and "mobility" in msg
