"""lbm_step_noalloc (the entry point for callers that cannot allocate device
memory) against lbm_step of a context, through the C ABI: the same state in
caller-owned buffers of the documented layout, the same number of steps, and
bitwise-identical results.  Two calls in a row on the same GPU, the second on
a smaller box, so a stale descriptor or tile list left in the static scratch
array by the first call would show."""
import numpy as np
import pytest

from paper_2501_00846_amd import lbm
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem

from tests.gpu_util import smooth_random_state

pytestmark = pytest.mark.gpu

DEFAULT_SCALE = np.array([1024.0] + [4096.0] * 3 + [65536.0] * 6)


def _dtypes(precision):
    if precision == "fp64":
        return np.float64, np.float64
    if precision == "fp32":
        return np.float32, np.float32
    return np.float32, (np.float16 if precision == "fp16_os" else "bf16")


def _to_bf16(x32):
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16  # round to nearest even (finite values)
    return u.astype(np.uint16)


def _from_bf16(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32)


def pack(state, prob, precision, nmom):
    """(11, nz, ny, nx) decoded state -> host byte images of the phi and mom
    buffers in the device layout (rows padded to the pitch; padding zero)."""
    nz, ny, nx = prob.nz, prob.ny, prob.nx
    pitch = lbm.row_pitch(precision, nx)
    tp, tm = _dtypes(precision)
    phi = np.zeros((nz, ny, pitch), dtype=tp)
    phi[:, :, :nx] = state[0].astype(tp)
    if precision in ("fp16_os", "bf16_os"):
        # pairs of fields (2p, 2p + 1) as one 32-bit word per node, the even
        # field in the low half: [z][p][y][x][half]
        mom = np.zeros((nz, nmom // 2, ny, pitch, 2), dtype=np.uint16 if tm == "bf16" else np.float16)
        for k in range(nmom):
            enc = state[1 + k].astype(np.float32) * np.float32(DEFAULT_SCALE[k])  # offset 0
            mom[:, k // 2, :, :nx, k % 2] = _to_bf16(enc) if tm == "bf16" else enc.astype(np.float16)
        return phi, mom
    mom = np.zeros((nz, nmom, ny, pitch), dtype=tm)
    for k in range(nmom):
        mom[:, k, :, :nx] = state[1 + k].astype(tm)
    return phi, mom


def unpack(phi, mom, prob, precision, nmom):
    nz, ny, nx = prob.nz, prob.ny, prob.nx
    out = np.zeros((11, nz, ny, nx))
    out[0] = phi[:, :, :nx].astype(np.float64)
    for k in range(nmom):
        m = mom[:, k // 2, :, :nx, k % 2] if precision in ("fp16_os", "bf16_os") else mom[:, k, :, :nx]
        if precision == "bf16_os":
            m = _from_bf16(m) * np.float32(1.0 / DEFAULT_SCALE[k])
        elif precision == "fp16_os":
            m = m.astype(np.float32) * np.float32(1.0 / DEFAULT_SCALE[k])
        out[1 + k] = m.astype(np.float64)
    return out


def run_pair(prob, precision, nsteps, seed):
    import torch

    nmom = 4 if prob.gradient_closure else 10
    state = smooth_random_state(prob, seed)
    # the context path: set the state, read back what it stored, step
    with lbm.Context(prob, precision) as ctx:
        ctx.set_state(0, state.reshape(-1))
        start = ctx.get_state(0)
        ctx.step(nsteps)
        ctx.synchronize()
        ref = ctx.get_state(0)
    # caller-owned buffers in the documented layout, filled from the host
    phi_h, mom_h = pack(start, prob, precision, nmom)
    dev = torch.device("cuda", 0)
    bufs = []
    for _ in range(2):
        bufs.append((torch.from_numpy(phi_h.view(np.uint8).copy()).to(dev),
                     torch.from_numpy(mom_h.view(np.uint8).copy()).to(dev)))
    # the host image must decode to the state the context stored
    assert np.array_equal(unpack(phi_h, mom_h, prob, precision, nmom), start)
    params = lbm.make_params(prob, precision)
    stream = torch.cuda.current_stream(dev)
    print("noalloc: %dx%dx%d %s %d steps" % (prob.nx, prob.ny, prob.nz, precision, nsteps), flush=True)
    lbm.lbm_step_noalloc(params, None, [bufs[0][0].data_ptr(), bufs[1][0].data_ptr()],
                         [bufs[0][1].data_ptr(), bufs[1][1].data_ptr()], parity=0, nsteps=nsteps,
                         stream=stream.cuda_stream)
    torch.cuda.synchronize()
    out = bufs[nsteps & 1]
    got = unpack(out[0].cpu().numpy().view(phi_h.dtype).reshape(phi_h.shape),
                 out[1].cpu().numpy().view(mom_h.dtype).reshape(mom_h.shape), prob, precision, nmom)
    return got, ref


CASES = [
    ("fp64", False), ("fp32", False), ("fp16_os", False), ("bf16_os", False), ("fp32", True),
]


@pytest.mark.parametrize("precision,gc", CASES)
def test_noalloc_step_equals_context_step_twice(precision, gc):
    big = Problem(70, 37, 29, (PERIODIC, WALL, WALL), gradient_closure=gc)
    small = Problem(24, 20, 9, (PERIODIC, PERIODIC, PERIODIC), gradient_closure=gc)
    for prob, nsteps, seed in ((big, 5, 11), (small, 4, 12)):
        got, ref = run_pair(prob, precision, nsteps, seed)
        assert np.all(np.isfinite(got))
        bad = np.argwhere(got != ref)
        assert bad.size == 0, "%s %dx%dx%d: %d values differ, first at %s: %r vs %r" % (
            precision, prob.nx, prob.ny, prob.nz, len(bad), bad[0], got[tuple(bad[0])], ref[tuple(bad[0])])
