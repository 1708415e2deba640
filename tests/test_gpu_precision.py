"""Reduced-precision storage modes against the FP64 oracle.

One step from the same stored state (the host quantises the input exactly as
the GPU stores it): the GPU's FP32 arithmetic plus the re-encoding of the
output must stay within FP32 rounding on the field scale plus one storage
half-ulp of each value."""
import sys

import numpy as np
import pytest

from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem
from tests.gpu_util import (DEFAULT_SCALE, field_tolerance, gpu_run_state, oracle_run_state, quantize_state,
                            smooth_random_state, FIELDS)

pytestmark = pytest.mark.gpu
P_, W_ = PERIODIC, WALL


@pytest.mark.parametrize("precision", ["fp32", "fp16_os", "bf16_os"])
@pytest.mark.parametrize("dims,bc", [((37, 29, 23), (P_, P_, P_)), ((33, 14, 11), (W_, W_, W_))])
def test_one_step_reduced_precision(precision, dims, bc):
    prob = Problem(*dims, bc=bc, rho_l=1.0, rho_g=1e-3, nu_l=1 / 60, nu_g=1 / 6, sigma=0.01,
                   gravity=(0.0, 0.0, -1e-5), rho_ref=1.0)
    state = smooth_random_state(prob, seed=sum(dims) + 1)
    got = gpu_run_state(prob, state, 1, precision)
    ref = oracle_run_state(prob, quantize_state(state, precision), 1)
    tol = field_tolerance(precision, ref)
    for k, name in enumerate(FIELDS):
        err = np.abs(got[k] - ref[k])
        worst = float((err / tol[k]).max())
        print("%s %s %s: max err %.3e (scale %.3e), worst err/tol %.3f" % (
            precision, dims, name, err.max(), np.abs(ref[k]).max(), worst), flush=True)
        assert worst <= 1.0, name
    sys.stdout.flush()


# a non-trivial encoding: offsets of the order of the field values, scales
# other than the defaults (powers of two)
ENC_OFFSET = np.array([2e-3, 1e-3, -2e-3, 5e-4, 1e-4, -1e-4, 2e-4, 5e-5, -5e-5, 1e-5])
ENC_SCALE = np.array([2048.0, 8192.0, 8192.0, 8192.0] + [32768.0] * 6)


@pytest.mark.parametrize("precision", ["fp16_os", "bf16_os"])
def test_one_step_with_offset_encoding(precision):
    """lbm_set_encoding with non-zero offsets: the stored state is the host
    quantisation (value - offset) * scale, and one step matches the oracle run
    from that quantised state, the output re-encoded with the same offsets."""
    from paper_2501_00846_amd import lbm

    prob = Problem(33, 14, 11, bc=(W_, W_, W_), rho_l=1.0, rho_g=1e-3, nu_l=1 / 60, nu_g=1 / 6,
                   sigma=0.01, gravity=(0.0, 0.0, -1e-5), rho_ref=1.0)
    state = smooth_random_state(prob, seed=41)
    q = quantize_state(state, precision, ENC_OFFSET, ENC_SCALE)
    with lbm.Context(prob, precision) as ctx:
        ctx.set_encoding(0, ENC_OFFSET, ENC_SCALE)
        ctx.set_state(0, state.reshape(-1))
        stored = ctx.get_state(0)
        assert np.array_equal(stored, q.reshape(stored.shape))
        ctx.step(1)
        got = ctx.get_state(0)
    ref = oracle_run_state(prob, q, 1)
    tol = field_tolerance(precision, ref, ENC_OFFSET)
    for k, name in enumerate(FIELDS):
        worst = float((np.abs(got[k] - ref[k]) / tol[k]).max())
        print("%s offset encoding %s: worst err/tol %.3f" % (precision, name, worst), flush=True)
        assert worst <= 1.0, name


@pytest.mark.parametrize("precision", ["fp16_os", "bf16_os"])
def test_set_encoding_reencodes_live_state(precision):
    """Changing the encoding of a box that holds a state re-encodes it: the
    state reads back as the host re-quantisation of the old values, and the
    next step equals a step from that state stored under the new encoding."""
    from paper_2501_00846_amd import lbm

    prob = Problem(37, 29, 23, rho_l=1.0, rho_g=1e-3, nu_l=1 / 60, nu_g=1 / 6, sigma=0.01)
    state = smooth_random_state(prob, seed=43)
    with lbm.Context(prob, precision) as ctx:
        ctx.set_state(0, state.reshape(-1))
        old = ctx.get_state(0)
        ctx.set_encoding(0, ENC_OFFSET, ENC_SCALE)
        new = ctx.get_state(0)
        expect = quantize_state(old, precision, ENC_OFFSET, ENC_SCALE).reshape(new.shape)
        assert np.array_equal(new, expect)
        ctx.step(2)
        stepped = ctx.get_state(0)
    with lbm.Context(prob, precision) as ctx:
        ctx.set_encoding(0, ENC_OFFSET, ENC_SCALE)
        ctx.set_state(0, new.reshape(-1))
        ctx.step(2)
        assert np.array_equal(ctx.get_state(0), stepped)


def test_set_encoding_is_ignored_outside_16_bit_modes():
    from paper_2501_00846_amd import lbm

    prob = Problem(9, 7, 5)
    state = smooth_random_state(prob, seed=45)
    for precision in ("fp64", "fp32"):
        with lbm.Context(prob, precision) as ctx:
            ctx.set_state(0, state.reshape(-1))
            before = ctx.get_state(0)
            ctx.set_encoding(0, ENC_OFFSET, ENC_SCALE)
            assert np.array_equal(ctx.get_state(0), before)


@pytest.mark.parametrize("precision", ["fp16_os", "bf16_os"])
def test_zero_offset_encode_equals_general_encode(precision):
    """The step's encode skips the subtraction when every offset is +0 (the
    default encoding).  Offsets of -0.0 take the general path, (v - (-0)) *
    scale, which equals v * scale in value (only -0 turns into +0): five
    steps of both boxes from the same state read back equal."""
    from paper_2501_00846_amd import lbm

    prob = Problem(33, 14, 11, bc=(W_, W_, W_), rho_l=1.0, rho_g=1e-3, nu_l=1 / 60, nu_g=1 / 6,
                   sigma=0.01, gravity=(0.0, 0.0, -1e-5), rho_ref=1.0)
    state = smooth_random_state(prob, seed=47)
    got = []
    for off in (np.zeros(10), np.full(10, -0.0)):
        with lbm.Context(prob, precision) as ctx:
            ctx.set_encoding(0, off, DEFAULT_SCALE)
            ctx.set_state(0, state.reshape(-1))
            ctx.step(5)
            got.append(ctx.get_state(0))
    assert np.array_equal(got[0], got[1])
