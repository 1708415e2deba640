"""Reduced-precision storage modes against the FP64 oracle.

One step from the same stored state (the host quantises the input exactly as
the GPU stores it): the GPU's FP32 arithmetic plus the re-encoding of the
output must stay within FP32 rounding on the field scale plus one storage
half-ulp of each value."""
import sys

import numpy as np
import pytest

from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem
from tests.gpu_util import (field_tolerance, gpu_run_state, oracle_run_state, quantize_state,
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
