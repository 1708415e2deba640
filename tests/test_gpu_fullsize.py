"""Parity at full workload sizes, in the launch configuration the benchmark
times: one step of the GPU from the seeded initial state, checked at sampled
nodes (walls, corners, interfaces, random) against the per-node oracle."""
import sys

import numpy as np
import pytest

from oracle import pointwise as PW
from paper_2501_00846_amd import lbm, workloads
from tests.gpu_util import LazyState, field_tolerance, quantize, sample_points, FIELDS

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(case, precision, tune=True, extra=()):
    prob = case.problem
    rng = np.random.default_rng(123)
    pts = sample_points(prob, rng, extra=extra)
    _log("%s %s: %d sampled nodes" % (case.name, precision, len(pts)))
    with lbm.Context(prob, precision) as ctx:
        ctx.init_case(0, case)
        if tune:
            ctx.autotune(2)      # the launch configuration the benchmark picks ...
            ctx.init_case(0, case)  # ... then restart from the initial state
        _log("tuning %s" % ctx.tuning())
        ctx.step(1)
        got = ctx.state_at(0, pts)
    q = lambda a, k: None if a is None else quantize(a, precision, k)
    u = case.u
    st = LazyState(q(case.phi, 0), None if case.pstar is None else q(case.pstar, 1),
                   tuple(None if u is None else q(u[a], 2 + a) for a in range(3)))
    ref = PW.step_points(st, prob, pts)
    refa = np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])
    tols = field_tolerance(precision, refa)
    for k, name in enumerate(FIELDS):
        scale = np.abs(refa[k]).max()
        tol = tols[k]
        err = np.abs(got[k] - refa[k])
        _log("  %-4s max err %.3e scale %.3e worst/tol %.3f" % (name, err.max(), scale, (err / tol).max()))
        assert (err <= tol).all(), name


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rising_bubble_128x128x256_one_step(precision):
    case = workloads.rising_bubble()
    extra = [(64, 64, 48 - 16), (64, 64, 48 + 16), (48, 64, 48), (80, 64, 48)]
    _check(case, precision, extra=extra)


@pytest.mark.parametrize("precision", ["fp32", "fp16_os"])
def test_drop_into_pool_512_one_step(precision):
    case = workloads.drop_into_pool()
    extra = [(256, 256, 127), (256, 256, 128), (256, 256, 220), (256, 256, 300), (0, 0, 511), (511, 511, 0)]
    _check(case, precision, tune=True, extra=extra)
