"""GPU parity of the gradient-closure variant (LBM_GRADIENT_CLOSURE: a2 from
the isotropic gradient of J, state phi, P, J) against the oracle's variant."""
import sys

import numpy as np
import pytest

from oracle import pointwise as PW
from oracle import scheme as S
from paper_2501_00846_amd import lbm, workloads
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem
from tests.gpu_util import (FIELDS, LazyState, field_tolerance, gpu_run_state, oracle_run_state,
                            quantize_state, rel_err, sample_points, smooth_random_state)

pytestmark = pytest.mark.gpu
P_, W_ = PERIODIC, WALL


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _prob(dims, bc, **kw):
    base = dict(rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1, sigma=0.01,
                gravity=(1e-5, -2e-5, 3e-5), rho_ref=0.5, gradient_closure=True)
    base.update(kw)
    return Problem(*dims, bc=bc, **base)


GRIDS = [
    ((37, 29, 23), (P_, P_, P_)),
    ((37, 29, 23), (W_, P_, W_)),
    ((33, 14, 11), (W_, W_, W_)),
    ((3, 4, 5), (P_, P_, P_)),
    ((5, 2, 7), (W_, W_, P_)),
    ((62, 7, 4), (P_, W_, P_)),
]


@pytest.mark.parametrize("dims,bc", GRIDS)
def test_one_step_fp64(dims, bc):
    prob = _prob(dims, bc)
    state = smooth_random_state(prob, seed=sum(dims) + 1)
    _log("closure one step fp64 %s bc=%s" % (dims, bc))
    got = gpu_run_state(prob, state, 1)
    ref = oracle_run_state(prob, state, 1)
    err = rel_err(got, ref)
    assert max(err.values()) <= 1e-12, err
    assert np.abs(got[5:]).max() == 0.0  # Q is not part of the state


@pytest.mark.parametrize("precision", ["fp32", "fp16_os"])
def test_one_step_reduced_precision(precision):
    prob = _prob((37, 29, 23), (W_, P_, W_))
    state = quantize_state(smooth_random_state(prob, seed=7), precision)
    _log("closure one step %s" % precision)
    got = gpu_run_state(prob, state, 1, precision=precision)
    ref = oracle_run_state(prob, state, 1)
    tol = field_tolerance(precision, ref)
    for k, name in enumerate(FIELDS[:5]):
        assert (np.abs(got[k] - ref[k]) <= tol[k]).all(), (name, np.abs(got[k] - ref[k]).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tile_shapes_bitwise(precision):
    prob = _prob((45, 23, 19), (W_, P_, W_))
    state = smooth_random_state(prob, 3)
    outs = []
    for t in [(32, 8, 64, 0), (34, 8, 7, 0), (34, 15, 16, 0), (32, 8, 5, 3)]:
        _log("closure tuning %s %s" % (t, precision))
        outs.append(gpu_run_state(prob, state, 3, precision=precision, tuning=t))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_static_droplet_100_steps_fp64():
    """C1 static droplet with the gradient closure: GPU and oracle agree within
    1e-10 (relative) on rho, u, phi and p after 100 steps."""
    case = workloads.static_droplet()
    prob = case.problem
    prob.gradient_closure = True
    _log("C1 closure 100 steps")
    with lbm.Context(prob, "fp64") as ctx:
        ctx.init_case(0, case)
        ctx.step(100)
        f = ctx.fields(0)
    st = S.run(S.initial_state(case.phi, case.u, case.pstar), prob, 100)
    ob = S.observables(st, prob)
    for name in ("rho", "phi", "u", "p"):
        a, b = f[name], ob[name]
        l2 = np.linalg.norm(a - b) / np.linalg.norm(b)
        mx = np.abs(a - b).max() / np.abs(b).max()
        assert l2 <= 1e-10 and mx <= 1e-10, (name, l2, mx)


def test_rising_bubble_full_size_one_step_fp64():
    """128 x 128 x 256 bubble with walls on every face, autotuned launch, one
    step checked at sampled nodes against the per-node oracle."""
    case = workloads.rising_bubble()
    prob = case.problem
    prob.gradient_closure = True
    pts = sample_points(prob, np.random.default_rng(5),
                        extra=[(64, 64, 32), (64, 64, 64), (48, 64, 48), (0, 0, 0), (127, 127, 255)])
    with lbm.Context(prob, "fp64") as ctx:
        ctx.init_case(0, case)
        ctx.autotune(2)
        ctx.init_case(0, case)
        _log("closure C2 tuning %s" % ctx.tuning())
        ctx.step(1)
        got = ctx.state_at(0, pts)
    ref = PW.step_points(LazyState(case.phi, None if case.pstar is None else case.pstar,
                                   tuple(None if case.u is None else case.u[a] for a in range(3))), prob, pts)
    refa = np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T])
    s_mom = max(np.abs(refa[1]).max(), np.abs(refa[2:5]).max())
    for k in range(5):
        scale = np.abs(refa[k]).max() if k == 0 else max(np.abs(refa[k]).max(), s_mom)
        err = np.abs(got[k] - refa[k]).max()
        _log("  %-3s err %.3e scale %.3e" % (FIELDS[k], err, scale))
        assert err <= 1e-12 * scale, (FIELDS[k], err, scale)
