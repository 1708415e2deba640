"""Fourth-order phase-field update (LBM_HIGH_ORDER_AC) on the GPU against the
FP64 oracle's higher-order variant, through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import scheme as S
from paper_2501_00846_amd import lbm, workloads
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem
from tests.gpu_util import (field_tolerance, gpu_run_state, oracle_run_state, quantize_state, rel_err,
                            smooth_random_state, FIELDS)

pytestmark = pytest.mark.gpu
P_, W_ = PERIODIC, WALL


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _prob(dims, bc, **kw):
    base = dict(rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1, sigma=0.01, mobility=0.05, width=3.0,
                gravity=(1e-5, -2e-5, 3e-5), rho_ref=0.5, high_order_ac=True)
    base.update(kw)
    return Problem(*dims, bc=bc, **base)


GRIDS = [
    ((37, 29, 23), (P_, P_, P_)),
    ((37, 29, 23), (W_, P_, W_)),
    ((33, 14, 11), (W_, W_, W_)),
    ((4, 5, 6), (W_, W_, W_)),     # wall axes at their minimum of 4 nodes
    ((3, 4, 5), (P_, P_, P_)),     # smaller than the wide stencil's reach
    ((62, 7, 4), (P_, W_, P_)),
]


@pytest.mark.parametrize("dims,bc", GRIDS)
def test_one_step_fp64(dims, bc):
    prob = _prob(dims, bc)
    state = smooth_random_state(prob, seed=sum(dims) + 3)
    _log("high-order one step fp64 %s bc=%s" % (dims, bc))
    got = gpu_run_state(prob, state, 1)
    ref = oracle_run_state(prob, state, 1)
    err = rel_err(got, ref)
    assert max(err.values()) <= 1e-12, err


@pytest.mark.parametrize("literal,gc", [(True, False), (False, True)])
def test_one_step_fp64_printed_advection_and_gradient_closure(literal, gc):
    prob = _prob((21, 17, 9), (P_, W_, W_), literal_advection=literal, gradient_closure=gc)
    state = smooth_random_state(prob, seed=7)
    if gc:
        state[5:] = 0.0  # the gradient closure keeps no Q
    got = gpu_run_state(prob, state, 2)
    ref = oracle_run_state(prob, state, 2)
    err = rel_err(got, ref)
    assert max(err.values()) <= 1e-12, err


def test_the_variant_changes_phi_only():
    """The flow solver keeps its second-order stencils: after one step from
    the same state, P, J and Q equal those of the second-order run bitwise
    and phi differs."""
    prob = _prob((37, 29, 23), (W_, P_, W_))
    state = smooth_random_state(prob, seed=5)
    ho = gpu_run_state(prob, state, 1)
    prob2 = _prob((37, 29, 23), (W_, P_, W_), high_order_ac=False)
    lo = gpu_run_state(prob2, state, 1)
    assert np.array_equal(ho[1:], lo[1:])
    assert np.abs(ho[0] - lo[0]).max() > 1e-6


@pytest.mark.parametrize("case_name", ["droplet", "walled_bubble"])
def test_100_steps_fp64(case_name):
    """100 FP64 steps match the oracle within 1e-10 (relative L2 and max) on
    rho, u, phi and p: a static droplet at density ratio 1000 (periodic) and
    a buoyant bubble between walls."""
    if case_name == "droplet":
        case = workloads.static_droplet(n=24, radius=6.0, seed=3, noise=1e-5)
    else:
        case = workloads.rising_bubble(nx=24, ny=20, nz=40, radius=6.0, zc=14.0, seed=9)
    case.problem.high_order_ac = True
    prob = case.problem
    _log("high-order %s 100 steps fp64" % case_name)
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


@pytest.mark.parametrize("precision,literal", [("fp32", False), ("fp16_os", False), ("fp32", True)])
def test_one_step_reduced_precision(precision, literal):
    """Stored state in FP32 / FP16 offset-scale: one step matches the oracle
    run from the host-quantised state within the storage modes' tolerance.
    The velocity and S are kept in FP32 and the phase update computes in
    FP32, the precision of the stored phi (flux form and printed advection)."""
    prob = _prob((33, 14, 11), (W_, W_, W_), rho_g=1e-3, nu_l=1 / 60, nu_g=1 / 6,
                 gravity=(0.0, 0.0, -1e-5), rho_ref=1.0, literal_advection=literal)
    state = smooth_random_state(prob, seed=44)
    _log("high-order one step %s literal=%s" % (precision, literal))
    got = gpu_run_state(prob, state, 1, precision)
    ref = oracle_run_state(prob, quantize_state(state, precision), 1)
    tol = field_tolerance(precision, ref)
    for k, name in enumerate(FIELDS):
        worst = float((np.abs(got[k] - ref[k]) / tol[k]).max())
        assert worst <= 1.0, (name, worst)


def test_phase_mass_conserved_with_walls():
    """sum phi is conserved to round-off over 200 steps with walls on every
    axis (the fourth-order flux divergence telescopes with mirrored ghosts)."""
    prob = _prob((20, 18, 24), (W_, W_, W_))
    state = smooth_random_state(prob, seed=8)
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_state(0, state.reshape(-1))
        m0 = ctx.diagnostics(0)["phase_mass"]
        ctx.step(200)
        m1 = ctx.diagnostics(0)["phase_mass"]
    assert abs(m1 - m0) <= 1e-12 * abs(m0), (m0, m1)


def test_ensemble_one_launch_equals_separate_boxes():
    """Two boxes in one context (one launch of each kernel per step) give
    bitwise the results of each box run alone."""
    probs = [_prob((24, 20, 9), (P_, P_, P_)), _prob((37, 29, 23), (P_, W_, W_))]
    states = [smooth_random_state(p, seed=60 + i) for i, p in enumerate(probs)]
    with lbm.Context(probs, "fp64") as ctx:
        for i, s in enumerate(states):
            ctx.set_state(i, s.reshape(-1))
        ctx.step(3)
        together = [ctx.get_state(i) for i in range(2)]
    for i, p in enumerate(probs):
        alone = gpu_run_state(p, states[i], 3)
        assert np.array_equal(together[i], alone), i
