"""Parity of the HIP fused step (through the C ABI) with the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import scheme as S
from paper_2501_00846_amd import lbm, workloads
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem
from tests.gpu_util import gpu_run_state, oracle_run_state, rel_err, smooth_random_state

pytestmark = pytest.mark.gpu

P_, W_ = PERIODIC, WALL


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


GRIDS = [
    ((37, 29, 23), (P_, P_, P_)),   # several tiles, ragged in x and y
    ((37, 29, 23), (W_, P_, W_)),
    ((33, 14, 11), (W_, W_, W_)),
    ((3, 4, 5), (P_, P_, P_)),      # smaller than one tile
    ((1, 1, 8), (P_, P_, P_)),
    ((5, 2, 7), (W_, W_, P_)),
    ((62, 7, 4), (P_, W_, P_)),
]


@pytest.mark.parametrize("dims,bc", GRIDS)
def test_one_step_fp64_random_state(dims, bc):
    prob = Problem(*dims, bc=bc, rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1, sigma=0.01,
                   gravity=(1e-5, -2e-5, 3e-5), rho_ref=0.5)
    state = smooth_random_state(prob, seed=sum(dims))
    _log("one step fp64 %s bc=%s" % (dims, bc))
    got = gpu_run_state(prob, state, 1)
    ref = oracle_run_state(prob, state, 1)
    err = rel_err(got, ref)
    assert max(err.values()) <= 1e-12, err


def test_one_step_literal_advection():
    prob = Problem(21, 17, 9, bc=(P_, W_, P_), rho_g=0.05, literal_advection=True)
    state = smooth_random_state(prob, seed=5)
    got = gpu_run_state(prob, state, 2)
    ref = oracle_run_state(prob, state, 2)
    err = rel_err(got, ref)
    assert max(err.values()) <= 1e-12, err


def test_static_droplet_100_steps_fp64():
    """Static droplet 32^3, density ratio 1000, viscosity ratio 100: FP64 GPU
    matches the oracle within 1e-10 (relative) on rho, u and phi after 100 steps."""
    case = workloads.static_droplet()
    prob = case.problem
    _log("C1 32^3 100 steps fp64")
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


def test_largest_plane_fp64():
    """nx * ny = 2^28, the largest plane the library accepts: per-lane byte
    offsets inside one FP64 plane reach 2^31.  One step from a smooth phase
    field, checked at sampled nodes (edges of the plane included) against the
    per-node oracle."""
    from oracle import pointwise as PW
    from tests.gpu_util import LazyState, sample_points

    n = 1 << 14
    prob = Problem(n, n, 1, bc=(P_, P_, P_), rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1,
                   sigma=0.01, gravity=(1e-6, 0.0, 2e-6))
    k = 2 * np.pi * 64 / n
    x = np.arange(n, dtype=np.float64)
    phi = (0.5 + 0.45 * np.sin(k * x)[None, :] * np.cos(k * x)[:, None])[None]
    pts = sample_points(prob, np.random.default_rng(9), n_random=16,
                        extra=[(n - 1, n - 1, 0), (n - 1, 0, 0), (0, n - 1, 0), (n // 2, n - 1, 0)])
    _log("largest plane %dx%dx1 fp64, %d points" % (n, n, len(pts)))
    with lbm.Context(prob, "fp64") as ctx:
        ctx.init_phase(0, phi, None, None)
        ctx.step(1)
        got = ctx.state_at(0, pts)
    ref = PW.step_points(LazyState(phi), prob, pts)
    refa = np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])
    # each moment is a signed sum of populations of size max(|P|, |J|): FP64
    # agreement is judged on that scale (some Q components are far smaller)
    s_mom = max(np.abs(refa[1]).max(), np.abs(refa[2:5]).max())
    for kf in range(11):
        scale = np.abs(refa[kf]).max() if kf == 0 else max(np.abs(refa[kf]).max(), s_mom)
        err = np.abs(got[kf] - refa[kf]).max()
        assert err <= 1e-12 * scale, (kf, err, scale)
