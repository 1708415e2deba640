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
    # agreement is measured on that scale (some Q components are far smaller)
    s_mom = max(np.abs(refa[1]).max(), np.abs(refa[2:5]).max())
    for kf in range(11):
        scale = np.abs(refa[kf]).max() if kf == 0 else max(np.abs(refa[kf]).max(), s_mom)
        err = np.abs(got[kf] - refa[kf]).max()
        assert err <= 1e-12 * scale, (kf, err, scale)


def _fields_vs_oracle(fields, case, nsteps, tol=1e-10):
    """rho, phi, u, p of the GPU run against the oracle run from the same
    initial fields: relative L2 and max norms within tol."""
    st = S.run(S.initial_state(case.phi, case.u, case.pstar), case.problem, nsteps)
    ob = S.observables(st, case.problem)
    for name in ("rho", "phi", "u", "p"):
        a, b = fields[name], ob[name]
        l2 = np.linalg.norm(a - b) / np.linalg.norm(b)
        mx = np.abs(a - b).max() / np.abs(b).max()
        assert l2 <= tol and mx <= tol, (case.name, name, l2, mx)


def test_static_droplet_500_steps_fp64():
    """The static droplet over its whole 500-step run: FP64 GPU and oracle
    agree within 1e-10 on rho, u, phi and p."""
    case = workloads.static_droplet()
    _log("C1 32^3 500 steps fp64")
    with lbm.Context(case.problem, "fp64") as ctx:
        ctx.init_case(0, case)
        ctx.step(500)
        f = ctx.fields(0)
    _fields_vs_oracle(f, case, 500)


def test_walled_bubble_100_steps_fp64():
    """The rising-bubble set-up (walls on every face, buoyancy on the light
    phase, density ratio 1000, viscosity ratio 100) on a 32 x 32 x 64 box,
    100 steps, autotuned launch: FP64 GPU and oracle agree within 1e-10."""
    case = workloads.rising_bubble(nx=32, ny=32, nz=64, radius=6.0, zc=20.0)
    _log("walled bubble 32x32x64 100 steps fp64")
    with lbm.Context(case.problem, "fp64") as ctx:
        ctx.init_case(0, case)
        ctx.autotune(steps=4)
        # the tuner advanced the state: restart from the initial fields
        ctx.init_case(0, case)
        ctx.step(100)
        f = ctx.fields(0)
    _fields_vs_oracle(f, case, 100)


def test_three_ensemble_boxes_100_steps_fp64():
    """The three smallest boxes of the 64-box ensemble (uneven edges 25-53),
    stepped together in one launch per step for 100 steps: each matches its
    own oracle run within 1e-10."""
    cases = [workloads.ensemble_box(k) for k in (58, 56, 62)]
    _log("ensemble boxes 58, 56, 62: 100 steps fp64")
    with lbm.Context([c.problem for c in cases], "fp64") as ctx:
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
        ctx.step(100)
        fields = [ctx.fields(i) for i in range(len(cases))]
    for f, c in zip(fields, cases):
        _fields_vs_oracle(f, c, 100)


def test_translation_equivariance_bitwise():
    """Periodic box: shifting the initial state by an integer offset shifts
    the state after three steps by the same offset, bit for bit (no node's
    update depends on where its tile starts)."""
    prob = Problem(37, 29, 23, bc=(P_, P_, P_), rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1,
                   sigma=0.01, gravity=(1e-5, -2e-5, 3e-5), rho_ref=0.5)
    state = smooth_random_state(prob, seed=11)
    shift = (7, 3, 5)  # z, y, x
    _log("translation equivariance 37x29x23 shift %s" % (shift,))
    a = gpu_run_state(prob, state, 3)
    b = gpu_run_state(prob, np.roll(state, shift, axis=(1, 2, 3)), 3)
    assert np.array_equal(np.roll(a, shift, axis=(1, 2, 3)), b)
