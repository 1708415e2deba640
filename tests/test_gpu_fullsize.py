"""Parity at full workload sizes, in the launch configuration the benchmark
times: one step of the GPU from the seeded initial state, checked at sampled
nodes (walls, corners, interfaces, random) against the per-node oracle."""
import os
import sys

import numpy as np
import pytest

from oracle import pointwise as PW
from paper_2501_00846_amd import lbm, workloads
from tests.gpu_util import LazyState, field_tolerance, force_scale, quantize, sample_points, FIELDS

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _reference(case, precision, pts):
    """Per-node oracle step at pts from the stored (quantised) initial state."""
    prob = case.problem
    q = lambda a, k: None if a is None else quantize(a, precision, k)
    u = case.u
    st = LazyState(q(case.phi, 0), None if case.pstar is None else q(case.pstar, 1),
                   tuple(None if u is None else q(u[a], 2 + a) for a in range(3)))
    ref = PW.step_points(st, prob, pts)
    return np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])


def _compare(got, refa, precision, force=None):
    """FP64: 1e-12 of phi's scale for phi and of the population scale
    max(|P|, |J|, the moment's own) for each moment -- a moment is a signed
    sum of populations of that size, so its FP64 rounding is relative to it
    (a small off-diagonal Q at sampled nodes carries the rounding of sums of
    O(|P|) terms).  Reduced precision: field_tolerance."""
    tols = field_tolerance(precision, refa, force=force)
    if precision == "fp64":
        s_mom = max(np.abs(refa[1]).max(), np.abs(refa[2:5]).max())
        for k in range(1, 11):
            tols[k] = 1e-12 * max(np.abs(refa[k]).max(), s_mom) + 1e-300
    for k, name in enumerate(FIELDS):
        scale = np.abs(refa[k]).max()
        tol = tols[k]
        err = np.abs(got[k] - refa[k])
        _log("  %-4s max err %.3e scale %.3e worst/tol %.3f" % (name, err.max(), scale, (err / tol).max()))
        assert (err <= tol).all(), name


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
    force = None if precision == "fp64" else force_scale(prob, case.phi, case.pstar, pts)
    _compare(got, _reference(case, precision, pts), precision, force)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rising_bubble_128x128x256_one_step(precision):
    case = workloads.rising_bubble()
    extra = [(64, 64, 48 - 16), (64, 64, 48 + 16), (48, 64, 48), (80, 64, 48)]
    _check(case, precision, extra=extra)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16_os", "bf16_os"])
def test_drop_into_pool_512_one_step(precision):
    case = workloads.drop_into_pool()
    extra = [(256, 256, 127), (256, 256, 128), (256, 256, 220), (256, 256, 300), (0, 0, 511), (511, 511, 0)]
    _check(case, precision, tune=True, extra=extra)


@pytest.mark.parametrize("precision", ["fp32", "fp16_os", "bf16_os"])
def test_droplet_collision_256_one_step(precision):
    case = workloads.droplet_collision()
    extra = [(120, 128, 128), (136, 128, 128), (128, 128, 128), (96, 128, 128), (160, 128, 128)]
    _check(case, precision, extra=extra)


def test_ensemble_64_boxes_one_launch_one_step():
    """All 64 boxes of uneven sizes in one launch per step, in the tile shape
    and z-chunk the FP32 benchmark autotunes to, each box checked at sampled
    nodes against the per-node oracle, in FP64 (1e-12 of each box's
    population scale).  The FP32 form of the same launch is checked by
    test_ensemble_64_boxes_fp32_from_developed_state below."""
    cases = workloads.ensemble()
    with lbm.Context([c.problem for c in cases], "fp32") as ctx:
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
        ctx.autotune(2)
        t = ctx.tuning()
    _log("ensemble fp32 tuning %s" % t)
    with lbm.Context([c.problem for c in cases], "fp64") as ctx:
        bx = 34 if (t["block_x"], t["block_y"]) == (66, 8) else t["block_x"]  # 66 x 8 has no FP64 form
        ctx.set_tuning(bx, t["block_y"], t["z_chunk"], t["persistent"])
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
        ctx.step(1)
        rng = np.random.default_rng(77)
        for i, c in enumerate(cases):
            pts = sample_points(c.problem, rng, n_random=4)
            got = ctx.state_at(i, pts)
            refa = _reference(c, "fp64", pts)
            s_mom = max(np.abs(refa[1]).max(), np.abs(refa[2:5]).max())
            for k, name in enumerate(FIELDS):
                scale = np.abs(refa[k]).max() if k == 0 else max(np.abs(refa[k]).max(), s_mom)
                err = np.abs(got[k] - refa[k]).max()
                assert err <= 1e-12 * scale, (i, name, err, scale)
        _log("64 boxes checked")


def _state_reference(prob, state, pts):
    """Per-node oracle step at pts from a full (11, nz, ny, nx) state."""
    st = LazyState(state[0], state[1], tuple(state[2:5]), tuple(state[5:11]))
    ref = PW.step_points(st, prob, pts)
    return np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])


def test_ensemble_64_boxes_fp32_from_developed_state():
    """The 64-box ensemble in FP32, one launch per step in the tile shape and
    z-chunk the FP32 benchmark autotunes to.  The boxes first run 60 FP64
    steps from their seeded fields, so the drops oscillate and carry flow
    (from rest, one step moves P and J by less than FP32 rounding of the
    forces); that state, stored in FP32, is stepped once and every box is
    checked at sampled nodes against the per-node oracle on the same stored
    values, to the FP32 tolerance."""
    from tests.gpu_util import quantize_state

    cases = workloads.ensemble()
    probs = [c.problem for c in cases]
    with lbm.Context(probs, "fp64") as ctx:
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
        ctx.step(60)
        states = [quantize_state(ctx.get_state(i), "fp32") for i in range(len(cases))]
    _log("ensemble: 60 FP64 steps done")
    with lbm.Context(probs, "fp32") as ctx:
        for i, st in enumerate(states):
            ctx.set_state(i, st.reshape(-1))
        ctx.autotune(2)
        _log("ensemble fp32 tuning %s" % ctx.tuning())
        for i, st in enumerate(states):
            ctx.set_state(i, st.reshape(-1))
        ctx.step(1)
        rng = np.random.default_rng(78)
        for i, c in enumerate(cases):
            pts = sample_points(c.problem, rng, n_random=4)
            got = ctx.state_at(i, pts)
            refa = _state_reference(c.problem, states[i], pts)
            tols = field_tolerance("fp32", refa, force=force_scale(c.problem, states[i][0], states[i][1], pts))
            for k, name in enumerate(FIELDS):
                err = np.abs(got[k] - refa[k])
                assert (err <= tols[k]).all(), (i, name, float(err.max()), float(tols[k].max()))
    _log("64 boxes checked in FP32")


class _F64:
    """Read-only view of an FP32 array whose elements read as FP64 scalars, so
    that the per-node oracle computes in FP64 on FP32-stored inputs."""

    def __init__(self, a):
        self.a = a
        self.shape = a.shape

    def __getitem__(self, key):
        return np.float64(self.a[key])


def test_raindrop_train_fp32_one_step():
    """The raindrop train of Sec. III.D at the benchmark's size (500 x 500 x
    3000, walls on +-z), FP32, in the launch configuration of the benchmark's
    sweep (34 x 15 workgroups, z-chunk 128).  Its inputs are built in FP32, so
    they are stored exactly.  One step, sampled nodes (substrate, drops,
    interfaces, top wall) against the per-node oracle."""
    case = workloads.raindrop_train(dtype=np.float32)
    prob = case.problem
    pts = sample_points(prob, np.random.default_rng(31), n_random=12,
                        extra=[(250, 250, 0), (250, 250, 1), (250, 250, 75), (250, 250, 50),
                               (250, 250, 100), (225, 250, 75), (250, 250, 2999), (499, 499, 2998)])
    _log("raindrop train %dx%dx%d fp32: %d sampled nodes" % (prob.nx, prob.ny, prob.nz, len(pts)))
    with lbm.Context(prob, "fp32") as ctx:
        ctx.set_tuning(34, 15, 128, 0)
        ctx.init_case(0, case)
        ctx.step(1)
        got = ctx.state_at(0, pts)
    st = LazyState(_F64(case.phi), None, tuple(_F64(case.u[a]) for a in range(3)))
    ref = PW.step_points(st, prob, pts)
    refa = np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])
    _compare(got, refa, "fp32", force_scale(prob, case.phi, case.pstar, pts))


def test_eo_ga_sweep_fp32_one_step():
    """The twelve Eo-Ga bubbles (Sec. III.A) at the benchmark's size (200 x
    200 x 400 each), FP32, in one launch per step in the launch configuration
    of the benchmark's sweep (32 x 8 workgroups, z-chunk 8).  One step, each
    box at sampled nodes against the per-node oracle on the FP32-stored
    inputs."""
    cases = workloads.eo_ga_sweep()
    with lbm.Context([c.problem for c in cases], "fp32") as ctx:
        ctx.set_tuning(32, 8, 8, 0)
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
        ctx.step(1)
        rng = np.random.default_rng(32)
        for i, c in enumerate(cases):
            pts = sample_points(c.problem, rng, n_random=6, extra=[(100, 100, 50), (100, 100, 150)])
            got = ctx.state_at(i, pts)
            _log("Eo-Ga box %d (%s)" % (i, c.name))
            _compare(got, _reference(c, "fp32", pts), "fp32", force_scale(c.problem, c.phi, c.pstar, pts))


GOLDEN_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "rising_bubble_128x128x256_100steps.json")


def test_rising_bubble_128x128x256_100_steps_fp64():
    """The full rising-bubble workload (128 x 128 x 256, walls on every face,
    density ratio 1000, Eo 10, Mo 1e-3), 100 FP64 steps in the launch the
    benchmark picks, against the FP64 oracle's run at 64 fixed nodes (walls,
    corners, the bubble's poles and equator, random), stored by
    tests/golden/make_rising_bubble_100.py: every state field and rho, u, p
    within 1e-10 of the field's largest magnitude over the box."""
    import json

    with open(GOLDEN_C2) as fh:
        gold = json.load(fh)
    case = workloads.rising_bubble()
    prob = case.problem
    pts = [tuple(p) for p in gold["nodes"]]
    _log("rising bubble 128x128x256: %d steps fp64 against the stored oracle run" % gold["steps"])
    with lbm.Context(prob, "fp64") as ctx:
        ctx.init_case(0, case)
        ctx.autotune(2)
        ctx.init_case(0, case)
        _log("tuning %s" % ctx.tuning())
        ctx.step(gold["steps"])
        got = ctx.state_at(0, pts)
        f = ctx.fields(0)
    for k, name in enumerate(FIELDS):
        ref = np.array(gold["state"][name])
        err = np.abs(got[k] - ref).max() / gold["max_abs"][name]
        _log("  %-4s max err / field scale %.3e" % (name, err))
        assert err <= 1e-10, name
    idx = tuple(np.array([[z for x, y, z in pts], [y for x, y, z in pts], [x for x, y, z in pts]]))
    obs = {"rho": f["rho"][idx], "ux": f["u"][0][idx], "uy": f["u"][1][idx], "uz": f["u"][2][idx],
           "p": f["p"][idx]}
    for name, v in obs.items():
        err = np.abs(v - np.array(gold["observables"][name])).max() / gold["max_abs"][name]
        _log("  %-4s max err / field scale %.3e" % (name, err))
        assert err <= 1e-10, name


POOL_EXTRA = [(256, 256, 127), (256, 256, 128), (256, 256, 220), (256, 256, 300), (0, 0, 511), (511, 511, 0)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_drop_into_pool_512_high_order_one_step(precision):
    """The fourth-order phase update on the 512^3 drop into a pool, in both
    modes the benchmark times: one step at sampled nodes (walls, interface,
    random) against the per-node oracle's fourth-order stencils."""
    case = workloads.drop_into_pool()
    case.problem.high_order_ac = True
    _check(case, precision, tune=True, extra=POOL_EXTRA)


class _Restricted:
    """Coarse phi as the mean of the 8 fine nodes of each cell, evaluated on
    demand (optionally rounded to the storage type)."""

    def __init__(self, fine_at, shape, rnd):
        self.fine_at, self.shape, self.rnd = fine_at, shape, rnd
        self._cache = {}

    def __getitem__(self, idx):
        z, y, x = (int(v) for v in idx)
        if (z, y, x) not in self._cache:
            kids = [self.fine_at(2 * x + dx, 2 * y + dy, 2 * z + dz)
                    for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
            self._cache[(z, y, x)] = self.rnd(np.mean(kids))
        return self._cache[(z, y, x)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_drop_into_pool_512_fine_phase_one_step(precision):
    """The finer phase grid on the 512^3 drop into a pool (1024^3 fine
    nodes), in both modes the benchmark times: from the seeded initial
    fields (the fine phi their interpolation, the coarse phi its restriction)
    one step, checked at sampled coarse nodes against the per-node fine
    oracle: the flow part, the new coarse phi (the mean of the 8 updated fine
    nodes of the cell), and those 8 fine nodes themselves.  Reduced
    precision: the fine and coarse phi the oracle starts from are rounded to
    FP32 like the stored ones."""
    case = workloads.drop_into_pool()
    case.problem.fine_phase = True
    prob = case.problem
    rng = np.random.default_rng(321)
    pts = sample_points(prob, rng, n_random=16, extra=POOL_EXTRA)
    _log("%s fine phase %s: %d sampled nodes" % (case.name, precision, len(pts)))
    with lbm.Context(prob, precision) as ctx:
        ctx.init_case(0, case)
        ctx.autotune(2)
        ctx.init_case(0, case)
        _log("tuning %s" % ctx.tuning())
        ctx.step(1)
        got = ctx.state_at(0, pts)
        kids = [(2 * x + dx, 2 * y + dy, 2 * z + dz) for x, y, z in pts for dz in (0, 1) for dy in (0, 1)
                for dx in (0, 1)]
        got_fine = ctx.fine_phase_at(0, kids)
    rnd = (lambda v: float(v)) if precision == "fp64" else (lambda v: float(np.float32(v)))
    phi0 = quantize(case.phi, precision, 0)
    cache = {}

    def fine0(X, Y, Z):
        if (X, Y, Z) not in cache:
            cache[(X, Y, Z)] = rnd(PW.prolong_at(lambda x, y, z: phi0[z, y, x], prob, X, Y, Z))
        return cache[(X, Y, Z)]

    q = lambda a, k: None if a is None else quantize(a, precision, k)
    u = case.u
    st = LazyState(_Restricted(fine0, prob.shape, rnd), q(case.pstar, 1),
                   tuple(None if u is None else q(u[a], 2 + a) for a in range(3)))
    ref = PW.step_points_fine(st, fine0, prob, pts)
    refa = np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])
    force = None if precision == "fp64" else force_scale(prob, st.phi, q(case.pstar, 1), pts)
    _compare(got, refa, precision, force)
    # the fine nodes themselves: the 8 children of every sampled coarse node
    po = PW.FinePointOracle(st, fine0, prob)
    ref_fine = np.array([po.phase_at(*k) for k in kids])
    tol = 1e-12 if precision == "fp64" else 2e-5
    err = np.abs(got_fine - ref_fine).max()
    _log("  fine phi at %d fine nodes: max err %.3e" % (len(kids), err))
    assert err <= tol * np.abs(ref_fine).max(), err


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16_os"])
def test_drop_into_pool_512_gradient_closure_one_step(precision):
    """The gradient closure (state phi, P, J; a2 from the isotropic velocity
    gradient) on the 512^3 drop into a pool, in the modes it is benchmarked
    in: one step at sampled nodes against the per-node oracle."""
    case = workloads.drop_into_pool()
    case.problem.gradient_closure = True
    _check(case, precision, tune=True, extra=POOL_EXTRA)


def test_rising_bubble_128x128x256_gradient_closure_fp32_one_step():
    """The gradient closure on the walled 128 x 128 x 256 bubble in FP32 (its
    FP64 form is in test_gpu_closure.py)."""
    case = workloads.rising_bubble()
    case.problem.gradient_closure = True
    _check(case, "fp32", extra=[(64, 64, 32), (64, 64, 64), (48, 64, 48)])
