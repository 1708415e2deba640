"""The second workloads on the GPU (Sec. III.D raindrop train onto a
substrate; Sec. III.A Eo-Ga deformation-regime sweep as one batched launch):
one step against the per-node oracle at sampled nodes, then a few hundred
steps that keep the state finite and the phase mass conserved."""
import sys

import numpy as np
import pytest

from oracle import pointwise as PW
from paper_2501_00846_amd import lbm, workloads
from tests.gpu_util import FIELDS, LazyState, sample_points

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _reference(case, pts):
    u = case.u
    st = LazyState(case.phi, case.pstar, tuple(None if u is None else u[a] for a in range(3)))
    ref = PW.step_points(st, case.problem, pts)
    return np.concatenate([ref["phi"][None], ref["P"][None], ref["J"].T,
                           np.stack([ref["Q"][:, 0, 0], ref["Q"][:, 1, 1], ref["Q"][:, 2, 2],
                                     ref["Q"][:, 0, 1], ref["Q"][:, 0, 2], ref["Q"][:, 1, 2]])])


def _check(got, refa, tag):
    s_mom = max(np.abs(refa[1]).max(), np.abs(refa[2:5]).max())
    for k, name in enumerate(FIELDS):
        scale = np.abs(refa[k]).max() if k == 0 else max(np.abs(refa[k]).max(), s_mom)
        err = np.abs(got[k] - refa[k]).max()
        assert err <= 1e-12 * scale, (tag, name, err, scale)


def test_raindrop_train():
    case = workloads.raindrop_train(nx=64, ny=64, nz=240, radius=8.0)
    prob = case.problem
    pts = sample_points(prob, np.random.default_rng(11),
                        extra=[(32, 32, 0), (32, 32, 1), (32, 32, 16), (32, 32, 24), (32, 32, 40), (32, 32, 239)])
    _log("raindrop train %s: %d points" % (prob.shape, len(pts)))
    with lbm.Context(prob, "fp64") as ctx:
        ctx.init_case(0, case)
        m0 = ctx.diagnostics(0)["phase_mass"]
        ctx.step(1)
        _check(ctx.state_at(0, pts), _reference(case, pts), "raindrop")
        ctx.step(399)
        d = ctx.diagnostics(0)
    assert d["nonfinite"] == 0
    assert abs(d["phase_mass"] - m0) <= 1e-11 * m0


def test_eo_ga_sweep_batched():
    cases = workloads.eo_ga_sweep(nx=32, ny=32, nz=64, radius=8.0, g=5e-5)
    with lbm.Context([c.problem for c in cases], "fp64") as ctx:
        for i, c in enumerate(cases):
            ctx.init_case(i, c)
        m0 = [ctx.diagnostics(i)["phase_mass"] for i in range(len(cases))]
        ctx.step(1)
        rng = np.random.default_rng(12)
        for i, c in enumerate(cases):
            pts = sample_points(c.problem, rng, n_random=6, extra=[(16, 16, 16), (16, 16, 8), (8, 16, 16)])
            _check(ctx.state_at(i, pts), _reference(c, pts), c.name)
        _log("12 sweep boxes checked after one step")
        ctx.step(299)
        for i, c in enumerate(cases):
            p = c.problem
            # at R = 8 the Ga = 100 liquid relaxes at omega ~ 1.98 (nu = 0.0016)
            # and is not resolved; the paper's R = 50 gives omega ~ 1.74 there
            if 1.0 / (3.0 * p.nu_l + 0.5) > 1.9:
                continue
            d = ctx.diagnostics(i)
            assert d["nonfinite"] == 0, c.name
            assert abs(d["phase_mass"] - m0[i]) <= 1e-11 * m0[i], c.name
