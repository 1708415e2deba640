"""Runtime properties of the HIP path: bitwise determinism across tile
shapes and launch modes, graph replay, every output node written, restart
from a checkpoint, batched ensembles, observables and diagnostics."""
import sys

import numpy as np
import pytest

from oracle import scheme as S
from paper_2501_00846_amd import lbm, workloads
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem
from tests.gpu_util import (array_state, oracle_run_state, rel_err, smooth_random_state,
                            state_array)

pytestmark = pytest.mark.gpu
P_, W_ = PERIODIC, WALL


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _prob(dims, bc, **kw):
    base = dict(rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1, sigma=0.01,
                gravity=(1e-5, -2e-5, 3e-5), rho_ref=0.5)
    base.update(kw)
    return Problem(*dims, bc=bc, **base)


TUNINGS = [(32, 8, 64, 0), (34, 8, 7, 0), (34, 15, 16, 0), (32, 8, 5, 3), (34, 8, 1, 0), (18, 14, 4, 0)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tile_shapes_give_bitwise_identical_results(precision):
    """The update of a node does not depend on which workgroup computes it."""
    prob = _prob((45, 23, 19), (W_, P_, W_))
    state = smooth_random_state(prob, 3)
    outs = []
    tunings = TUNINGS + ([(66, 8, 9, 0)] if precision != "fp64" else [])
    for t in tunings:
        _log("tuning %s %s" % (t, precision))
        with lbm.Context(prob, precision) as ctx:
            ctx.set_tuning(*t)
            ctx.set_state(0, state.reshape(-1))
            ctx.step(3)
            outs.append(ctx.get_state(0))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_graph_replay_equals_eager_launches():
    """hipGraph replays (32-step chunks plus a remainder) give the same bits as
    eager launches, replay after replay with eager work in between."""
    prob = _prob((33, 17, 29), (P_, W_, P_))
    state = smooth_random_state(prob, 4)
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_graphs(False)
        ctx.set_state(0, state.reshape(-1))
        ref = []
        for _ in range(3):
            ctx.step(37)
            ref.append(ctx.get_state(0))
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_graphs(True)
        ctx.set_state(0, state.reshape(-1))
        for k in range(3):
            ctx.step(37)
            got = ctx.get_state(0)
            assert np.array_equal(got, ref[k]), k
            _ = ctx.diagnostics(0)  # eager work between replays


def test_every_output_node_is_written():
    """Poison the write buffer with NaN: a step must overwrite every node."""
    prob = _prob((37, 13, 11), (W_, W_, P_))
    state = smooth_random_state(prob, 6)
    nan_state = np.full_like(state, np.nan)
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_state(0, nan_state.reshape(-1))  # buffer A <- NaN
        ctx.step(1)                              # buffer B <- NaN results
        ctx.set_state(0, state.reshape(-1))      # buffer B <- valid
        ctx.step(1)                              # reads B, overwrites all of A
        got = ctx.get_state(0)
    assert np.isfinite(got).all()
    ref = oracle_run_state(prob, state, 1)
    assert max(rel_err(got, ref).values()) <= 1e-12


def test_checkpoint_resume_is_bitwise():
    prob = _prob((29, 31, 13), (P_, P_, W_))
    state = smooth_random_state(prob, 8)
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_state(0, state.reshape(-1))
        ctx.step(10)
        mid = ctx.get_state(0)
        ctx.step(10)
        full = ctx.get_state(0)
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_state(0, mid.reshape(-1))
        ctx.step(10)
        resumed = ctx.get_state(0)
    assert np.array_equal(resumed, full)


ENSEMBLE = [((24, 30, 27), (P_, P_, P_)), ((40, 9, 33), (W_, P_, P_)), ((7, 5, 9), (P_, P_, W_)),
            ((65, 33, 12), (W_, W_, W_)), ((3, 2, 4), (P_, P_, P_))]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16_os"])
def test_ensemble_one_launch_equals_separate_boxes(precision):
    """One launch over the tile list of every box equals each box stepped on
    its own, and equals one launch per box (the unbatched baseline), bit for
    bit in every storage mode."""
    probs = [_prob(d, bc, sigma=0.005 * (i + 1)) for i, (d, bc) in enumerate(ENSEMBLE)]
    states = [smooth_random_state(p, 10 + i) for i, p in enumerate(probs)]
    single = []
    for p, s in zip(probs, states):
        with lbm.Context(p, precision) as ctx:
            ctx.set_state(0, s.reshape(-1))
            ctx.step(4)
            single.append(ctx.get_state(0))
    for mode in ("batched", "unbatched"):
        with lbm.Context(probs, precision) as ctx:
            for i, s in enumerate(states):
                ctx.set_state(i, s.reshape(-1))
            if mode == "batched":
                ctx.step(4)
            else:
                ctx.step_unbatched(4)
            for i in range(len(probs)):
                assert np.array_equal(ctx.get_state(i), single[i]), (mode, i)
    if precision != "fp64":
        return
    # and the small boxes against the oracle
    for i in (2, 4):
        ref = oracle_run_state(probs[i], states[i], 4)
        assert max(rel_err(single[i], ref).values()) <= 1e-11


def test_observables_and_diagnostics_match_oracle():
    case = workloads.static_droplet(n=24, radius=6.0, seed=3, noise=1e-4)
    prob = case.problem
    with lbm.Context(prob, "fp64") as ctx:
        ctx.init_case(0, case)
        ctx.step(5)
        f = ctx.fields(0)
        d = ctx.diagnostics(0)
        st = ctx.get_state(0)
    ref_state = S.run(S.initial_state(case.phi, case.u, case.pstar), prob, 5)
    ob = S.observables(ref_state, prob)
    for name in ("rho", "phi", "u", "p"):
        assert np.abs(f[name] - ob[name]).max() <= 1e-11 * np.abs(ob[name]).max(), name
    dg = S.diagnostics(array_state(st), prob)
    # sums of signed values may cancel to ~0: absolute slack scales with the
    # sum of magnitudes (summation order differs between GPU and NumPy)
    abs_p = 1e-13 * np.abs(st[1]).sum()
    for key in ("phase_mass", "pstar_sum", "kinetic", "umax", "p_l", "p_g", "n_l", "n_g"):
        assert d[key] == pytest.approx(dg[key], rel=1e-10, abs=abs_p + 1e-30), key
    for key in ("momentum", "centroid_l", "velocity_l", "centroid_g", "velocity_g"):
        assert np.allclose(d[key], dg[key], rtol=1e-9, atol=1e-16), key
    assert d["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diagnostics_of_all_boxes_in_one_launch(precision):
    """lbm_diagnostics_all reduces every box of an ensemble in one launch and
    gives, box by box, bitwise what lbm_diagnostics gives; each box agrees with
    the oracle's diagnostics of its own (decoded) state."""
    dims = [(24, 20, 9), (37, 29, 23), (8, 8, 8), (61, 13, 17)]
    bcs = [(P_, P_, P_), (P_, W_, W_), (W_, P_, P_), (W_, W_, W_)]
    probs = [_prob(d, b) for d, b in zip(dims, bcs)]
    with lbm.Context(probs, precision) as ctx:
        for i, p in enumerate(probs):
            ctx.set_state(i, smooth_random_state(p, 40 + i).reshape(-1))
        ctx.step(3)
        together = ctx.diagnostics_all()
        alone = [ctx.diagnostics(i) for i in range(len(probs))]
        states = [ctx.get_state(i) for i in range(len(probs))]
    assert len(together) == len(probs)
    for i, (t, a) in enumerate(zip(together, alone)):
        assert t == a, i
        dg = S.diagnostics(array_state(states[i]), probs[i])
        abs_p = 1e-13 * np.abs(states[i][1]).sum()
        for key in ("phase_mass", "pstar_sum", "kinetic", "umax", "p_l", "p_g", "n_l", "n_g"):
            assert t[key] == pytest.approx(dg[key], rel=1e-10, abs=abs_p + 1e-30), (i, key)
        for key in ("momentum", "centroid_l", "velocity_l", "centroid_g", "velocity_g"):
            assert np.allclose(t[key], dg[key], rtol=1e-9, atol=1e-16), (i, key)


def test_nonfinite_state_is_reported():
    prob = _prob((8, 8, 8), (P_, P_, P_))
    state = smooth_random_state(prob, 1)
    state[1, 3, 4, 5] = np.nan
    with lbm.Context(prob, "fp64") as ctx:
        ctx.set_state(0, state.reshape(-1))
        with pytest.raises(lbm.LbmError) as ei:
            ctx.diagnostics(0)
        assert ei.value.status == -5
        with pytest.raises(lbm.LbmError) as ei:
            ctx.diagnostics_all()
        assert ei.value.status == -5
        with pytest.raises(lbm.LbmError):
            ctx.fields(0)


def test_step_before_init_is_rejected():
    prob = _prob((8, 8, 8), (P_, P_, P_))
    with lbm.Context(prob, "fp64") as ctx:
        with pytest.raises(lbm.LbmError) as ei:
            ctx.step(1)
        assert ei.value.status == -6


def test_rising_bubble_conservation_fp64():
    """Full-size rising bubble (walls, buoyancy): phase mass and sum p* are
    conserved to round-off over 200 steps."""
    case = workloads.rising_bubble()
    with lbm.Context(case.problem, "fp64") as ctx:
        ctx.init_case(0, case)
        d0 = ctx.diagnostics(0)
        ctx.step(200)
        d1 = ctx.diagnostics(0)
    assert abs(d1["phase_mass"] - d0["phase_mass"]) <= 1e-12 * d0["phase_mass"]
    assert abs(d1["pstar_sum"] - d0["pstar_sum"]) <= 1e-13 * case.problem.n_nodes
    assert d1["velocity_g"][2] > 0  # the bubble starts to rise
