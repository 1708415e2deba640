"""Helpers shared by the GPU tests (host side only)."""
import numpy as np

from oracle import scheme as S
from paper_2501_00846_amd import lbm

FIELDS = lbm.FIELDS


def state_array(st):
    """oracle State -> (11, nz, ny, nx) in the ABI field order."""
    return np.concatenate([st.phi[None], st.P[None], st.J, S.q_six(st.Q)])


def array_state(a):
    return S.State(a[0].copy(), a[1].copy(), a[2:5].copy(), S.q_full(a[5:11]))


def smooth_random_state(prob, seed, amp_u=0.02, amp_p=0.01, amp_q=1e-3):
    """Random but smooth state (phi in (0, 1)) so forces stay moderate."""
    rng = np.random.default_rng(seed)
    shape = prob.shape
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float) for n in shape), indexing="ij")
    k = rng.uniform(0.3, 1.1, size=(3, 3))
    ph = rng.uniform(0, 2 * np.pi, size=3)
    arg = sum(np.sin(k[i, 0] * x + k[i, 1] * y + k[i, 2] * z + ph[i]) for i in range(3)) / 3.0
    phi = 0.5 + 0.45 * arg + 0.02 * rng.uniform(-1, 1, shape)
    P = amp_p * rng.uniform(-1, 1, shape)
    J = amp_u * rng.uniform(-1, 1, (3,) + shape)
    Q6 = amp_q * rng.uniform(-1, 1, (6,) + shape)
    return np.concatenate([phi[None], P[None], J, Q6])


def rel_err(got, ref):
    """Per-field max-norm error relative to the field's max magnitude."""
    out = {}
    for k, name in enumerate(FIELDS):
        scale = max(np.abs(ref[k]).max(), 1e-300)
        out[name] = float(np.abs(got[k] - ref[k]).max() / scale)
    return out


def gpu_run_state(prob, state, nsteps, precision="fp64", tuning=None, graphs=True):
    with lbm.Context(prob, precision) as ctx:
        if tuning is not None:
            ctx.set_tuning(*tuning)
        ctx.set_graphs(graphs)
        ctx.set_state(0, state.reshape(-1))
        ctx.step(nsteps)
        return ctx.get_state(0)


def oracle_run_state(prob, state, nsteps):
    st = array_state(state)
    for _ in range(nsteps):
        st = S.step(st, prob)
    return state_array(st)
