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


# ---------------------------------------------------------------------------
# Storage quantisation done on the host (never read back from the GPU): the
# oracle starts from exactly the values the GPU stores at set_state / init.
# ---------------------------------------------------------------------------
DEFAULT_SCALE = np.array([1024.0] + [4096.0] * 3 + [65536.0] * 6)


def _bf16_round(x32):
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32)


def quantize(values, precision, field, offset=None, scale=None):
    """Stored-and-decoded value of `values` for field index (0 = phi, 1..10 moments).

    The 16-bit modes store (f32(v) - offset) * scale rounded to FP16 / BF16
    (the subtraction rounded to FP32, the power-of-two scale exact) and decode
    f32(stored) * (1/scale) + offset in FP32 (the product is exact, so a fused
    multiply-add and a separate add round alike).  offset / scale: the 10
    per-moment values of lbm_set_encoding (default 0 and DEFAULT_SCALE)."""
    v = np.asarray(values, dtype=np.float64)
    if precision == "fp64":
        return v.copy()
    f32 = v.astype(np.float32)
    if precision == "fp32" or field == 0:
        return f32.astype(np.float64)
    off = np.float32(0.0 if offset is None else offset[field - 1])
    s = np.float32(DEFAULT_SCALE[field - 1] if scale is None else scale[field - 1])
    x = (f32 - off) * s
    if precision == "fp16_os":
        h = x.astype(np.float16).astype(np.float32)
    elif precision == "bf16_os":
        h = _bf16_round(x)
    else:
        raise ValueError(precision)
    return (h * (np.float32(1.0) / s) + off).astype(np.float64)


def quantize_state(state, precision, offset=None, scale=None):
    return np.stack([quantize(state[k], precision, k, offset, scale) for k in range(11)])


# relative half-ulp of the storage format per field
def storage_rel(precision, field):
    if precision == "fp64":
        return 2.0 ** -53
    if precision == "fp32" or field == 0:
        return 2.0 ** -24
    return 2.0 ** -11 if precision == "fp16_os" else 2.0 ** -8


class _Vec:
    """Read-only (k, z, y, x) view built from per-component arrays (or None = 0)."""

    def __init__(self, comps, shape):
        self.comps = comps
        self.shape = shape

    def __getitem__(self, key):
        rest = key[1:]
        return np.array([0.0 if c is None else float(c[rest]) for c in self.comps])


class _Ten:
    def __init__(self, comps6, shape):
        self.c = comps6

    def __getitem__(self, key):
        rest = key[2:]
        q = [0.0 if c is None else float(c[rest]) for c in self.c]
        return np.array([[q[0], q[3], q[4]], [q[3], q[1], q[5]], [q[4], q[5], q[2]]])


class LazyState:
    """Minimal State for the per-node oracle on big boxes: phi, P (arrays or
    None), J (3 arrays or None), Q6 (6 arrays or None)."""

    def __init__(self, phi, P=None, J=(None, None, None), Q6=(None,) * 6):
        self.phi = phi
        shape = phi.shape
        self.P = P if P is not None else np.broadcast_to(np.float64(0.0), shape)
        self.J = _Vec(list(J), shape)
        self.Q = _Ten(list(Q6), shape)


def sample_points(prob, rng, n_random=24, extra=()):
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    pts = set()
    for c in [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, 0), (nx - 1, 0, nz - 1),
              (nx // 2, ny // 2, 0), (nx // 2, ny // 2, 1), (nx // 2, ny // 2, nz - 1),
              (nx // 2, ny // 2, nz - 2), (0, ny // 3, nz // 2), (nx - 1, ny // 3, nz // 2),
              (nx // 3, 0, nz // 2), (nx // 3, ny - 1, nz // 2), (1, 1, 1)]:
        pts.add(c)
    for _ in range(n_random):
        pts.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    for c in extra:
        pts.add(tuple(int(v) for v in c))
    # the fixed probes assume at least 3 nodes per axis: clamp them into the box
    clamp = lambda v, n: max(0, min(v, n - 1))
    return sorted({(clamp(x, nx), clamp(y, ny), clamp(z, nz)) for x, y, z in pts})


def field_tolerance(precision, ref, offset=None, force=None):
    """Per-field absolute tolerance for one step from the same stored state.

    FP64: 1e-12 of the field scale.  Reduced precision (FP32 arithmetic):
    phi within 2e-5; every moment within 1e-5 of the
    leading population scale max(|P|, |J|) -- each moment, Q included, is a
    signed sum of populations of that size, and the chemical potential is a
    near-cancelling difference whose FP32 rounding is amplified by 1/rho_g in
    the light phase (measured up to 3e-6 of that scale for density ratio
    1000) -- plus one storage half-ulp of the stored value (v - offset) in the
    16-bit modes (offset: the 10 per-moment offsets, default 0).  ref may be
    (11, ...).

    force (optional, one value per node of ref, from force_scale): the
    magnitude of the terms that FP32 arithmetic sums into the acceleration
    a = F/rho around each node.  Each moment then also gets 4 FP32 rounding
    units (2^-24) of it: the Laplacian (two roundings of its filtered sums),
    the chemical-potential difference and its product with grad(phi)/rho each
    round once, and the populations carry a with weights of order one.  Where
    the populations themselves are small (a bubble at rest, strong surface
    tension) this term, not the population scale, bounds the rounding."""
    ref = np.asarray(ref)
    tol = np.empty_like(ref)
    s_mom = max(np.abs(ref[1]).max(), np.abs(ref[2:5]).max())
    f_term = 0.0 if force is None else 4.0 * 2.0 ** -24 * np.asarray(force)
    for k in range(11):
        scale = np.abs(ref[k]).max()
        if precision == "fp64":
            tol[k] = 1e-12 * scale + 1e-300
        elif k == 0:
            tol[k] = 2e-5 * scale + 1.01 * storage_rel(precision, k) * np.abs(ref[k]) + 1e-300
        else:
            off = 0.0 if offset is None or precision not in ("fp16_os", "bf16_os") else offset[k - 1]
            tol[k] = (1e-5 * max(scale, s_mom) + f_term
                      + 1.01 * storage_rel(precision, k) * np.abs(ref[k] - off) + 1e-300)
    return tol


def _axis_index(i, n, wall):
    """Node index along an axis of n nodes: periodic wrap, or the half-way
    mirror of a wall (-1 -> 0, -2 -> 1)."""
    if not wall:
        return i % n
    if i < 0:
        i = -1 - i
    elif i >= n:
        i = 2 * n - 1 - i
    return min(max(i, 0), n - 1)


def force_scale(prob, phi, pstar, pts):
    """Per sampled node (x, y, z): the largest, over the node and its 26
    neighbours (whose post-collision populations stream into it), of
    (|beta4 phi (phi-1)(phi-1/2)| + kappa (6 phi + |lap phi|) + |p*| drho/3)
    |grad phi| / rho(phi) -- the sizes of the surface-tension and pressure
    force terms per unit mass before they cancel, with the Laplacian's own
    summands (6 phi) in place of its value.  phi, pstar: (nz, ny, nx) arrays
    (or indexable alike; pstar None means 0).  Wall axes mirror."""
    beta4 = 48.0 * prob.sigma / prob.width
    kappa = 1.5 * prob.sigma * prob.width
    drho = prob.rho_l - prob.rho_g
    dims = (prob.nx, prob.ny, prob.nz)
    walls = tuple(b == 1 for b in prob.bc)
    w1 = (1.0, 4.0, 1.0)
    out = np.empty(len(pts))
    for j, (x, y, z) in enumerate(pts):
        idx = [[_axis_index(c + d, dims[a], walls[a]) for d in range(-2, 3)] for a, c in enumerate((x, y, z))]
        patch = np.array([[[float(phi[zz, yy, xx]) for xx in idx[0]] for yy in idx[1]] for zz in idx[2]])
        ps = None if pstar is None else np.array(
            [[[float(pstar[zz, yy, xx]) for xx in idx[0][1:4]] for yy in idx[1][1:4]] for zz in idx[2][1:4]])
        best = 0.0
        for kz in range(1, 4):
            for ky in range(1, 4):
                for kx in range(1, 4):
                    c = patch[kz, ky, kx]
                    g = np.zeros(3)
                    lap = 0.0
                    for cz in (-1, 0, 1):
                        for cy in (-1, 0, 1):
                            for cx in (-1, 0, 1):
                                w = w1[cx + 1] * w1[cy + 1] * w1[cz + 1] / 216.0
                                v = patch[kz + cz, ky + cy, kx + cx]
                                g += 3.0 * w * v * np.array([cx, cy, cz])
                                lap += 6.0 * w * (v - c)
                    rho = prob.rho_g + min(max(c, 0.0), 1.0) * drho
                    p = 0.0 if ps is None else abs(ps[kz - 1, ky - 1, kx - 1])
                    t = (abs(beta4 * c * (c - 1.0) * (c - 0.5)) + kappa * (6.0 * abs(c) + abs(lap))
                         + p * drho / 3.0) * np.linalg.norm(g) / rho
                    best = max(best, t)
        out[j] = best
    return out
