"""Pins of the fourth-order phase-field stencils of the higher-order
Allen-Cahn variant (the higher-order discretisation named as future work at
the end of Sec. II.A; readings H1-H3 of oracle/scheme.py).

The expected values are closed forms written here from the definitions, not
calls into the oracle's stencil code.  The isotropic D3Q27 stencils of
Sec. II.C map a plane wave exp(i k.x) to i s(k) (gradient) and l(k)
(Laplacian), with m(k) = 2/3 + cos(k)/3,

    s_a(k) = sin(k_a) prod_{b != a} m(k_b),   l(k) = 6 (m(k_x) m(k_y) m(k_z) - 1);

the same stencils at spacing 2 (scaled by 1/2 and 1/4) give s_a(2k)/2 and
l(2k)/4, so the fourth-order combinations have the symbols

    s4(k) = (4 s(k) - s(2k)/2) / 3,   l4(k) = (4 l(k) - l(2k)/4) / 3,

with s4(k) = k + O(|k|^5) and l4(k) = -|k|^2 + O(|k|^6).  Independently of the
symbols, the gradient must be exact on every polynomial of degree <= 4 and
the Laplacian on degree <= 5; the second-order stencils are not."""
import itertools

import numpy as np
import pytest

from oracle import pointwise as PW
from oracle import scheme as S
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem, tanh_profile


def _m(k):
    return 2.0 / 3.0 + np.cos(k) / 3.0


def s2(k):
    kx, ky, kz = k
    return np.array([np.sin(kx) * _m(ky) * _m(kz), np.sin(ky) * _m(kx) * _m(kz),
                     np.sin(kz) * _m(kx) * _m(ky)])


def s4(k):
    k = np.asarray(k, float)
    return (4.0 * s2(k) - 0.5 * s2(2.0 * k)) / 3.0


def l2(k):
    return 6.0 * (_m(k[0]) * _m(k[1]) * _m(k[2]) - 1.0)


def l4(k):
    k = np.asarray(k, float)
    return (4.0 * l2(k) - 0.25 * l2(2.0 * k)) / 3.0


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


def _wave(prob, modes, theta):
    k = 2 * np.pi * np.array(modes, dtype=float) / np.array([prob.nx, prob.ny, prob.nz], dtype=float)
    x, y, z = _grid(prob.shape)
    return k, k[0] * x + k[1] * y + k[2] * z + theta


@pytest.mark.parametrize("modes", [(1, 2, 1), (3, 1, 2), (0, 0, 4)])
def test_plane_wave_symbols(modes):
    prob = Problem(12, 10, 14)
    k, arg = _wave(prob, modes, 0.7)
    phi = np.cos(arg)
    fp = S.pad(phi, prob, 4)
    g = S.grad4(fp, 4)
    lap = S.laplacian4(fp, 4)
    expect_g = -np.sin(arg)[None] * s4(k).reshape(3, 1, 1, 1)
    assert np.abs(g - expect_g).max() < 1e-14
    assert np.abs(lap - l4(k) * phi).max() < 1e-13
    # the divergence of a field along one axis has the same symbol
    v = np.zeros((3,) + prob.shape)
    v[1] = phi
    d = S.divergence4(np.stack([S.pad(v[a], prob, 4) for a in range(3)]), 4)
    assert np.abs(d + np.sin(arg) * s4(k)[1]).max() < 1e-14


def test_symbols_are_fourth_order():
    """|s4(k) - k| and |l4(k) + |k|^2| shrink 32x and 64x when k halves
    (fifth- and sixth-order remainders); the second-order ones only 8x and 16x."""
    d = np.array([0.6, -0.3, 0.45])
    for k in (0.2 * d, 0.1 * d):
        pass
    e4 = [np.abs(s4(k) - k).max() for k in (0.2 * d, 0.1 * d)]
    e2 = [np.abs(s2(k) - k).max() for k in (0.2 * d, 0.1 * d)]
    f4 = [abs(l4(k) + k @ k) for k in (0.2 * d, 0.1 * d)]
    f2 = [abs(l2(k) + k @ k) for k in (0.2 * d, 0.1 * d)]
    assert e4[0] / e4[1] == pytest.approx(32.0, rel=0.02)
    assert e2[0] / e2[1] == pytest.approx(8.0, rel=0.02)
    assert f4[0] / f4[1] == pytest.approx(64.0, rel=0.02)
    assert f2[0] / f2[1] == pytest.approx(16.0, rel=0.02)


def _monomials(max_degree):
    return [e for e in itertools.product(range(max_degree + 1), repeat=3) if sum(e) <= max_degree]


def _poly_padded(coef, exps, n, h):
    """Polynomial sum c x^a y^b z^c on the nodes -h .. n+h-1 of each axis,
    centred at (n-1)/2, as an array padded by h (no wrap: the stencils read
    the polynomial itself beyond the interior)."""
    r = np.arange(-h, n + h, dtype=float) - (n - 1) / 2.0
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    val = sum(c * x ** a * y ** b * z ** e for c, (a, b, e) in zip(coef, exps))
    dx = sum(c * a * x ** max(a - 1, 0) * y ** b * z ** e for c, (a, b, e) in zip(coef, exps) if a)
    dy = sum(c * b * x ** a * y ** max(b - 1, 0) * z ** e for c, (a, b, e) in zip(coef, exps) if b)
    dz = sum(c * e * x ** a * y ** b * z ** max(e - 1, 0) for c, (a, b, e) in zip(coef, exps) if e)
    lap = sum(c * (a * (a - 1) * x ** max(a - 2, 0) * y ** b * z ** e
                   + b * (b - 1) * x ** a * y ** max(b - 2, 0) * z ** e
                   + e * (e - 1) * x ** a * y ** b * z ** max(e - 2, 0)) for c, (a, b, e) in zip(coef, exps))
    cut = (slice(h, h + n),) * 3
    return val, np.stack([dx[cut], dy[cut], dz[cut]]), lap[cut]


def test_exact_on_polynomials():
    rng = np.random.default_rng(7)
    n, h = 6, 4
    exps4 = _monomials(4)
    coef = rng.uniform(-1, 1, len(exps4))
    val, g_exact, lap_exact = _poly_padded(coef, exps4, n, h)
    scale = np.abs(g_exact).max()
    assert np.abs(S.grad4(val, h) - g_exact).max() < 1e-12 * scale
    assert np.abs(S.laplacian4(val, h) - lap_exact).max() < 1e-12 * np.abs(lap_exact).max()
    # the second-order stencils are not exact on quartics: the pin is sharp
    assert np.abs(S.grad(val, h) - g_exact).max() > 1e-2 * scale
    # the Laplacian is also exact on quintics
    exps5 = [e for e in _monomials(5) if sum(e) == 5]
    coef5 = rng.uniform(-1, 1, len(exps5))
    val5, _, lap5 = _poly_padded(coef5, exps5, n, h)
    assert np.abs(S.laplacian4(val5, h) - lap5).max() < 1e-11 * np.abs(lap5).max()
    assert np.abs(S.laplacian(val5, h) - lap5).max() > 1e-2 * np.abs(lap5).max()


def _advection_only(dims, literal, gravity=(0.0, 0.0, 0.0)):
    return Problem(*dims, bc=(PERIODIC,) * 3, rho_l=0.7, rho_g=0.7, nu_l=0.05, nu_g=0.08,
                   sigma=0.0, mobility=0.0, width=4.0, gravity=gravity, rho_ref=0.0,
                   literal_advection=literal, high_order_ac=True)


def _steppers(prob):
    yield "scheme", lambda st: S.step(st, prob)
    if prob.n_nodes <= 400:
        yield "pointwise", lambda st: PW.step_full(st, prob)


def _uniform(prob, U):
    return np.broadcast_to(np.asarray(U, float).reshape(3, 1, 1, 1), (3,) + prob.shape).copy()


@pytest.mark.parametrize("literal", [False, True])
def test_uniform_flow_advects_plane_wave(literal):
    """One step of phi' = phi - V.grad4(phi) on A + B cos(k.x + t) adds
    B (V.s4(k)) sin(k.x + t) exactly, with V = J (no force)."""
    prob = _advection_only((8, 6, 7), literal)
    U = np.array([0.031, -0.017, 0.023])
    k, arg = _wave(prob, (1, 1, 2), 0.4)
    phi = 0.5 + 0.3 * np.cos(arg)
    expect = phi + 0.3 * float(U @ s4(k)) * np.sin(arg)
    second = phi + 0.3 * float(U @ s2(k)) * np.sin(arg)
    assert np.abs(expect - second).max() > 1e-4  # the second-order update is told apart
    for name, step in _steppers(prob):
        st = step(S.initial_state(phi, _uniform(prob, U)))
        assert np.abs(st.phi - expect).max() < 1e-15, name


@pytest.mark.parametrize("literal", [False, True])
def test_uniform_force_advects_with_half_force_shift(literal):
    g = np.array([0.012, 0.018, -0.024])
    prob = _advection_only((6, 5, 7), literal, gravity=tuple(g))
    U = np.array([0.01, -0.02, 0.015])
    k, arg = _wave(prob, (1, 2, 1), 1.1)
    phi = 0.45 + 0.35 * np.cos(arg)
    expect = phi + 0.35 * float((U + 0.5 * g) @ s4(k)) * np.sin(arg)
    for name, step in _steppers(prob):
        st = step(S.initial_state(phi, _uniform(prob, U)))
        assert np.abs(st.phi - expect).max() < 1e-15, name


def test_diffusion_of_plane_wave():
    """sigma = 0, no flow, mobility M: the sharpening flux phi(1-phi)n of a
    constant-plus-wave field is not linear, so take a wave of amplitude small
    enough to leave a uniform field: phi = c exactly gives phi' = c; and the
    diffusion part alone (kappa_AC = 0 needs M = 0 with W -> inf) is checked
    through the Laplacian symbol on a width so large that the sharpening
    term is below rounding."""
    prob = Problem(9, 8, 10, bc=(PERIODIC,) * 3, rho_l=1.0, rho_g=1.0, nu_l=0.1, nu_g=0.1,
                   sigma=0.0, mobility=0.05, width=1e30, high_order_ac=True)
    k, arg = _wave(prob, (2, 1, 3), 0.2)
    phi = 0.5 + 0.2 * np.cos(arg)
    st = S.step(S.initial_state(phi), prob)
    expect = phi + 0.05 * 0.2 * l4(k) * np.cos(arg)
    assert np.abs(st.phi - expect).max() < 1e-15


def _random_state(prob, seed):
    rng = np.random.default_rng(seed)
    x, y, z = _grid(prob.shape)
    phi = 0.5 + 0.4 * np.sin(0.9 * x + 0.3) * np.cos(0.7 * y - 0.2 * z) + 0.05 * rng.uniform(-1, 1, prob.shape)
    st = S.initial_state(phi, 0.03 * rng.uniform(-1, 1, (3,) + prob.shape), 0.01 * rng.uniform(-1, 1, prob.shape))
    st.Q = S.q_full(1e-3 * rng.uniform(-1, 1, (6,) + prob.shape))
    return st


@pytest.mark.parametrize("bc", [(PERIODIC, PERIODIC, PERIODIC), (WALL, PERIODIC, WALL), (WALL, WALL, WALL)])
def test_phase_mass_conserved(bc):
    """The flux form of the fourth-order update conserves sum phi to rounding
    (the divergence telescopes; at walls with the ghost rules of H3)."""
    prob = Problem(7, 6, 8, bc=bc, rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1, sigma=0.01,
                   mobility=0.05, width=3.0, gravity=(0.0, 0.0, -1e-4), rho_ref=1.0, high_order_ac=True)
    st = _random_state(prob, 3)
    m0 = st.phi.sum()
    for _ in range(5):
        st = S.step(st, prob)
    assert abs(st.phi.sum() - m0) < 1e-13 * prob.n_nodes
    # the second-order update differs from the fourth-order one
    prob2 = Problem(**{**prob.__dict__, "high_order_ac": False})
    assert np.abs(S.step(_random_state(prob, 3), prob2).phi - S.step(_random_state(prob, 3), prob).phi).max() > 1e-4


@pytest.mark.parametrize("dims,bc", [((5, 4, 6), (WALL, PERIODIC, WALL)), ((4, 5, 4), (WALL, WALL, WALL)),
                                     ((3, 2, 5), (PERIODIC, PERIODIC, WALL))])
def test_push_equals_pull(dims, bc):
    """Whole-array step (push, padded arrays) = per-node pull step with explicit
    index maps, full physics, fourth-order phase update."""
    prob = Problem(*dims, bc=bc, rho_l=1.0, rho_g=0.01, nu_l=0.02, nu_g=0.1, sigma=0.01,
                   mobility=0.05, width=3.0, gravity=(1e-4, 0.0, -2e-4), rho_ref=1.0, high_order_ac=True)
    st = _random_state(prob, 11)
    a = S.step(st, prob)
    b = PW.step_full(st, prob)
    assert np.abs(a.phi - b.phi).max() < 1e-14
    assert np.abs(a.J - b.J).max() < 1e-14


def test_planar_interface_converges_at_fourth_order():
    """A slab at rest with tanh interfaces (R1), sigma = 0, run to its
    discrete equilibrium: the departure from the tanh profile is truncation
    error, which the interface width W controls (W nodes resolve the
    profile).  Doubling W divides it by ~16 for the fourth-order update (10.4
    measured at W = 4 -> 8, approaching 16) and by ~4 for the second-order one
    (3.5), and at W = 8 the fourth-order profile is ten times closer."""
    drift = {}
    for W, nz, N in ((4.0, 48, 400), (8.0, 96, 1500)):
        z = np.arange(nz, dtype=float)
        slab = tanh_profile(z - nz / 4 + 0.5, W) * tanh_profile(3 * nz / 4 - 0.5 - z, W)
        for ho in (False, True):
            prob = Problem(2, 2, nz, bc=(PERIODIC,) * 3, rho_l=1.0, rho_g=1.0, nu_l=0.1, nu_g=0.1,
                           sigma=0.0, mobility=0.05, width=W, high_order_ac=ho)
            st = S.initial_state(np.broadcast_to(slab.reshape(nz, 1, 1), prob.shape).copy())
            for _ in range(N):
                st = S.step(st, prob)
            drift[W, ho] = np.abs(st.phi[:, 0, 0] - slab).max()
    assert drift[4.0, True] / drift[8.0, True] > 8.0, drift
    assert 3.0 < drift[4.0, False] / drift[8.0, False] < 4.5, drift
    assert drift[8.0, True] < drift[8.0, False] / 5.0, drift
