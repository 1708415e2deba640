"""Pins of the oracle's gradient-closure variant (Problem.gradient_closure):
a2 = -(cs^2/omega)(grad J + grad J^T) in place of the stored second moment
(the velocity-gradient form of a2 given with Eq. noneqts; readings G1-G4 of
scheme.py).  Each test fails on a wrong sign or prefactor of a2, a transposed
gradient, a wrong ghost rule for J, or a streaming/indexing slip."""
import numpy as np
import pytest

from oracle import pointwise as PW
from oracle import scheme as S
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem, random_state, tanh_profile
from tests.test_oracle_physics import layered_poiseuille

pytestmark = pytest.mark.filterwarnings("ignore")


def _state(phi, J, P=None):
    shape = phi.shape
    return S.State(phi, np.zeros(shape) if P is None else P, J, np.zeros((3, 3) + shape))


def test_velocity_gradient_plane_wave_symbol():
    """J_a = U_a cos(k.x): the isotropic gradient gives
    d_b J_a = -U_a sin(k.x) sin(k_b) prod_{c != b} m(k_c), m = 2/3 + cos/3,
    and a2 = -(cs^2/omega)(d_a J_b + d_b J_a) exactly (periodic grid)."""
    nx, ny, nz = 8, 6, 10
    prob = Problem(nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = np.array([2 * np.pi * 1 / nx, 2 * np.pi * 2 / ny, 2 * np.pi * 3 / nz])
    th = k[0] * x + k[1] * y + k[2] * z
    U = np.array([0.3, -0.2, 0.5])
    J = U.reshape(3, 1, 1, 1) * np.cos(th)
    m = 2 / 3 + np.cos(k) / 3
    sym = np.array([np.sin(k[b]) * np.prod([m[c] for c in range(3) if c != b]) for b in range(3)])
    gJ = S.velocity_gradient(J, prob)
    for a in range(3):
        for b in range(3):
            assert np.allclose(gJ[a, b], -U[a] * sym[b] * np.sin(th), atol=1e-14)
    om = 1.3
    A = S.gradient_closure_tensor(gJ, om)
    for a in range(3):
        for b in range(3):
            ref = -(1 / 3) / om * (-(U[a] * sym[b] + U[b] * sym[a]) * np.sin(th))
            assert np.allclose(A[a, b], ref, atol=1e-14)


def test_wall_ghosts_of_J_are_odd():
    """At a wall J's ghost is minus the mirrored value (R11), so a profile
    linear in the wall-normal coordinate through zero at the half-way wall,
    J_x = g (y + 1/2), has the exact gradient g at the first node."""
    prob = Problem(3, 6, 3, bc=(PERIODIC, WALL, PERIODIC))
    yy = np.arange(6, dtype=float)
    J = np.zeros((3, 3, 6, 3))
    J[0] = (0.01 * (yy + 0.5)).reshape(1, 6, 1)
    gJ = S.velocity_gradient(J, prob)
    assert np.allclose(gJ[0, 1][:, 0, :], 0.01, atol=1e-15)
    assert np.allclose(gJ[0, 0], 0.0, atol=1e-15) and np.allclose(gJ[0, 2], 0.0, atol=1e-15)


def test_uniform_flow_and_force():
    """Uniform J: a2 = 0; with a uniform acceleration the velocity gains exactly
    a per step (R4 holds in the variant) and P stays put."""
    prob = Problem(4, 3, 5, rho_l=1.0, rho_g=1.0, gravity=(1e-5, -2e-5, 3e-5), rho_ref=0.0,
                   gradient_closure=True)
    shape = prob.shape
    J = np.array([0.01, 0.02, -0.015]).reshape(3, 1, 1, 1) * np.ones((3,) + shape)
    st = _state(np.ones(shape), J, 0.003 * np.ones(shape))
    nf = S.node_fields(st, prob)
    assert np.abs(nf["A"]).max() < 1e-18
    st1 = S.step(st, prob)
    g = np.array(prob.gravity).reshape(3, 1, 1, 1)
    assert np.allclose(st1.J, J + g, rtol=0, atol=1e-17)
    assert np.allclose(st1.P, 0.003, rtol=0, atol=1e-17)
    assert np.abs(st1.Q).max() == 0.0


@pytest.mark.parametrize("bc", [(PERIODIC,) * 3, (WALL, PERIODIC, WALL), (WALL,) * 3])
def test_push_equals_pull(bc):
    """Whole-array push form and per-node pull form agree (tiny grids)."""
    prob, phi, ps, J, _ = random_state(6, 5, 7, 11, bc=bc, rho_l=1.0, rho_g=0.05, nu_l=0.02,
                                       nu_g=0.1, sigma=0.01, gravity=(1e-5, -2e-5, 3e-5),
                                       rho_ref=0.5, gradient_closure=True)
    st = _state(phi, J, ps)
    a = S.step(st, prob)
    b = PW.step_full(st, prob)
    for x, y in ((a.phi, b.phi), (a.P, b.P), (a.J, b.J)):
        assert np.abs(x - y).max() < 1e-14


@pytest.mark.parametrize("bc", [(PERIODIC,) * 3, (WALL, WALL, PERIODIC)])
def test_conservation(bc):
    """sum phi and sum P are conserved to round-off; with every force zero
    (sigma = 0, equal densities, no gravity) and periodic, sum J is too."""
    prob, phi, ps, J, _ = random_state(7, 6, 5, 4, bc=bc, rho_l=1.0, rho_g=0.1, nu_l=0.05,
                                       nu_g=0.1, sigma=0.01, gradient_closure=True)
    st = _state(0.2 + 0.6 * phi, J * 0.2, ps)
    m0, p0 = st.phi.sum(), st.P.sum()
    for _ in range(5):
        st = S.step(st, prob)
    assert abs(st.phi.sum() - m0) < 1e-12 * abs(m0)
    assert abs(st.P.sum() - p0) < 1e-13
    prob1 = Problem(7, 6, 5, rho_l=1.0, rho_g=1.0, nu_l=0.05, nu_g=0.08, sigma=0.0,
                    gradient_closure=True)
    st = _state(0.2 + 0.6 * phi, J * 0.2, ps)
    j0 = st.J.sum(axis=(1, 2, 3))
    for _ in range(5):
        st = S.step(st, prob1)
    assert np.allclose(st.J.sum(axis=(1, 2, 3)), j0, rtol=0, atol=1e-14)


def _decay_rate_error(L, t0, t1):
    prob = Problem(1, L, 1, nu_l=0.05, nu_g=0.05, gradient_closure=True)
    y = np.arange(L)
    k = 2 * np.pi / L
    J = np.zeros((3, 1, L, 1))
    J[0, 0, :, 0] = 1e-4 * np.sin(k * y)
    st = _state(np.ones((1, L, 1)), J)
    amps = []
    for t in range(t1 + 1):
        if t in (t0, t1):
            amps.append(2 / L * np.sum(st.J[0, 0, :, 0] * np.sin(k * y)))
        st = S.step(st, prob)
    rate = np.log(amps[0] / amps[1]) / (t1 - t0)
    return rate / (0.05 * k ** 2) - 1.0


def test_shear_wave_decay():
    """phi = 1: the shear wave decays as exp(-nu k^2 t), nu = cs^2 (1/omega - 1/2),
    up to the second-order truncation of the finite-difference gradient:
    within 1 % at 64 nodes per wavelength, and the error shrinks about 4x
    when the grid spacing halves (measured 2.0 % at 32, 0.5 % at 64)."""
    e32 = _decay_rate_error(32, 100, 400)
    e64 = _decay_rate_error(64, 400, 1600)
    assert abs(e64) < 0.01, e64
    assert 3.0 < e32 / e64 < 5.0, (e32, e64)


def test_closure_agrees_with_moment_scheme():
    """The moment scheme's own non-equilibrium tensor of a decaying shear wave
    (A = Q + a a/4 with a = 0) matches -(cs^2/omega)(grad u + grad u^T) of its
    velocity: this fixes the sign and prefactor of G1 independently of the
    variant's code path."""
    L = 32
    prob = Problem(1, L, 1, nu_l=0.05, nu_g=0.05)
    y = np.arange(L)
    k = 2 * np.pi / L
    J = np.zeros((3, 1, L, 1))
    J[0, 0, :, 0] = 1e-4 * np.sin(k * y)
    st = _state(np.ones((1, L, 1)), J)
    for _ in range(200):
        st = S.step(st, prob)
    om = S.relaxation(0.05)
    A_ce = S.gradient_closure_tensor(S.velocity_gradient(st.J, prob), om)
    qxy = st.Q[0, 1, 0, :, 0]
    ref = A_ce[0, 1, 0, :, 0]
    assert np.abs(qxy - ref).max() < 0.02 * np.abs(ref).max()


@pytest.mark.parametrize("rho_g,nu_g", [(1.0, 0.04), (0.25, 0.05)])
def test_layered_poiseuille(rho_g, nu_g):
    """Two layers between no-slip walls driven by a uniform acceleration: the
    steady profile matches the sharp-interface closed form (density ratio 4
    exercises the viscous correction with the gradient-closure a2)."""
    Ny = 32
    h = Ny / 2
    g = 2e-6
    prob = Problem(1, Ny, 1, bc=(PERIODIC, WALL, PERIODIC), rho_l=1.0, rho_g=rho_g,
                   nu_l=0.1, nu_g=nu_g, sigma=1e-4, width=3.0, mobility=0.02,
                   gravity=(g, 0.0, 0.0), rho_ref=0.0, gradient_closure=True)
    yc = np.arange(Ny) - (Ny - 1) / 2
    phi0 = tanh_profile(-yc, prob.width).reshape(1, Ny, 1)
    ua = layered_poiseuille(yc, h, 1.0 * 0.1, rho_g * nu_g, 1.0 * g, rho_g * g)
    J = np.zeros((3, 1, Ny, 1))
    J[0, 0, :, 0] = ua
    st = S.initial_state(phi0, J)
    for _ in range(6000):
        st = S.step(st, prob)
    u = S.observables(st, prob)["u"][0, 0, :, 0]
    err = np.abs(u - ua).max() / np.abs(ua).max()
    assert err < 0.03, err
