"""Pins of the finer phase-field grid variant (the finer grid named as future
work at the end of Sec. II.A; readings F1-F6 of oracle/scheme.py).

Expected values are closed forms written here from the readings, not calls
into the oracle's stencil code.  Fine node I of an axis sits at I/2 - 1/4
(cell centred, F1).  On the fine grid the isotropic D3Q27 stencils of
Sec. II.C map a plane wave sin(k.x) to s(kh)/h cos(k.x) (gradient) and
l(kh)/h^2 sin(k.x) (Laplacian), h = 1/2, with m(k) = 2/3 + cos(k)/3,

    s_a(k) = sin(k_a) prod_{b != a} m(k_b),   l(k) = 6 (m(k_x) m(k_y) m(k_z) - 1).
"""
import numpy as np
import pytest

from oracle import pointwise as PW
from oracle import scheme as S
from paper_2501_00846_amd.workloads import PERIODIC, WALL, Problem

H = 0.5


def _m(k):
    return 2.0 / 3.0 + np.cos(k) / 3.0


def _s(k):
    kx, ky, kz = k
    return np.array([np.sin(kx) * _m(ky) * _m(kz), np.sin(ky) * _m(kx) * _m(kz),
                     np.sin(kz) * _m(kx) * _m(ky)])


def _l(k):
    return 6.0 * (_m(k[0]) * _m(k[1]) * _m(k[2]) - 1.0)


def _fine_positions(prob):
    """(x, y, z) of the fine nodes, arrays of shape (2nz, 2ny, 2nx) (F1)."""
    z, y, x = np.meshgrid(np.arange(2 * prob.nz), np.arange(2 * prob.ny), np.arange(2 * prob.nx),
                          indexing="ij")
    return x / 2.0 - 0.25, y / 2.0 - 0.25, z / 2.0 - 0.25


def _quiet_problem(nx, ny, nz, bc=(PERIODIC,) * 3, mobility=0.0, width=4.0):
    """Equal densities, no surface tension, no gravity: a = 0 and u = J."""
    return Problem(nx, ny, nz, bc=bc, rho_l=1.0, rho_g=1.0, nu_l=0.1, nu_g=0.1, sigma=0.0,
                   mobility=mobility, width=width, fine_phase=True)


def _state(prob, phif, J):
    st = S.initial_state(S.restrict(phif), u=J)
    return st


@pytest.mark.parametrize("bc", [(PERIODIC,) * 3, (WALL,) * 3, (PERIODIC, WALL, WALL)])
def test_interpolation_keeps_the_total(bc):
    prob = Problem(7, 6, 5, bc=bc)
    g = np.random.default_rng(3).random((5, 6, 7))
    f = S.prolong(g, prob)
    assert f.shape == (10, 12, 14)
    assert abs(f.sum() / 8.0 - g.sum()) <= 1e-13 * g.sum()


def test_interpolation_is_exact_on_linear_fields():
    """Trilinear interpolation reproduces a linear field at the fine node
    positions of F1 (away from the wall ghosts, here a periodic axis would
    wrap, so the check covers the interior)."""
    prob = Problem(7, 6, 5, bc=(WALL,) * 3)
    z, y, x = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    lin = 0.3 + 0.1 * x - 0.2 * y + 0.05 * z
    fx, fy, fz = _fine_positions(prob)
    exact = 0.3 + 0.1 * fx - 0.2 * fy + 0.05 * fz
    got = S.prolong(lin, prob)
    assert np.abs(got - exact)[1:-1, 1:-1, 1:-1].max() < 1e-15


def test_wall_ghost_velocity_vanishes_on_the_wall():
    """A velocity interpolated with the odd ghost (minus the mirrored value)
    is half the first node's value at the first fine node (x = -1/4), i.e. it
    falls linearly to zero on the wall at x = -1/2."""
    prob = Problem(6, 4, 4, bc=(WALL, PERIODIC, PERIODIC))
    u = np.random.default_rng(4).random((4, 4, 6))
    f = S.prolong(u, prob, odd=True)
    # along y and z the field is interpolated as usual; compare against the
    # same interpolation of the first coarse column, halved
    col = S.prolong(np.repeat(u[:, :, :1], 6, axis=2), Problem(6, 4, 4))
    assert np.allclose(f[:, :, 0], 0.5 * col[:, :, 0], rtol=0, atol=1e-15)


def test_restriction_of_the_interpolation_of_a_quadratic():
    """Per axis R(P(g)) = g + (g(i-1) - 2g(i) + g(i+1))/8, so x^2 + y^2 + z^2
    gains 3/4 away from the boundary (F6)."""
    prob = Problem(8, 7, 6, bc=(WALL,) * 3)
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij")
    q = (x * x + y * y + z * z).astype(np.float64)
    got = S.restrict(S.prolong(q, prob))
    assert np.abs(got - (q + 0.75))[1:-1, 1:-1, 1:-1].max() < 1e-12


def test_restriction_conserves_the_phase_mass():
    f = np.random.default_rng(5).random((6, 8, 10))
    assert abs(S.restrict(f).sum() - f.sum() / 8.0) < 1e-13


def test_fine_advection_of_a_plane_wave():
    """Uniform u = J (no forces), M = 0: one fine step is
    phi - (U . s(kh)/h) B cos(k.x) exactly (F3: the interpolation of a uniform
    u is that u; F4: the 1/h scaling; F1: the node positions)."""
    prob = _quiet_problem(8, 6, 5)
    fx, fy, fz = _fine_positions(prob)
    k = np.array([2 * np.pi / 4.0, 2 * np.pi / 3.0, -2 * np.pi / 2.5])  # periods of the box
    A, B = 0.5, 0.2
    arg = k[0] * fx + k[1] * fy + k[2] * fz
    phif = A + B * np.sin(arg)
    U = np.array([0.03, -0.02, 0.015])
    J = np.broadcast_to(U.reshape(3, 1, 1, 1), (3,) + prob.shape).copy()
    _, got = S.step_fine(_state(prob, phif, J), phif, prob)
    expect = phif - np.dot(U, _s(k * H)) / H * B * np.cos(arg)
    assert np.abs(got - expect).max() < 1e-15


def test_fine_diffusion_of_a_plane_wave():
    """u = 0, W so large that the sharpening coefficient 4M/W vanishes: one
    fine step is phi + M l(kh)/h^2 B sin(k.x)."""
    M = 0.05
    prob = _quiet_problem(8, 6, 5, mobility=M, width=1e30)
    fx, fy, fz = _fine_positions(prob)
    k = np.array([2 * np.pi / 8.0, -2 * np.pi / 3.0, 2 * np.pi / 5.0])
    A, B = 0.5, 0.2
    arg = k[0] * fx + k[1] * fy + k[2] * fz
    phif = A + B * np.sin(arg)
    J = np.zeros((3,) + prob.shape)
    _, got = S.step_fine(_state(prob, phif, J), phif, prob)
    expect = phif + M * _l(k * H) / (H * H) * B * np.sin(arg)
    assert np.abs(got - expect).max() < 1e-15


@pytest.mark.parametrize("bc", [(PERIODIC,) * 3, (WALL,) * 3, (WALL, PERIODIC, WALL)])
def test_fine_step_conserves_the_phase_mass(bc):
    """Random smooth fine phase field and velocity, walls or not: the fine
    flux divergence telescopes (F5), and the coarse phi is the restriction."""
    prob = Problem(7, 6, 5, bc=bc, sigma=0.01, mobility=0.05, gravity=(0.0, 0.0, -1e-4),
                   rho_ref=1.0, fine_phase=True)
    rng = np.random.default_rng(6)
    phif = 0.5 + 0.4 * np.sin(rng.random((10, 12, 14)) * 2.0)
    J = 0.02 * (rng.random((3, 5, 6, 7)) - 0.5)
    st, got = S.step_fine(_state(prob, phif, J), phif, prob)
    assert abs(got.sum() - phif.sum()) < 1e-13 * phif.sum()
    assert np.array_equal(st.phi, S.restrict(got))


def _slab(x, x1, x2, W):
    return 0.5 * (np.tanh(2 * (x - x1) / W) - np.tanh(2 * (x - x2) / W))


def test_fine_grid_carries_an_interface_more_accurately():
    """A slab of phase 1 in a periodic box, carried by a uniform u for 40
    steps, no surface tension (the equilibrium profile of the conservative
    Allen-Cahn equation just translates).  Against the exactly translated
    profile, the fine grid's error is well below the coarse scheme's."""
    W, M, U, N, L = 4.0, 0.02, 0.05, 40, 48
    common = dict(bc=(PERIODIC,) * 3, rho_l=1.0, rho_g=1.0, nu_l=0.1, nu_g=0.1, sigma=0.0,
                  mobility=M, width=W)
    coarse = Problem(L, 2, 2, **common)
    fine = Problem(L, 2, 2, fine_phase=True, **common)
    x1, x2 = 12.0, 30.0
    xc = np.broadcast_to(np.arange(L, dtype=np.float64), (2, 2, L))
    J = np.zeros((3, 2, 2, L))
    J[0] = U
    # coarse scheme
    st = S.initial_state(_slab(xc, x1, x2, W), u=J)
    st = S.run(st, coarse, N)
    err_c = np.abs(st.phi - _slab(xc, x1 + U * N, x2 + U * N, W)).max()
    # fine grid
    fx, _, _ = _fine_positions(fine)
    phif = _slab(fx, x1, x2, W)
    stf, phif = S.run_fine(_state(fine, phif, J), phif, fine, N)
    err_f = np.abs(phif - _slab(fx, x1 + U * N, x2 + U * N, W)).max()
    assert err_f < 0.5 * err_c, (err_f, err_c)


def test_tangential_flow_next_to_a_wall():
    """Walls on x, a uniform coarse velocity U along y, phi a wave along y,
    M = 0.  The fine velocity falls to U/2 at the first fine column (the
    coarse ghost is -U, F3) and the fine ghost column carries -U/2 (F5).  The
    D3Q27 weights factor into (1/6, 2/3, 1/6) per axis, so the y-divergence at
    a column sees the x-average of the velocity over that column and its two
    neighbours: 5U/12 at the first column, 11U/12 at the second, U beyond."""
    prob = _quiet_problem(6, 4, 3, bc=(WALL, PERIODIC, PERIODIC))
    fx, fy, fz = _fine_positions(prob)
    k = 2 * np.pi / 2.0
    B, U = 0.2, 0.04
    phif = 0.5 + B * np.sin(k * fy)
    J = np.zeros((3,) + prob.shape)
    J[1] = U
    _, got = S.step_fine(_state(prob, phif, J), phif, prob)
    ubar = np.full(12, U)
    ubar[[0, -1]] = 5 * U / 12
    ubar[[1, -2]] = 11 * U / 12
    expect = phif - ubar.reshape(1, 1, 12) * B * np.cos(k * fy) * np.sin(k * H) / H
    assert np.abs(got - expect).max() < 1e-15


@pytest.mark.parametrize("bc", [(PERIODIC,) * 3, (WALL,) * 3, (WALL, PERIODIC, WALL)])
def test_interpolation_node_by_node(bc):
    """pointwise.prolong_at (one fine node at a time, explicit taps and ghost
    signs) equals the axis-by-axis whole-array interpolation, even and odd."""
    prob = Problem(5, 4, 3, bc=bc)
    g = np.random.default_rng(9).random((3, 4, 5)) - 0.3
    for odd in (False, True):
        whole = S.prolong(g, prob, odd=odd)
        at = lambda x, y, z: g[z, y, x]
        for Z in range(6):
            for Y in range(8):
                for X in range(10):
                    v = PW.prolong_at(at, prob, X, Y, Z, odd=odd)
                    assert abs(v - whole[Z, Y, X]) < 1e-15, (odd, X, Y, Z)


@pytest.mark.parametrize("bc", [(PERIODIC,) * 3, (WALL,) * 3, (PERIODIC, WALL, WALL)])
def test_node_by_node_step_equals_whole_array_step(bc):
    """The per-node form of the fine step (pointwise.FinePointOracle: explicit
    ghost mapping per fine node, gradient on the mirrored field) equals
    scheme.step_fine at every coarse node, random smooth state, forces on."""
    prob = Problem(5, 4, 6, bc=bc, rho_l=1.0, rho_g=0.1, nu_l=0.02, nu_g=0.1, sigma=0.01,
                   mobility=0.05, width=3.0, gravity=(1e-4, -2e-4, 3e-4), rho_ref=0.5, fine_phase=True)
    rng = np.random.default_rng(12)
    phif = 0.5 + 0.4 * np.sin(rng.random((12, 8, 10)) * 3.0)
    J = 0.02 * (rng.random((3, 6, 4, 5)) - 0.5)
    st = S.initial_state(S.restrict(phif), u=J)
    st.P = 0.01 * (rng.random(st.P.shape) - 0.5)
    st.Q = 1e-3 * (rng.random(st.Q.shape) - 0.5)
    st.Q = 0.5 * (st.Q + st.Q.transpose(1, 0, 2, 3, 4))
    ref, _ = S.step_fine(st, phif, prob)
    pts = [(x, y, z) for z in range(6) for y in range(4) for x in range(5)]
    got = PW.step_points_fine(st, lambda X, Y, Z: phif[Z, Y, X], prob, pts)
    for k, (x, y, z) in enumerate(pts):
        assert abs(got["phi"][k] - ref.phi[z, y, x]) < 1e-14
        assert abs(got["P"][k] - ref.P[z, y, x]) < 1e-15
        assert np.abs(got["J"][k] - ref.J[:, z, y, x]).max() < 1e-15
        assert np.abs(got["Q"][k] - ref.Q[:, :, z, y, x]).max() < 1e-15
