"""Whole-array FP64 oracle of one time step (test infrastructure only).

Follows the four phases of Sec. II.D in the paper's order:
  1. moments and forces  (Eqs. moments0, moments1, press_corr, jaqminforce,
     visc_corr; the chemical potential of Sec. II.C),
  2. pre-regularisation  (Eq. hermite_neq2 with the shifted equilibrium),
  3. fused stream/collide in push form (Eqs. LBexp, pushLB with the equilibria
     of Eq. eqts, the recursive non-equilibrium of Eq. noneqts and the Guo
     source of Eq. guoforce),
  4. interface tracking by FTCS (Sec. II.A conservative Allen-Cahn, Sec. II.D
     update formula), with the isotropic stencils of Sec. II.C.

State between steps (the thread-safe principle of Sec. II.B: the update needs
only hydrodynamic moments, never stored populations):
  phi            phase field
  P   = sum_i f_i                       (normalised pressure p*, Eq. moments0)
  J   = sum_i f_i c_i                   (first moment of the streamed f)
  Q   = sum_i f_i H2_i - J J            (second moment about J)
The velocity is u = J + a/2 with a = F/rho (Eq. moments1, reading R3 below).

Readings where the paper is silent, ambiguous or garbled (the same list is in
the design notes of the repository):
  R1  The interface width delta of Sec. II.A/II.C is W; the equilibrium profile
      is 0.5(1 + tanh(2 d / W)) with Euclidean signed distance d.  With
      beta = 12 sigma/W and kappa = 3 sigma W / 2 this is the exact zero of the
      chemical potential and carries surface tension sigma.
  R2  kappa in the Allen-Cahn equation is 4 D / W (kappa_AC); kappa in the
      chemical potential is 3 sigma W / 2 (kappa_mu).  D is the mobility M.
  R3  Force and velocity: the Guo source and the velocity shift use the
      acceleration a = F / rho (velocity-based equilibrium with p* = p /(rho
      cs^2)), and u = J + a/2 (the printed "1/2 sum_i S_i" vanishes
      identically; its first moment is meant).
  R4  Post-collision state f_post = f_eq + (1 - omega) f_neq + S/2, i.e. the
      shifted equilibrium f_eq - S/2 plus relaxed non-equilibrium plus the
      full source, with f_neq rebuilt from a2 = sum_i H2_i (f_i - feq_i + S_i/2)
      (Eq. hermite_neq2).  A uniform acceleration then raises u by exactly a
      per step.
  R5  Eq. noneqts is read with the weight w_i and the Hermite tensor H2_i
      (c c - cs^2 I), so that f_neq has zero mass and momentum; the same
      (1 - omega) relaxes the second- and third-order parts.
  R6  The second-derivative stencil of Sec. II.C is read as the isotropic
      Laplacian (2/cs^2) sum_i w_i (Psi(x + c_i) - Psi(x)); the gradient is
      (1/cs^2) sum_i w_i Psi(x + c_i) c_i; both with the D3Q27 weights.
  R7  The viscous correction (Eq. visc_corr) contracts the second index with
      grad(rho); its population bracket is taken with f_eq at (p*, J), which
      makes it the stored Q (so it is available before u, in the order of
      Sec. II.D).
  R8  Kinematic viscosity is interpolated linearly in phi,
      nu = nu_g + phi (nu_l - nu_g), and omega = 1/(nu/cs^2 + 1/2).
  R9  The advection term is taken in conservative flux form div(phi u) (the
      equation is called conservative); the printed u.grad(phi) form is kept
      behind the literal_advection flag.
  R10 The normal is n = grad(phi) / (|grad(phi)| + 1e-12).
  R11 Walls: half-way bounce-back, f_i(x) = f_post_opp(i)(x) when x - c_i lies
      behind a wall; the phase field uses mirror ghosts (phi(-1) = phi(0),
      phi(-2) = phi(1)), which is the neutral-wetting (zero normal derivative)
      condition of Sec. III.D; ghost velocity is minus the mirrored velocity
      and the ghost normal is computed from the mirrored phase field.
  R12 Body force: F_b = (rho - rho_ref) g (buoyancy acting on the light phase
      when rho_ref is the liquid density).
  R13 Phase-field time level: all terms at level n (explicit Euler), computed
      from the same node quantities the flow step uses.
  R14 The material laws rho(phi) and nu(phi) are evaluated at phi clamped to
      [0, 1], the range the model assigns to phi (Sec. II.A); the density
      gradient in the pressure and viscous corrections is the derivative of
      the linear law, (rho_l - rho_g) grad(phi).  FTCS advection at cell
      Peclet number u/M > 2 over- and undershoots slightly; unclamped, an
      undershoot below -rho_g/(rho_l - rho_g) makes rho <= 0 at density ratio
      1000 and an overshoot can make nu < 0.

Gradient-closure variant (Problem.gradient_closure; the alternative a2 of
Eq. noneqts, stated there as a velocity-gradient expression):
  G1  a2_ab = -(cs^2/omega) (d_a u_b + d_b u_a): the Chapman-Enskog value of
      the non-equilibrium second moment for populations normalised like these
      (sum f = p*, sum f c = u).  The printed prefactor -1/(omega cs^2) acting
      on grad(rho u) is read as this density-normalised form.
  G2  The gradient is taken of the stored first moment J (the isotropic
      gradient of R6, ghosts by R11: minus the mirrored value), not of
      u = J + a/2: a at a neighbour needs that neighbour's viscous force,
      which needs its own velocity gradient, so J keeps the step explicit;
      the two differ by grad(a)/2, first order in the force.
  G3  The viscous correction (Eq. visc_corr) uses the same a2 in place of the
      moment-based tensor.
  G4  The state is phi, P, J (5 fields); Q is neither stored nor used and is
      kept zero in State.

Higher-order Allen-Cahn variant (Problem.high_order_ac; the higher-order
discrete derivatives named as future work at the end of Sec. II.A, for which
the paper gives no scheme):
  H1  The three discrete derivatives of the phase-field update -- the
      divergence of the advective and sharpening fluxes, the Laplacian, and
      the gradient inside the normal n -- are fourth-order: each is the
      Richardson combination (4 D_1 - D_2)/3 of the isotropic D3Q27 stencil of
      R6 at spacing 1 (D_1) and the same stencil at spacing 2 (D_2: points
      x + 2 c_i, same weights, divided by 2 for a first derivative and by 4
      for the Laplacian).  The leading errors of D_1 and D_2 are isotropic and
      in the ratio 1 : 4, so the combination cancels them: the gradient is
      exact on polynomials of degree <= 4 and the Laplacian on degree <= 5.
  H2  The flow solver is unchanged: the forces (surface tension, pressure and
      viscous corrections) keep the second-order stencils of Sec. II.C.
  H3  Ghosts at walls extend R11 to the depth the wider stencils reach:
      phi(-k) = phi(k - 1) for k = 1..4 (wall axes need at least 4 nodes),
      ghost velocity minus the mirrored one, ghost normal from the mirrored
      phi.  The flux divergence still telescopes, so sum phi is conserved.

Finer phase-field grid (Problem.fine_phase; the finer grid for the phase field
named as future work at the end of Sec. II.A, for which the paper gives no
scheme):
  F1  The phase field lives on a grid refined by 2 along every axis, cell
      centred: coarse node i (the centre of the cell [i - 1/2, i + 1/2]) has
      the two fine nodes 2i and 2i + 1 at i - 1/4 and i + 1/4.  The fine grid
      has spacing h = 1/2 and 8 N nodes; periodic axes stay periodic (period
      2n); a wall half-way beyond coarse node 0 is half-way beyond fine node
      0 as well, so the fine ghosts mirror as in R11 (phi(-1) = phi(0), ...).
  F2  The flow solver (phases 1-3) is unchanged and reads the coarse phi, the
      restriction of the fine field: the mean of the 8 fine nodes of each
      coarse cell.  This conserves the phase mass exactly
      (sum phi_coarse = sum phi_fine / 8).
  F3  The velocity of the phase-field update on the fine grid is the
      trilinear interpolation of the coarse u = J + a/2 of the same step
      (R13): along each axis fine node 2i takes 3/4 u(i) + 1/4 u(i - 1) and
      2i + 1 takes 3/4 u(i) + 1/4 u(i + 1), with the coarse ghost velocity of
      R11 (minus the mirrored one) beyond a wall.
  F4  The fine update is the FTCS step of phase_update at spacing h with the
      time step of the flow solver (1): the stencils of R6 divided by h (first
      derivatives) and h^2 (Laplacian), M and W unchanged in lattice units, so
      the interface keeps its width and spans twice as many fine nodes.
      Stability of the diffusive part needs M / h^2 = 4 M below about 0.35
      (the largest magnitude of the isotropic Laplacian's symbol is 5.78).
  F5  Fine ghosts at walls follow R11 on the fine grid: phi mirrored, the
      ghost flux phi u from the mirrored node with u negated, the ghost
      normal from the mirrored phi.  The flux divergence telescopes, so the
      fine phase mass is conserved.
  F6  A coarse phi given at initialisation (or in a restart from the coarse
      state) is carried to the fine grid with the interpolation of F3 (ghosts
      mirrored, not negated), and the coarse phi becomes the restriction of
      that fine field, so that the coarse phi is always the restriction of
      the fine one.  Per axis the restriction of the interpolation is
      g + (g(i-1) - 2 g(i) + g(i+1)) / 8.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .lattice import C, CS2, H2_ALL, H3_ALL, OPP, Q as NQ, W

PERIODIC = 0
WALL = 1
EPS_NORMAL = 1e-12
BULK_THRESHOLD = 0.02  # diagnostics: bulk phase means use phi >= 1-t or phi <= t

Q6_INDEX = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


@dataclasses.dataclass
class State:
    phi: np.ndarray  # (nz, ny, nx)
    P: np.ndarray    # (nz, ny, nx)
    J: np.ndarray    # (3, nz, ny, nx)
    Q: np.ndarray    # (3, 3, nz, ny, nx), symmetric

    def copy(self):
        return State(self.phi.copy(), self.P.copy(), self.J.copy(), self.Q.copy())


def q_full(q6):
    """(6, ...) ordered xx, yy, zz, xy, xz, yz  ->  symmetric (3, 3, ...)."""
    q = np.empty((3, 3) + q6.shape[1:])
    for k, (a, b) in enumerate(Q6_INDEX):
        q[a, b] = q6[k]
        q[b, a] = q6[k]
    return q


def q_six(q):
    return np.stack([q[a, b] for a, b in Q6_INDEX])


def initial_state(phi, u=None, pstar=None):
    """Initial state: P = p*_0 (default 0), J = u_0 (default 0), Q = 0.

    With f = f_eq(p*_0, u_0) at t = 0 the second moment about J vanishes.
    """
    phi = np.asarray(phi, dtype=np.float64)
    shape = phi.shape
    P = np.zeros(shape) if pstar is None else np.asarray(pstar, np.float64).copy()
    J = np.zeros((3,) + shape) if u is None else np.asarray(u, np.float64).copy()
    return State(phi.copy(), P, J, np.zeros((3, 3) + shape))


# ----------------------------------------------------------------------------
# Ghost layers and isotropic stencils (Sec. II.C, reading R6; walls R11)
# ----------------------------------------------------------------------------

def pad(f, prob, h, odd=(False, False, False)):
    """Pad the last three axes (z, y, x) of f by h ghost layers.

    Periodic axes wrap.  Wall axes mirror about the half-way wall
    (g(-1) = g(0), g(-2) = g(1)); a quantity odd under reflection across that
    axis gets its ghost layers negated.  odd is given per axis (x, y, z).
    """
    out = np.asarray(f, dtype=np.float64)
    lead = out.ndim - 3
    for arr_axis, ax in ((lead + 0, 2), (lead + 1, 1), (lead + 2, 0)):
        widths = [(0, 0)] * out.ndim
        widths[arr_axis] = (h, h)
        if prob.bc[ax] == PERIODIC:
            out = np.pad(out, widths, mode="wrap")
        else:
            out = np.pad(out, widths, mode="symmetric")
            if odd[ax]:
                idx = [slice(None)] * out.ndim
                idx[arr_axis] = slice(0, h)
                out[tuple(idx)] *= -1.0
                idx[arr_axis] = slice(out.shape[arr_axis] - h, None)
                out[tuple(idx)] *= -1.0
    return out


def shifted(fp, h, c, e=0):
    """Values g(x + c) for x over the interior grown by e, from an array padded by h."""
    nz, ny, nx = (s - 2 * h for s in fp.shape[-3:])
    cx, cy, cz = (int(v) for v in c)
    return fp[..., h - e + cz:h + nz + e + cz, h - e + cy:h + ny + e + cy,
              h - e + cx:h + nx + e + cx]


def grad(fp, h, e=0):
    """Isotropic gradient (1/cs^2) sum_i w_i g(x + c_i) c_i."""
    out = None
    for i in range(NQ):
        v = shifted(fp, h, C[i], e)
        term = (W[i] / CS2) * C[i].astype(np.float64).reshape(3, 1, 1, 1) * v
        out = term if out is None else out + term
    return out


def laplacian(fp, h, e=0):
    """Isotropic Laplacian (2/cs^2) sum_i w_i (g(x + c_i) - g(x))."""
    centre = shifted(fp, h, (0, 0, 0), e)
    out = np.zeros_like(centre)
    for i in range(NQ):
        out += (2.0 * W[i] / CS2) * (shifted(fp, h, C[i], e) - centre)
    return out


def divergence(vp, h, e=0):
    """Isotropic divergence (1/cs^2) sum_i w_i v(x + c_i) . c_i of a padded (3, ...) field."""
    out = None
    for i in range(NQ):
        v = shifted(vp, h, C[i], e)
        term = (W[i] / CS2) * sum(float(C[i][a]) * v[a] for a in range(3))
        out = term if out is None else out + term
    return out


def grad_wide(fp, h, e=0):
    """The gradient stencil of R6 at spacing 2: (1/(2 cs^2)) sum_i w_i g(x + 2 c_i) c_i (H1)."""
    out = None
    for i in range(NQ):
        v = shifted(fp, h, 2 * C[i], e)
        term = (W[i] / (2.0 * CS2)) * C[i].astype(np.float64).reshape(3, 1, 1, 1) * v
        out = term if out is None else out + term
    return out


def laplacian_wide(fp, h, e=0):
    """The Laplacian of R6 at spacing 2: (2/(4 cs^2)) sum_i w_i (g(x + 2 c_i) - g(x)) (H1)."""
    centre = shifted(fp, h, (0, 0, 0), e)
    out = np.zeros_like(centre)
    for i in range(NQ):
        out += (2.0 * W[i] / (4.0 * CS2)) * (shifted(fp, h, 2 * C[i], e) - centre)
    return out


def divergence_wide(vp, h, e=0):
    """The divergence of R6 at spacing 2: (1/(2 cs^2)) sum_i w_i v(x + 2 c_i) . c_i (H1)."""
    out = None
    for i in range(NQ):
        v = shifted(vp, h, 2 * C[i], e)
        term = (W[i] / (2.0 * CS2)) * sum(float(C[i][a]) * v[a] for a in range(3))
        out = term if out is None else out + term
    return out


def grad4(fp, h, e=0):
    """Fourth-order isotropic gradient (4 D_1 - D_2) / 3 (H1)."""
    return (4.0 * grad(fp, h, e) - grad_wide(fp, h, e)) / 3.0


def laplacian4(fp, h, e=0):
    """Fourth-order isotropic Laplacian (4 L_1 - L_2) / 3 (H1)."""
    return (4.0 * laplacian(fp, h, e) - laplacian_wide(fp, h, e)) / 3.0


def divergence4(vp, h, e=0):
    """Fourth-order isotropic divergence (4 D_1 - D_2) / 3 (H1)."""
    return (4.0 * divergence(vp, h, e) - divergence_wide(vp, h, e)) / 3.0


# ----------------------------------------------------------------------------
# Local (per node) physics; every function broadcasts over node arrays
# ----------------------------------------------------------------------------

def clamp01(phi):
    """phi restricted to the model's range [0, 1] (reading R14)."""
    return np.minimum(np.maximum(phi, 0.0), 1.0)


def density(phi, prob):
    """rho = rho_l phi + (1 - phi) rho_g  (Sec. II.C, below Eq. press_corr),
    at phi clamped to [0, 1] (R14)."""
    phi = clamp01(phi)
    return prob.rho_l * phi + (1.0 - phi) * prob.rho_g


def density_gradient(grad_phi, prob):
    """grad(rho) = (rho_l - rho_g) grad(phi): derivative of the linear law (R14)."""
    return (prob.rho_l - prob.rho_g) * grad_phi


def viscosity(phi, prob):
    """Reading R8: linear interpolation of the kinematic viscosity, at phi
    clamped to [0, 1] (R14)."""
    return prob.nu_g + clamp01(phi) * (prob.nu_l - prob.nu_g)


def relaxation(nu):
    """omega from nu = cs^2 (1/omega - 1/2) (reading R8)."""
    return 1.0 / (nu / CS2 + 0.5)


def chemical_potential(phi, lap_phi, prob):
    """mu = 4 beta (phi - phi_l)(phi - phi_g)(phi - phi_0) - kappa lap(phi)
    with phi_l = 1, phi_g = 0, phi_0 = 1/2, beta = 12 sigma/W,
    kappa = 3 sigma W / 2 (Sec. II.C; readings R1, R2)."""
    beta = 12.0 * prob.sigma / prob.width
    kappa = 1.5 * prob.sigma * prob.width
    return 4.0 * beta * (phi - 1.0) * (phi - 0.0) * (phi - 0.5) - kappa * lap_phi


def total_force(phi, grad_phi, lap_phi, grad_rho, P, Q, prob):
    """F = F^s + F^p + F^nu + F^b (Sec. II.C; readings R7, R12).

    F^s = mu grad(phi)                               (Eq. jaqminforce)
    F^p = -p* cs^2 grad(rho)                         (Eq. press_corr)
    F^nu_a = -(nu omega / cs^2) sum_b Q_ab d_b rho   (Eq. visc_corr)
    F^b = (rho - rho_ref) g                          (Sec. III.A)
    """
    mu = chemical_potential(phi, lap_phi, prob)
    rho = density(phi, prob)
    nu = viscosity(phi, prob)
    om = relaxation(nu)
    fs = mu * grad_phi
    fp = -P * CS2 * grad_rho
    fv = -(nu * om / CS2) * np.einsum("ab...,b...->a...", Q, grad_rho)
    g = np.asarray(prob.gravity, dtype=np.float64).reshape((3,) + (1,) * np.ndim(phi))
    fb = (rho - prob.rho_ref) * g
    return fs + fp + fv + fb


def f_eq(P, u):
    """Third-order Hermite equilibrium of Eq. eqts (velocity based, with p*)."""
    out = np.empty((NQ,) + np.shape(P))
    for i in range(NQ):
        c = C[i].astype(np.float64)
        cu = np.einsum("a,a...->...", c, u)
        h2uu = np.einsum("ab,a...,b...->...", H2_ALL[i], u, u)
        h3uuu = np.einsum("abg,a...,b...,g...->...", H3_ALL[i], u, u, u)
        out[i] = W[i] * (P + cu / CS2 + h2uu / (2 * CS2 ** 2) + h3uuu / (6 * CS2 ** 3))
    return out


def third_order_neq(A, u):
    """a3_abg = u_a A_bg + u_b A_ag + u_g A_ab (recursive relation, Eq. noneqts)."""
    return (np.einsum("a...,bg...->abg...", u, A) + np.einsum("b...,ag...->abg...", u, A)
            + np.einsum("g...,ab...->abg...", u, A))


def f_neq(A, u):
    """Regularised non-equilibrium of Eq. noneqts (reading R5)."""
    a3 = third_order_neq(A, u)
    out = np.empty((NQ,) + A.shape[2:])
    for i in range(NQ):
        h2a = np.einsum("ab,ab...->...", H2_ALL[i], A)
        h3a = np.einsum("abg,abg...->...", H3_ALL[i], a3)
        out[i] = W[i] * (h2a / (2 * CS2 ** 2) + h3a / (6 * CS2 ** 3))
    return out


def guo_source(u, a):
    """Guo forcing of Eq. guoforce, with the acceleration a in place of F (R3)."""
    out = np.empty((NQ,) + u.shape[1:])
    for i in range(NQ):
        c = C[i].astype(np.float64).reshape((3,) + (1,) * (u.ndim - 1))
        cu = np.sum(c * u, axis=0)
        out[i] = W[i] * np.sum(((c - u) / CS2 + cu * c / CS2 ** 2) * a, axis=0)
    return out


def second_moment(f):
    """sum_i H2_i f_i  ->  (3, 3, ...)."""
    return np.einsum("iab,i...->ab...", H2_ALL, f)


def velocity_gradient(J, prob):
    """grad J as (a, b, ...) = d_b J_a: the isotropic gradient (R6) of each
    component, ghost values minus the mirrored value at walls (R11; G2)."""
    return np.stack([grad(pad(J[a], prob, 1, odd=(True, True, True)), 1) for a in range(3)])


def gradient_closure_tensor(grad_J, omega):
    """a2 = -(cs^2/omega) (d_a J_b + d_b J_a)  (Eq. noneqts, velocity-gradient form; G1, G2)."""
    return -(CS2 / omega) * (grad_J + np.swapaxes(grad_J, 0, 1))


def collide_closed(P, J, A, F, rho, omega):
    """Post-collision populations with the regularisation tensor given:
    u = J + a/2, f_post = feq(P, u) + (1 - omega) f_neq(A, u) + S/2
    (Eqs. moments1, LBexp, noneqts, guoforce; R3, R4)."""
    a = F / rho
    u = J + 0.5 * a
    feq = f_eq(P, u)
    S = guo_source(u, a)
    fpost = feq + (1.0 - omega) * f_neq(A, u) + 0.5 * S
    return fpost, u, A, a


def collide(P, J, Q, F, rho, omega):
    """Moments -> velocity -> pre-regularisation -> post-collision populations.

    u  = J + a/2, a = F/rho                          (Eq. moments1, R3)
    a2 = [sum_i H2_i f_i] - sum_i H2_i (feq_i - S_i/2)  (Eq. hermite_neq2),
         where sum_i H2_i f_i = Q + J J by the definition of Q
    f_post = feq + (1 - omega) f_neq(a2) + S/2       (Eq. LBexp, R4)
    Returns (f_post, u, a2, a).
    """
    a = F / rho
    u = J + 0.5 * a
    feq = f_eq(P, u)
    S = guo_source(u, a)
    A = Q + np.einsum("a...,b...->ab...", J, J) - second_moment(feq - 0.5 * S)
    fneq = f_neq(A, u)
    fpost = feq + (1.0 - omega) * fneq + 0.5 * S
    return fpost, u, A, a


# ----------------------------------------------------------------------------
# Whole-array step
# ----------------------------------------------------------------------------

def node_fields(st, prob):
    """Per-node quantities of phase 1 (moments and forces) on the interior."""
    phip = pad(st.phi, prob, 2)
    gphi = grad(phip, 2)
    lphi = laplacian(phip, 2)
    rho = density(st.phi, prob)
    grho = density_gradient(gphi, prob)
    nu = viscosity(st.phi, prob)
    om = relaxation(nu)
    A = None
    if prob.gradient_closure:
        A = gradient_closure_tensor(velocity_gradient(st.J, prob), om)
        F = total_force(st.phi, gphi, lphi, grho, st.P, A, prob)   # G3
    else:
        F = total_force(st.phi, gphi, lphi, grho, st.P, st.Q, prob)
    return dict(phip=phip, grad_phi=gphi, lap_phi=lphi, rho=rho, grad_rho=grho,
                nu=nu, omega=om, F=F, A=A)


def stream_push(fpost, prob):
    """Eq. pushLB: f_i(x + c_i) = f_post_i(x); at walls half-way bounce-back
    (R11): a population whose destination lies behind a wall returns to its
    own node in the opposite direction."""
    shape = fpost.shape[1:]
    nz, ny, nx = shape
    f = np.zeros_like(fpost)
    for i in range(NQ):
        cx, cy, cz = (int(v) for v in C[i])
        leave = np.zeros(shape, dtype=bool)
        for ax, cc, n in ((2, cx, nx), (1, cy, ny), (0, cz, nz)):
            if prob.bc[2 - ax] == WALL and cc != 0:
                idx = [slice(None)] * 3
                idx[ax] = n - 1 if cc > 0 else 0
                leave[tuple(idx)] = True
        stay = np.where(leave, 0.0, fpost[i])
        f[i] += np.roll(stay, shift=(cz, cy, cx), axis=(0, 1, 2))
        f[OPP[i]] += np.where(leave, fpost[i], 0.0)
    return f


def moments(f):
    """P = sum f (Eq. moments0), J = sum f c, Q = sum H2 f - J J."""
    P = f.sum(axis=0)
    J = np.einsum("ia,i...->a...", C.astype(np.float64), f)
    Q = second_moment(f) - np.einsum("a...,b...->ab...", J, J)
    return P, J, Q


def normal(grad_phi):
    """Interface normal n = grad(phi) / (|grad(phi)| + eps) (reading R10)."""
    mag = np.sqrt(np.sum(grad_phi ** 2, axis=0))
    return grad_phi / (mag + EPS_NORMAL)


def phase_update(st, nf, u, prob):
    """Interface tracking: FTCS step of the conservative Allen-Cahn equation
    (Sec. II.A and the update formula of Sec. II.D; readings R2, R9, R11, R13).

    phi' = phi - div(phi u) + M lap(phi) - kappa_AC div(phi (1 - phi) n)
    """
    phip = nf["phip"]
    M = prob.mobility
    kac = 4.0 * M / prob.width
    phi1 = shifted(phip, 2, (0, 0, 0), 1)               # phi on interior + 1 ghost layer
    n1 = normal(grad(phip, 2, 1))                        # ghost normal from mirrored phi
    up = np.stack([pad(u[a], prob, 1, odd=(True, True, True)) for a in range(3)])
    sharp = phi1 * (1.0 - phi1) * n1
    if prob.literal_advection:
        adv = np.sum(u * nf["grad_phi"], axis=0)
    else:
        adv = divergence(phi1 * up, 1)
    return st.phi - adv + M * nf["lap_phi"] - kac * divergence(sharp, 1)


def phase_update_high_order(st, u, prob):
    """The FTCS step of phase_update with the fourth-order derivatives of H1
    (ghosts H3):

    phi' = phi - div4(phi u) + M lap4(phi) - kappa_AC div4(phi (1 - phi) n4),
    n4 = grad4(phi) / (|grad4(phi)| + eps).
    The fluxes are needed up to two nodes beyond the box (the reach of
    div4), their normals up to four (the reach of grad4 from there).
    """
    M = prob.mobility
    kac = 4.0 * M / prob.width
    phip = pad(st.phi, prob, 4)
    phi2 = shifted(phip, 4, (0, 0, 0), 2)               # phi on interior + 2 ghost layers
    n2 = normal(grad4(phip, 4, 2))                       # ghost normals from mirrored phi
    up = np.stack([pad(u[a], prob, 2, odd=(True, True, True)) for a in range(3)])
    sharp = phi2 * (1.0 - phi2) * n2
    if prob.literal_advection:
        adv = np.sum(u * grad4(phip, 4), axis=0)
    else:
        adv = divergence4(phi2 * up, 2)
    return st.phi - adv + M * laplacian4(phip, 4) - kac * divergence4(sharp, 2)


# ----------------------------------------------------------------------------
# Finer phase-field grid (F1-F6)
# ----------------------------------------------------------------------------

FINE_H = 0.5  # fine grid spacing in lattice units (F1)


def prolong(g, prob, odd=False):
    """Trilinear interpolation of a coarse (nz, ny, nx) field onto the fine
    grid (2nz, 2ny, 2nx) of F1 (F3; ghosts beyond a wall mirrored, negated if
    odd).  The axes are refined one after the other; each pass consumes that
    axis's ghost layers."""
    out = pad(g, prob, 1, odd=(odd, odd, odd))
    for axis in range(3):  # array axes z, y, x of the padded field
        n = out.shape[axis] - 2
        lo, mid, hi = ([slice(None)] * 3 for _ in range(3))
        lo[axis], mid[axis], hi[axis] = slice(0, n), slice(1, n + 1), slice(2, n + 2)
        centre = out[tuple(mid)]
        shape = list(centre.shape)
        shape[axis] *= 2
        fine = np.empty(shape)
        even, oddn = [slice(None)] * 3, [slice(None)] * 3
        even[axis], oddn[axis] = slice(0, None, 2), slice(1, None, 2)
        fine[tuple(even)] = 0.75 * centre + 0.25 * out[tuple(lo)]  # fine node 2i at i - 1/4
        fine[tuple(oddn)] = 0.75 * centre + 0.25 * out[tuple(hi)]  # fine node 2i + 1 at i + 1/4
        out = fine
    return out


def restrict(phif):
    """Mean of the 8 fine nodes of every coarse cell (F2)."""
    nz, ny, nx = (s // 2 for s in phif.shape)
    return phif.reshape(nz, 2, ny, 2, nx, 2).mean(axis=(1, 3, 5))


def initial_fine_phase(phi, prob):
    """Fine phase field from a coarse one, and the coarse phi the flow solver
    then sees (F6)."""
    phif = prolong(phi, prob)
    return phif, restrict(phif)


def phase_update_fine(phif, u, prob):
    """FTCS step of the conservative Allen-Cahn equation on the fine grid
    (F1, F3-F5):

    phi_f' = phi_f - div_h(phi_f u_f) + M lap_h(phi_f) - kappa_AC div_h(phi_f (1 - phi_f) n_f),
    div_h = div / h, lap_h = lap / h^2, n_f = grad_h(phi_f) / (|grad_h(phi_f)| + eps),
    u_f the interpolation of the coarse u of this step.
    """
    h = FINE_H
    M = prob.mobility
    kac = 4.0 * M / prob.width
    phip = pad(phif, prob, 2)
    phi1 = shifted(phip, 2, (0, 0, 0), 1)               # fine phi on interior + 1 ghost layer
    n1 = normal(grad(phip, 2, 1) / h)                    # ghost normal from mirrored phi
    uf = np.stack([prolong(u[a], prob, odd=True) for a in range(3)])
    up = np.stack([pad(uf[a], prob, 1, odd=(True, True, True)) for a in range(3)])
    sharp = phi1 * (1.0 - phi1) * n1
    adv = divergence(phi1 * up, 1) / h
    lap = laplacian(phip, 2) / (h * h)
    return phif - adv + M * lap - kac * divergence(sharp, 1) / h


def step_fine(st, phif, prob):
    """One time step with the phase field on the fine grid: phases 1-3 of
    Sec. II.D on the coarse grid from st (whose phi is restrict(phif), F2),
    then the fine phase update with that step's u (F3, F4), then the
    restriction.  Returns the new coarse state and fine field."""
    nf = node_fields(st, prob)
    if prob.gradient_closure:
        fpost, u, _, _ = collide_closed(st.P, st.J, nf["A"], nf["F"], nf["rho"], nf["omega"])
    else:
        fpost, u, _, _ = collide(st.P, st.J, st.Q, nf["F"], nf["rho"], nf["omega"])
    f = stream_push(fpost, prob)
    P, J, Q = moments(f)
    if prob.gradient_closure:
        Q = np.zeros_like(Q)  # G4
    phif_new = phase_update_fine(phif, u, prob)
    return State(restrict(phif_new), P, J, Q), phif_new


def run_fine(st, phif, prob, nsteps):
    for _ in range(nsteps):
        st, phif = step_fine(st, phif, prob)
    return st, phif


def step(st, prob):
    """One full time step, phases 1-4 of Sec. II.D."""
    nf = node_fields(st, prob)
    if prob.gradient_closure:
        fpost, u, _, _ = collide_closed(st.P, st.J, nf["A"], nf["F"], nf["rho"], nf["omega"])
    else:
        fpost, u, _, _ = collide(st.P, st.J, st.Q, nf["F"], nf["rho"], nf["omega"])
    f = stream_push(fpost, prob)
    P, J, Q = moments(f)
    if prob.gradient_closure:
        Q = np.zeros_like(Q)  # G4
    if getattr(prob, "high_order_ac", False):
        phi = phase_update_high_order(st, u, prob)
    else:
        phi = phase_update(st, nf, u, prob)
    return State(phi, P, J, Q)


def run(st, prob, nsteps):
    for _ in range(nsteps):
        st = step(st, prob)
    return st


# ----------------------------------------------------------------------------
# Observables and diagnostics
# ----------------------------------------------------------------------------

def observables(st, prob):
    """rho(phi), u = J + a/2 from the current state, p = rho cs^2 p* (Sec. II.C)."""
    nf = node_fields(st, prob)
    a = nf["F"] / nf["rho"]
    u = st.J + 0.5 * a
    p = nf["rho"] * CS2 * st.P
    return dict(rho=nf["rho"], u=u, phi=st.phi.copy(), p=p)


def diagnostics(st, prob, threshold=BULK_THRESHOLD):
    ob = observables(st, prob)
    rho, u, phi, p = ob["rho"], ob["u"], ob["phi"], ob["p"]
    nz, ny, nx = phi.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x, y, z]).astype(np.float64)
    speed = np.sqrt(np.sum(u ** 2, axis=0))
    wl = phi
    wg = 1.0 - phi
    heavy = phi >= 1.0 - threshold
    light = phi <= threshold
    finite = all(np.isfinite(a).all() for a in (st.phi, st.P, st.J, st.Q))
    return dict(
        phase_mass=phi.sum(),
        pstar_sum=st.P.sum(),
        momentum=(rho * u).reshape(3, -1).sum(axis=1),
        kinetic=0.5 * np.sum(rho * speed ** 2),
        umax=speed.max(),
        centroid_l=(wl * pos).reshape(3, -1).sum(axis=1) / wl.sum(),
        velocity_l=(wl * u).reshape(3, -1).sum(axis=1) / wl.sum(),
        centroid_g=(wg * pos).reshape(3, -1).sum(axis=1) / wg.sum(),
        velocity_g=(wg * u).reshape(3, -1).sum(axis=1) / wg.sum(),
        p_l=p[heavy].mean() if heavy.any() else 0.0,
        p_g=p[light].mean() if light.any() else 0.0,
        n_l=float(heavy.sum()),
        n_g=float(light.sum()),
        nonfinite=0 if finite else 1,
    )
