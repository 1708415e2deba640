"""Seeded synthetic inputs for the droplet / bubble workloads.

This module only builds initial fields and physical parameters.  It holds no
part of the lattice Boltzmann / Allen-Cahn update: both the HIP path and the
CPU oracle take its output as input, so it is the one module they share.

Phase convention (Sec. II.C, density interpolation): phi = 1 is the liquid
(subscript l), phi = 0 the gas (subscript g); rho = rho_l*phi + rho_g*(1-phi).

Initial interfaces use the equilibrium tanh profile of Sec. II.A with the
interface width W standing for delta and the Euclidean signed distance d
(positive inside the phi = 1 phase):  phi = 0.5*(1 + tanh(2 d / W)).

Arrays are C-ordered (nz, ny, nx), x fastest, matching the node index
n = x + nx*(y + ny*z).  Velocity is three SoA planes (3, nz, ny, nx).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

PERIODIC = 0
WALL = 1


@dataclasses.dataclass
class Problem:
    """Physical parameters of one box in lattice units (dx = dt = 1)."""

    nx: int
    ny: int
    nz: int
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)  # per axis x, y, z
    rho_l: float = 1.0        # density of the phi = 1 phase
    rho_g: float = 1e-3       # density of the phi = 0 phase
    nu_l: float = 1.0 / 60.0  # kinematic viscosity of the phi = 1 phase
    nu_g: float = 1.0 / 6.0   # kinematic viscosity of the phi = 0 phase
    sigma: float = 0.01       # surface tension
    mobility: float = 0.02    # interface diffusivity D (= M)
    width: float = 4.0        # interface width delta (= W)
    gravity: tuple = (0.0, 0.0, 0.0)
    rho_ref: float = 0.0      # body force density is (rho - rho_ref) * gravity
    literal_advection: bool = False  # u.grad(phi) instead of div(phi u)
    gradient_closure: bool = False   # a2 from the velocity gradient; state phi, P, J only
    high_order_ac: bool = False      # fourth-order stencils in the phase-field update
    fine_phase: bool = False         # phase field on a grid refined by 2 per axis

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Case:
    """A seeded initial condition: problem parameters plus fields."""

    name: str
    problem: Problem
    phi: np.ndarray                 # (nz, ny, nx) float64
    u: Optional[np.ndarray] = None  # (3, nz, ny, nx) float64 or None (= 0)
    pstar: Optional[np.ndarray] = None  # (nz, ny, nx) float64 or None (= 0)
    seed: int = 0


def tanh_profile(d, width):
    """Equilibrium profile for signed distance d (> 0 inside phi = 1)."""
    return 0.5 * (1.0 + np.tanh(2.0 * d / width))


def coords(nx, ny, nz, dtype=np.float64):
    z, y, x = np.meshgrid(np.arange(nz, dtype=dtype), np.arange(ny, dtype=dtype),
                          np.arange(nx, dtype=dtype), indexing="ij")
    return x, y, z


def static_droplet(n=32, radius=8.0, seed=1, noise=1e-6, rho_ratio=1000.0,
                   mu_ratio=100.0, nu_gas=1.0 / 6.0, sigma=0.01, mobility=0.02,
                   width=4.0, center=None, nx=None, ny=None, nz=None):
    """Static droplet (phi = 1 inside) in a periodic box, with seeded noise on u."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    rng = np.random.default_rng(seed)
    c = center if center is not None else ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2)
    x, y, z = coords(nx, ny, nz)
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    phi = tanh_profile(radius - r, width)
    u = rng.uniform(-noise, noise, size=(3, nz, ny, nx)) if noise else None
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    nu_l = nu_gas * mu_ratio / rho_ratio
    prob = Problem(nx, ny, nz, (PERIODIC,) * 3, rho_l, rho_g, nu_l, nu_gas,
                   sigma, mobility, width)
    return Case("static_droplet_%dx%dx%d" % (nx, ny, nz), prob, phi, u, None, seed)


def rising_bubble(nx=128, ny=128, nz=256, radius=16.0, zc=48.0, seed=2,
                  eotvos=10.0, morton=1e-3, g=1e-6, rho_ratio=1000.0,
                  mu_ratio=100.0, width=4.0, mobility=0.02):
    """Gas bubble (phi = 0 inside) rising in liquid between no-slip walls.

    sigma from Eo = rho_l g R^2 / sigma (Sec. III.A) and the liquid viscosity
    from the Morton number Mo = g mu_l^4 (rho_l - rho_g) / (rho_l^2 sigma^3);
    the gas viscosity follows from the dynamic viscosity ratio.  Buoyancy acts
    on the light phase only: rho_ref = rho_l.
    """
    rng = np.random.default_rng(seed)
    j = rng.uniform(-0.5, 0.5, size=3)
    c = ((nx - 1) / 2 + j[0], (ny - 1) / 2 + j[1], zc + j[2])
    x, y, z = coords(nx, ny, nz)
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    phi = tanh_profile(r - radius, width)
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    sigma = rho_l * g * radius ** 2 / eotvos
    mu_l = (morton * rho_l ** 2 * sigma ** 3 / (g * (rho_l - rho_g))) ** 0.25
    nu_l = mu_l / rho_l
    nu_g = nu_l * rho_ratio / mu_ratio
    prob = Problem(nx, ny, nz, (WALL, WALL, WALL), rho_l, rho_g, nu_l, nu_g,
                   sigma, mobility, width, (0.0, 0.0, -g), rho_l)
    return Case("rising_bubble_%dx%dx%d" % (nx, ny, nz), prob, phi, None, None, seed)


def droplet_collision(n=256, radius=24.0, seed=3, speed=0.02, rho_ratio=800.0,
                      mu_ratio=50.0, nu_gas=1.0 / 6.0, sigma=0.005,
                      mobility=0.02, width=4.0, nx=None, ny=None, nz=None):
    """Two drops approaching along x with a seeded impact offset along y."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    rng = np.random.default_rng(seed)
    b = rng.uniform(0.0, 0.3 * radius)
    cx, cy, cz = nx / 2, ny / 2, nz / 2
    sep = 32.0 * nx / 256.0 if nx < 256 else 32.0
    centers = [(cx - sep, cy - b / 2, cz), (cx + sep, cy + b / 2, cz)]
    x, y, z = coords(nx, ny, nz)
    phis = []
    for c in centers:
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        phis.append(tanh_profile(radius - r, width))
    phi = np.maximum(phis[0], phis[1])
    u = np.zeros((3, nz, ny, nx))
    u[0] = speed * phis[0] - speed * phis[1]
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    nu_l = nu_gas * mu_ratio / rho_ratio
    prob = Problem(nx, ny, nz, (PERIODIC,) * 3, rho_l, rho_g, nu_l, nu_gas,
                   sigma, mobility, width)
    return Case("droplet_collision_%dx%dx%d" % (nx, ny, nz), prob, phi, u, None, seed)


def ensemble_box(k, lo=24, hi=96, rho_ratio=1000.0, mu_ratio=100.0,
                 nu_gas=1.0 / 6.0, sigma=0.01, mobility=0.02, width=4.0):
    """Box k of the oscillating-droplet ensemble (seed 4000 + k).

    Edges are iid integers in [lo, hi]; one ellipsoidal drop at the box centre,
    radius U(0.15, 0.35) * min edge, aspect ratio U(1, 1.5) with volume
    preserving semi-axes (R a^(2/3), R a^(-1/3), R a^(-1/3)).
    """
    rng = np.random.default_rng(4000 + k)
    nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, size=3))
    radius = rng.uniform(0.15, 0.35) * min(nx, ny, nz)
    aspect = rng.uniform(1.0, 1.5)
    axes = (radius * aspect ** (2 / 3), radius * aspect ** (-1 / 3),
            radius * aspect ** (-1 / 3))
    c = ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2)
    x, y, z = coords(nx, ny, nz)
    q = np.sqrt(((x - c[0]) / axes[0]) ** 2 + ((y - c[1]) / axes[1]) ** 2
                + ((z - c[2]) / axes[2]) ** 2)
    d = radius * (1.0 - q)
    phi = tanh_profile(d, width)
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    nu_l = nu_gas * mu_ratio / rho_ratio
    prob = Problem(nx, ny, nz, (PERIODIC,) * 3, rho_l, rho_g, nu_l, nu_gas,
                   sigma, mobility, width)
    return Case("ensemble_box_%d" % k, prob, phi, None, None, 4000 + k)


def ensemble(n_boxes=64, lo=24, hi=96):
    return [ensemble_box(k, lo, hi) for k in range(n_boxes)]


def drop_into_pool(n=512, pool_depth=128, radius=40.0, zc=260.0, seed=5,
                   speed=0.05, rho_ratio=1000.0, mu_ratio=100.0,
                   nu_gas=1.0 / 6.0, sigma=0.008, mobility=0.05, width=4.0,
                   g=1e-6, nx=None, ny=None, nz=None, dtype=np.float64):
    """Drop falling into a liquid pool; walls on +-z, periodic x and y.

    The mobility is not fixed by the workload; M = 0.05 keeps the cell Peclet
    number of the explicit phase-field advection at u/M = 1 for the 0.05 fall
    speed (at M = 0.02 it is 2.5 and the run loses stability within a few
    hundred steps)."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    rng = np.random.default_rng(seed)
    scale = nz / 512.0
    zp = pool_depth * scale - 0.5
    x, y, z = coords(nx, ny, nz, dtype)
    pool = tanh_profile(zp - z, width)
    c = ((nx - 1) / 2, (ny - 1) / 2, zc * scale)
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    del x, y
    drop = tanh_profile(radius * scale - r, width)
    del r
    phi = np.maximum(pool, drop)
    del pool
    phi = phi + 1e-4 * rng.uniform(-1.0, 1.0, size=phi.shape).astype(dtype) * 4.0 * phi * (1.0 - phi)
    u = np.zeros((3,) + phi.shape, dtype=dtype)
    u[2] = -speed * drop
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    nu_l = nu_gas * mu_ratio / rho_ratio
    prob = Problem(nx, ny, nz, (PERIODIC, PERIODIC, WALL), rho_l, rho_g, nu_l,
                   nu_gas, sigma, mobility, width, (0.0, 0.0, -g), rho_g)
    return Case("drop_into_pool_%dx%dx%d" % (nx, ny, nz), prob, phi, u, None, seed)


def raindrop_train(nx=500, ny=500, nz=3000, n_drops=5, radius=25.0, spacing=2.0,
                   weber=40.0, speed=0.05, z_first=None, seed=6, rho_ratio=1000.0,
                   mu_ratio=100.0, nu_gas=1.0 / 6.0, mobility=0.05, width=4.0, g=1e-6,
                   dtype=np.float64):
    """A train of drops falling onto a solid substrate (Sec. III.D).

    No-slip walls on -z (the substrate) and +z, periodic x and y; the mirror
    ghosts of the phase field make the walls impermeable and neutrally wetting.
    Drop k (k = 0 nearest the substrate) of diameter D = 2 radius is centred
    at z_first + k * spacing * D over the middle of the box (seeded jitter of
    +-0.5 cells in x and y), moving down at `speed` under gravity g; the
    surface tension gives the Weber number We = rho_l speed^2 D / sigma.  The
    default box is the paper's 500 x 500 x 3000 with five drops two diameters
    apart.  M = 0.05 keeps the cell Peclet number of the phase-field advection
    at speed / M = 1.
    """
    rng = np.random.default_rng(seed)
    diam = 2.0 * radius
    z_first = radius + diam if z_first is None else z_first
    jit = rng.uniform(-0.5, 0.5, size=(n_drops, 2))
    x = np.arange(nx, dtype=dtype).reshape(1, 1, nx)
    y = np.arange(ny, dtype=dtype).reshape(1, ny, 1)
    phi = np.zeros((nz, ny, nx), dtype=dtype)
    reach = radius + 10.0 * width  # tanh tail below 1e-17 beyond this distance
    for k in range(n_drops):
        cz = z_first + k * spacing * diam
        z0, z1 = max(0, int(cz - reach)), min(nz, int(cz + reach) + 1)
        if z0 >= z1:
            continue
        z = np.arange(z0, z1, dtype=dtype).reshape(-1, 1, 1)
        r = np.sqrt((x - ((nx - 1) / 2 + jit[k, 0])) ** 2 + (y - ((ny - 1) / 2 + jit[k, 1])) ** 2
                    + (z - cz) ** 2)
        np.maximum(phi[z0:z1], tanh_profile(radius - r, width).astype(dtype), out=phi[z0:z1])
    u = np.zeros((3,) + phi.shape, dtype=dtype)
    u[2] = -speed * phi
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    nu_l = nu_gas * mu_ratio / rho_ratio
    sigma = rho_l * speed ** 2 * diam / weber
    prob = Problem(nx, ny, nz, (PERIODIC, PERIODIC, WALL), rho_l, rho_g, nu_l, nu_gas,
                   sigma, mobility, width, (0.0, 0.0, -g), rho_g)
    return Case("raindrop_train_%dx%dx%d" % (nx, ny, nz), prob, phi, u, None, seed)


# Eo-Ga points of the deformation-regime sweep (Sec. III.A); (30, 100) is the
# peripheral-breakup case the paper names
EO_GA_POINTS = [(eo, ga) for eo in (1.0, 10.0, 30.0, 100.0) for ga in (10.0, 30.0, 100.0)]


def eo_ga_bubble(eotvos, galilei, nx=200, ny=200, nz=400, radius=50.0, g=4e-6, seed=7,
                 rho_ratio=1000.0, mu_ratio=100.0, width=4.0, mobility=0.05):
    """Gas bubble of the Eo-Ga deformation-regime sweep (Sec. III.A).

    Periodic in every direction; D = 100 in a 200 x 200 x 400 box by default.
    sigma from Eo = rho_l g R^2 / sigma, the liquid viscosity from
    Ga = sqrt(g R) R / nu_l, the gas viscosity from the dynamic viscosity
    ratio; buoyancy on the light phase only (rho_ref = rho_l).  Seeded jitter
    of +-0.5 cells of the centre, which sits a quarter of the box height up.
    The paper does not give g; g = 4e-6 keeps sigma <= 0.01 down to Eo = 1 at
    R = 50 (with g = 5e-5, Eo = 1 needs sigma = 0.125, and that box loses
    stability within a few hundred steps at density ratio 1000).
    """
    rng = np.random.default_rng(seed)
    j = rng.uniform(-0.5, 0.5, size=3)
    c = ((nx - 1) / 2 + j[0], (ny - 1) / 2 + j[1], nz / 4 + j[2])
    x = np.arange(nx, dtype=np.float64).reshape(1, 1, nx)
    y = np.arange(ny, dtype=np.float64).reshape(1, ny, 1)
    z = np.arange(nz, dtype=np.float64).reshape(nz, 1, 1)
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    phi = tanh_profile(r - radius, width)
    rho_l, rho_g = 1.0, 1.0 / rho_ratio
    sigma = rho_l * g * radius ** 2 / eotvos
    nu_l = np.sqrt(g * radius) * radius / galilei
    nu_g = nu_l * rho_ratio / mu_ratio
    prob = Problem(nx, ny, nz, (PERIODIC,) * 3, rho_l, rho_g, nu_l, nu_g, sigma, mobility,
                   width, (0.0, 0.0, -g), rho_l)
    return Case("eo_ga_bubble_Eo%g_Ga%g" % (eotvos, galilei), prob, phi, None, None, seed)


def eo_ga_sweep(points=None, **kw):
    """One bubble per (Eo, Ga) point, seeds 7, 8, ...; equal boxes, so the
    whole sweep runs as one batched launch per step."""
    pts = EO_GA_POINTS if points is None else points
    return [eo_ga_bubble(eo, ga, seed=7 + i, **kw) for i, (eo, ga) in enumerate(pts)]


def random_state(nx, ny, nz, seed, bc=(PERIODIC,) * 3, amp_u=0.02, amp_p=0.01,
                 amp_q=1e-3, **kw):
    """Smooth-ish random state for invariance and parity tests.

    Returns (problem, phi, pstar, J, Q6) where Q6 holds (xx, yy, zz, xy, xz, yz).
    """
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    phi = rng.uniform(0.0, 1.0, size=shape)
    pstar = amp_p * rng.uniform(-1, 1, size=shape)
    J = amp_u * rng.uniform(-1, 1, size=(3,) + shape)
    Q = amp_q * rng.uniform(-1, 1, size=(6,) + shape)
    prob = Problem(nx, ny, nz, tuple(bc), **kw)
    return prob, phi, pstar, J, Q


CONFIGS = {
    "C1": lambda: static_droplet(),
    "C2": lambda: rising_bubble(),
    "C3": lambda: droplet_collision(),
    "C5": lambda: drop_into_pool(),
}
