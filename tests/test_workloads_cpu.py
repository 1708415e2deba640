"""The seeded inputs carry the parameters and dimensionless numbers of the
configurations they stand for, and their geometry is where the recipe puts
it."""
import numpy as np

from paper_2501_00846_amd import workloads as WL


def test_raindrop_train_recipe():
    c = WL.raindrop_train(nx=48, ny=40, nz=300, radius=6.0, spacing=2.0, weber=40.0, speed=0.05)
    p = c.problem
    assert p.bc == (WL.PERIODIC, WL.PERIODIC, WL.WALL)
    assert p.rho_l * 0.05 ** 2 * 12.0 / p.sigma == np.float64(40.0)
    assert abs(p.rho_ref - p.rho_g) == 0 and p.gravity[2] < 0
    prof = c.phi[:, 20, 24]
    inside = np.where(prof > 0.5)[0]
    # five drops of ~2R nodes each, centres 2 D apart starting at R + D = 18
    runs = np.split(inside, np.where(np.diff(inside) > 1)[0] + 1)
    assert len(runs) == 5
    centres = [r.mean() for r in runs]
    assert np.allclose(np.diff(centres), 24.0, atol=1.0) and abs(centres[0] - 18.0) < 1.0
    assert np.allclose(c.u[2], -0.05 * c.phi) and np.abs(c.u[:2]).max() == 0.0
    assert 0.0 <= c.phi.min() and c.phi.max() <= 1.0


def test_eo_ga_recipe():
    for case, (eo, ga) in zip(WL.eo_ga_sweep(nx=24, ny=24, nz=48, radius=6.0), WL.EO_GA_POINTS):
        p = case.problem
        g, R = -p.gravity[2], 6.0
        assert np.isclose(p.rho_l * g * R * R / p.sigma, eo, rtol=1e-12)
        assert np.isclose(np.sqrt(g * R) * R / p.nu_l, ga, rtol=1e-12)
        assert np.isclose((p.nu_l * p.rho_l) / (p.nu_g * p.rho_g), 100.0, rtol=1e-12)
        assert p.bc == (WL.PERIODIC,) * 3 and p.rho_ref == p.rho_l
        # gas bubble: phi small at the centre, liquid far away
        assert case.phi[12, 12, 12] < 0.01 and case.phi[40, 0, 0] > 0.99
    assert (30.0, 100.0) in WL.EO_GA_POINTS


def test_static_droplet_recipe():
    """32^3 periodic, R 8, W 4, density ratio 1000, viscosity ratio 100,
    sigma 0.01, M 0.02, u noise of 1e-6, drop at the box centre."""
    c = WL.static_droplet()
    p = c.problem
    assert (p.nx, p.ny, p.nz) == (32, 32, 32) and p.bc == (WL.PERIODIC,) * 3
    assert p.rho_l / p.rho_g == 1000.0
    assert np.isclose((p.nu_l * p.rho_l) / (p.nu_g * p.rho_g), 100.0, rtol=1e-12)
    assert (p.sigma, p.mobility, p.width) == (0.01, 0.02, 4.0)
    assert np.abs(c.u).max() <= 1e-6 and np.abs(c.u).max() > 0
    # symmetric about the centre (15.5, 15.5, 15.5); phi = 1/2 at radius 8
    assert np.allclose(c.phi, c.phi[::-1, ::-1, ::-1], atol=1e-14)
    assert np.isclose(c.phi[16, 16, 16], 1.0, atol=1e-3) and c.phi[0, 0, 0] < 1e-3


def test_rising_bubble_recipe():
    """128 x 128 x 256 with walls on every face; gas bubble of R 16 at z 48
    (jittered by at most half a cell); g = 1e-6 along -z on the gas;
    sigma and the liquid viscosity from Eo = rho_l g R^2 / sigma = 10 and
    Mo = g mu_l^4 (rho_l - rho_g) / (rho_l^2 sigma^3) = 1e-3; dynamic
    viscosity ratio 100, density ratio 1000."""
    c = WL.rising_bubble()
    p = c.problem
    g, R = 1e-6, 16.0
    assert (p.nx, p.ny, p.nz) == (128, 128, 256) and p.bc == (WL.WALL,) * 3
    assert p.gravity == (0.0, 0.0, -g) and p.rho_ref == p.rho_l
    assert np.isclose(p.rho_l * g * R * R / p.sigma, 10.0, rtol=1e-12)
    mu_l = p.nu_l * p.rho_l
    assert np.isclose(g * mu_l ** 4 * (p.rho_l - p.rho_g) / (p.rho_l ** 2 * p.sigma ** 3), 1e-3, rtol=1e-10)
    assert np.isclose(mu_l / (p.nu_g * p.rho_g), 100.0, rtol=1e-12)
    assert np.isclose(p.sigma, 2.56e-5, rtol=1e-12) and np.isclose(p.nu_l, 2.024e-3, rtol=1e-3)
    # bubble centre: the lightest node lies within a cell of (63.5, 63.5, 48)
    z, y, x = np.unravel_index(np.argmin(c.phi), c.phi.shape)
    assert abs(x - 63.5) <= 1.5 and abs(y - 63.5) <= 1.5 and abs(z - 48) <= 1.5


def test_collision_and_pool_recipes():
    """Collision: 256^3 periodic, two R 24 drops at +-0.02, density ratio 800,
    viscosity ratio 50, sigma 0.005.  Pool: 512^3 with walls on +-z, pool of
    128 cells, R 40 drop at z 260 falling at 0.05 under g 1e-6, sigma 0.008
    (checked on the builders' small-size variants where the sizes scale)."""
    c = WL.droplet_collision(n=64, radius=6.0)
    p = c.problem
    assert p.bc == (WL.PERIODIC,) * 3 and p.rho_l / p.rho_g == 800.0
    assert np.isclose((p.nu_l * p.rho_l) / (p.nu_g * p.rho_g), 50.0, rtol=1e-12) and p.sigma == 0.005
    assert np.isclose(np.abs(c.u[0]).max(), 0.02, rtol=1e-2)  # 0.02 times the drop's own phi
    full = WL.droplet_collision.__defaults__
    assert 256 in full and 24.0 in full
    d = WL.drop_into_pool(n=64)  # geometry scales with nz / 512: pool 16, R 5, drop at z 32.5
    q = d.problem
    assert q.bc == (WL.PERIODIC, WL.PERIODIC, WL.WALL) and q.sigma == 0.008 and q.rho_ref == q.rho_g
    assert q.gravity[2] == -1e-6 and np.isclose(d.u[2].min(), -0.05, rtol=2e-2)  # 0.05 times the drop's phi
    assert d.phi[4, 32, 32] > 0.99 and d.phi[22, 32, 32] < 0.01 and d.phi[32, 32, 32] > 0.98
    assert WL.drop_into_pool.__defaults__[:4] == (512, 128, 40.0, 260.0)


def test_ensemble_recipe():
    """64 boxes, edges iid in [24, 96], one ellipsoidal drop per box of radius
    (0.15-0.35) x min edge and aspect ratio 1-1.5, seeds 4000 + k."""
    boxes = WL.ensemble()
    assert len(boxes) == 64
    for c in boxes:
        p = c.problem
        assert all(24 <= n <= 96 for n in (p.nx, p.ny, p.nz)) and p.bc == (WL.PERIODIC,) * 3
        vol = (c.phi > 0.5).sum()
        r_eq = (3 * vol / (4 * np.pi)) ** (1 / 3)
        m = min(p.nx, p.ny, p.nz)
        assert 0.12 * m <= r_eq <= 0.38 * m, (c.name, r_eq, m)
    assert len({(c.problem.nx, c.problem.ny, c.problem.nz) for c in boxes}) > 50
