"""The seeded inputs of the second workloads carry the dimensionless numbers
they are named for, and their geometry is where the recipe puts it."""
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
