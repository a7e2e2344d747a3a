"""Checks of the seeded Plummer sampler against the Plummer model's closed forms."""
import numpy as np
from scipy import stats

from oracle import forces
from synth import plummer_unit, draw_theta, PRIOR_BOUNDS


def test_radius_distribution_matches_plummer_mass_profile():
    xi, _ = plummer_unit(20000, 7)
    r = np.sqrt((xi * xi).sum(1))
    rmax = 10.0
    Mtr = rmax ** 3 / (rmax ** 2 + 1) ** 1.5

    def cdf(x):
        x = np.minimum(x, rmax)
        return (x ** 3 / (x ** 2 + 1) ** 1.5) / Mtr

    # the mean shift after recentring is ~1e-2, below the KS resolution at this n
    res = stats.kstest(r, cdf)
    assert res.pvalue > 1e-3, res


def test_virial_equilibrium_and_zero_centre_of_mass():
    n = 3000
    xi, zeta = plummer_unit(n, 8)
    m = np.full(n, 1.0 / n)
    np.testing.assert_allclose(xi.mean(0), 0, atol=1e-15)
    np.testing.assert_allclose(zeta.mean(0), 0, atol=1e-15)
    K = 0.5 * np.sum(m * (zeta * zeta).sum(1))
    W = forces.pair_potential_energy(xi, m, 1.0, 1e-3)
    # untruncated Plummer sphere: W = -3 pi / 32, 2K/|W| = 1
    assert abs(2 * K / abs(W) - 1) < 0.08
    assert abs(W / (-3 * np.pi / 32) - 1) < 0.08


def test_speed_never_exceeds_escape_speed():
    xi, zeta = plummer_unit(5000, 9)
    # before recentring every speed is below the local escape speed; the mean
    # removed is tiny, so allow a small margin
    r2 = (xi * xi).sum(1)
    v = np.sqrt((zeta * zeta).sum(1))
    assert np.all(v < np.sqrt(2.0) * (1 + r2) ** -0.25 + 0.05)


def test_seeded_determinism_and_prior_bounds():
    a = plummer_unit(100, 3)
    b = plummer_unit(100, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    th = draw_theta(1000, 50)
    for k, (lo, hi) in enumerate(PRIOR_BOUNDS):
        assert th[:, k].min() >= lo and th[:, k].max() <= hi
