"""CPU checks of the host-side parameter maps used by the surrogate and the fit."""
import numpy as np

from oracle import surrogate as S
from synth import draw_theta


def test_normalisation_matches_oracle_and_inverts():
    from paper_2511_22468_amd import surrogate as P
    th = draw_theta(50, 3)
    np.testing.assert_allclose(P.normalise(th), S.normalise_theta(th), rtol=0, atol=1e-14)
    np.testing.assert_allclose(P.denormalise(P.normalise(th)), th, rtol=1e-12)


def test_theta_jacobian_matches_finite_differences():
    from paper_2511_22468_amd import fit
    u = np.array([0.3, -0.4, 0.1, 0.7])
    J = fit.dtheta_du(u[None])
    for k in range(4):
        e = np.zeros(4)
        e[k] = 1e-6
        fd = (fit.theta_internal((u + e)[None]) - fit.theta_internal((u - e)[None])) / 2e-6
        np.testing.assert_allclose(fd[k], J[k], rtol=1e-7)
        assert np.all(np.delete(fd, k) == 0)


def test_orbit_frame_matches_oracle():
    from paper_2511_22468_amd.surrogate import orbit_frame
    e1, e2, n = S.frame((12.0, 0, 0), (0, -180.0, 60.0))
    np.testing.assert_allclose(orbit_frame((12.0, 0, 0), (0, -180.0, 60.0)),
                               np.concatenate([e1, e2, n]), atol=1e-15)


def test_bootstrap_row_maps_match_the_single_row_maps():
    from paper_2511_22468_amd import bootstrap as B, fit
    rng = np.random.default_rng(4)
    u = rng.uniform(-1, 1, (6, 4))
    th, J = B.theta_rows(u), B.dtheta_du_rows(u)
    for r in range(6):
        np.testing.assert_allclose(th[r], fit.theta_internal(u[r][None]), rtol=1e-15)
        np.testing.assert_allclose(J[r], fit.dtheta_du(u[r][None]), rtol=1e-15)


def test_inference_grid_covers_the_prior_box():
    from paper_2511_22468_amd.infer import grid_points
    g = grid_points(4)
    assert g.shape == (256, 4) and len({tuple(r) for r in g}) == 256
    assert g.min() == -1.0 and g.max() == 1.0
    for k in range(4):
        np.testing.assert_allclose(np.unique(g[:, k]), np.linspace(-1, 1, 4))
