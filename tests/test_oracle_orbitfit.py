"""Pins of the oracle's orbit fit (chi2 track likelihood, Levenberg-Marquardt,
Fisher matrix; Sec. 2.2.2).

The frame and observables are pinned by the geometry of the present-day point,
by the library unwrap of the atan2 longitude and by a circular orbit in a
spherical halo (closed form); the interpolation by exactness at orbit points;
the Jacobian by central differences; the Hessian by the Gauss-Newton identity
H = 2 J^T J that holds exactly where all residuals vanish; Levenberg-Marquardt
by recovering the parameters of a noise-free track.
"""
import numpy as np
import pytest

from oracle import constants as C, forces, orbitfit as of

G = C.G
W_NOW = np.array([12.0, 0.0, 0.0, 0.0, -180.0, 60.0])
P_TRUE = np.log10([1.0e12, 16.0, 6.5e10, 3.0, 0.28])
SIGMA = (2e-3, 0.05, 1.0)        # phi2 [rad], d [kpc], v_r [km/s]
DT_TOTAL = C.gyr(0.5)
N_STEPS = 250


def mock_track(p=P_TRUE, K=16, lo=-0.9, hi=0.5):
    phi1 = np.linspace(lo, hi, K)
    Y, seg = of.model_track(p, W_NOW, G, DT_TOTAL, N_STEPS, phi1)
    assert all(s >= 0 for _, s in seg)
    return np.column_stack([phi1, Y])


ARGS = lambda tr: (tr, SIGMA, W_NOW, G, DT_TOTAL, N_STEPS)


def test_frame_is_right_handed_and_present_day_point_is_at_origin():
    e1, e2, n = of.frame(W_NOW)
    M = np.array([e1, e2, n])
    np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-15)
    np.testing.assert_allclose(np.cross(e1, e2), n, atol=1e-15)
    X, V = of.branch(W_NOW, of.potential(P_TRUE, G), 1e-3, 3)
    ph, Y = of.observables(X, V, (e1, e2, n))
    assert ph[0] == 0.0 and abs(Y[0, 0]) < 1e-16 and Y[0, 1] == 12.0
    assert ph[1] > 0          # the orbit moves towards +phi1 (e2 is the in-plane velocity)


def test_phi1_equals_unwrapped_atan2_longitude():
    pot = of.potential(P_TRUE, G)
    X, V = of.branch(W_NOW, pot, C.myr(2.0), 1500)     # several wraps
    fr = of.frame(W_NOW)
    ph, _ = of.observables(X, V, fr)
    ref = np.unwrap(np.arctan2(X @ fr[1], X @ fr[0]))
    assert ph[-1] > 4 * np.pi
    np.testing.assert_allclose(ph, ref, rtol=0, atol=1e-11)


def test_circular_orbit_in_spherical_halo():
    """NFW only, circular velocity in the plane: phi2 = 0, d = R, v_r = 0 up to
    the leapfrog's O(dt^2), phi1 = v_c t / R."""
    R, rs, M = 12.0, 16.0, 1e12
    x = R / rs
    vc = np.sqrt(G * M * (np.log1p(x) - x / (1 + x)) / R)
    w = np.array([R, 0, 0, 0, vc, 0.0])
    pot = forces.Potential(G=G, eps=0.0, m_nfw=M, rs_nfw=rs, m_mn=0.0)
    dt, n = C.myr(0.25), 400
    X, V = of.branch(w, pot, dt, n)
    fr = (np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0]))
    ph, Y = of.observables(X, V, fr)
    assert np.abs(Y[:, 0]).max() == 0.0
    dev = np.abs(Y[:, 1] - R).max()
    assert dev < 1e-5 * R and np.abs(Y[:, 2]).max() < 1e-3
    t = dt * np.arange(n + 1)
    np.testing.assert_allclose(ph, vc * t / R, rtol=1e-5, atol=1e-12)
    # the deviations are the leapfrog's O(dt^2): half the step, a quarter of them
    X2, V2 = of.branch(w, pot, dt / 2, 2 * n)
    ph2, Y2 = of.observables(X2, V2, fr)
    assert 3.6 < dev / np.abs(Y2[:, 1] - R).max() < 4.4
    assert 3.6 < np.abs(ph[-1] - vc * t[-1] / R) / np.abs(ph2[-1] - vc * t[-1] / R) < 4.4


def test_interpolation_is_exact_at_orbit_points_and_sides_follow_sign():
    pot = of.potential(P_TRUE, G)
    dt = DT_TOTAL / N_STEPS
    fr = of.frame(W_NOW)
    phf, Yf = of.observables(*of.branch(W_NOW, pot, dt, N_STEPS), fr)
    phb, Yb = of.observables(*of.branch(W_NOW, pot, -dt, N_STEPS), fr)
    assert phb[1] < 0
    pts = np.array([phf[5], phf[17], phb[9]])
    Y, seg = of.model_track(P_TRUE, W_NOW, G, DT_TOTAL, N_STEPS, pts)
    np.testing.assert_allclose(Y[0], Yf[5], rtol=1e-14)
    np.testing.assert_allclose(Y[1], Yf[17], rtol=1e-14)
    np.testing.assert_allclose(Y[2], Yb[9], rtol=1e-14)
    assert [s[0] for s in seg] == [1, 1, -1]
    # a longitude the branches never reach gives an infinite chi2
    far = np.array([[1e3, 0.0, 12.0, 0.0]])
    assert np.isinf(of.chi2(P_TRUE, far, SIGMA, W_NOW, G, DT_TOTAL, N_STEPS))


def test_chi2_zero_on_own_track_and_jacobian_matches_central_differences():
    tr = mock_track()
    assert of.chi2(P_TRUE, *ARGS(tr)) == 0.0
    p = P_TRUE + np.array([0.03, -0.02, 0.05, 0.04, -0.03])
    r, J = of.jacobian(p, *ARGS(tr))
    h = 1e-6
    for i in range(5):
        e = np.zeros(5)
        e[i] = h
        fd = (of.residuals(p + e, *ARGS(tr)) - of.residuals(p - e, *ARGS(tr))) / (2 * h)
        np.testing.assert_allclose(J[:, i], fd, rtol=1e-5, atol=1e-6 * np.abs(J).max())
    np.testing.assert_allclose(of.gradient(p, *ARGS(tr)), 2 * J.T @ r, rtol=1e-14)


def test_hessian_at_zero_residual_equals_gauss_newton():
    tr = mock_track()
    H = of.hessian(P_TRUE, *ARGS(tr))
    _, J = of.jacobian(P_TRUE, *ARGS(tr))
    GN = 2 * J.T @ J
    assert np.abs(H - GN).max() <= 1e-6 * np.abs(GN).max()
    F, Cov = of.fisher(H)
    np.testing.assert_allclose(F @ Cov, np.eye(5), atol=1e-6)


def test_hessian_away_from_minimum_matches_differences_of_chi2():
    tr = mock_track()
    p = P_TRUE + np.array([0.02, 0.01, -0.02, 0.01, 0.02])
    H = of.hessian(p, *ARGS(tr))
    h = 1e-3
    f = lambda q: of.chi2(q, *ARGS(tr))
    for i, j in [(0, 0), (0, 2), (1, 3), (4, 4)]:
        ei, ej = np.zeros(5), np.zeros(5)
        ei[i], ej[j] = h, h
        fd = (f(p + ei + ej) - f(p + ei - ej) - f(p - ei + ej) + f(p - ei - ej)) / (4 * h * h)
        assert abs(fd - H[i, j]) <= 2e-3 * np.abs(H).max(), (i, j, fd, H[i, j])


@pytest.mark.parametrize("start", [0, 1])
def test_levenberg_marquardt_recovers_noise_free_track(start):
    tr = mock_track()
    rng = np.random.default_rng(100 + start)
    p0 = P_TRUE + rng.uniform(-0.12, 0.12, 5)
    assert of.chi2(p0, *ARGS(tr)) > 10.0
    # the halo mass and scale radius are nearly degenerate on a short arc: the
    # walk along the valley takes a few dozen steps
    p, c = of.levenberg_marquardt(p0, *ARGS(tr), n_iter=60)
    assert c < 1e-20
    np.testing.assert_allclose(p, P_TRUE, rtol=0, atol=1e-9)
