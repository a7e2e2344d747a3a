"""Pins of the oracle's integrator, adjoint, loss and pipeline.

The integrator is pinned by the closed-form two-body (Kepler) orbit, its order
of convergence, conservation laws and time reversibility; the adjoint by
complex-step derivatives of the oracle's own forward map (exact to rounding
because every function on the path is analytic) and the dot-product identity;
the MMD by its identities and by the closed-form expectation for Gaussian
samples.
"""
import numpy as np

from oracle import adjoint, constants as C, forces, integrate, mmd, pipeline
from oracle.forces import Potential
from synth import plummer_unit

G = 4.3009e-6


def kepler_relative(t, a, e, GM):
    n = np.sqrt(GM / a ** 3)
    M = n * t
    E = M.copy() if np.ndim(M) else M
    for _ in range(60):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    return np.array([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), 0.0])


def kepler_run(dt, n_steps, a=1.0, e=0.5, m1=0.3, m2=0.7):
    GM = m1 + m2
    r0 = a * (1 - e)
    v0 = np.sqrt(GM * (1 + e) / (a * (1 - e)))
    rel_x = np.array([r0, 0, 0])
    rel_v = np.array([0, v0, 0])
    pos = np.array([-m2 / GM * rel_x, m1 / GM * rel_x])
    vel = np.array([-m2 / GM * rel_v, m1 / GM * rel_v])
    pot = Potential(G=1.0, eps=0.0)
    x, v = integrate.simulate(pos, vel, np.array([m1, m2]), pot, dt, n_steps, with_ext=False)
    rel = x[1] - x[0]
    return rel, kepler_relative(dt * n_steps, a, e, GM)


def test_kepler_two_body_closed_form_and_second_order():
    P = 2 * np.pi
    errs = []
    for k in (1000, 2000, 4000):
        rel, exact = kepler_run(P / k, k // 2)       # half an orbit, ends at apocentre
        errs.append(np.sqrt(((rel - exact) ** 2).sum()))
    assert errs[-1] < 5e-5
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (errs, r1, r2)


def test_kepler_energy_has_no_secular_drift():
    m = np.array([0.3, 0.7])
    a, e = 1.0, 0.5
    r0, v0 = a * (1 - e), np.sqrt((1 + e) / (a * (1 - e)))
    pos = np.array([[-0.7 * r0, 0, 0], [0.3 * r0, 0, 0]])
    vel = np.array([[0, -0.7 * v0, 0], [0, 0.3 * v0, 0]])
    pot = Potential(G=1.0, eps=0.0)
    E0 = integrate.total_energy(pos, vel, m, pot, with_ext=False)
    errs = []
    integrate.simulate(pos, vel, m, pot, 2 * np.pi / 500, 5000, with_ext=False,
                       callback=lambda n, x, v: errs.append(
                           integrate.total_energy(x, v, m, pot, with_ext=False) / E0 - 1))
    errs = np.abs(np.array(errs))
    first, last = errs[:500].max(), errs[-500:].max()
    assert last < 1.5 * first and first < 1e-3


def _cluster(n=40, seed=0, m_tot=2e4):
    xi, zeta = plummer_unit(n, seed)
    a_p = 0.01
    x = np.array(C.W_NOW_X) + a_p * xi
    v = np.array(C.W_NOW_V) + np.sqrt(G * m_tot / a_p) * zeta
    return x, v, np.full(n, m_tot / n)


def test_momentum_conserved_in_isolation():
    x, v, m = _cluster()
    pot = Potential()
    P0 = (m[:, None] * v).sum(0)
    x1, v1 = integrate.simulate(x, v, m, pot, C.myr(0.5), 100, with_ext=False)
    P1 = (m[:, None] * v1).sum(0)
    assert np.abs(P1 - P0).max() < 1e-12 * np.abs(m[:, None] * v).sum()


def test_angular_momentum_z_conserved_in_axisymmetric_host():
    x, v, m = _cluster()
    pot = Potential()
    Lz = lambda x, v: np.sum(m * (x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0]))
    L0 = Lz(x, v)
    x1, v1 = integrate.simulate(x, v, m, pot, C.myr(0.5), 200)
    assert abs(Lz(x1, v1) - L0) < 1e-12 * abs(L0) * 200


def test_time_reversibility():
    x, v, m = _cluster()
    pot = Potential()
    x1, v1 = integrate.simulate(x, v, m, pot, C.myr(0.5), 60)
    x2, v2 = integrate.simulate(x1, -v1, m, pot, C.myr(0.5), 60)
    assert np.abs(x2 - x).max() < 1e-9
    assert np.abs(-v2 - v).max() < 1e-6


def test_restart_from_a_stored_state_is_bitwise():
    # the fixed-step map is a function of the state alone: stopping after k steps
    # and continuing from the stored (x, v) reproduces the uninterrupted run
    x, v, m = _cluster()
    pot = Potential()
    dt = C.myr(0.5)
    stored = {}
    xT, vT = integrate.simulate(x, v, m, pot, dt, 30,
                                callback=lambda k, xk, vk: stored.update({k: (xk.copy(), vk.copy())}))
    for k in (1, 10, 29):
        xk, vk = stored[k]
        x2, v2 = integrate.simulate(xk, vk, m, pot, dt, 30 - k)
        assert np.array_equal(x2, xT) and np.array_equal(v2, vT)


# -------------------------------------------------------------------- adjoint

def _cs(fun, h=1e-30):
    return np.imag(fun(1j * h)) / h


def test_adjoint_matches_complex_step_of_the_forward_map():
    rng = np.random.default_rng(11)
    x, v, m = _cluster(n=12, seed=3)
    pot = Potential(m_nfw=1.1e12, m_mn=6.0e10)
    dt, n_steps = C.myr(1.0), 25
    wx, wv = rng.normal(size=x.shape), rng.normal(size=v.shape)
    dx, dv = rng.normal(size=x.shape) * 1e-3, rng.normal(size=v.shape)
    dm = rng.normal(size=m.shape)

    def run(z, px=0, pv=0, pm=0, pn=0.0, pd=0.0, pdt=0.0, prs=0.0, pa=0.0, pb=0.0):
        pp = pot.replace(m_nfw=pot.m_nfw + z * pn, m_mn=pot.m_mn + z * pd,
                         rs_nfw=pot.rs_nfw + z * prs, a_mn=pot.a_mn + z * pa,
                         b_mn=pot.b_mn + z * pb)
        xT, vT = integrate.simulate(x + z * px, v + z * pv, m + z * pm, pp, dt + z * pdt, n_steps)
        return np.sum(wx * xT) + np.sum(wv * vT)

    xT, vT, traj = integrate.simulate(x, v, m, pot, dt, n_steps, keep=True)
    g = adjoint.simulate_vjp(traj, m, pot, dt, wx, wv)
    np.testing.assert_allclose(np.sum(g["x0"] * dx) + np.sum(g["v0"] * dv),
                               _cs(lambda z: run(z, px=dx, pv=dv)), rtol=1e-10)
    np.testing.assert_allclose(np.sum(g["mass"] * dm), _cs(lambda z: run(z, pm=dm)), rtol=1e-10)
    np.testing.assert_allclose(g["m_nfw"], _cs(lambda z: run(z, pn=1.0)), rtol=1e-10)
    np.testing.assert_allclose(g["m_mn"], _cs(lambda z: run(z, pd=1.0)), rtol=1e-10)
    np.testing.assert_allclose(g["dt"], _cs(lambda z: run(z, pdt=1.0)), rtol=1e-10)
    np.testing.assert_allclose(g["rs_nfw"], _cs(lambda z: run(z, prs=1.0)), rtol=1e-10)
    np.testing.assert_allclose(g["a_mn"], _cs(lambda z: run(z, pa=1.0)), rtol=1e-10)
    np.testing.assert_allclose(g["b_mn"], _cs(lambda z: run(z, pb=1.0)), rtol=1e-10)


def test_pair_vjp_dot_product_identity():
    rng = np.random.default_rng(12)
    x, _, m = _cluster(n=30, seed=4)
    delta, w = rng.normal(size=x.shape), rng.normal(size=x.shape)
    jd = np.imag(forces.pair_accel(x + 1e-30j * delta, m, G, 1e-3)) / 1e-30
    jtw = adjoint.pair_vjp(x, m, G, 1e-3, w)
    np.testing.assert_allclose(np.sum(jd * w), np.sum(delta * jtw), rtol=1e-11)
    dm = rng.normal(size=m.shape)
    jm = np.imag(forces.pair_accel(x, m + 1e-30j * dm, G, 1e-3)) / 1e-30
    np.testing.assert_allclose(np.sum(jm * w), np.sum(dm * adjoint.pair_mass_vjp(x, G, 1e-3, w)),
                               rtol=1e-11)


def test_pipeline_gradient_matches_complex_step():
    xi, zeta = plummer_unit(10, 21)
    target = np.array(C.W_NOW_X) + 0.05 * np.random.default_rng(5).normal(size=(16, 3))
    pot = Potential()
    theta = np.array([C.myr(40.0), 3e4, 1.1e12, 7e10])
    L, g = pipeline.loss_and_grad(theta, xi, zeta, pot, 20, target, 0.2)
    names = ["t_end", "m_prog", "m_nfw", "m_mn"]
    for k, name in enumerate(names):
        th = theta.astype(complex)
        th[k] += 1e-30j * theta[k]
        cs = np.imag(pipeline.loss(th, xi, zeta, pot, 20, target, 0.2)) / (1e-30 * theta[k])
        np.testing.assert_allclose(g[name], cs, rtol=1e-9, err_msg=name)


# ----------------------------------------------------------------------- MMD

def test_mmd_identities_and_gradient():
    rng = np.random.default_rng(13)
    X, Y = rng.normal(size=(40, 3)), rng.normal(size=(30, 3)) + 0.3
    assert abs(mmd.mmd2(X, X, 0.5)) < 1e-15
    assert mmd.mmd2(X, Y, 0.5) > 0
    x, y = X[:1], Y[:1]
    d2 = np.sum((x - y) ** 2)
    np.testing.assert_allclose(mmd.mmd2(x, y, 0.7), 2 - 2 * np.exp(-d2 / (2 * 0.49)), rtol=1e-14)
    g = mmd.mmd2_grad(X, Y, 0.5)
    D = rng.normal(size=X.shape)
    cs = np.imag(mmd.mmd2(X + 1e-30j * D, Y, 0.5)) / 1e-30
    np.testing.assert_allclose(np.sum(g * D), cs, rtol=1e-12)


def test_mmd_expectation_for_gaussian_clouds():
    # E k(x,y) for x ~ N(mu1, s1^2 I), y ~ N(mu2, s2^2 I) in 3-D:
    #   (h^2/(h^2+s1^2+s2^2))^{3/2} exp(-|mu1-mu2|^2 / (2 (h^2+s1^2+s2^2)))
    rng = np.random.default_rng(14)
    h, s1, s2 = 0.2, 0.15, 0.25
    mu = np.array([0.1, -0.05, 0.0])
    n, m = 3000, 2000
    X = rng.normal(scale=s1, size=(n, 3))
    Y = mu + rng.normal(scale=s2, size=(m, 3))

    def Ek(sa, sb, dmu2):
        q = h * h + sa * sa + sb * sb
        return (h * h / q) ** 1.5 * np.exp(-dmu2 / (2 * q))

    expect = ((1 / n) + (1 - 1 / n) * Ek(s1, s1, 0) + (1 / m) + (1 - 1 / m) * Ek(s2, s2, 0)
              - 2 * Ek(s1, s2, mu @ mu))
    got = mmd.mmd2(X, Y, h)
    assert abs(got - expect) < 0.03 * expect, (got, expect)
