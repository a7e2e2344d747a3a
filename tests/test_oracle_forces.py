"""Pins of the oracle's force and potential code against physics and mathematics.

None of these tests re-types the formula under test: each one checks the
oracle against a different route to the same quantity (a potential
differentiated by complex step, an enclosed mass integrated numerically,
Poisson's equation, a conservation law, a textbook special case).
"""
import numpy as np
import pytest
from scipy import integrate as spi

from oracle import forces
from oracle.forces import Potential

G = 4.3009e-6


def cs_grad(f, x, h=1e-30):
    """Complex-step gradient of a scalar function of a flat float vector."""
    x = np.asarray(x, dtype=float)
    g = np.zeros_like(x)
    for k in range(x.size):
        xc = x.astype(complex)
        xc.flat[k] += 1j * h
        g.flat[k] = np.imag(f(xc)) / h
    return g


def cs_jvp(f, x, v, h=1e-30):
    """Complex-step directional derivative of a vector function."""
    return np.imag(f(np.asarray(x, complex) + 1j * h * np.asarray(v))) / h


# ------------------------------------------------------------------ pair sum

def test_two_body_closed_form():
    eps = 0.3
    pos = np.array([[0.0, 0.0, 0.0], [2.0, -1.0, 0.5]])
    m = np.array([3.0, 5.0])
    a = forces.pair_accel(pos, m, 1.7, eps)
    r = np.array([2.0, -1.0, 0.5])
    r2 = 4.0 + 1.0 + 0.25
    # magnitude G m_other r / (r^2+eps^2)^{3/2}, directed at the other body
    np.testing.assert_allclose(a[0], 1.7 * 5.0 * r / (r2 + eps * eps) ** 1.5, rtol=1e-14)
    np.testing.assert_allclose(a[1], -1.7 * 3.0 * r / (r2 + eps * eps) ** 1.5, rtol=1e-14)


def test_pair_force_is_minus_gradient_of_pair_energy():
    rng = np.random.default_rng(0)
    pos = rng.normal(size=(7, 3))
    m = rng.uniform(0.5, 2.0, 7)
    eps = 0.05
    a = forces.pair_accel(pos, m, G, eps)

    def W(flat):
        return forces.pair_potential_energy(flat.reshape(7, 3), m, G, eps)

    grad = cs_grad(W, pos.ravel()).reshape(7, 3)
    np.testing.assert_allclose(m[:, None] * a, -grad, rtol=1e-12, atol=1e-12 * np.abs(grad).max())


def test_newton_third_law_and_translation_invariance():
    rng = np.random.default_rng(1)
    pos = rng.normal(scale=0.01, size=(300, 3))
    m = rng.uniform(1.0, 3.0, 300)
    a = forces.pair_accel(pos, m, G, 1e-3)
    net = np.abs((m[:, None] * a).sum(axis=0)).max()
    assert net / np.sum(m * np.sqrt((a * a).sum(1))) < 1e-15 * 300
    a2 = forces.pair_accel(pos + np.array([0.3, -0.2, 0.1]), m, G, 1e-3)
    np.testing.assert_allclose(a2, a, rtol=1e-9, atol=1e-9 * np.abs(a).max())


def test_symmetric_configuration_gives_zero_force_at_centre():
    # centre particle surrounded by the 8 vertices of a cube
    verts = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    pos = np.vstack([np.zeros((1, 3)), verts])
    a = forces.pair_accel(pos, np.ones(9), 1.0, 0.1)
    assert np.abs(a[0]).max() < 1e-15


def test_distant_cluster_acts_as_point_mass():
    rng = np.random.default_rng(2)
    cl = rng.normal(scale=0.01, size=(200, 3))
    cl -= cl.mean(0)
    pos = np.vstack([cl, [[50.0, 0.0, 0.0]]])
    m = np.ones(201)
    a = forces.pair_accel(pos, m, G, 1e-3, rows=np.array([200]))[0]
    # monopole: G M / D^2 toward the cluster; quadrupole correction ~ (0.01/50)^2
    np.testing.assert_allclose(a, [-G * 200 / 50.0 ** 2, 0, 0], rtol=1e-6, atol=1e-12)


def test_zero_softening_masks_self_term():
    pos = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    a = forces.pair_accel(pos, np.array([1.0, 1.0]), 1.0, 0.0)
    np.testing.assert_allclose(a, [[1.0, 0, 0], [-1.0, 0, 0]], rtol=1e-15)


def test_longdouble_brute_force_small_n():
    rng = np.random.default_rng(3)
    for n in (2, 5, 16):
        pos = rng.normal(size=(n, 3))
        m = rng.uniform(0.1, 1.0, n)
        a64 = forces.pair_accel(pos, m, G, 1e-2)
        ald = forces.pair_accel(pos.astype(np.longdouble), m.astype(np.longdouble), G, 1e-2)
        np.testing.assert_allclose(a64, ald.astype(float), rtol=1e-13, atol=0)


# ------------------------------------------------------------------ NFW halo

def test_nfw_accel_is_minus_gradient_of_potential():
    rng = np.random.default_rng(4)
    for p in rng.normal(scale=10.0, size=(6, 3)):
        f = lambda q: forces.nfw_potential(q.reshape(1, 3), G, 1e12, 16.0)[0]
        g = cs_grad(f, p)
        np.testing.assert_allclose(forces.nfw_accel(p[None], G, 1e12, 16.0)[0], -g, rtol=1e-12)


def test_nfw_enclosed_mass_by_quadrature():
    # rho = rho0 / ((r/rs)(1+r/rs)^2) with M = 4 pi rho0 rs^3 (scale mass)
    M, rs = 1e12, 16.0
    rho0 = M / (4 * np.pi * rs ** 3)
    for r in (0.5, 5.0, 12.0, 40.0, 200.0):
        Menc, _ = spi.quad(lambda s: 4 * np.pi * s * s * rho0 / ((s / rs) * (1 + s / rs) ** 2), 0, r,
                           epsabs=0, epsrel=1e-13, limit=200)
        a = forces.nfw_accel(np.array([[r, 0.0, 0.0]]), G, M, rs)[0]
        np.testing.assert_allclose(-a[0], G * Menc / r ** 2, rtol=1e-10)


def test_nfw_centre_limit_and_circular_velocity():
    a = forces.nfw_accel(np.array([[1e-7, 0, 0], [0.0, 0, 0]]), G, 1e12, 16.0)
    np.testing.assert_allclose(-a[0, 0], G * 1e12 / (2 * 16.0 ** 2), rtol=1e-6)
    assert np.all(a[1] == 0)
    # series and closed form agree at the switch point
    x = np.array([0.99999e-4, 1.00001e-4])
    mu = forces._nfw_mu(x)
    np.testing.assert_allclose(mu[0] / x[0] ** 2, mu[1] / x[1] ** 2, rtol=1e-5)


# --------------------------------------------------------- Miyamoto-Nagai ---

def test_mn_accel_is_minus_gradient_of_potential():
    rng = np.random.default_rng(5)
    for p in rng.normal(scale=5.0, size=(6, 3)):
        f = lambda q: forces.mn_potential(q.reshape(1, 3), G, 6.5e10, 3.0, 0.28)[0]
        np.testing.assert_allclose(forces.mn_accel(p[None], G, 6.5e10, 3.0, 0.28)[0], -cs_grad(f, p),
                                   rtol=1e-12)


def test_mn_reduces_to_plummer_and_point_mass():
    rng = np.random.default_rng(6)
    p = rng.normal(scale=2.0, size=(5, 3))
    r2 = (p * p).sum(1)
    a = forces.mn_accel(p, G, 1e10, 0.0, 0.7)
    np.testing.assert_allclose(a, -G * 1e10 * p / ((r2 + 0.49) ** 1.5)[:, None], rtol=1e-13)
    a = forces.mn_accel(p, G, 1e10, 0.0, 0.0)
    np.testing.assert_allclose(a, -G * 1e10 * p / (r2 ** 1.5)[:, None], rtol=1e-13)


def test_mn_poisson_equation():
    # div a = -4 pi G rho with the Miyamoto-Nagai (1975) density
    M, a_, b = 6.5e10, 3.0, 0.28
    rng = np.random.default_rng(7)
    for p in rng.normal(scale=[4.0, 4.0, 0.5], size=(5, 3)):
        f = lambda q: forces.mn_accel(q.reshape(1, 3), G, M, a_, b)[0]
        div = sum(cs_jvp(f, p, e)[k] for k, e in enumerate(np.eye(3)))
        R2 = p[0] ** 2 + p[1] ** 2
        S = np.sqrt(p[2] ** 2 + b * b)
        rho = b * b * M / (4 * np.pi) * (a_ * R2 + (a_ + 3 * S) * (a_ + S) ** 2) / (
            (R2 + (a_ + S) ** 2) ** 2.5 * S ** 3)
        np.testing.assert_allclose(div, -4 * np.pi * G * rho, rtol=1e-10)


def test_nfw_poisson_equation():
    M, rs = 1e12, 16.0
    rho0 = M / (4 * np.pi * rs ** 3)
    rng = np.random.default_rng(8)
    for p in rng.normal(scale=10.0, size=(5, 3)):
        f = lambda q: forces.nfw_accel(q.reshape(1, 3), G, M, rs)[0]
        div = sum(cs_jvp(f, p, e)[k] for k, e in enumerate(np.eye(3)))
        r = np.sqrt((p * p).sum())
        np.testing.assert_allclose(div, -4 * np.pi * G * rho0 / ((r / rs) * (1 + r / rs) ** 2),
                                   rtol=1e-10)


# ----------------------------------------------------------------- Hessians

@pytest.mark.parametrize("which", ["nfw", "mn"])
def test_external_hessian_vector_products(which):
    rng = np.random.default_rng(9)
    p = rng.normal(scale=6.0, size=(8, 3))
    w = rng.normal(size=(8, 3))
    if which == "nfw":
        f = lambda q: forces.nfw_accel(q, G, 1e12, 16.0)
        hv = forces.nfw_hvp(p, w, G, 1e12, 16.0)
    else:
        f = lambda q: forces.mn_accel(q, G, 6.5e10, 3.0, 0.28)
        hv = forces.mn_hvp(p, w, G, 6.5e10, 3.0, 0.28)
    # per-particle functions: the Jacobian is block diagonal, so J w is a JVP
    np.testing.assert_allclose(hv, cs_jvp(f, p, w), rtol=1e-11, atol=1e-12 * np.abs(hv).max())


def test_nfw_scale_radius_derivative_against_complex_step():
    # positions from the centre (the small-x series of mu) out to 20 scale radii
    rng = np.random.default_rng(13)
    dirs = rng.normal(size=(9, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    radii = np.array([1e-6, 1e-3, 0.5, 4.0, 12.0, 16.0, 40.0, 120.0, 320.0])
    p = dirs * radii[:, None]
    got = forces.nfw_accel_drs(p, G, 1e12, 16.0)
    ref = np.imag(forces.nfw_accel(p, G, 1e12, 16.0 + 1e-30j)) / 1e-30
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())
    assert np.all(forces.nfw_accel_drs(np.zeros((1, 3)), G, 1e12, 16.0) == 0.0)


@pytest.mark.parametrize("b", [0.28, 0.0])
def test_mn_scale_length_derivatives_against_complex_step(b):
    # points above, below and in the disk plane (b = 0: the razor-thin disk, whose
    # b-derivative vanishes off the plane and is taken as zero on it)
    rng = np.random.default_rng(14)
    p = rng.normal(scale=6.0, size=(10, 3))
    p[:3, 2] = 0.0
    da, db = forces.mn_accel_dab(p, G, 6.5e10, 3.0, b)
    ra = np.imag(forces.mn_accel(p, G, 6.5e10, 3.0 + 1e-30j, b)) / 1e-30
    rb = np.imag(forces.mn_accel(p, G, 6.5e10, 3.0, b + 1e-30j)) / 1e-30
    np.testing.assert_allclose(da, ra, rtol=1e-10, atol=1e-14 * np.abs(ra).max())
    if b > 0:
        np.testing.assert_allclose(db, rb, rtol=1e-10, atol=1e-14 * np.abs(rb).max())
    else:
        np.testing.assert_allclose(db[3:], rb[3:], atol=1e-14 * np.abs(ra).max())
        assert np.all(db[:3] == 0.0)


def test_external_potential_defaults_and_circular_speed():
    pot = Potential()
    p = np.array([[12.0, 0.0, 0.0]])
    vc_nfw = np.sqrt(-forces.nfw_accel(p, G, pot.m_nfw, pot.rs_nfw)[0, 0] * 12.0)
    vc_mn = np.sqrt(-forces.mn_accel(p, G, pot.m_mn, pot.a_mn, pot.b_mn)[0, 0] * 12.0)
    # circular speeds of the host potential at the progenitor's present radius
    assert abs(vc_nfw - 216.72) < 0.01
    assert abs(vc_mn - 144.60) < 0.01
