"""Equilibrium Plummer-sphere samples in unit form.

The paper's benchmark and inference runs start from a Plummer sphere in
equilibrium (Sec. 2.1 and the inference pipeline of Fig. 2, step 3).  Samples
are drawn with the method of Aarseth, Henon and Wielen (1974):

* the radius from the inverse cumulative mass profile,
  r = (U^(-2/3) - 1)^(-1/2), rejecting r > r_max (default 10 scale radii);
* the speed as a fraction q of the local escape speed sqrt(2) (1 + r^2)^(-1/4),
  with q drawn by rejection from g(q) = q^2 (1 - q^2)^(7/2) under the bound 0.1;
* isotropic, independent directions for position and velocity.

Units are G = M = a = 1: the returned xi and zeta are x / a_P and
v / sqrt(G M / a_P).  The sample mean of each is removed, so the centre of
mass is at rest at the origin.  Seeds feed numpy's PCG64 generator.
"""
import numpy as np


def _isotropic(rng, n):
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)


def plummer_unit(n, seed, r_max=10.0):
    """Return (xi, zeta), each float64 of shape (n, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = np.empty(0)
    while radii.shape[0] < n:
        u = rng.uniform(0.0, 1.0, 2 * n + 16)
        u = u[u > 0.0]
        r = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        radii = np.concatenate([radii, r[r <= r_max]])
    r = radii[:n]
    q = np.empty(0)
    while q.shape[0] < n:
        qq = rng.uniform(0.0, 1.0, 4 * n + 16)
        yy = rng.uniform(0.0, 0.1, 4 * n + 16)
        q = np.concatenate([q, qq[yy < qq * qq * (1.0 - qq * qq) ** 3.5]])
    q = q[:n]
    speed = q * np.sqrt(2.0) * (1.0 + r * r) ** -0.25
    xi = r[:, None] * _isotropic(rng, n)
    zeta = speed[:, None] * _isotropic(rng, n)
    xi -= xi.mean(axis=0)
    zeta -= zeta.mean(axis=0)
    return xi, zeta


def random_directions(n, seed):
    """n seeded unit vectors in 3-D, shape (n, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _isotropic(rng, n)


def sample_rows(n, k, seed):
    """k distinct seeded row indices out of n, sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=min(k, n), replace=False))
