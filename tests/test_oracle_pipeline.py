"""Pins of the oracle's initial-condition assembly (Fig. 2, step 3: the recovered
centre of mass is populated with an equilibrium Plummer sphere of mass M_Plummer).

The physical scales of the assembled sphere are checked against the Plummer
model's own closed forms, not against a retyped copy of the assembly formula:
with unit samples drawn for G = M = a = 1, a sphere of total mass M and scale
radius a_P must carry the potential energy and the kinetic energy that the
Plummer model fixes for that mass and radius, in physical units.  The samples
are truncated at 10 scale radii, so the expected energies are the quadratures of
the truncated profile (the untruncated values -3 pi G M^2 / (32 a) and half its
magnitude are 2.7 % away); the velocity dispersion at radius r is the isotropic
Jeans value <v^2>(r) = G M / (2 sqrt(r^2 + a^2)).  A slip in the velocity scale
(sqrt(G M a_P) for sqrt(G M / a_P)), the particle mass, or the position scale
changes one of the energies by orders of magnitude.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.spatial.distance import pdist

from oracle import constants as C
from oracle.pipeline import assemble_ic
from synth import plummer_unit

R_MAX = 10.0   # truncation radius of the unit samples, in scale radii


def _mu(r):
    """Mass fraction inside r of an untruncated Plummer sphere (unit scale radius)."""
    return r ** 3 / (r * r + 1.0) ** 1.5


def _dmu(r):
    return 3.0 * r * r / (r * r + 1.0) ** 2.5


def truncated_energies():
    """(W, K) of a Plummer sphere truncated at R_MAX, with its mass renormalised to 1,
    in units of G M^2 / a: W = -int M(r) dM / r, K = 1/2 int <v^2>(r) dM."""
    f_r = _mu(R_MAX)
    W = -integrate.quad(lambda r: (_mu(r) / f_r) * (_dmu(r) / f_r) / r, 0.0, R_MAX,
                        epsabs=1e-13, epsrel=1e-12)[0]
    K = 0.5 * integrate.quad(lambda r: 0.5 / np.sqrt(1.0 + r * r) * _dmu(r) / f_r, 0.0, R_MAX,
                             epsabs=1e-13, epsrel=1e-12)[0]
    return W, K


def test_truncated_energies_reduce_to_the_untruncated_closed_form():
    # the quadratures themselves: without the truncation they give -3 pi / 32 and
    # 3 pi / 64, the Plummer sphere's potential and kinetic energy (virial 2K = -W)
    W = -integrate.quad(lambda r: _mu(r) * _dmu(r) / r, 0.0, np.inf, epsabs=1e-13)[0]
    K = 0.5 * integrate.quad(lambda r: 0.5 / np.sqrt(1.0 + r * r) * _dmu(r), 0.0, np.inf,
                             epsabs=1e-13)[0]
    assert W == pytest.approx(-3.0 * np.pi / 32.0, rel=1e-9)
    assert K == pytest.approx(3.0 * np.pi / 64.0, rel=1e-9)
    Wt, Kt = truncated_energies()
    assert 0.97 < Wt / W < 1.05 and 0.97 < Kt / K < 1.05


@pytest.mark.parametrize("m_prog,a_p,seed", [(3e4, C.A_PLUMMER, 41), (1e5, 0.03, 42)])
def test_assemble_ic_physical_scales(m_prog, a_p, seed):
    n = 4096
    xi, zeta = plummer_unit(n, seed)
    w_x = np.array(C.W_NOW_X)
    w_v = np.array(C.W_NOW_V)
    x0, v0, m = assemble_ic(w_x, w_v, m_prog, xi, zeta, C.G, a_p)
    # mass: n equal particles summing to M_Plummer
    assert np.all(m == m[0])
    assert m.sum() == pytest.approx(m_prog, rel=1e-13)
    # centre of mass and its velocity at the recovered phase-space point
    np.testing.assert_allclose(x0.mean(0), w_x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v0.mean(0), w_v, rtol=0, atol=1e-10)
    # energies in the centre-of-mass frame against the truncated Plummer model
    scale = C.G * m_prog ** 2 / a_p
    W_exp, K_exp = truncated_energies()
    W = -C.G * m[0] * m[0] * np.sum(1.0 / pdist(x0 - x0.mean(0)))
    dv = v0 - v0.mean(0)
    K = 0.5 * np.sum(m[:, None] * dv * dv)
    # sampling scatter of either energy at n = 4096 is about 2 %
    assert W / (W_exp * scale) == pytest.approx(1.0, abs=0.05)
    assert K / (K_exp * scale) == pytest.approx(1.0, abs=0.05)
    assert (2 * K / -W) / (2 * K_exp / -W_exp) == pytest.approx(1.0, abs=0.05)
