"""Seeded draws of the four inference parameters.

The paper infers Theta = (t_end, M_Plummer, M_NFW, M_MN) (Sec. 2.2.1).  The
surrogate's training set draws them from box priors: t_end uniform in Gyr, the
three masses log-uniform in solar masses.
"""
import numpy as np

PRIOR_BOUNDS = (
    (1.0, 4.0),          # t_end [Gyr], uniform
    (1.0e4, 1.0e5),      # M_Plummer [Msun], log-uniform
    (5.0e11, 2.0e12),    # M_NFW [Msun], log-uniform
    (3.0e10, 1.0e11),    # M_MN [Msun], log-uniform
)


def draw_theta(n, seed):
    """(n, 4) float64 array of (t_end [Gyr], M_Plummer, M_NFW, M_MN)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, 4))
    lo, hi = PRIOR_BOUNDS[0]
    out[:, 0] = rng.uniform(lo, hi, n)
    for k in range(1, 4):
        lo, hi = PRIOR_BOUNDS[k]
        out[:, k] = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n)
    return out
