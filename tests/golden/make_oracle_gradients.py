"""Writes tests/golden/oracle_gradients_n8192.txt from the oracle alone.

The differentiation workload at full particle number (Sec. 2: gradients of
the inference loss with respect to t_end, M_Plummer, M_NFW and M_MN; the
pipeline of Fig. 2, steps 2-4): 8192 Plummer particles (unit sample seed 3),
eps = 1e-3 kpc, n steps of t_end / n with t_end = n x 1.1 x (2 Gyr / 2000),
M_Plummer = 3.6e4, M_NFW = 0.9e12, M_MN = 7.15e10 Msun, and the squared MMD
(h = 0.2 kpc) against a 4096-point Gaussian cloud of sigma 0.02 kpc about
(12, 0, 0) kpc (PCG64 seed 30).  For n = 20 and 50 the file holds the loss and
the four gradient components, and the same for the initial positions
perturbed at the FP32 rounding scale (every unit-sample coordinate scaled by
1 +- 2^-24, signs from PCG64 seeds 100 + k): the spread between those runs is
the oracle's own sensitivity to one FP32 rounding of the initial state, which
grows with the horizon because the bound core is chaotic.

Usage: python tests/golden/make_oracle_gradients.py [--jobs J]
(about 20 minutes on 6 cores).
"""
import argparse
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_gradients_n8192.txt")
N, M_TGT, STEPS, DRAWS = 8192, 4096, (20, 50), 2


def inputs():
    from synth import plummer_unit
    xi, zeta = plummer_unit(N, 3)
    rng = np.random.Generator(np.random.PCG64(30))
    target = np.array([12.0, 0.0, 0.0]) + 0.02 * rng.normal(size=(M_TGT, 3))
    return xi, zeta, target


def theta_for(T):
    from oracle import constants as C
    return np.array([T * 1.1 * C.gyr(2.0) / 2000, 3e4 * 1.2, 1e12 * 0.9, 6.5e10 * 1.1])


def perturbed(xi, k):
    rng = np.random.Generator(np.random.PCG64(100 + k))
    s = rng.choice(np.array([-1.0, 1.0]), size=xi.shape)
    return xi * (1.0 + s * 2.0 ** -24)


def one(job):
    T, k = job
    from oracle import pipeline as opipe
    from oracle.forces import Potential
    xi, zeta, target = inputs()
    if k >= 0:
        xi = perturbed(xi, k)
    L, g = opipe.loss_and_grad(theta_for(T), xi, zeta, Potential(eps=1e-3), T, target, 0.2)
    return T, k, L, [g["t_end"], g["m_prog"], g["m_nfw"], g["m_mn"]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    jobs = [(T, k) for T in STEPS for k in range(-1, DRAWS)]
    with Pool(a.jobs) as p:
        res = p.map(one, jobs, chunksize=1)
    with open(OUT, "w") as f:
        f.write("# Oracle pipeline loss and gradient, N = 8192 differentiation workload\n")
        f.write("# (written by tests/golden/make_oracle_gradients.py, which states the\n")
        f.write("# configuration).  draw -1: the unperturbed initial state; draw k >= 0:\n")
        f.write("# unit-sample positions scaled by 1 +- 2^-24 (signs from PCG64 seed 100 + k).\n")
        f.write("# steps draw loss dL/dt_end dL/dM_Plummer dL/dM_NFW dL/dM_MN\n")
        for T, k, L, g in res:
            f.write(f"{T} {k} {float(L)!r} " + " ".join(repr(float(x)) for x in g) + "\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
