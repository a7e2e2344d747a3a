"""Units and default parameters of the oracle (test infrastructure only).

Internal units are kpc, km/s and solar masses, the units in which the
workloads of the paper's stream experiment (Sec. 2.2.1) are stated.  The time
unit is then 1 kpc / (km/s).  The paper gives no unit convention; the reading
taken here is: kpc = 3.0856775814913673e16 km, Myr = 3.15576e13 s (Julian
year), and G = 4.3009e-6 kpc (km/s)^2 / Msun exactly.
"""

KPC_KM = 3.0856775814913673e16
MYR_S = 3.15576e13
# one internal time unit, kpc/(km/s), expressed in Myr
TIME_UNIT_MYR = KPC_KM / MYR_S
G = 4.3009e-6


def myr(t_myr):
    """Convert Myr to internal time units."""
    return t_myr / TIME_UNIT_MYR


def gyr(t_gyr):
    """Convert Gyr to internal time units."""
    return t_gyr * 1000.0 / TIME_UNIT_MYR


# Host potential of the stream experiments (Sec. 2.2.1 names an NFW halo and a
# Miyamoto-Nagai disk; the shape values follow the workload definitions).
M_NFW = 1.0e12
RS_NFW = 16.0
M_MN = 6.5e10
A_MN = 3.0
B_MN = 0.28

# Present-day phase-space point of the progenitor centre of mass.
W_NOW_X = (12.0, 0.0, 0.0)
W_NOW_V = (0.0, -180.0, 60.0)

# Plummer scale radius of the progenitor.
A_PLUMMER = 0.01
