"""Units of the library: kpc, km/s, Msun; time in kpc/(km/s).

kpc = 3.0856775814913673e16 km and Myr = 3.15576e13 s (Julian year), so one
time unit is about 977.79 Myr.  G = 4.3009e-6 kpc (km/s)^2 / Msun.
"""
KPC_KM = 3.0856775814913673e16
MYR_S = 3.15576e13
TIME_UNIT_MYR = KPC_KM / MYR_S
G = 4.3009e-6


def myr(t):
    """Myr -> internal time units."""
    return t / TIME_UNIT_MYR


def gyr(t):
    """Gyr -> internal time units."""
    return t * 1000.0 / TIME_UNIT_MYR
