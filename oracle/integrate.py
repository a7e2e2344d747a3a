"""Kick-drift-kick integrator of the oracle (test infrastructure only).

Sec. 2.2.1 evolves the system with a second-order Velocity-Verlet integrator
and a fixed number of equal time steps.  Velocity-Verlet is the same map as the
kick-drift-kick leapfrog; the oracle writes it in the unmerged textbook form,
evaluating a(x_0) once at the start:

    v_half  = v_n + dt/2 a(x_n)
    x_{n+1} = x_n + dt v_half
    v_{n+1} = v_half + dt/2 a(x_{n+1})
"""
import numpy as np

from . import forces


def simulate(pos, vel, mass, pot, dt, n_steps, with_ext=True, self_gravity=True,
             keep=False, callback=None):
    """Advance (pos, vel) by n_steps of size dt.

    Returns (pos_T, vel_T) or, with keep=True, (pos_T, vel_T, traj) where traj
    holds per step n: x_n, the half-step velocity and a(x_n) for n = 0..n_steps
    (the half-step velocity list has n_steps entries).
    """
    x = np.array(pos, copy=True)
    v = np.array(vel, copy=True)
    a = forces.accel(x, mass, pot, with_ext, self_gravity)
    xs, vhs, acs = ([x.copy()], [], [a.copy()]) if keep else (None, None, None)
    for n in range(n_steps):
        vh = v + (0.5 * dt) * a
        x = x + dt * vh
        a = forces.accel(x, mass, pot, with_ext, self_gravity)
        v = vh + (0.5 * dt) * a
        if keep:
            xs.append(x.copy())
            vhs.append(vh.copy())
            acs.append(a.copy())
        if callback is not None:
            callback(n + 1, x, v)
    if keep:
        return x, v, dict(x=xs, vh=vhs, a=acs)
    return x, v


def step(pos, vel, mass, pot, dt, with_ext=True):
    """One kick-drift-kick step."""
    return simulate(pos, vel, mass, pot, dt, 1, with_ext)


def total_energy(pos, vel, mass, pot, with_ext=True):
    K, W, X = forces.energies(pos, vel, mass, pot)
    return K + W + (X if with_ext else 0.0)
