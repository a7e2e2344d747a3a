"""Discrete adjoint of the oracle's integrator (test infrastructure only).

Sec. 2 states that the final particle state is differentiable with respect to
the initial conditions, the integration time, the particle masses and the
external-potential parameters, which the paper obtains by reverse-mode
differentiation through the whole simulation.  The oracle computes the same
quantity, the exact derivative of the discrete kick-drift-kick map, by writing
the reverse sweep out step by step (no merging of the two half kicks that meet
at a common x_n).  Nothing here is approximated: every formula below is the
chain rule applied to the forward code of forces.py and integrate.py, and the
test-suite pins it against complex-step derivatives of that forward code.

Pair Jacobian, with d_kj = x_j - x_k, s = |d|^2 + eps^2 and
K(d) = s^(-3/2) I - 3 s^(-5/2) d d^T:

    (J^T w)_k = G sum_j K(d_kj) (m_k w_j - m_j w_k)

Mass cotangent of the pair sum:

    (da/dm)^T w |_k = -G sum_j (d_kj . w_j) s_kj^(-3/2)
"""
import numpy as np

from . import forces


def pair_vjp(pos, mass, G, eps, w, rows=None, block=256):
    """(J^T w)_k for all k, or for the index array `rows` only."""
    pos = np.asarray(pos)
    w = np.asarray(w)
    mass = np.asarray(mass)
    idx = np.arange(pos.shape[0]) if rows is None else np.asarray(rows)
    out = np.zeros((idx.shape[0], 3), dtype=np.result_type(pos, w, mass, float))
    eps2 = eps * eps
    for b0 in range(0, idx.shape[0], block):
        kk = idx[b0:b0 + block]
        d = pos[None, :, :] - pos[kk, None, :]                 # x_j - x_k
        s = d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2 + eps2
        if eps2 == 0:
            s = s.copy()
            s[np.arange(kk.shape[0]), kk] = 1.0
        r3 = s ** -1.5
        r5 = s ** -2.5
        u = mass[kk, None, None] * w[None, :, :] - mass[None, :, None] * w[kk, None, :]
        du = d[..., 0] * u[..., 0] + d[..., 1] * u[..., 1] + d[..., 2] * u[..., 2]
        term = r3[..., None] * u - 3.0 * (r5 * du)[..., None] * d
        if eps2 == 0:
            term[np.arange(kk.shape[0]), kk, :] = 0.0
        out[b0:b0 + block] = G * term.sum(axis=1)
    return out


def pair_mass_vjp(pos, G, eps, w, block=256):
    pos = np.asarray(pos)
    w = np.asarray(w)
    n = pos.shape[0]
    out = np.zeros(n, dtype=np.result_type(pos, w, float))
    eps2 = eps * eps
    for b0 in range(0, n, block):
        kk = np.arange(b0, min(n, b0 + block))
        d = pos[None, :, :] - pos[kk, None, :]
        s = d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2 + eps2
        if eps2 == 0:
            s = s.copy()
            s[np.arange(kk.shape[0]), kk] = 1.0
        dw = d[..., 0] * w[None, :, 0] + d[..., 1] * w[None, :, 1] + d[..., 2] * w[None, :, 2]
        t = dw * s ** -1.5
        if eps2 == 0:
            t[np.arange(kk.shape[0]), kk] = 0.0
        out[b0:b0 + block] = -G * t.sum(axis=1)
    return out


def accel_vjp(pos, mass, pot, w, with_ext=True, self_gravity=True):
    """Cotangents of a(x; m, M_NFW, M_MN) for an incoming cotangent w.

    Returns (gx, gm, g_mnfw, g_mmn).  Both host masses enter linearly, so
    da/dM = a_component / M.
    """
    gx = np.zeros(np.shape(pos), dtype=np.result_type(pos, w, float))
    gm = np.zeros(np.shape(pos)[0], dtype=gx.dtype)
    if self_gravity:
        gx = gx + pair_vjp(pos, mass, pot.G, pot.eps, w)
        gm = gm + pair_mass_vjp(pos, pot.G, pot.eps, w)
    g_nfw = g_mn = 0.0
    if with_ext:
        gx = gx + forces.ext_hvp(pos, w, pot)
        if pot.m_nfw != 0:
            g_nfw = np.sum(forces.nfw_accel(pos, pot.G, 1.0, pot.rs_nfw) * w)
        if pot.m_mn != 0:
            g_mn = np.sum(forces.mn_accel(pos, pot.G, 1.0, pot.a_mn, pot.b_mn) * w)
    return gx, gm, g_nfw, g_mn


def ext_shape_vjp(pos, pot, w):
    """Cotangents of the host's shape parameters for an incoming cotangent w of
    the accelerations: (sum w . da/drs_nfw, sum w . da/da_mn, sum w . da/db_mn)."""
    g_rs = g_a = g_b = 0.0
    if pot.m_nfw != 0:
        g_rs = np.sum(forces.nfw_accel_drs(pos, pot.G, pot.m_nfw, pot.rs_nfw) * w)
    if pot.m_mn != 0:
        da, db = forces.mn_accel_dab(pos, pot.G, pot.m_mn, pot.a_mn, pot.b_mn)
        g_a, g_b = np.sum(da * w), np.sum(db * w)
    return g_rs, g_a, g_b


def simulate_vjp(traj, mass, pot, dt, gx_T, gv_T, with_ext=True, self_gravity=True):
    """Reverse sweep through a trajectory recorded by integrate.simulate(keep=True).

    Returns a dict with the cotangents of x_0, v_0, the particle masses, the
    two host masses, the host's three shape parameters and the step size dt.
    """
    xs, vhs, acs = traj["x"], traj["vh"], traj["a"]
    lx = np.array(gx_T, copy=True)
    lv = np.array(gv_T, copy=True)
    lm = np.zeros(np.shape(mass), dtype=np.result_type(lx, float))
    l_nfw = l_mn = l_dt = 0.0
    l_shape = np.zeros(3, dtype=lx.dtype)

    def shape(x, w):
        return np.array(ext_shape_vjp(x, pot, w)) if with_ext else 0.0

    for n in range(len(vhs) - 1, -1, -1):
        # v_{n+1} = v_half + dt/2 a(x_{n+1})
        gx, gm, gn, gd = accel_vjp(xs[n + 1], mass, pot, lv, with_ext, self_gravity)
        lx = lx + 0.5 * dt * gx
        lm = lm + 0.5 * dt * gm
        l_nfw = l_nfw + 0.5 * dt * gn
        l_mn = l_mn + 0.5 * dt * gd
        l_shape = l_shape + 0.5 * dt * shape(xs[n + 1], lv)
        l_dt = l_dt + 0.5 * np.sum(acs[n + 1] * lv)
        # x_{n+1} = x_n + dt v_half
        l_dt = l_dt + np.sum(vhs[n] * lx)
        lv = lv + dt * lx
        # v_half = v_n + dt/2 a(x_n)
        gx, gm, gn, gd = accel_vjp(xs[n], mass, pot, lv, with_ext, self_gravity)
        lx = lx + 0.5 * dt * gx
        lm = lm + 0.5 * dt * gm
        l_nfw = l_nfw + 0.5 * dt * gn
        l_mn = l_mn + 0.5 * dt * gd
        l_shape = l_shape + 0.5 * dt * shape(xs[n], lv)
        l_dt = l_dt + 0.5 * np.sum(acs[n] * lv)
    return dict(x0=lx, v0=lv, mass=lm, m_nfw=l_nfw, m_mn=l_mn, dt=l_dt,
                rs_nfw=l_shape[0], a_mn=l_shape[1], b_mn=l_shape[2])
