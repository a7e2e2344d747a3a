"""Forward model and gradient of the stream-inference pipeline (test infrastructure only).

The inference pipeline of the paper (Fig. 2, steps 2-4; Sec. 2.2.1):

1. the present-day centre of mass w_now of the progenitor is integrated
   backward in time for t_end in the host potential (M_NFW, M_MN) as a single
   particle;
2. the recovered point is populated with an equilibrium Plummer sphere of mass
   M_Plummer;
3. the system is evolved forward for t_end with a fixed number of steps;
4. the final positions are compared with the observed stream by the MMD.

Readings where the paper is silent: the back-integration treats the
progenitor as a test particle (the paper's "single particle of mass
M_Plummer" feels no force that depends on its own mass in a static potential);
the number of steps n is fixed and dt = t_end / n for both legs, so t_end
enters smoothly; particle masses are M_Plummer / N and the velocity scale of
the Plummer sample is sqrt(G M_Plummer / a_P).

theta = (t_end, M_Plummer, M_NFW, M_MN) with t_end in internal time units.
"""
import numpy as np

from . import adjoint, constants as C, integrate, mmd


def back_integrate(theta, pot, n_steps, w_now=(C.W_NOW_X, C.W_NOW_V), keep=False):
    t_end, _, m_nfw, m_mn = theta
    pot_t = pot.replace(m_nfw=m_nfw, m_mn=m_mn)
    dt = t_end / n_steps
    wx = np.asarray(w_now[0], dtype=np.result_type(t_end, m_nfw, m_mn, float))[None, :]
    wv = np.asarray(w_now[1], dtype=wx.dtype)[None, :]
    return integrate.simulate(wx, wv, np.zeros(1), pot_t, -dt, n_steps,
                              self_gravity=False, keep=keep)


def assemble_ic(w_x, w_v, m_prog, xi, zeta, G, a_p=C.A_PLUMMER):
    n = xi.shape[0]
    x0 = w_x + a_p * xi
    v0 = w_v + np.sqrt(G * m_prog / a_p) * zeta
    m = np.full(n, m_prog / n, dtype=np.result_type(m_prog, float))
    return x0, v0, m


def forward(theta, xi, zeta, pot, n_steps, a_p=C.A_PLUMMER, keep=False):
    t_end, m_prog, m_nfw, m_mn = theta
    pot_t = pot.replace(m_nfw=m_nfw, m_mn=m_mn)
    dt = t_end / n_steps
    back = back_integrate(theta, pot, n_steps, keep=keep)
    x0, v0, m = assemble_ic(back[0], back[1], m_prog, xi, zeta, pot.G, a_p)
    fwd = integrate.simulate(x0, v0, m, pot_t, dt, n_steps, keep=keep)
    if keep:
        return fwd[0], fwd[1], dict(back=back, fwd=fwd, m=m, x0=x0, v0=v0)
    return fwd[0], fwd[1]


def loss(theta, xi, zeta, pot, n_steps, target, h, a_p=C.A_PLUMMER):
    xT, _ = forward(theta, xi, zeta, pot, n_steps, a_p)
    return mmd.mmd2(xT, target, h)


def loss_and_grad(theta, xi, zeta, pot, n_steps, target, h, a_p=C.A_PLUMMER):
    """Return (L, dict of dL/dtheta components and dL/d(x0, v0))."""
    t_end, m_prog, m_nfw, m_mn = theta
    pot_t = pot.replace(m_nfw=m_nfw, m_mn=m_mn)
    dt = t_end / n_steps
    xT, vT, rec = forward(theta, xi, zeta, pot, n_steps, a_p, keep=True)
    L = mmd.mmd2(xT, target, h)
    gxT = mmd.mmd2_grad(xT, target, h)
    adj = adjoint.simulate_vjp(rec["fwd"][2], rec["m"], pot_t, dt, gxT, np.zeros_like(vT))
    n = xi.shape[0]
    g_mprog = (np.sum(adj["mass"]) / n
               + np.sum(adj["v0"] * zeta) * 0.5 * np.sqrt(pot.G / (a_p * m_prog)))
    lwx = np.sum(adj["x0"], axis=0)[None, :]
    lwv = np.sum(adj["v0"], axis=0)[None, :]
    adjb = adjoint.simulate_vjp(rec["back"][2], np.zeros(1), pot_t, -dt, lwx, lwv,
                                self_gravity=False)
    g = dict(
        t_end=(adj["dt"] - adjb["dt"]) / n_steps,
        m_prog=g_mprog,
        m_nfw=adj["m_nfw"] + adjb["m_nfw"],
        m_mn=adj["m_mn"] + adjb["m_mn"],
        x0=adj["x0"], v0=adj["v0"],
    )
    return L, g
