"""Differentiable forward model of the stream-inference pipeline.

The pipeline of the paper (Fig. 2, steps 2-4; Sec. 2.2.1): integrate the
present-day centre of mass backward for t_end in the host potential as a single
particle, populate the recovered point with an equilibrium Plummer sphere of
mass M_Plummer, evolve it forward for t_end with a fixed number of steps, and
compare the final positions with the observed stream through the MMD.
theta = (t_end, M_Plummer, M_NFW, M_MN), t_end in internal time units.

Every stage is a call into libdnb (autograd.py); torch only forms dt = t_end/n
and chains the scalar cotangents.
"""
import torch

from . import autograd as AG
from .engine import Potential
from .units import G as G_DEFAULT

W_NOW = (12.0, 0.0, 0.0, 0.0, -180.0, 60.0)


class StreamModel:
    def __init__(self, engine_ctx, xi, zeta, target, n_steps, pot=None, h=0.2, a_p=0.01,
                 ckpt_every=1, w_now=W_NOW):
        self.ctx = engine_ctx
        self.xi, self.zeta, self.target = xi, zeta, target
        self.n_steps, self.h, self.a_p, self.K = int(n_steps), float(h), float(a_p), int(ckpt_every)
        self.pot = pot if pot is not None else Potential()
        self.w_now = torch.tensor(w_now, dtype=torch.float64, device=xi.device)

    def final_positions(self, theta):
        t_end, m_prog, m_nfw, m_mn = theta[0], theta[1], theta[2], theta[3]
        dt = t_end / self.n_steps
        w0 = AG.orbit(self.ctx, self.w_now, m_nfw, m_mn, -dt, self.pot, self.n_steps)
        pos, vel, mass = AG.place_plummer(self.ctx, w0, m_prog, self.xi, self.zeta, self.a_p,
                                          self.pot.G)
        pos_T, _ = AG.simulate(self.ctx, pos, vel, mass, m_nfw, m_mn, dt, self.pot, self.n_steps,
                               self.K, m_scale=m_prog)
        return pos_T

    def loss(self, theta):
        return AG.mmd(self.ctx, self.final_positions(theta), self.target, self.h)

    def loss_and_grad(self, theta):
        th = theta.detach().clone().requires_grad_(True)
        L = self.loss(th)
        (g,) = torch.autograd.grad(L, th)
        return L.detach(), g


def make_target(engine_ctx, xi, zeta, theta, n_steps, pot=None, a_p=0.01):
    """Final positions of a pipeline run at theta (used as a mock observed stream)."""
    m = StreamModel(engine_ctx, xi, zeta, None, n_steps, pot=pot, a_p=a_p)
    with torch.no_grad():
        return m.final_positions(theta).detach()
