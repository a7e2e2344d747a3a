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
import numpy as np
import torch

from . import autograd as AG
from .engine import Potential

W_NOW = (12.0, 0.0, 0.0, 0.0, -180.0, 60.0)


class StreamModel:
    def __init__(self, engine_ctx, xi, zeta, target, n_steps, pot=None, h=0.2, a_p=0.01,
                 ckpt_every=1, w_now=W_NOW, reversal=False):
        self.ctx = engine_ctx
        self.xi, self.zeta, self.target = xi, zeta, target
        self.n_steps, self.h, self.a_p, self.K = int(n_steps), float(h), float(a_p), int(ckpt_every)
        self.reversal = bool(reversal)
        self.pot = pot if pot is not None else Potential()
        self.w_now = torch.tensor(w_now, dtype=torch.float64, device=xi.device)

    def final_positions(self, theta):
        t_end, m_prog, m_nfw, m_mn = theta[0], theta[1], theta[2], theta[3]
        dt = t_end / self.n_steps
        w0 = AG.orbit(self.ctx, self.w_now, m_nfw, m_mn, -dt, self.pot, self.n_steps)
        pos, vel, mass = AG.place_plummer(self.ctx, w0, m_prog, self.xi, self.zeta, self.a_p,
                                          self.pot.G)
        pos_T, _ = AG.simulate(self.ctx, pos, vel, mass, m_nfw, m_mn, dt, self.pot, self.n_steps,
                               self.K, m_scale=m_prog, reversal=self.reversal)
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


def run_ensemble(engine_ctx, thetas, xi, zeta, n_steps, pot=None, a_p=0.01, w_now=W_NOW):
    """Final positions of pipeline runs at many parameter rows, advanced as
    batched ensembles (FP32C pair terms).  thetas: (M, 4) host array of
    (t_end [internal], M_Plummer, M_NFW, M_MN).  Yields (first row, positions
    (B, 3, n)) per chunk of as many members as the context holds."""
    pot = pot if pot is not None else Potential()
    dev = xi.device
    th = np.asarray(thetas, float).reshape(-1, 4)
    M, n = th.shape[0], xi.shape[1]
    pots = [pot.replace(m_nfw=r[2], m_mn=r[3]) for r in th]
    dts = [r[0] / n_steps for r in th]
    cap = engine_ctx.batch_capacity(n)
    if cap < 1:
        raise ValueError(f"the context cannot hold one system of {n} particles")
    cap = min(cap, M)
    w_now_t = torch.tensor(w_now, dtype=torch.float64, device=dev)
    m_prog = torch.tensor(th[:, 1], dtype=torch.float64, device=dev)
    for s in range(0, M, cap):
        e = min(M, s + cap)
        w0 = w_now_t.repeat(e - s, 1)
        w_init = engine_ctx.orbit_batch(w0, pots[s:e], [-d for d in dts[s:e]], n_steps)
        pos, vel, mass = engine_ctx.place_plummer_batch(w_init, xi, zeta, m_prog[s:e].contiguous(),
                                                        a_p, pot.G)
        engine_ctx.simulate_batch(pos, vel, mass, pots[s:e], dts[s:e], n_steps)
        yield s, pos


def grid_search(engine_ctx, thetas, xi, zeta, target, n_steps, pot=None, h=0.2, a_p=0.01,
                w_now=W_NOW):
    """MMD loss of the pipeline at every parameter row (the grid-search stage of
    the inference, Sec. 2.2.1): a host array of M losses.  target is one observed
    stream (3, m) or one per row (M, 3, m)."""
    th = np.asarray(thetas, float).reshape(-1, 4)
    out = torch.empty(th.shape[0], dtype=torch.float64, device=xi.device)
    per_target = target.dim() == 3
    for s, pos in run_ensemble(engine_ctx, th, xi, zeta, n_steps, pot, a_p, w_now):
        e = s + pos.shape[0]
        tgt = target[s:e].contiguous() if per_target else target
        out[s:e] = engine_ctx.mmd_batch(pos, tgt, h)
    return out.cpu().numpy()


def batch_loss_and_grad(engine_ctx, thetas, xi, zeta, target, n_steps, pot=None, h=0.2,
                        a_p=0.01, w_now=W_NOW, chunk=None):
    """MMD loss and its gradient with respect to theta = (t_end, M_Plummer, M_NFW,
    M_MN) at every parameter row, one batched pass per chunk (the gradient of
    StreamModel.loss for many theta at once).  Each chunk runs the backward orbit
    (keeping its trajectory), the placement, the N-body run (keeping its tape),
    the MMD with its position gradient, then the three adjoints in reverse.
    target is one observed stream (3, m) for every row or one per row (M, 3, m);
    w_now one present-day centre (6 values) or one per row ((M, 6) host array).
    chunk bounds the members per pass (default: as many as the context holds and
    half of the free device memory takes, the tape being 72 n T bytes per member).
    Returns host arrays (losses (M,), grads (M, 4)).

    With dt = t_end / n, the orbit runs with -dt and the N-body run with +dt, so
    dL/dt_end = (dL/ddt_sim - dL/ddt_orb) / n; the particle masses are M / n each,
    so the mass term of the N-body adjoint, sum_k m_k dL/dm_k, enters dL/dM
    divided by M beside the placement's own dL/dM."""
    pot = pot if pot is not None else Potential()
    dev = xi.device
    th = np.asarray(thetas, float).reshape(-1, 4)
    M, n = th.shape[0], xi.shape[1]
    T = int(n_steps)
    pots = [pot.replace(m_nfw=r[2], m_mn=r[3]) for r in th]
    dts = [r[0] / T for r in th]
    cap = engine_ctx.batch_capacity(n)
    if cap < 1:
        raise ValueError(f"the context cannot hold one system of {n} particles")
    if not chunk:
        # every member keeps its whole trajectory for the adjoint (9 n doubles per
        # step, plus the orbit and the per-member buffers): take at most half of
        # the free device memory
        free, _ = torch.cuda.mem_get_info(dev)
        per_member = 8 * (9 * n * T + 3 * n + 3 * (T + 1) + 40 * n)
        chunk = max(1, int(0.5 * free // per_member))
    cap = min(cap, M, int(chunk))
    w_rows = np.broadcast_to(np.asarray(w_now, float).reshape(-1, 6), (M, 6))
    w_now_t = torch.tensor(np.ascontiguousarray(w_rows), dtype=torch.float64, device=dev)
    per_target = target.dim() == 3
    m_prog = torch.tensor(th[:, 1], dtype=torch.float64, device=dev)
    losses = np.empty(M)
    grads = np.empty((M, 4))
    for s in range(0, M, cap):
        e = min(M, s + cap)
        B = e - s
        odts = [-d for d in dts[s:e]]
        w_init, traj = engine_ctx.orbit_batch(w_now_t[s:e].contiguous(), pots[s:e], odts, T,
                                              keep=True)
        mp = m_prog[s:e].contiguous()
        pos, vel, mass = engine_ctx.place_plummer_batch(w_init, xi, zeta, mp, a_p, pot.G)
        tape = engine_ctx.simulate_batch(pos, vel, mass, pots[s:e], dts[s:e], T, tape=True)
        tgt = target[s:e].contiguous() if per_target else target
        loss, gpos_T = engine_ctx.mmd_batch_grad(pos, tgt, h)
        g0, gv0, gsim = engine_ctx.simulate_batch_vjp(mass, pots[s:e], dts[s:e], T, tape, pos,
                                                      gpos_T)
        del tape
        gw, gm_place = engine_ctx.place_plummer_batch_vjp(zeta, mp, a_p, g0, gv0, pot.G)
        _, gorb = engine_ctx.orbit_batch_vjp(traj, pots[s:e], odts, T, gw)
        g = torch.stack([(gsim[:, 2] - gorb[:, 2]) / T,
                         gm_place + gsim[:, 3] / mp,
                         gsim[:, 0] + gorb[:, 0],
                         gsim[:, 1] + gorb[:, 1]], dim=1)
        losses[s:e] = loss.cpu().numpy()
        grads[s:e] = g.cpu().numpy()
    return losses, grads
