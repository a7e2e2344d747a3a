"""torch.autograd.Function wrappers around the library's forward and adjoint calls.

The paper obtains gradients of the final particle state with respect to the
initial conditions, the integration time, the particle masses and the
external-potential parameters by reverse-mode differentiation through the
simulation (Sec. 2).  Here each differentiable stage is one Function whose
backward is the library's hand-written adjoint (the exact discrete adjoint of
the kick-drift-kick map), so torch only chains a handful of tensors; no torch
arithmetic runs on particle data.

Tensors: positions/velocities (3, n) float64 CUDA, masses (n,), scalars 0-d
float64 CUDA tensors.  The potential shape parameters (rs_nfw, a_mn, b_mn, eps, G)
are held fixed; the two host masses and the step size are differentiable.
"""
import torch

from .engine import Potential


def _scalar(t):
    return float(t.detach().item()) if isinstance(t, torch.Tensor) else float(t)


class Simulate(torch.autograd.Function):
    """(pos0, vel0, mass, m_nfw, m_mn, dt, m_scale) -> (pos_T, vel_T) after n_steps steps.

    m_scale (optional 0-d tensor) declares that all particle masses are
    proportional to it (e.g. the progenitor mass, m_k = M / n); its cotangent is
    (sum_k m_k dL/dm_k) / m_scale, which the adjoint gets from one reduction
    instead of a per-particle mass gradient.  Per-particle mass gradients are
    computed only when `mass` itself requires grad."""

    @staticmethod
    def forward(ctx, pos0, vel0, mass, m_nfw, m_mn, dt, m_scale, engine_ctx, pot, n_steps,
                ckpt_every, reversal=False):
        p = pot.replace(m_nfw=_scalar(m_nfw), m_mn=_scalar(m_mn))
        pos, vel = pos0.detach().clone(), vel0.detach().clone()
        tape = engine_ctx.simulate(pos, vel, mass.detach(), p, _scalar(dt), n_steps,
                                   ckpt_every=ckpt_every)
        ctx.save_for_backward(mass, pos, vel)
        ctx.engine_ctx, ctx.pot, ctx.dt = engine_ctx, p, _scalar(dt)
        ctx.n_steps, ctx.K, ctx.tape = n_steps, ckpt_every, tape
        ctx.reversal = bool(reversal)
        ctx.mass_req = mass.requires_grad
        ctx.m_scale = None if m_scale is None else _scalar(m_scale)
        return pos, vel

    @staticmethod
    def backward(ctx, gpos, gvel):
        mass, posT, velT = ctx.saved_tensors
        if gpos is None:
            gpos = torch.zeros_like(posT)
        gx0, gv0, gm, gpar = ctx.engine_ctx.simulate_vjp(
            mass.detach(), ctx.pot, ctx.dt, ctx.n_steps, ctx.K, ctx.tape, posT,
            gpos.contiguous(), None if gvel is None else gvel.contiguous(),
            with_mass=ctx.mass_req, vel_T=velT if ctx.reversal else None)
        ctx.tape = None
        gs = None if ctx.m_scale is None else gpar[3] / ctx.m_scale
        return gx0, gv0, gm, gpar[0], gpar[1], gpar[2], gs, None, None, None, None, None


class MMD(torch.autograd.Function):
    """(pos, target) -> squared MMD (Gaussian kernel, bandwidth h); grad w.r.t. pos."""

    @staticmethod
    def forward(ctx, pos, target, h, engine_ctx):
        loss, g = engine_ctx.mmd(pos.detach(), target.detach(), h, grad=True)
        ctx.save_for_backward(g)
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        return g * gl, None, None, None


class Orbit(torch.autograd.Function):
    """(w0[6], m_nfw, m_mn, dt) -> w[6] after n_steps KDK steps in the host potential."""

    @staticmethod
    def forward(ctx, w0, m_nfw, m_mn, dt, engine_ctx, pot, n_steps):
        p = pot.replace(m_nfw=_scalar(m_nfw), m_mn=_scalar(m_mn))
        w, traj = engine_ctx.orbit(w0.detach().contiguous(), p, _scalar(dt), n_steps, keep=True)
        ctx.save_for_backward(traj)
        ctx.engine_ctx, ctx.pot, ctx.dt, ctx.n_steps = engine_ctx, p, _scalar(dt), n_steps
        return w

    @staticmethod
    def backward(ctx, gw):
        (traj,) = ctx.saved_tensors
        gw0, gpar = ctx.engine_ctx.orbit_vjp(traj, ctx.pot, ctx.dt, ctx.n_steps, gw.contiguous())
        return gw0, gpar[0], gpar[1], gpar[2], None, None, None


class PlacePlummer(torch.autograd.Function):
    """(w[6], m_tot) -> (pos, vel, mass) of a Plummer sphere from unit samples."""

    @staticmethod
    def forward(ctx, w, m_tot, xi, zeta, a_p, engine_ctx, G):
        pos, vel, mass = engine_ctx.place_plummer(w.detach().contiguous(), xi, zeta,
                                                  _scalar(m_tot), a_p, G)
        # the masses' dependence on m_tot is carried by Simulate's m_scale input
        ctx.mark_non_differentiable(mass)
        ctx.save_for_backward(zeta)
        ctx.engine_ctx, ctx.m_tot, ctx.a_p, ctx.G = engine_ctx, _scalar(m_tot), a_p, G
        return pos, vel, mass

    @staticmethod
    def backward(ctx, gpos, gvel, gmass):
        (zeta,) = ctx.saved_tensors
        if gpos is None:
            gpos = torch.zeros_like(zeta)
        if gvel is None:
            gvel = torch.zeros_like(zeta)
        gw, gm = ctx.engine_ctx.place_plummer_vjp(zeta, ctx.m_tot, ctx.a_p, gpos.contiguous(),
                                                  gvel.contiguous(), None, G=ctx.G)
        return gw, gm[0], None, None, None, None, None


class Accelerations(torch.autograd.Function):
    """(pos, mass) -> a = a_int + a_ext (3, n) at fixed potential parameters;
    the backward is dnb_accelerations_vjp (gradients of both inputs)."""

    @staticmethod
    def forward(ctx, pos, mass, engine_ctx, pot, with_ext):
        p, m = pos.detach().contiguous(), mass.detach().contiguous()
        ctx.save_for_backward(p, m)
        ctx.engine_ctx, ctx.pot, ctx.with_ext = engine_ctx, pot, with_ext
        return engine_ctx.accelerations(p, m, pot, with_ext=with_ext)

    @staticmethod
    def backward(ctx, gacc):
        p, m = ctx.saved_tensors
        g, gm = ctx.engine_ctx.accelerations_vjp(p, m, ctx.pot, gacc.contiguous(),
                                                 with_ext=ctx.with_ext,
                                                 with_mass=ctx.needs_input_grad[1])
        return g, gm, None, None, None


def accelerations(engine_ctx, pos, mass, pot: Potential, with_ext=True):
    return Accelerations.apply(pos, mass, engine_ctx, pot, with_ext)


def simulate(engine_ctx, pos0, vel0, mass, m_nfw, m_mn, dt, pot: Potential, n_steps,
             ckpt_every=1, m_scale=None, reversal=False):
    """reversal: the backward pass rebuilds the trajectory between checkpoints by
    stepping it backward from the final state instead of recomputing it forward
    (one pair launch per step instead of two; the gradient of a trajectory that
    differs from the run's by rounding grown over at most ckpt_every steps)."""
    return Simulate.apply(pos0, vel0, mass, m_nfw, m_mn, dt, m_scale, engine_ctx, pot, n_steps,
                          ckpt_every, reversal)


def mmd(engine_ctx, pos, target, h):
    return MMD.apply(pos, target, h, engine_ctx)


def orbit(engine_ctx, w0, m_nfw, m_mn, dt, pot: Potential, n_steps):
    return Orbit.apply(w0, m_nfw, m_mn, dt, engine_ctx, pot, n_steps)


def place_plummer(engine_ctx, w, m_tot, xi, zeta, a_p, G):
    return PlacePlummer.apply(w, m_tot, xi, zeta, a_p, engine_ctx, G)
