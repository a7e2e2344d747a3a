"""Bootstrap refinement of the stream inference, every realisation at once.

The inference pipeline of the paper (Fig. 2; Sec. 2.2.1) draws bootstrap
realisations of the observed stream, each resampled with its observational
errors, and refines a grid-search estimate for each one with 10 plain
gradient-descent steps, keeping the parameters of the lowest MMD met.  The
realisations are independent problems, so they advance together here: one
batched pipeline gradient (pipeline.batch_loss_and_grad) per descent step serves
all of them.

Steps are taken in the normalised coordinates u of the prior box (t_end linear,
masses logarithmic, as in the surrogate and the time-to-fit experiment) along
each realisation's negative gradient direction, with a step length that is
halved whenever a step would raise the loss: the paper quotes its learning rate
without the coordinates it applies to, and a normalised step serves every
horizon and mass scale alike.
"""
import numpy as np

from .pipeline import W_NOW, batch_loss_and_grad
from .surrogate import PRIOR, denormalise
from .units import gyr


def theta_rows(u):
    """(B, 4) normalised rows -> (t_end [internal], M_Plummer, M_NFW, M_MN)."""
    th = denormalise(u)
    th[:, 0] = gyr(th[:, 0])
    return th


def dtheta_du_rows(u):
    """Diagonal of d theta / d u for every row, (B, 4)."""
    th = denormalise(u)
    d = np.empty_like(th)
    d[:, 0] = gyr(1.5)
    for k in range(1, 4):
        lo, hi = np.log10(PRIOR[k][0]), np.log10(PRIOR[k][1])
        d[:, k] = th[:, k] * np.log(10.0) * 0.5 * (hi - lo)
    return d


def resample(target, sigma, noise):
    """Bootstrap realisations of an observed stream (Fig. 2, step 6): target
    (3, m) device tensor, sigma the positional error [kpc], noise (B, 3, m)
    standard normal draws (device tensor).  Returns (B, 3, m)."""
    return (target.unsqueeze(0) + sigma * noise).contiguous()


def refine(engine_ctx, u0, xi, zeta, targets, n_steps, lr, iters=10, pot=None, h=0.2,
           a_p=0.01, w_now=W_NOW, chunk=None):
    """iters descent steps for every row of u0 (B, 4) against targets[b]
    (B, 3, m).  Each step moves a realisation by its current step length along
    its negative gradient direction; a step that would raise that realisation's
    loss is not taken and its length is halved (the descent of the time-to-fit
    experiment).  Every step costs one batched pipeline gradient for all rows.
    Returns (u (B, 4) at the lowest loss met, that loss (B,), history
    (iters + 1, B) of the losses at the evaluated points, accepted (iters, B))."""
    u = np.clip(np.array(u0, float).reshape(-1, 4), -1.0, 1.0)

    def evaluate(uu):
        L, g = batch_loss_and_grad(engine_ctx, theta_rows(uu), xi, zeta, targets, n_steps, pot,
                                   h, a_p, w_now, chunk)
        return L, g * dtheta_du_rows(uu)

    L, gu = evaluate(u)
    hist, accepted = [L.copy()], []
    step = np.full(u.shape[0], float(lr))
    for _ in range(iters):
        gn = np.sqrt((gu * gu).sum(1))
        ok = np.isfinite(gn) & (gn > 0)
        cand = u.copy()
        cand[ok] = np.clip(u[ok] - step[ok, None] * gu[ok] / gn[ok, None], -1.0, 1.0)
        Lc, gc = evaluate(cand)
        acc = ok & (Lc <= L)
        u[acc], L[acc], gu[acc] = cand[acc], Lc[acc], gc[acc]
        step[~acc] *= 0.5
        hist.append(Lc)
        accepted.append(acc)
    return u, L, np.array(hist), np.array(accepted)
