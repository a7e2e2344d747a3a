"""Bootstrap refinement of the stream inference, every realisation at once.

The inference pipeline of the paper (Fig. 2; Sec. 2.2.1) draws bootstrap
realisations of the observed stream, each resampled with its observational
errors, and refines a grid-search estimate for each one with 10 plain
gradient-descent steps, keeping the parameters of the lowest MMD met.  The
realisations are independent problems, so they advance together here: one
batched pipeline gradient (pipeline.batch_loss_and_grad) per descent step serves
all of them.

Steps are taken in the normalised coordinates u of the prior box (t_end linear,
masses logarithmic, as in the surrogate and the time-to-fit experiment), each of
fixed length lr along its realisation's negative gradient direction: the paper
quotes its learning rate without the coordinates it applies to, and a
normalised step serves every horizon and mass scale alike.
"""
import numpy as np
import torch

from .pipeline import W_NOW, batch_loss_and_grad, grid_search
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
    (B, 3, m), then the loss at the last point.  Returns (u_best (B, 4),
    L_best (B,), history (iters + 1, B) of losses)."""
    u = np.clip(np.array(u0, float).reshape(-1, 4), -1.0, 1.0)
    hist = []
    best_u, best_L = u.copy(), np.full(u.shape[0], np.inf)
    for it in range(iters + 1):
        th = theta_rows(u)
        if it < iters:
            L, g = batch_loss_and_grad(engine_ctx, th, xi, zeta, targets, n_steps, pot, h, a_p,
                                       w_now, chunk)
        else:
            L = grid_search(engine_ctx, th, xi, zeta, targets, n_steps, pot, h, a_p, w_now)
        better = L < best_L
        best_u[better], best_L[better] = u[better], L[better]
        hist.append(L)
        if it == iters:
            break
        gu = g * dtheta_du_rows(u)
        gn = np.sqrt((gu * gu).sum(1, keepdims=True))
        ok = np.isfinite(gn[:, 0]) & (gn[:, 0] > 0)
        step = np.zeros_like(u)
        step[ok] = lr * gu[ok] / gn[ok]
        u = np.clip(u - step, -1.0, 1.0)
    return best_u, best_L, np.array(hist)
