"""Orbit fit of a stream progenitor (bindings of include/dnb_orbitfit.h).

The paper's second inference example (Sec. 2.2.2) evolves only the progenitor,
forward and backward in time from its present-day point, compares the orbit
with the stream track through a chi-squared statistic, minimises it by
Levenberg-Marquardt from many random starts and reads confidence contours off
the inverse Fisher matrix F = 1/2 d2 chi2 / dp dp.  Parameters are
p = log10(M_NFW, rs_NFW, M_MN, a_MN, b_MN).  Every integration, derivative,
damped solve and inverse runs in the library's kernels; torch only allocates.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .units import G as G_DEFAULT, gyr

NPAR = 5
TRACK_MAX = 64
# Starts of the fit are drawn between p_true / START_FACTOR and p_true * START_FACTOR
# (Sec. 2.2.2: from half to twice the true parameters).
START_FACTOR = 2.0


@dataclass(frozen=True)
class TrackModel:
    w_now: tuple = (12.0, 0.0, 0.0, 0.0, -180.0, 60.0)
    dt_total: float = gyr(2.0)
    n_steps: int = 2000
    sigma: tuple = (2e-3, 0.05, 1.0)  # phi2 [rad], d [kpc], v_r [km/s]
    G: float = G_DEFAULT

    def c(self):
        m = _lib.dnb_track_model()
        m.w_now[:] = [float(v) for v in self.w_now]
        m.G, m.dt_total, m.n_steps = float(self.G), float(self.dt_total), int(self.n_steps)
        m.sigma[:] = [float(v) for v in self.sigma]
        return m


def _dev(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")
    return t


def _track(track):
    K = track.shape[0]
    _dev(track, (K, 4), "track")
    return K


def observe(ctx, model, phi1, p):
    """Model (phi2, d, v_r) at the longitudes phi1 (K,) for p (5,): a (K, 3) tensor."""
    K = phi1.shape[0]
    _dev(phi1, (K,), "phi1"); _dev(p, (NPAR,), "p")
    y = torch.empty(K, 3, dtype=torch.float64, device=phi1.device)
    _lib.check(_lib.lib().dnb_track_observe(ctx._h, model.c(), K, _lib.ptr(phi1), _lib.ptr(p),
                                            _lib.ptr(y), _lib.stream_handle()))
    return y


def chi2(ctx, model, track, p, derivatives=True):
    """chi2 (B,), J^T r (B, 5) and packed J^T J (B, 15) at p (B, 5)."""
    K, B = _track(track), p.shape[0]
    _dev(p, (B, NPAR), "p")
    dev = p.device
    c = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty(B, NPAR, dtype=torch.float64, device=dev) if derivatives else None
    h = torch.empty(B, 15, dtype=torch.float64, device=dev) if derivatives else None
    _lib.check(_lib.lib().dnb_track_chi2(ctx._h, model.c(), K, _lib.ptr(track), B, _lib.ptr(p),
                                         _lib.ptr(c), _lib.ptr(g), _lib.ptr(h),
                                         _lib.stream_handle()))
    return c, g, h


def unpack_sym(h):
    """(..., 15) packed upper triangle -> (..., 5, 5) symmetric."""
    iu = np.triu_indices(NPAR)
    out = torch.zeros(*h.shape[:-1], NPAR, NPAR, dtype=h.dtype, device=h.device)
    out[..., iu[0], iu[1]] = h
    out[..., iu[1], iu[0]] = h
    return out


def hessian(ctx, model, track, p, covariance=True):
    """Exact Hessian (B, 5, 5) of chi2 and the Fisher covariance (B, 5, 5) in dex^2."""
    K, B = _track(track), p.shape[0]
    _dev(p, (B, NPAR), "p")
    H = torch.empty(B, NPAR, NPAR, dtype=torch.float64, device=p.device)
    C = torch.empty_like(H) if covariance else None
    _lib.check(_lib.lib().dnb_track_hessian(ctx._h, model.c(), K, _lib.ptr(track), B, _lib.ptr(p),
                                            _lib.ptr(H), _lib.ptr(C), _lib.stream_handle()))
    return H, C


def lm(ctx, model, track, p0, n_iter=60, lambda0=1e-3):
    """Levenberg-Marquardt from every start p0 (B, 5): (fits (B, 5), chi2 (B,))."""
    K, B = _track(track), p0.shape[0]
    _dev(p0, (B, NPAR), "p0")
    p = p0.clone()
    c = torch.empty(B, dtype=torch.float64, device=p0.device)
    _lib.check(_lib.lib().dnb_track_lm(ctx._h, model.c(), K, _lib.ptr(track), B, _lib.ptr(p),
                                       int(n_iter), float(lambda0), _lib.ptr(c),
                                       _lib.stream_handle()))
    return p, c


def fit(ctx, model, track, p_true, n_starts=1000, n_iter=60, seed=0, lambda0=1e-3):
    """The paper's recipe: starts drawn log-uniformly in [theta/2, 2 theta] around
    p_true, Levenberg-Marquardt from each, the lowest chi2 kept, and the Fisher
    covariance there.  Returns (best p, its chi2, covariance, all fits, all chi2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = np.log10(START_FACTOR)
    starts = np.asarray(p_true, float)[None, :] + rng.uniform(-half, half, (n_starts, NPAR))
    p0 = torch.tensor(starts, dtype=torch.float64, device=track.device)
    fits, c = lm(ctx, model, track, p0, n_iter, lambda0)
    k = int(torch.argmin(torch.nan_to_num(c, nan=float("inf"))).item())
    best = fits[k:k + 1].contiguous()
    _, C = hessian(ctx, model, track, best)
    return best[0], c[k], C[0], fits, c
