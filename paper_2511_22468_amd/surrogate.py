"""Learned surrogate of the stream experiment (bindings of include/dnb_surrogate.h).

The paper names coupling the differentiable N-body code with a neural network
as future work (Sec. 3).  Here a 4 -> 256 -> 256 -> 256 -> 2048 GELU network
maps the four inference parameters of Sec. 2.2.1 to the density image of the
final stream; it is trained on runs of the engine itself and used to
warm-start the N-body gradient fit.  Every product, activation, loss and
optimiser step runs in the library's kernels (BF16 MFMA with FP32
accumulation); torch only allocates.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from .pipeline import run_ensemble
from .units import gyr

PRIOR = ((1.0, 4.0), (1.0e4, 1.0e5), (5.0e11, 2.0e12), (3.0e10, 1.0e11))
NPIX = 2048


def normalise(theta_gyr):
    """(M, 4) array of (t_end [Gyr], M_Plummer, M_NFW, M_MN) -> inputs in [-1, 1]."""
    th = np.atleast_2d(np.asarray(theta_gyr, float))
    u = np.empty_like(th)
    u[:, 0] = (th[:, 0] - 2.5) / 1.5
    for k in range(1, 4):
        lo, hi = np.log10(PRIOR[k][0]), np.log10(PRIOR[k][1])
        u[:, k] = 2.0 * (np.log10(th[:, k]) - lo) / (hi - lo) - 1.0
    return u


def denormalise(u):
    u = np.atleast_2d(np.asarray(u, float))
    th = np.empty_like(u)
    th[:, 0] = 2.5 + 1.5 * u[:, 0]
    for k in range(1, 4):
        lo, hi = np.log10(PRIOR[k][0]), np.log10(PRIOR[k][1])
        th[:, k] = 10.0 ** (lo + (u[:, k] + 1.0) * 0.5 * (hi - lo))
    return th


def orbit_frame(w_x, w_v):
    """(e1, e2, n) of the orbit-aligned frame at the present-day point, as 9 doubles."""
    x = np.asarray(w_x, float)
    v = np.asarray(w_v, float)
    n = np.cross(x, v)
    n /= np.linalg.norm(n)
    e1 = x / np.linalg.norm(x)
    e2 = np.cross(n, e1)
    return np.concatenate([e1, e2, n])


def density_grid(pos, frame9, workspace=None):
    """(32, 64) FP32 density image of positions pos (3, n) (see dnb_density_grid)."""
    n = pos.shape[1]
    grid = torch.empty(32, 64, dtype=torch.float32, device=pos.device)
    if workspace is None:
        workspace = torch.empty(int(_lib.lib().dnb_grid_workspace_bytes()), dtype=torch.uint8,
                                device=pos.device)
    f = (ctypes.c_double * 9)(*[float(v) for v in frame9])
    _lib.check(_lib.lib().dnb_density_grid(n, _lib.ptr(pos), f, _lib.ptr(grid),
                                           _lib.ptr(workspace), _lib.stream_handle()))
    return grid


class MLP:
    """FP32 master parameters, their BF16 copy, Adam moments and per-batch workspaces."""

    def __init__(self, flat_params, device):
        self.device = device
        self.P = int(_lib.lib().dnb_mlp_param_count())
        assert flat_params.shape == (self.P,)
        self.p = torch.tensor(flat_params, dtype=torch.float32, device=device)
        self.pb = torch.empty(self.P, dtype=torch.int16, device=device)
        self.m = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.v = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.grads = torch.empty(self.P, dtype=torch.float32, device=device)
        self.t = 0
        self._ws = {}
        _lib.check(_lib.lib().dnb_mlp_to_bf16(self.P, _lib.ptr(self.p), _lib.ptr(self.pb),
                                              _lib.stream_handle()))

    def ws(self, B):
        if B not in self._ws:
            nb = int(_lib.lib().dnb_mlp_workspace_bytes(B))
            self._ws[B] = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._ws[B]

    def forward(self, x):
        B = x.shape[0]
        y = torch.empty(B, NPIX, dtype=torch.float32, device=self.device)
        _lib.check(_lib.lib().dnb_mlp_forward(_lib.ptr(self.p), _lib.ptr(self.pb), B,
                                              _lib.ptr(x), _lib.ptr(y), _lib.ptr(self.ws(B)),
                                              _lib.stream_handle()))
        return y

    def backward(self, dy, want_dx=False, want_grads=True):
        """After forward(x) on the same batch size: fills self.grads (unless
        want_grads is False); returns dx or None."""
        B = dy.shape[0]
        dx = torch.empty(B, 4, dtype=torch.float32, device=self.device) if want_dx else None
        grads = self.grads if want_grads else None
        _lib.check(_lib.lib().dnb_mlp_backward(_lib.ptr(self.pb), B, _lib.ptr(dy),
                                               _lib.ptr(self.ws(B)), _lib.ptr(grads),
                                               _lib.ptr(dx), _lib.stream_handle()))
        return dx

    @staticmethod
    def mse(y, t):
        loss = torch.empty(1, dtype=torch.float64, device=y.device)
        dy = torch.empty_like(y)
        _lib.check(_lib.lib().dnb_mlp_mse(y.numel(), _lib.ptr(y), _lib.ptr(t), _lib.ptr(loss),
                                          _lib.ptr(dy), _lib.stream_handle()))
        return loss, dy

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _lib.check(_lib.lib().dnb_mlp_adam(self.P, _lib.ptr(self.p), _lib.ptr(self.pb),
                                           _lib.ptr(self.m), _lib.ptr(self.v),
                                           _lib.ptr(self.grads), lr, b1, b2, eps, self.t,
                                           _lib.stream_handle()))

    def train(self, X, Y, epochs, batch, lr, seed=0, lr_final=None):
        """Minibatch Adam on (X (M, 4), Y (M, 2048)) FP32 device tensors; returns epoch losses."""
        rng = np.random.Generator(np.random.PCG64(seed))
        M = X.shape[0]
        nb = M // batch
        losses = []
        for ep in range(epochs):
            lr_ep = lr if lr_final is None else lr * (lr_final / lr) ** (ep / max(1, epochs - 1))
            perm = torch.tensor(rng.permutation(M), device=self.device)
            tot = torch.zeros((), dtype=torch.float64, device=self.device)
            for b in range(nb):
                idx = perm[b * batch:(b + 1) * batch]
                xb, yb = X[idx].contiguous(), Y[idx].contiguous()
                y = self.forward(xb)
                loss, dy = self.mse(y, yb)
                self.backward(dy)
                self.adam(lr_ep)
                tot += loss[0]
            losses.append(float(tot.item()) / nb)
        return losses

    def invert(self, target, n_starts=64, iters=300, lr=0.05, seed=0):
        """Minimise mean((MLP(u) - target)^2) over u in [-1, 1]^4 from n_starts seeded
        starts by Adam on u (gradients through the network).  Returns (best u, its loss)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        B = ((n_starts + 15) // 16) * 16
        u = torch.tensor(rng.uniform(-0.9, 0.9, size=(B, 4)), dtype=torch.float32,
                         device=self.device)
        tgt = target.reshape(NPIX).contiguous()
        ws = torch.empty(int(_lib.lib().dnb_mlp_invert_workspace_bytes(B)), dtype=torch.uint8,
                         device=self.device)
        _lib.check(_lib.lib().dnb_mlp_invert(_lib.ptr(self.p), _lib.ptr(self.pb), B,
                                             _lib.ptr(tgt), _lib.ptr(u), int(iters), float(lr),
                                             _lib.ptr(ws), _lib.stream_handle()))
        tgt = tgt.reshape(1, NPIX).expand(B, NPIX)
        y = self.forward(u)
        err = ((y - tgt) ** 2).mean(dim=1)
        k = int(torch.argmin(err[:n_starts]).item())
        return u[k].detach().cpu().numpy().astype(np.float64), float(err[k].item())


def generate_dataset(engine_ctx, thetas_gyr, xi, zeta, n_steps, pot, frame9,
                     w_now=(12.0, 0.0, 0.0, 0.0, -180.0, 60.0), a_p=0.01):
    """Density images of pipeline runs (back-integration, Plummer placement,
    n_steps forward steps) at each parameter row; returns (X, Y) FP32 device tensors.
    The runs are advanced as batched ensembles, as many members per launch as
    the context holds (pair terms in FP32C)."""
    dev = xi.device
    th = np.array(thetas_gyr, float).reshape(-1, 4)
    th_int = th.copy()
    th_int[:, 0] = [gyr(t) for t in th[:, 0]]
    Y = torch.empty(th.shape[0], NPIX, dtype=torch.float32, device=dev)
    ws = torch.empty(int(_lib.lib().dnb_grid_workspace_bytes()), dtype=torch.uint8, device=dev)
    for s, pos in run_ensemble(engine_ctx, th_int, xi, zeta, n_steps, pot, a_p, w_now):
        for b in range(pos.shape[0]):
            Y[s + b] = density_grid(pos[b], frame9, ws).reshape(NPIX)
    X = torch.tensor(normalise(th), dtype=torch.float32, device=dev)
    return X, Y
