"""Density grid and MLP surrogate of the oracle (test infrastructure only).

The paper names coupling the N-body code with a neural network as future work
(Sec. 3); the surrogate here maps the four inference parameters of Sec. 2.2.1
to a smoothed density image of the final stream, and the plain N-body gradient
fit remains the test of it.  Nothing in this module is given by the paper;
the readings taken are:

Grid.  A fixed orbit-aligned frame built from the present-day phase-space
point w_now = (x, v): n = x cross v / |x cross v|, e1 = x / |x|, e2 = n cross e1.
phi1 = atan2(x.e2, x.e1) in 64 bins over [-pi, pi); phi2 = asin(x.n / |x|) in
32 bins over [-0.1, 0.1] rad; particles outside are dropped.  Integer counts
are blurred with a separable Gaussian of sigma = 1 bin (kernel radius 3,
weights exp(-k^2/2) normalised to sum 1), periodic in phi1 and zero-padded in
phi2, and the image is normalised to sum 1 (all zeros if empty).

MLP.  4 -> 256 -> 256 -> 256 -> 2048, exact-erf GELU after the first three
layers, linear output, mean squared error.  BF16 rounding (round to nearest
even) is applied where the GPU kernels round: the weights, and the left
operand of every matrix product (layer inputs in the forward pass, output
gradients in the backward pass); everything else is exact here (FP64).
Inputs are normalised: t_end [Gyr] -> (t - 2.5) / 1.5, and each log10 mass is
mapped linearly from its prior bounds onto [-1, 1].
"""
import math

import numpy as np
from scipy.special import erf

PRIOR = ((1.0, 4.0), (1.0e4, 1.0e5), (5.0e11, 2.0e12), (3.0e10, 1.0e11))
LAYERS = (4, 256, 256, 256, 2048)
NPHI1, NPHI2 = 64, 32
PHI2_MAX = 0.1


# ------------------------------------------------------------------- grid --

def frame(w_x, w_v):
    x = np.asarray(w_x, float)
    v = np.asarray(w_v, float)
    n = np.cross(x, v)
    n = n / np.sqrt(n @ n)
    e1 = x / np.sqrt(x @ x)
    e2 = np.cross(n, e1)
    return e1, e2, n


def density_grid(pos, w_x, w_v):
    """(32, 64) normalised, blurred histogram of final positions pos (N, 3)."""
    e1, e2, nh = frame(w_x, w_v)
    pos = np.asarray(pos, float)
    r = np.sqrt((pos * pos).sum(1))
    phi1 = np.arctan2(pos @ e2, pos @ e1)
    phi2 = np.arcsin(np.clip((pos @ nh) / r, -1.0, 1.0))
    i1 = np.floor((phi1 + np.pi) / (2 * np.pi) * NPHI1).astype(int)
    i2 = np.floor((phi2 + PHI2_MAX) / (2 * PHI2_MAX) * NPHI2).astype(int)
    ok = (i1 >= 0) & (i1 < NPHI1) & (i2 >= 0) & (i2 < NPHI2)
    counts = np.zeros((NPHI2, NPHI1))
    np.add.at(counts, (i2[ok], i1[ok]), 1.0)
    k = np.exp(-0.5 * np.arange(-3, 4) ** 2)
    k /= k.sum()
    out1 = np.zeros_like(counts)
    for d, wk in zip(range(-3, 4), k):            # periodic along phi1
        out1 += wk * np.roll(counts, d, axis=1)
    out = np.zeros_like(out1)
    for d, wk in zip(range(-3, 4), k):            # zero padding along phi2
        if d >= 0:
            out[d:, :] += wk * out1[:NPHI2 - d, :]
        else:
            out[:d, :] += wk * out1[-d:, :]
    s = out.sum()
    return out / s if s > 0 else out


# -------------------------------------------------------------------- MLP --

def normalise_theta(theta_gyr):
    """theta rows (t_end [Gyr], M_Plummer, M_NFW, M_MN) -> network inputs in ~[-1, 1]."""
    th = np.atleast_2d(np.asarray(theta_gyr, float))
    u = np.empty_like(th)
    u[:, 0] = (th[:, 0] - 2.5) / 1.5
    for k in range(1, 4):
        lo, hi = np.log10(PRIOR[k][0]), np.log10(PRIOR[k][1])
        u[:, k] = 2.0 * (np.log10(th[:, k]) - lo) / (hi - lo) - 1.0
    return u


def bf16(a):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def forward(params, X, emulate_bf16=True):
    """params: list of (W (in, out), b (out,)).  Returns (Y, cache)."""
    r = bf16 if emulate_bf16 else np.asarray
    h = np.asarray(X)
    cache = []
    for li, (W, b) in enumerate(params):
        a = r(h)
        z = a @ r(W) + b
        cache.append((a, z))
        h = gelu(z) if li < len(params) - 1 else z
    return h, cache


def mse(Y, T):
    d = np.asarray(Y, float) - np.asarray(T, float)
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dY, emulate_bf16=True):
    """Gradients of the loss whose output cotangent is dY.  Returns (grads, dX)."""
    r = bf16 if emulate_bf16 else np.asarray
    grads = [None] * len(params)
    g = np.asarray(dY, float)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        a, z = cache[li]
        if li < len(params) - 1:
            g = g * gelu_grad(z)
        gb = r(g)
        grads[li] = (a.T @ gb, g.sum(axis=0))
        g = gb @ r(W).T
    return grads, g


def adam(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on FP64 master parameters; state is a list of (m_W, v_W, m_b, v_b)."""
    new = []
    for (W, b), (gW, gb), st in zip(params, grads, state):
        out = []
        for k, (p, gp) in enumerate(((W, gW), (b, gb))):
            m, v = st[2 * k], st[2 * k + 1]
            m[...] = b1 * m + (1 - b1) * gp
            v[...] = b2 * v + (1 - b2) * gp * gp
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new
