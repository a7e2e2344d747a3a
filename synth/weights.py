"""Seeded initial weights of the surrogate network.

Weights are drawn from N(0, 2 / fan_in) (the last, linear layer from
N(0, 1 / fan_in)); biases start at zero.  Returned as a list of (W [in][out],
b [out]) float32 arrays, the order and layout of the library's parameter vector.
"""
import numpy as np

LAYERS = (4, 256, 256, 256, 2048)


def mlp_init(seed, layers=LAYERS):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for li, (a, b) in enumerate(zip(layers[:-1], layers[1:])):
        gain = 2.0 if li < len(layers) - 2 else 1.0
        W = rng.normal(scale=np.sqrt(gain / a), size=(a, b)).astype(np.float32)
        out.append((W, np.zeros(b, dtype=np.float32)))
    return out


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unflatten(flat, layers=LAYERS):
    out, o = [], 0
    for a, b in zip(layers[:-1], layers[1:]):
        W = flat[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((W, flat[o:o + b]))
        o += b
    return out
