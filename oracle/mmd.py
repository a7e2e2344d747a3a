"""Maximum mean discrepancy of the oracle (test infrastructure only).

Sec. 2.2.1 compares the simulated and observed streams, as point clouds, with
the maximum mean discrepancy and differentiates it.  The paper does not state
the kernel or the estimator.  The reading taken: Gaussian kernel
k(x, y) = exp(-|x - y|^2 / (2 h^2)) on 3-D positions, bandwidth h, and the
biased (V-statistic) estimate of the squared MMD,

    L = 1/n^2 sum_ij k(x_i, x_j) + 1/m^2 sum_ab k(y_a, y_b)
        - 2/(n m) sum_ia k(x_i, y_a),

whose gradient is

    dL/dx_i = -2/(n^2 h^2) sum_j k_ij (x_i - x_j)
              + 2/(n m h^2) sum_a k_ia (x_i - y_a).
"""
import numpy as np


def _kernel_sum(X, Y, h, block=512):
    tot = np.zeros((), dtype=np.result_type(X, Y, float))
    for b0 in range(0, X.shape[0], block):
        d = X[b0:b0 + block, None, :] - Y[None, :, :]
        r2 = d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2
        tot = tot + np.sum(np.exp(-r2 / (2.0 * h * h)))
    return tot


def mmd2(X, Y, h):
    X = np.asarray(X)
    Y = np.asarray(Y)
    n, m = X.shape[0], Y.shape[0]
    return (_kernel_sum(X, X, h) / (n * n) + _kernel_sum(Y, Y, h) / (m * m)
            - 2.0 * _kernel_sum(X, Y, h) / (n * m))


def mmd2_grad(X, Y, h, block=512):
    """dL/dX, shape (n, 3)."""
    X = np.asarray(X)
    Y = np.asarray(Y)
    n, m = X.shape[0], Y.shape[0]
    g = np.zeros(X.shape, dtype=np.result_type(X, Y, float))
    for b0 in range(0, n, block):
        xb = X[b0:b0 + block]
        d = xb[:, None, :] - X[None, :, :]
        k = np.exp(-(d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2) / (2.0 * h * h))
        g[b0:b0 + block] -= 2.0 / (n * n * h * h) * np.einsum("ij,ijk->ik", k, d)
        d = xb[:, None, :] - Y[None, :, :]
        k = np.exp(-(d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2) / (2.0 * h * h))
        g[b0:b0 + block] += 2.0 / (n * m * h * h) * np.einsum("ij,ijk->ik", k, d)
    return g
