"""Pins of the oracle's density grid and MLP against independent library routes."""
import numpy as np
import torch
from scipy.ndimage import gaussian_filter1d

from oracle import surrogate as S

W_X, W_V = (12.0, 0.0, 0.0), (0.0, -180.0, 60.0)


def sky(phi1, phi2, r=10.0):
    e1, e2, n = S.frame(W_X, W_V)
    return r * (np.cos(phi2) * (np.cos(phi1) * e1 + np.sin(phi1) * e2) + np.sin(phi2) * n)


def test_frame_is_orthonormal_and_places_known_points():
    e1, e2, n = S.frame(W_X, W_V)
    M = np.stack([e1, e2, n])
    np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-15)
    # the present-day velocity lies in the (e1, e2) plane
    assert abs(np.dot(W_V, n)) < 1e-12
    rng = np.random.default_rng(0)
    p1 = rng.uniform(-np.pi, np.pi, 2000)
    p2 = rng.uniform(-0.1, 0.1, 2000)
    pos = np.stack([sky(a, b, rr) for a, b, rr in zip(p1, p2, rng.uniform(5, 30, 2000))])
    counts, _, _ = np.histogram2d(p2, p1, bins=[32, 64], range=[[-0.1, 0.1], [-np.pi, np.pi]])
    k = np.exp(-0.5 * np.arange(-3, 4) ** 2)
    # the oracle blurs and normalises; undo neither, compare to an independent blur
    ref = gaussian_filter1d(counts, 1.0, axis=1, mode="wrap", truncate=3.0)
    ref = gaussian_filter1d(ref, 1.0, axis=0, mode="constant", truncate=3.0)
    ref /= ref.sum()
    np.testing.assert_allclose(S.density_grid(pos, W_X, W_V), ref, atol=1e-15)
    assert abs(k.sum() - 2.5066) < 1e-3   # sanity of the sigma = 1 kernel


def test_grid_edge_cases():
    assert S.density_grid(np.array([[0.0, 0.0, 30.0]]) * 0 + sky(0.0, 0.5), W_X, W_V).sum() == 0
    g = S.density_grid(sky(-np.pi + 1e-9, 0.0)[None], W_X, W_V)
    assert g[:, 63].sum() > 0 and g[:, 0].sum() > g[:, 3].sum()   # wraps around in phi1


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, 5000), [0.0, -0.0, 1.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x), ref)


def test_gelu_matches_torch_and_its_derivative():
    z = np.linspace(-6, 6, 201)
    ref = torch.nn.functional.gelu(torch.tensor(z)).numpy()
    np.testing.assert_allclose(S.gelu(z), ref, rtol=1e-12, atol=1e-16)
    cs = np.imag(S.gelu(z + 1e-30j)) / 1e-30
    np.testing.assert_allclose(S.gelu_grad(z), cs, rtol=1e-13, atol=1e-16)


def _params(seed, layers=(4, 16, 16, 16, 32)):
    rng = np.random.default_rng(seed)
    return [(rng.normal(scale=1 / np.sqrt(a), size=(a, b)), rng.normal(scale=0.1, size=b))
            for a, b in zip(layers[:-1], layers[1:])]


def test_mlp_backward_matches_complex_step():
    P = _params(2)
    rng = np.random.default_rng(3)
    X, T = rng.normal(size=(5, 4)), rng.normal(size=(5, 32))

    def loss(Pc, Xc):
        Y, _ = S.forward(Pc, Xc, emulate_bf16=False)
        return np.sum((Y - T) ** 2) / Y.size

    Y, cache = S.forward(P, X, emulate_bf16=False)
    _, dY = S.mse(Y, T)
    grads, dX = S.backward(P, cache, dY, emulate_bf16=False)
    for li in range(4):
        D = rng.normal(size=P[li][0].shape)
        Pc = [(W.astype(complex), b.astype(complex)) for W, b in P]
        Pc[li] = (Pc[li][0] + 1e-30j * D, Pc[li][1])
        np.testing.assert_allclose(np.sum(grads[li][0] * D), np.imag(loss(Pc, X)) / 1e-30, rtol=1e-10)
        db = rng.normal(size=P[li][1].shape)
        Pc = [(W.astype(complex), b.astype(complex)) for W, b in P]
        Pc[li] = (Pc[li][0], Pc[li][1] + 1e-30j * db)
        np.testing.assert_allclose(np.sum(grads[li][1] * db), np.imag(loss(Pc, X)) / 1e-30, rtol=1e-10)
    DX = rng.normal(size=X.shape)
    np.testing.assert_allclose(np.sum(dX * DX), np.imag(loss(P, X + 1e-30j * DX)) / 1e-30, rtol=1e-10)


def test_adam_matches_torch():
    P = _params(4, (4, 8, 3))
    rng = np.random.default_rng(5)
    tp = [torch.tensor(a, requires_grad=True) for W, b in P for a in (W, b)]
    opt = torch.optim.Adam(tp, lr=1e-2)
    state = [tuple(np.zeros_like(a) for a in (W, W, b, b)) for W, b in P]
    for t in range(1, 4):
        grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in P]
        P = S.adam(P, grads, state, 1e-2, t)
        for p, g in zip(tp, [g for gg in grads for g in gg]):
            p.grad = torch.tensor(g)
        opt.step()
    for a, p in zip([a for W, b in P for a in (W, b)], tp):
        np.testing.assert_allclose(a, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_theta_normalisation_maps_prior_box_to_unit_cube():
    lo = [1.0, 1e4, 5e11, 3e10]
    hi = [4.0, 1e5, 2e12, 1e11]
    np.testing.assert_allclose(S.normalise_theta(lo), [[-1, -1, -1, -1]], atol=1e-15)
    np.testing.assert_allclose(S.normalise_theta(hi), [[1, 1, 1, 1]], atol=1e-15)
