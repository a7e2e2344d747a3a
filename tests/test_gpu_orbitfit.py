"""Orbit fit (include/dnb_orbitfit.h) against the oracle (run on an MI355X).

The model observables, chi2 with its Jacobian products, the exact Hessian, the
Fisher covariance and Levenberg-Marquardt are compared with the FP64 oracle
(complex-step Jacobian, differences of complex-step gradients for the
Hessian, the same Levenberg-Marquardt recipe) on a 16-point noise-free mock
track spanning both branches.
"""
import numpy as np
import pytest
import torch

from oracle import constants as C, orbitfit as oof

from gpu_util import say

pytestmark = pytest.mark.gpu

W_NOW = np.array([12.0, 0.0, 0.0, 0.0, -180.0, 60.0])
P_TRUE = np.log10([1.0e12, 16.0, 6.5e10, 3.0, 0.28])
SIGMA = (2e-3, 0.05, 1.0)
DT_TOTAL = C.gyr(0.5)
N_STEPS = 250
OARGS = lambda tr: (tr, SIGMA, W_NOW, C.G, DT_TOTAL, N_STEPS)


@pytest.fixture(scope="module")
def fx():
    from paper_2511_22468_amd import engine, orbitfit as gof
    ctx = engine.Context(1024, "fp64")
    model = gof.TrackModel(w_now=tuple(W_NOW), dt_total=DT_TOTAL, n_steps=N_STEPS, sigma=SIGMA,
                           G=C.G)
    phi1 = np.linspace(-0.9, 0.5, 16)
    Y, _ = oof.model_track(P_TRUE, W_NOW, C.G, DT_TOTAL, N_STEPS, phi1)
    track = np.column_stack([phi1, Y])
    yield gof, ctx, model, track, torch.tensor(track, device="cuda")
    ctx.close()


def dev(a):
    return torch.tensor(np.asarray(a, float), device="cuda")


def test_observables_match_oracle(fx):
    gof, ctx, model, track, trk = fx
    say("[orbitfit] observe")
    p = P_TRUE + np.array([0.05, -0.03, 0.02, 0.04, -0.05])
    phi1 = np.array([-1.3, -0.4, -0.01, 0.0, 0.2, 0.9, 2.5, 1e3])
    Y, seg = oof.model_track(p, W_NOW, C.G, DT_TOTAL, N_STEPS, phi1)
    y = gof.observe(ctx, model, dev(phi1), dev(p)).cpu().numpy()
    assert seg[-1][1] == -1 and np.all(np.isinf(y[-1]))
    np.testing.assert_allclose(y[:-1], Y[:-1], rtol=1e-11, atol=1e-13)


def test_chi2_and_jacobian_products_match_oracle(fx):
    gof, ctx, model, track, trk = fx
    say("[orbitfit] chi2")
    rng = np.random.default_rng(4)
    P = P_TRUE[None, :] + rng.uniform(-0.1, 0.1, (6, 5))
    P[0] = P_TRUE
    c, g, h = gof.chi2(ctx, model, trk, dev(P))
    c, g, H = c.cpu().numpy(), g.cpu().numpy(), gof.unpack_sym(h).cpu().numpy()
    assert c[0] < 1e-20
    for b in range(1, 6):
        r, J = oof.jacobian(P[b], *OARGS(track))
        np.testing.assert_allclose(c[b], r @ r, rtol=1e-10)
        np.testing.assert_allclose(g[b], J.T @ r, rtol=1e-8, atol=1e-9 * np.abs(J.T @ r).max())
        JtJ = J.T @ J
        np.testing.assert_allclose(H[b], JtJ, rtol=1e-8, atol=1e-9 * np.abs(JtJ).max())


def test_exact_hessian_and_fisher_covariance(fx):
    gof, ctx, model, track, trk = fx
    say("[orbitfit] hessian")
    p_off = P_TRUE + np.array([0.02, 0.01, -0.02, 0.01, 0.02])
    H, Cov = gof.hessian(ctx, model, trk, dev(np.stack([P_TRUE, p_off])))
    H, Cov = H.cpu().numpy(), Cov.cpu().numpy()
    for b, p in enumerate((P_TRUE, p_off)):
        ref = oof.hessian(p, *OARGS(track))
        assert np.abs(H[b] - ref).max() <= 1e-6 * np.abs(ref).max(), b
        np.testing.assert_allclose(H[b], H[b].T, rtol=0, atol=0)
    # at zero residual the Hessian is exactly twice J^T J
    _, J = oof.jacobian(P_TRUE, *OARGS(track))
    assert np.abs(H[0] - 2 * J.T @ J).max() <= 1e-8 * np.abs(H[0]).max()
    F, Cref = oof.fisher(H[0])
    np.testing.assert_allclose(Cov[0] @ F, np.eye(5), atol=1e-8)
    np.testing.assert_allclose(Cov[0], Cref, rtol=1e-8, atol=1e-12 * np.abs(Cref).max())


def test_levenberg_marquardt_matches_oracle_iterates(fx):
    gof, ctx, model, track, trk = fx
    say("[orbitfit] lm")
    rng = np.random.default_rng(100)
    P0 = P_TRUE[None, :] + rng.uniform(-0.12, 0.12, (3, 5))
    for n_iter in (6, 60):
        p, c = gof.lm(ctx, model, trk, dev(P0), n_iter=n_iter)
        p, c = p.cpu().numpy(), c.cpu().numpy()
        for b in range(3):
            pr, cr = oof.levenberg_marquardt(P0[b], *OARGS(track), n_iter=n_iter)
            np.testing.assert_allclose(p[b], pr, rtol=0, atol=1e-8)
            if n_iter == 60:
                assert c[b] < 1e-18
                np.testing.assert_allclose(p[b], P_TRUE, rtol=0, atol=1e-9)


def test_fit_from_many_starts_recovers_truth(fx):
    gof, ctx, model, track, trk = fx
    say("[orbitfit] fit 512 starts")
    best, c, Cov, fits, cs = gof.fit(ctx, model, trk, P_TRUE, n_starts=512, n_iter=60, seed=3)
    np.testing.assert_allclose(best.cpu().numpy(), P_TRUE, rtol=0, atol=1e-8)
    assert c.item() < 1e-16
    assert torch.isfinite(Cov).all()
    assert (torch.diagonal(Cov) > 0).all()


def test_argument_checks(fx):
    gof, ctx, model, track, trk = fx
    from paper_2511_22468_amd._lib import DnbError
    p = dev(P_TRUE[None])
    with pytest.raises(DnbError, match="K = 65"):
        gof.chi2(ctx, model, torch.zeros(65, 4, dtype=torch.float64, device="cuda"), p)
    bad = gof.TrackModel(w_now=tuple(W_NOW), sigma=(0.0, 1.0, 1.0))
    with pytest.raises(DnbError, match="sigma"):
        gof.chi2(ctx, bad, trk, p)
    radial = gof.TrackModel(w_now=(12.0, 0, 0, 5.0, 0, 0))
    with pytest.raises(DnbError, match="angular momentum"):
        gof.chi2(ctx, radial, trk, p)


def test_single_point_and_unreachable_tracks(fx):
    gof, ctx, model, track, trk = fx
    # one track point: chi2 and the exact Hessian still match the oracle
    one = track[5:6]
    p = P_TRUE + np.array([0.02, -0.01, 0.01, 0.0, 0.01])
    c, g, h = gof.chi2(ctx, model, dev(one), dev(p[None]))
    r, J = oof.jacobian(p, *OARGS(one))
    np.testing.assert_allclose(c.item(), r @ r, rtol=1e-10)
    np.testing.assert_allclose(g[0].cpu().numpy(), J.T @ r, rtol=1e-8,
                               atol=1e-9 * np.abs(J.T @ r).max())
    # a point the orbit never reaches: chi2 is infinite, the start stays put, the
    # Hessian is NaN
    far = np.vstack([track[:3], [[50.0, 0.0, 12.0, 0.0]]])
    P0 = dev(np.stack([P_TRUE, p]))
    c, _, _ = gof.chi2(ctx, model, dev(far), P0)
    assert torch.isinf(c).all()
    fits, cf = gof.lm(ctx, model, dev(far), P0, n_iter=5)
    assert torch.equal(fits, P0) and torch.isinf(cf).all()
    H, C = gof.hessian(ctx, model, dev(far), P0)
    assert torch.isnan(H).all() and torch.isnan(C).all()
