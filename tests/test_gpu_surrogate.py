"""GPU parity of the surrogate kernels (BF16 MFMA MLP, MSE, Adam, density grid)
against the FP64 oracle with BF16 rounding emulated at the same points."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from synth import flatten, mlp_init, unflatten

from gpu_util import say

pytestmark = pytest.mark.gpu


def _mlp(seed=0):
    from paper_2511_22468_amd.surrogate import MLP
    params = mlp_init(seed)
    # non-zero biases so that the bias paths are exercised
    rng = np.random.default_rng(seed + 100)
    params = [(W, rng.normal(scale=0.1, size=b.shape).astype(np.float32)) for W, b in params]
    return params, MLP(flatten(params), torch.device("cuda"))


ULP = 2.0 ** -8   # one bfloat16 unit in the last place, relative (8-bit significand)


def _ratio(got, ref, allow):
    """Largest |got - ref| / allowance over the elements."""
    return float(np.max(np.abs(np.asarray(got, float) - ref) / allow))


@pytest.mark.parametrize("B", [16, 80])
def test_mlp_forward_backward_match_oracle(B):
    """Every element of the output, of each layer's dW and db and of dX against
    the oracle with BF16 rounding at the kernels' rounding points.  The
    allowance of an element is one BF16 unit on every operand its product sums
    (2^-8 sum |a| |w| for a product of a and w; for db, 2^-8 sum |g|): a BF16
    operand whose FP32 value lies at a rounding boundary may round the other way
    on the GPU, which accumulates in FP32 where the oracle is exact."""
    say(f"[mlp] forward/backward B={B}")
    params, net = _mlp(1)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(B, 4)).astype(np.float32)
    T = rng.normal(scale=0.01, size=(B, 2048)).astype(np.float32)
    P64 = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    Y_ref, cache = S.forward(P64, X.astype(np.float64))
    L_ref, dY_ref = S.mse(Y_ref, T)
    grads_ref, dX_ref = S.backward(P64, cache, dY_ref)

    x = torch.tensor(X, device="cuda")
    y = net.forward(x)
    loss, dy = net.mse(y, torch.tensor(T, device="cuda"))
    dx = net.backward(dy, want_dx=True)
    Y = y.cpu().numpy()
    Wb = [S.bf16(W) for W, _ in P64]
    a_last = cache[-1][0]
    r_y = _ratio(Y, Y_ref, ULP * (np.abs(a_last) @ np.abs(Wb[-1])) + 1e-30)
    assert abs(loss.item() / L_ref - 1) <= 5e-3
    # the backward signal of each layer as the oracle forms it (BF16-rounded)
    gs, g = [], np.asarray(dY_ref, float)
    for li in range(len(P64) - 1, -1, -1):
        if li < len(P64) - 1:
            g = g * S.gelu_grad(cache[li][1])
        gs.append(S.bf16(g))
        g = gs[-1] @ Wb[li].T
    gs = gs[::-1]
    gr = unflatten(net.grads.cpu().numpy())
    worst = {"y": r_y}
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(gr, grads_ref)):
        a = np.abs(cache[li][0])
        aw = ULP * (a.T @ np.abs(gs[li])) + 1e-30
        ab = ULP * np.abs(gs[li]).sum(0) + 1e-30
        worst[f"dW{li}"] = _ratio(gW, rW, aw)
        worst[f"db{li}"] = _ratio(gb, rb, ab)
    worst["dx"] = _ratio(dx.cpu().numpy(), dX_ref, ULP * (np.abs(gs[0]) @ np.abs(Wb[0]).T) + 1e-30)
    say("  largest |GPU - oracle| per element in units of its allowance: "
        + ", ".join(f"{k} {v:.3f}" for k, v in worst.items()))
    for k, v in worst.items():
        assert v <= 1.0, (k, v)


def test_adam_step_matches_oracle():
    params, net = _mlp(3)
    rng = np.random.default_rng(4)
    P64 = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    state = [tuple(np.zeros_like(a) for a in (W, W, b, b)) for W, b in P64]
    for t in range(1, 4):
        grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in P64]
        P64 = S.adam(P64, grads, state, 1e-3, t)
        net.grads.copy_(torch.tensor(flatten([(a.astype(np.float32), c.astype(np.float32))
                                              for a, c in grads])))
        net.adam(1e-3)
    got = net.p.cpu().numpy().astype(np.float64)
    ref = flatten([(W.astype(np.float32), b.astype(np.float32)) for W, b in P64]).astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-6
    # the BF16 copy is the rounded master
    pb = net.pb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(pb.view(np.float32).astype(np.float64), S.bf16(got))


def test_density_grid_matches_oracle():
    from paper_2511_22468_amd.surrogate import density_grid, orbit_frame
    rng = np.random.default_rng(5)
    e1, e2, n = S.frame((12.0, 0, 0), (0, -180.0, 60.0))
    phi1 = rng.uniform(-np.pi, np.pi, 6000)
    phi2 = rng.normal(scale=0.05, size=6000)
    r = rng.uniform(5, 30, 6000)
    pos = (r[:, None] * (np.cos(phi2)[:, None] * (np.cos(phi1)[:, None] * e1 + np.sin(phi1)[:, None] * e2)
                         + np.sin(phi2)[:, None] * n))
    ref = S.density_grid(pos, (12.0, 0, 0), (0, -180.0, 60.0))
    f9 = orbit_frame((12.0, 0, 0), (0, -180.0, 60.0))
    got = density_grid(torch.tensor(np.ascontiguousarray(pos.T), device="cuda"), f9).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-7 * max(1.0, ref.max()) + 1e-9
    # nothing inside: all zeros
    far = torch.tensor(np.ascontiguousarray(np.array([[0.0, 0.0, 10.0]]).T), device="cuda")
    assert float(density_grid(far, f9).abs().sum().item()) == 0.0


def test_training_reduces_loss():
    _, net = _mlp(6)
    rng = np.random.default_rng(7)
    X = torch.tensor(rng.uniform(-1, 1, size=(256, 4)), dtype=torch.float32, device="cuda")
    # smooth synthetic target images
    Y = torch.sin(X[:, :1] * 3 + torch.linspace(0, 6, 2048, device="cuda")[None]) * 0.01
    losses = net.train(X, Y.contiguous(), epochs=30, batch=64, lr=1e-3)
    say(f"[mlp] training loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.2 * losses[0]


def test_inversion_entry_equals_the_step_by_step_loop():
    """dnb_mlp_invert runs the same kernels in the same order as the loop of
    forward, mse, backward (input cotangent only), Adam on the inputs and the
    clamp to [-1, 1]: its inputs after 25 steps equal the loop's bit for bit, and
    the parameter gradients skipped by the backward leave dx unchanged."""
    from paper_2511_22468_amd import _lib
    from paper_2511_22468_amd.surrogate import NPIX
    _, net = _mlp(8)
    rng = np.random.default_rng(9)
    B, iters, lr = 32, 25, 0.05
    u0 = torch.tensor(rng.uniform(-0.9, 0.9, size=(B, 4)), dtype=torch.float32, device="cuda")
    target = torch.tensor(rng.normal(scale=0.01, size=NPIX), dtype=torch.float32, device="cuda")
    # the library loop
    u = u0.clone()
    ws = torch.empty(int(_lib.lib().dnb_mlp_invert_workspace_bytes(B)), dtype=torch.uint8,
                     device="cuda")
    _lib.check(_lib.lib().dnb_mlp_invert(_lib.ptr(net.p), _lib.ptr(net.pb), B, _lib.ptr(target),
                                         _lib.ptr(u), iters, lr, _lib.ptr(ws),
                                         _lib.stream_handle()))
    # the same steps through the single-call bindings
    v = u0.clone()
    tgt = target.reshape(1, NPIX).expand(B, NPIX).contiguous()
    vb = torch.empty(B * 4, dtype=torch.int16, device="cuda")
    mv = torch.zeros(B * 4, dtype=torch.float32, device="cuda")
    vv = torch.zeros(B * 4, dtype=torch.float32, device="cuda")
    for it in range(1, iters + 1):
        y = net.forward(v)
        _, dy = net.mse(y, tgt)
        dx = net.backward(dy, want_dx=True, want_grads=(it % 2 == 0))
        _lib.check(_lib.lib().dnb_mlp_adam(B * 4, _lib.ptr(v), _lib.ptr(vb), _lib.ptr(mv),
                                           _lib.ptr(vv), _lib.ptr(dx), lr, 0.9, 0.999, 1e-8,
                                           it, _lib.stream_handle()))
        v.clamp_(-1.0, 1.0)
    assert torch.equal(u, v)
    assert float((u - u0).abs().max().item()) > 0


def test_warm_start_gains_over_plain_descent():
    """What the trained network gains over the method without it: the quick
    time-to-fit configuration (fit N = 2048, 1000 steps; 64 training runs of
    N = 1024; the engine's own runs as training data).  Both arms descend until
    they converge (step length below 1/64 of its start, or 30 iterations).  The
    warm arm, the surrogate's inversion followed by the same descent, must reach
    the plain fit's final loss in less wall time than the plain fit takes, and
    end at a loss no worse than it."""
    from paper_2511_22468_amd import fit
    r = fit.run(quick=True, seed=50)
    p, w = r["plain"], r["warm"]
    say(f"[fit] plain {p['iterations']} iterations {p['seconds']:.2f} s to {p['final_loss']:.3e} "
        f"(converged {p['converged']}); warm {w['iterations']} iterations {w['seconds']:.2f} s "
        f"to {w['final_loss']:.3e} (converged {w['converged']}, inversion "
        f"{w['inversion_seconds']:.2f} s), plain fit loss reached after "
        f"{r['warm_seconds_to_plain_fit_loss']} s: {r['speedup_excl_training']}x excluding "
        f"training, {r['speedup_incl_training']}x including it")
    assert r["warm_seconds_to_plain_fit_loss"] is not None
    assert w["final_loss"] <= p["final_loss"]
    assert r["speedup_excl_training"] > 1.0


def test_one_surrogate_serves_several_targets():
    """The multi-target time-to-fit study at the quick configuration: a surrogate
    trained once per training set (the fit's 1000 steps and 250 steps over the
    same t_end) warm-starts two held-out targets.  Every arm is a deterministic
    function of its seeds, so the first target with the full-step training set
    repeats the single-target run bit for bit, and the summaries follow from the
    per-target rows by their stated formulas."""
    from paper_2511_22468_amd import fit
    say("[fit] study: quick, targets 50 and 60, training sets of 1000 and 250 steps")
    r = fit.study(seeds=(50, 60), quick=True)
    one = fit.run(quick=True, seed=50)
    t0 = r["targets"][0]
    assert [s["n_train_steps"] for s in r["surrogates"]] == [1000, 250]
    assert t0["plain"]["final_loss"] == one["plain_fit_loss"]
    assert t0["plain"]["iterations"] == one["plain"]["iterations"]
    assert t0["warm"][0]["final_loss"] == one["warm"]["final_loss"]
    assert t0["warm"][0]["iterations"] == one["warm"]["iterations"]
    for k, s in enumerate(r["surrogates"]):
        plain = sum(t["plain"]["seconds"] for t in r["targets"])
        warm, reached = 0.0, 0
        for t in r["targets"]:
            w = t["warm"][k]
            if w["seconds_to_plain_fit_loss"] is None:
                warm += w["seconds"] + t["plain"]["seconds"]
            else:
                assert w["seconds_to_plain_fit_loss"] <= w["seconds"]
                warm += w["seconds_to_plain_fit_loss"]
                reached += 1
        cost = s["data_seconds"] + s["train_seconds"]
        assert s["targets_reaching_plain_fit_loss"] == reached
        np.testing.assert_allclose(s["amortised_speedup_incl_training"], plain / (cost + warm),
                                   rtol=1e-12)
        say(f"[fit] {s['n_train_steps']}-step training set: data {s['data_seconds']:.2f} s, "
            f"training {s['train_seconds']:.2f} s, {reached}/2 targets reach the plain fit's "
            f"loss, amortised {s['amortised_speedup_incl_training']:.2f}x including training")
