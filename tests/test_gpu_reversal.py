"""The reverse sweep that rebuilds the trajectory by stepping it backward
(dnb_simulate_vjp_reversed; the kick-drift-kick step is time-reversible,
Sec. 2.2.1) against the oracle's exact discrete adjoint and against the sweep
that recomputes the trajectory forward.

* FP64 with a checkpoint at every step: nothing is rebuilt and the fused pair
  launch sums the same terms in the same order as the forward kernel, so the
  gradient equals dnb_simulate_vjp's bit for bit.
* Rebuilt segments (checkpoints every K > 1 steps, T a multiple of K or not,
  K beyond T): the rebuilt positions carry the rounding of at most K backward
  steps; against the oracle the bounds are those of the recomputing sweep
  (FP64 1e-10 on the raw adjoint and 1e-8 on the pipeline gradient, FP32C
  1e-3), each component on its own scale.
* The call is refused (DNB_ERR_STATE) when vel_T is not the velocity array the
  tape's forward run moved.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import adjoint as oadj, integrate as oint
from oracle import pipeline as opipe
from oracle.forces import Potential as OPot
from synth import plummer_unit

from gpu_util import rel_norm, say, to_dev, to_host

pytestmark = pytest.mark.gpu

G = 4.3009e-6
W_X = np.array([12.0, 0.0, 0.0])
W_V = np.array([0.0, -180.0, 60.0])


@pytest.fixture(scope="module")
def dnb():
    import paper_2511_22468_amd as pk
    from paper_2511_22468_amd import engine
    ctx = {p: engine.Context(9000, p) for p in ("fp64", "fp32c")}
    yield pk, engine, ctx
    for c in ctx.values():
        c.close()


def plummer_state(n, seed, m_tot=2e4, a_p=0.01):
    xi, zeta = plummer_unit(n, seed)
    return W_X + a_p * xi, W_V + np.sqrt(G * m_tot / a_p) * zeta, np.full(n, m_tot / n)


def gpu_pot(engine, op):
    return engine.Potential(G=op.G, eps=op.eps, m_nfw=op.m_nfw, rs_nfw=op.rs_nfw, m_mn=op.m_mn,
                            a_mn=op.a_mn, b_mn=op.b_mn)


def test_fp64_with_every_step_stored_equals_the_recomputing_sweep(dnb):
    pk, engine, ctx = dnb
    say("[reversal] n=600 T=13 K=1 fp64: bitwise against dnb_simulate_vjp")
    x, v, m = plummer_state(600, 9)
    m = m * np.random.default_rng(4).uniform(0.5, 1.5, m.shape)
    rng = np.random.default_rng(10)
    wx, wv = to_dev(rng.normal(size=x.shape)), to_dev(rng.normal(size=x.shape))
    op = OPot()
    pot = gpu_pot(engine, op)
    c = ctx["fp64"]
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    dt = pk.myr(0.5)
    tape = c.simulate(px, pv, pm, pot, dt, 13, ckpt_every=1)
    a = c.simulate_vjp(pm, pot, dt, 13, 1, tape, px, wx, wv, with_mass=True)
    b = c.simulate_vjp(pm, pot, dt, 13, 1, tape, px, wx, wv, with_mass=True, vel_T=pv)
    for name, s, r in zip(("gpos_0", "gvel_0", "gmass", "gparams"), a, b):
        assert torch.equal(s, r), (name, (s - r).abs().max().item())


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("K", [4, 10, 15])
@pytest.mark.parametrize("masses", ["equal", "unequal"])
def test_reversed_adjoint_matches_oracle(dnb, prec, K, masses):
    pk, engine, ctx = dnb
    n, T = 40, 10
    say(f"[reversal] n={n} T={T} K={K} prec={prec} masses={masses}")
    x, v, m = plummer_state(n, 7)
    if masses == "unequal":
        m = m * np.random.default_rng(9).uniform(0.5, 1.5, m.shape)
    rng = np.random.default_rng(8)
    wx, wv = rng.normal(size=x.shape), rng.normal(size=x.shape)
    op = OPot()
    dt = pk.myr(1.0)
    _, _, traj = oint.simulate(x, v, m, op, dt, T, keep=True)
    ref = oadj.simulate_vjp(traj, m, op, dt, wx, wv)
    c = ctx[prec]
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    pot = gpu_pot(engine, op)
    tape = c.simulate(px, pv, pm, pot, dt, T, ckpt_every=K)
    gx0, gv0, gm, gp = c.simulate_vjp(pm, pot, dt, T, K, tape, px, to_dev(wx), to_dev(wv),
                                      with_mass=True, vel_T=pv)
    gp = gp.cpu().numpy()
    tol = 1e-10 if prec == "fp64" else 1e-3
    errs = {"x0": rel_norm(to_host(gx0), ref["x0"]), "v0": rel_norm(to_host(gv0), ref["v0"]),
            "mass": rel_norm(to_host(gm), ref["mass"])}
    refp = [ref["m_nfw"], ref["m_mn"], ref["dt"], np.sum(m * ref["mass"]), ref["rs_nfw"],
            ref["a_mn"], ref["b_mn"]]
    for k, r in enumerate(refp):
        errs[f"p{k}"] = abs(gp[k] / r - 1)
    say(f"  largest relative error {max(errs.values()):.2e} ({max(errs, key=errs.get)})")
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, bad


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("n,T,K", [(1, 5, 2), (2, 7, 3), (300, 1, 5), (257, 9, 4)])
def test_reversed_adjoint_edge_cases(dnb, prec, n, T, K):
    """A single particle (no pair force), two particles, one step (nothing
    rebuilt, the final state only), a ragged particle count; zero softening (the
    self term masked in the fused launch as in the forward one).  The ragged
    FP32C case keeps eps = 1e-3: without softening the closest pairs of its 257
    particles carry FP32 rounding that the unsoftened dynamics grow to about
    9e-3 of the gradient over the 9 steps in every FP32C sweep alike (measured:
    full tape 9.17e-3, recomputed segments 9.17e-3, stepped backward 9.26e-3
    against the oracle), which is the precision's limit there, not the sweep's."""
    pk, engine, ctx = dnb
    eps = 1e-3 if (prec == "fp32c" and n > 2 and T > 1) else 0.0
    say(f"[reversal] edge n={n} T={T} K={K} prec={prec} eps={eps}")
    x, v, m = plummer_state(max(n, 2), 11)
    x, v, m = x[:n], v[:n], m[:n] * (1.0 + 0.3 * np.arange(n) / max(n, 1))
    rng = np.random.default_rng(12)
    wx, wv = rng.normal(size=x.shape), rng.normal(size=x.shape)
    op = OPot(eps=eps)
    dt = pk.myr(1.0)
    _, _, traj = oint.simulate(x, v, m, op, dt, T, keep=True)
    ref = oadj.simulate_vjp(traj, m, op, dt, wx, wv)
    c = ctx[prec]
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    pot = gpu_pot(engine, op)
    tape = c.simulate(px, pv, pm, pot, dt, T, ckpt_every=K)
    gx0, gv0, gm, gp = c.simulate_vjp(pm, pot, dt, T, K, tape, px, to_dev(wx), to_dev(wv),
                                      with_mass=True, vel_T=pv)
    tol = 1e-10 if prec == "fp64" else 1e-3
    errs = [rel_norm(to_host(gx0), ref["x0"]), rel_norm(to_host(gv0), ref["v0"]),
            abs(gp[2].item() / ref["dt"] - 1)]
    if n > 1:
        errs.append(rel_norm(to_host(gm), ref["mass"]))
    say(f"  largest relative error {max(errs):.2e}")
    assert max(errs) <= tol, errs


@pytest.mark.parametrize("prec,K", [("fp64", 10), ("fp64", 30), ("fp32c", 10), ("fp32c", 30)])
def test_reversed_pipeline_gradient_matches_oracle(dnb, prec, K):
    """Fig. 2 steps 2-4 end to end with the backward-stepping sweep: every
    component of dL/dtheta on its own scale against the oracle pipeline."""
    from paper_2511_22468_amd.pipeline import StreamModel
    pk, engine, ctx = dnb
    n, T = 300, 30
    say(f"[reversal] pipeline n={n} T={T} K={K} prec={prec}")
    xi, zeta = plummer_unit(n, 31)
    target = W_X + 0.05 * np.random.default_rng(32).normal(size=(128, 3))
    theta = np.array([pk.myr(30.0), 3e4, 1.1e12, 6.0e10])
    L_ref, g = opipe.loss_and_grad(theta, xi, zeta, OPot(), T, target, 0.2)
    g_ref = np.array([g["t_end"], g["m_prog"], g["m_nfw"], g["m_mn"]])
    model = StreamModel(ctx[prec], to_dev(xi), to_dev(zeta), to_dev(target), T,
                        pot=engine.Potential(), ckpt_every=K, reversal=True)
    L, gg = model.loss_and_grad(torch.tensor(theta, device="cuda"))
    tol = 1e-8 if prec == "fp64" else 1e-3
    g = gg.cpu().numpy()
    say(f"  loss rel err {abs(L.item() / L_ref - 1):.2e}, per-component gradient rel err "
        f"{np.abs(g / g_ref - 1)}")
    assert abs(L.item() / L_ref - 1) <= tol
    np.testing.assert_allclose(g, g_ref, rtol=tol)


@pytest.mark.parametrize("T", [20, 50])
def test_reversed_pipeline_gradient_n8192_against_oracle(T):
    """The differentiation workload at its full particle number (N = 8192,
    checkpoints every 10 steps) with the backward-stepping sweep, against the
    oracle's stored pipeline gradient: FP64 within 1e-8, FP32C within 1e-3,
    every component on its own scale."""
    import paper_2511_22468_amd as pk
    from paper_2511_22468_amd import engine
    from paper_2511_22468_amd.pipeline import StreamModel
    from test_gpu_configs import golden_gradients
    gold = golden_gradients()
    L_ref, g_ref = gold[(T, -1)]
    xi, zeta = plummer_unit(8192, 3)
    rng = np.random.Generator(np.random.PCG64(30))
    target = W_X + 0.02 * rng.normal(size=(4096, 3))
    theta = torch.tensor([T * 1.1 * pk.gyr(2.0) / 2000, 3e4 * 1.2, 1e12 * 0.9, 6.5e10 * 1.1],
                         dtype=torch.float64, device="cuda")
    for prec, tol in (("fp64", 1e-8), ("fp32c", 1e-3)):
        say(f"[reversal] N=8192 T={T} {prec}: pipeline gradient vs oracle")
        c = engine.Context(8192, prec)
        model = StreamModel(c, to_dev(xi), to_dev(zeta), to_dev(target), T,
                            pot=engine.Potential(eps=1e-3), h=0.2, ckpt_every=10,
                            reversal=True)
        L, g = model.loss_and_grad(theta)
        rel = np.abs(g.cpu().numpy() / g_ref - 1)
        say(f"  loss rel err {abs(L.item() / L_ref - 1):.2e}; per-component rel err {rel}")
        assert abs(L.item() / L_ref - 1) <= tol
        assert rel.max() <= tol
        c.close()


def test_reversed_sweep_refuses_another_velocity_array(dnb):
    pk, engine, ctx = dnb
    from paper_2511_22468_amd import _lib
    lib = _lib.lib()
    n, T, K = 300, 6, 3
    say(f"[reversal] refusal n={n} T={T} K={K}")
    x, v, m = plummer_state(n, 5)
    c = ctx["fp64"]
    pot = gpu_pot(engine, OPot())
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    dt = pk.myr(0.5)
    tape = c.simulate(px, pv, pm, pot, dt, T, ckpt_every=K)
    g = torch.ones(3, n, dtype=torch.float64, device="cuda")
    other = pv.clone()
    work = torch.zeros(int(lib.dnb_vjp_reversed_workspace_doubles(n)), dtype=torch.float64,
                       device="cuda")
    outs = [torch.zeros(3, n, dtype=torch.float64, device="cuda") for _ in range(2)]
    gpar = torch.zeros(7, dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    call = lambda vel: lib.dnb_simulate_vjp_reversed(
        c._h, n, P(pm), pot.c(), dt, T, K, P(tape), P(px), P(vel), P(g), None, P(work),
        P(outs[0]), P(outs[1]), None, P(gpar), None)
    assert call(other) == _lib.DNB_ERR_STATE
    assert b"vel_T" in lib.dnb_last_error()
    # the matching call goes through and gives the engine's result
    assert call(pv) == _lib.DNB_OK
    ref = c.simulate_vjp(pm, pot, dt, T, K, tape, px, g, vel_T=pv)
    assert torch.equal(outs[0], ref[0]) and torch.equal(outs[1], ref[1])
    # a run that moves the final velocities (here another system's step with
    # them) makes the backward-stepping sweep refuse the tape; the recomputing
    # sweep, which does not read them, still takes it
    qx = px.clone()
    c.step(qx, pv, pm, pot, dt)
    assert call(pv) == _lib.DNB_ERR_STATE
    assert b"vel_T" in lib.dnb_last_error()
    c.simulate_vjp(pm, pot, dt, T, K, tape, px, g)
