"""Batched ensembles (dnb_simulate_batch, dnb_orbit_batch, dnb_mmd_batch and the
grid search built on them) against the oracle and against single-system runs
(run on an MI355X).

Every member of an ensemble is an independent system with its own potential,
softening and step size.  Members are checked against the FP64 oracle at the
FP32C tolerance of the single-system tests and, where the source slicing of the
ensemble equals that of a lone system (n = 300: ten 32-source slices in both
for up to 64 members), bitwise against dnb_simulate in FP32C.
"""
import numpy as np
import pytest
import torch

from oracle import integrate as oint
from oracle.forces import Potential as OPot
from synth import plummer_unit

from gpu_util import rel_rows, say, to_dev
from paper_2511_22468_amd._lib import DnbError

pytestmark = pytest.mark.gpu

G = 4.3009e-6
W_X = np.array([12.0, 0.0, 0.0])
W_V = np.array([0.0, -180.0, 60.0])


def member(n, seed, m_tot=2e4, a_p=0.01, unequal=False):
    xi, zeta = plummer_unit(n, seed)
    x = W_X + a_p * xi
    v = W_V + np.sqrt(G * m_tot / a_p) * zeta
    m = np.full(n, m_tot / n)
    if unequal:
        m = m * np.random.default_rng(seed).uniform(0.5, 1.5, n)
    return x, v, m


def member_pot(b):
    return OPot(eps=(0.5 + 0.25 * (b % 3)) * 1e-3, m_nfw=(0.9 + 0.05 * b) * 1e12,
                rs_nfw=14.0 + b, m_mn=(5.0 + 0.5 * b) * 1e10)


def gpu_pot(engine, op):
    return engine.Potential(G=op.G, eps=op.eps, m_nfw=op.m_nfw, rs_nfw=op.rs_nfw, m_mn=op.m_mn,
                            a_mn=op.a_mn, b_mn=op.b_mn)


def stack(states):
    xs = np.stack([np.ascontiguousarray(s[0].T) for s in states])
    vs = np.stack([np.ascontiguousarray(s[1].T) for s in states])
    ms = np.stack([s[2] for s in states])
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    return dev(xs), dev(vs), dev(ms)


@pytest.fixture(scope="module")
def eng():
    import paper_2511_22468_amd as pk
    from paper_2511_22468_amd import engine
    ctx = engine.Context(65536, "fp32c")
    yield pk, engine, ctx
    ctx.close()


def test_members_match_oracle_and_single_runs(eng):
    pk, engine, ctx = eng
    B, n, T = 5, 300, 40
    say(f"[batch] B={B} n={n} T={T}")
    states = [member(n, 40 + b, unequal=(b == 2)) for b in range(B)]
    ops = [member_pot(b) for b in range(B)]
    dts = [pk.myr(0.5) * (1.0 + 0.1 * b) * (-1 if b == 4 else 1) for b in range(B)]
    px, pv, pm = stack(states)
    ctx.simulate_batch(px, pv, pm, [gpu_pot(engine, o) for o in ops], dts, T)
    torch.cuda.synchronize()
    for b in range(B):
        x, v, m = states[b]
        sx, sv = to_dev(x), to_dev(v)
        ctx.simulate(sx, sv, to_dev(m), gpu_pot(engine, ops[b]), dts[b], T)
        assert torch.equal(sx, px[b]) and torch.equal(sv, pv[b]), f"member {b} not bitwise"
        # against FP64: FP32C pair terms (~1e-8 relative) amplified by the core's
        # chaos over 40 steps (members with eps = 5e-4 and 0.65 Myr steps reach
        # 7e-7); the bound of the workloads is 1e-4
        xr, vr = oint.simulate(x, v, m, ops[b], dts[b], T)
        gx, gv = px[b].cpu().numpy().T, pv[b].cpu().numpy().T
        assert rel_rows(gx, xr).max() <= 1e-5, b
        assert rel_rows(gv, vr).max() <= 1e-3, b


def test_large_ensemble_sampled_members(eng):
    pk, engine, ctx = eng
    B, n, T = 64, 1000, 12
    say(f"[batch] B={B} n={n} T={T}")
    states = [member(n, 100 + b, unequal=(b % 7 == 3)) for b in range(B)]
    ops = [member_pot(b % 9) for b in range(B)]
    dts = [pk.myr(1.0) * (1.0 + 0.01 * b) for b in range(B)]
    px, pv, pm = stack(states)
    ctx.simulate_batch(px, pv, pm, [gpu_pot(engine, o) for o in ops], dts, T)
    torch.cuda.synchronize()
    for b in (0, 3, 37, 63):
        x, v, m = states[b]
        xr, vr = oint.simulate(x, v, m, ops[b], dts[b], T)
        assert rel_rows(px[b].cpu().numpy().T, xr).max() <= 1e-5, b
        assert rel_rows(pv[b].cpu().numpy().T, vr).max() <= 1e-3, b


def test_zero_steps_and_limits(eng):
    pk, engine, ctx = eng
    states = [member(64, 7 + b) for b in range(3)]
    px, pv, pm = stack(states)
    x0 = px.clone()
    pots = [engine.Potential(eps=1e-3)] * 3
    ctx.simulate_batch(px, pv, pm, pots, [0.01] * 3, 0)
    assert torch.equal(px, x0)
    with pytest.raises(DnbError, match="eps must be > 0"):
        ctx.simulate_batch(px, pv, pm, [engine.Potential(eps=0.0)] * 3, [0.01] * 3, 1)
    # 65536-particle context, n = 1000: 4 blocks of 256 per member, 256 blocks in all
    cap = ctx.batch_capacity(1000)
    assert cap == 64
    big = torch.zeros(cap + 1, 3, 1000, dtype=torch.float64, device="cuda")
    with pytest.raises(DnbError, match="does not fit"):
        ctx.simulate_batch(big, big.clone(), torch.ones(cap + 1, 1000, dtype=torch.float64,
                                                        device="cuda"),
                           [engine.Potential()] * (cap + 1), [0.01] * (cap + 1), 1)
    assert torch.equal(px, x0)


def test_orbit_batch_matches_single_orbits_and_oracle(eng):
    pk, engine, ctx = eng
    B, T = 7, 250
    rng = np.random.default_rng(3)
    w0 = np.concatenate([W_X + rng.normal(0, 1, (B, 3)), W_V + rng.normal(0, 10, (B, 3))], 1)
    ops = [member_pot(b) for b in range(B)]
    dts = [-pk.myr(1.0) * (1 + 0.2 * b) for b in range(B)]
    w0d = torch.tensor(w0, device="cuda")
    wo = ctx.orbit_batch(w0d, [gpu_pot(engine, o) for o in ops], dts, T)
    for b in range(B):
        single, _ = ctx.orbit(w0d[b].contiguous(), gpu_pot(engine, ops[b]), dts[b], T, keep=False)
        assert torch.equal(single, wo[b])
        xr, vr = oint.simulate(w0[b, None, :3], w0[b, None, 3:], np.zeros(1), ops[b], dts[b], T,
                               self_gravity=False)
        np.testing.assert_allclose(wo[b, :3].cpu().numpy(), xr[0], rtol=1e-12)
        np.testing.assert_allclose(wo[b, 3:].cpu().numpy(), vr[0], rtol=1e-12)


def test_mmd_batch_matches_oracle(eng):
    pk, engine, ctx = eng
    from oracle import mmd as ommd
    rng = np.random.default_rng(21)
    B, n, m = 5, 700, 300
    X = W_X + rng.normal(scale=0.3, size=(B, n, 3)) * rng.uniform(0.8, 1.2, (B, 1, 1))
    Y = W_X + 0.1 + rng.normal(scale=0.25, size=(m, 3))
    pos = torch.tensor(np.ascontiguousarray(X.transpose(0, 2, 1)), device="cuda")
    tgt = torch.tensor(np.ascontiguousarray(Y.T), device="cuda")
    loss = ctx.mmd_batch(pos, tgt, 0.2).cpu().numpy()
    for b in range(B):
        ref = ommd.mmd2(X[b], Y, 0.2)
        assert abs(loss[b] / ref - 1) <= 1e-12, b
        single, _ = ctx.mmd(pos[b], tgt, 0.2, grad=False)
        assert abs(loss[b] / single.item() - 1) <= 1e-13, b
    # a member identical to the target gives zero
    same = torch.tensor(np.ascontiguousarray(Y.T)[None], device="cuda")
    assert abs(ctx.mmd_batch(same, tgt, 0.2).item()) <= 1e-14


def test_grid_search_matches_oracle_pipeline(eng):
    pk, engine, ctx = eng
    from oracle import pipeline as opipe
    from paper_2511_22468_amd.pipeline import grid_search, StreamModel
    n, T, B = 300, 60, 6
    say(f"[grid] B={B} n={n} T={T}")
    xi, zeta = plummer_unit(n, 8)
    rng = np.random.default_rng(9)
    Y = W_X + rng.normal(scale=0.05, size=(400, 3))
    op = OPot()
    thetas = np.array([[pk.gyr(0.05 + 0.01 * b), 2e4 * (1 + 0.1 * b), 1e12 * (1 + 0.05 * b),
                        6.5e10 * (1 - 0.03 * b)] for b in range(B)])
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    losses = grid_search(ctx, thetas, t3(xi), t3(zeta), t3(Y), T, gpu_pot(engine, op), h=0.2)
    model = StreamModel(ctx, t3(xi), t3(zeta), t3(Y), T, pot=gpu_pot(engine, op), h=0.2)
    for b in range(B):
        # the batched runs repeat the single-system FP32C runs bit for bit; only
        # the loss sums are ordered differently
        single = model.loss(torch.tensor(thetas[b], device="cuda")).item()
        assert abs(losses[b] / single - 1) <= 1e-12, (b, losses[b], single)
        # against the FP64 oracle: FP32C positions differ by ~1e-7 relative (more
        # where the core is chaotic), moving the loss by |grad L| |dx| ~ (1/h) 1e-6
        ref = opipe.loss(tuple(thetas[b]), xi, zeta, op, T, Y, 0.2)
        say(f"  member {b}: loss {losses[b]:.10e} oracle {ref:.10e} "
            f"difference {abs(losses[b] - ref):.2e}")
        assert abs(losses[b] - ref) <= 2e-5, (b, losses[b], ref)


def test_single_particle_members_follow_the_host_potential(eng):
    """n = 1: no pair force (the self term vanishes for eps > 0), so every member is a
    test particle in its own potential."""
    pk, engine, ctx = eng
    B, T = 4, 100
    rng = np.random.default_rng(12)
    x = W_X + rng.normal(0, 1, (B, 1, 3))
    v = W_V + rng.normal(0, 10, (B, 1, 3))
    ops = [member_pot(b) for b in range(B)]
    dts = [pk.myr(1.0) * (1 + 0.3 * b) for b in range(B)]
    px, pv, pm = stack([(x[b], v[b], np.array([5e3])) for b in range(B)])
    ctx.simulate_batch(px, pv, pm, [gpu_pot(engine, o) for o in ops], dts, T)
    for b in range(B):
        xr, vr = oint.simulate(x[b], v[b], np.array([5e3]), ops[b], dts[b], T, self_gravity=False)
        np.testing.assert_allclose(px[b].cpu().numpy().T, xr, rtol=1e-12)
        np.testing.assert_allclose(pv[b].cpu().numpy().T, vr, rtol=1e-12)
    assert ctx.batch_capacity(0) == 0


def test_mmd_batch_single_points_closed_form(eng):
    """n = m = 1: MMD^2 = 2 - 2 exp(-|x - y|^2 / (2 h^2))."""
    pk, engine, ctx = eng
    pos = torch.tensor([[[0.0], [0.0], [0.0]], [[0.3], [0.0], [0.0]], [[0.1], [0.2], [-0.2]]],
                       dtype=torch.float64, device="cuda")
    tgt = torch.zeros(3, 1, dtype=torch.float64, device="cuda")
    got = ctx.mmd_batch(pos, tgt, 0.2).cpu().numpy()
    d2 = (pos.cpu().numpy() ** 2).sum(axis=(1, 2))
    np.testing.assert_allclose(got, 2 - 2 * np.exp(-d2 / (2 * 0.2 ** 2)), rtol=1e-14, atol=1e-16)


def test_place_plummer_batch_equals_single_placements(eng):
    pk, engine, ctx = eng
    n, B = 700, 5
    xi, zeta = plummer_unit(n, 61)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    rng = np.random.default_rng(62)
    w = torch.tensor(np.concatenate([W_X + rng.normal(0, 1, (B, 3)),
                                     W_V + rng.normal(0, 10, (B, 3))], 1), device="cuda")
    m = torch.tensor(rng.uniform(1e4, 1e5, B), device="cuda")
    pos, vel, mass = ctx.place_plummer_batch(w, t3(xi), t3(zeta), m, 0.01, G)
    for b in range(B):
        p, v, mm = ctx.place_plummer(w[b], t3(xi), t3(zeta), m[b].item(), 0.01, G)
        assert torch.equal(p, pos[b]) and torch.equal(v, vel[b]) and torch.equal(mm, mass[b])


def test_batched_adjoint_equals_single_system_adjoints(eng):
    """dnb_simulate_batch_vjp repeats dnb_simulate_vjp member by member: with the
    same source slicing (n = 300) every member's gradient is bitwise that of a lone
    system; the gradient of a linear functional is also checked against the
    oracle's discrete adjoint."""
    pk, engine, ctx = eng
    from oracle import adjoint as oadj
    B, n, T = 4, 300, 25
    states = [member(n, 80 + b, unequal=(b == 1)) for b in range(B)]
    ops = [member_pot(b) for b in range(B)]
    dts = [pk.myr(0.5) * (1.0 + 0.2 * b) for b in range(B)]
    pots = [gpu_pot(engine, o) for o in ops]
    px, pv, pm = stack(states)
    tape = ctx.simulate_batch(px, pv, pm, pots, dts, T, tape=True)
    rng = np.random.default_rng(81)
    gx = torch.tensor(rng.normal(size=(B, 3, n)), device="cuda")
    gv = torch.tensor(rng.normal(size=(B, 3, n)), device="cuda")
    g0, gv0, gpar = ctx.simulate_batch_vjp(pm, pots, dts, T, tape, px, gx, gv)
    for b in range(B):
        x, v, m = states[b]
        sx, sv = to_dev(x), to_dev(v)
        stape = ctx.simulate(sx, sv, to_dev(m), pots[b], dts[b], T, ckpt_every=1)
        assert torch.equal(sx, px[b])
        s0, sv0, _, sp = ctx.simulate_vjp(to_dev(m), pots[b], dts[b], T, 1, stape, sx,
                                          gx[b].contiguous(), gv[b].contiguous())
        assert torch.equal(s0, g0[b]) and torch.equal(sv0, gv0[b]), f"member {b}"
        # the batched sweep returns the first four parameters (masses, dt, mass scale)
        assert torch.equal(sp[:4], gpar[b]), f"member {b} parameters"
    # the oracle's exact discrete adjoint for one member (FP64 reference)
    x, v, m = states[2]
    xr, vr, traj = oint.simulate(x, v, m, ops[2], dts[2], T, keep=True)
    ref = oadj.simulate_vjp(traj, m, ops[2], dts[2], gx[2].cpu().numpy().T, gv[2].cpu().numpy().T)
    got = g0[2].cpu().numpy().T
    assert np.sqrt(((got - ref["x0"]) ** 2).sum()) <= 1e-3 * np.sqrt((ref["x0"] ** 2).sum())


def test_batched_pipeline_gradient_matches_single_model_and_oracle(eng):
    """pipeline.batch_loss_and_grad (orbit, placement, N-body run, MMD and their
    three adjoints, all batched) against StreamModel.loss_and_grad member by member
    and, for one member, against the oracle pipeline's exact gradient."""
    pk, engine, ctx = eng
    from oracle import pipeline as opipe
    from paper_2511_22468_amd.pipeline import StreamModel, batch_loss_and_grad
    n, T, B = 300, 30, 4
    say(f"[batch-grad] B={B} n={n} T={T}")
    xi, zeta = plummer_unit(n, 31)
    Y = W_X + 0.05 * np.random.default_rng(32).normal(size=(128, 3))
    op = OPot()
    thetas = np.array([[pk.myr(30.0 * (1 + 0.1 * b)), 3e4 * (1 - 0.1 * b), 1.1e12 * (1 + 0.03 * b),
                        6.0e10 * (1 + 0.05 * b)] for b in range(B)])
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    losses, grads = batch_loss_and_grad(ctx, thetas, t3(xi), t3(zeta), t3(Y), T,
                                        gpu_pot(engine, op), h=0.2, chunk=3)
    model = StreamModel(ctx, t3(xi), t3(zeta), t3(Y), T, pot=gpu_pot(engine, op), h=0.2,
                        ckpt_every=1)
    for b in range(B):
        L, g = model.loss_and_grad(torch.tensor(thetas[b], device="cuda"))
        assert abs(losses[b] / L.item() - 1) <= 1e-12, b
        # same trajectories bit for bit; the MMD gradient sums are ordered
        # differently, which moves FP32 roundings of the adjoint's pair terms
        sg, sr = grads[b] * thetas[b], g.cpu().numpy() * thetas[b]
        assert np.abs(sg - sr).max() <= 1e-6 * np.abs(sr).max(), (b, sg, sr)
    L_ref, g = opipe.loss_and_grad(thetas[0], xi, zeta, op, T, Y, 0.2)
    g_ref = np.array([g["t_end"], g["m_prog"], g["m_nfw"], g["m_mn"]])
    assert abs(losses[0] / L_ref - 1) <= 1e-3
    sg, sr = grads[0] * thetas[0], g_ref * thetas[0]
    assert np.abs(sg - sr).max() <= 1e-3 * np.abs(sr).max()


def test_batched_component_adjoints_equal_single_ones(eng):
    """The three per-member adjoints the batched pipeline gradient chains: the MMD
    position gradient (against dnb_mmd and the oracle), the test-particle orbit VJP
    and the Plummer placement VJP (against their single-system entries)."""
    pk, engine, ctx = eng
    from oracle import mmd as ommd
    B, n, m, T = 3, 300, 200, 40
    say(f"[batch-vjp] B={B} n={n} m={m} T={T}")
    rng = np.random.default_rng(90)
    pos = torch.tensor(W_X[None, :, None] + 0.1 * rng.normal(size=(B, 3, n)), device="cuda")
    Y = W_X + 0.1 * rng.normal(size=(m, 3))
    tgt = torch.tensor(np.ascontiguousarray(Y.T), device="cuda")
    loss, g = ctx.mmd_batch_grad(pos, tgt, 0.2)
    for b in range(B):
        sl, sg = ctx.mmd(pos[b].contiguous(), tgt, 0.2)
        # the batched and single entries sum in different orders; MMD^2 (~1e-3) is a
        # difference of kernel means of order 0.1-1, so one ulp of those sums is
        # ~1e-13 of the loss
        assert abs(loss[b].item() / sl.item() - 1) <= 1e-12
        # per-row errors against the largest row: rows near a kernel-sum cancellation
        # have small gradients with few correct digits in any summation order
        got, single = g[b].cpu().numpy().T, sg.cpu().numpy().T
        scale = np.sqrt((single ** 2).sum(1)).max()
        assert np.sqrt(((got - single) ** 2).sum(1)).max() <= 1e-12 * scale, b
        ref = ommd.mmd2_grad(pos[b].cpu().numpy().T, Y, 0.2)
        assert np.sqrt(((got - ref) ** 2).sum(1)).max() <= 1e-12 * scale, b
    # orbits: each member its own potential and signed step
    ops = [member_pot(b) for b in range(B)]
    pots = [gpu_pot(engine, o) for o in ops]
    dts = [pk.myr(2.0) * (1 + 0.2 * b) * (-1 if b == 1 else 1) for b in range(B)]
    w0 = torch.tensor(np.concatenate([W_X, W_V])[None, :] + rng.normal(size=(B, 6)),
                      device="cuda")
    w_out, traj = ctx.orbit_batch(w0, pots, dts, T, keep=True)
    gw_out = torch.tensor(rng.normal(size=(B, 6)), device="cuda")
    gw0, gpar = ctx.orbit_batch_vjp(traj, pots, dts, T, gw_out)
    for b in range(B):
        s_out, s_traj = ctx.orbit(w0[b].contiguous(), pots[b], dts[b], T)
        assert torch.equal(s_traj, traj[b])
        s0, sp = ctx.orbit_vjp(s_traj, pots[b], dts[b], T, gw_out[b].contiguous())
        np.testing.assert_allclose(gw0[b].cpu().numpy(), s0.cpu().numpy(), rtol=1e-13, atol=0)
        np.testing.assert_allclose(gpar[b].cpu().numpy(), sp.cpu().numpy(), rtol=1e-13, atol=0)
    # placement: shared unit samples, per-member centre and mass
    xi, zeta = plummer_unit(n, 91)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    m_tot = torch.tensor([2e4, 3.5e4, 5e3], device="cuda", dtype=torch.float64)
    gpos = torch.tensor(rng.normal(size=(B, 3, n)), device="cuda")
    gvel = torch.tensor(rng.normal(size=(B, 3, n)), device="cuda")
    gw, gm = ctx.place_plummer_batch_vjp(t3(zeta), m_tot, 0.01, gpos, gvel)
    for b in range(B):
        sw, sm = ctx.place_plummer_vjp(t3(zeta), m_tot[b].item(), 0.01, gpos[b].contiguous(),
                                       gvel[b].contiguous())
        np.testing.assert_allclose(gw[b].cpu().numpy(), sw.cpu().numpy(), rtol=1e-12, atol=0)
        assert abs(gm[b].item() / sm.item() - 1) <= 1e-12, b


def test_mmd_batch_with_a_target_per_member(eng):
    """Bootstrap form of the batched loss: member b against its own target tgt[b]
    (loss and gradient equal dnb_mmd on that pair; a member whose target is its
    own positions has zero loss and gradient)."""
    pk, engine, ctx = eng
    B, n, m = 4, 300, 260
    say(f"[mmd-per-member] B={B} n={n} m={m}")
    rng = np.random.default_rng(95)
    pos = torch.tensor(W_X[None, :, None] + 0.1 * rng.normal(size=(B, 3, n)), device="cuda")
    tgt = torch.tensor(W_X[None, :, None] + 0.1 * rng.normal(size=(B, 3, m)), device="cuda")
    loss, g = ctx.mmd_batch_grad(pos, tgt, 0.2)
    assert torch.equal(ctx.mmd_batch(pos, tgt, 0.2), loss)
    for b in range(B):
        sl, sg = ctx.mmd(pos[b].contiguous(), tgt[b].contiguous(), 0.2)
        assert abs(loss[b].item() / sl.item() - 1) <= 1e-12, b
        got, single = g[b].cpu().numpy().T, sg.cpu().numpy().T
        scale = np.sqrt((single ** 2).sum(1)).max()
        assert np.sqrt(((got - single) ** 2).sum(1)).max() <= 1e-12 * scale, b
    # targets equal to the members' own positions (m = n)
    l0, g0 = ctx.mmd_batch_grad(pos, pos.clone(), 0.2)
    assert l0.abs().max().item() <= 1e-14
    assert g0.abs().max().item() <= 1e-12
    with pytest.raises(ValueError):
        ctx.mmd_batch(pos, tgt[:2].contiguous(), 0.2)


def test_bootstrap_refinement_equals_row_by_row_descent(eng):
    """bootstrap.refine advances every realisation with one batched gradient per
    step; the same descent row by row through StreamModel.loss_and_grad must
    visit the same points (up to the FP32 roundings of the adjoint) and the loss
    must not end above its start."""
    pk, engine, ctx = eng
    from paper_2511_22468_amd import bootstrap as BS
    from paper_2511_22468_amd.pipeline import StreamModel, make_target
    n, T, B, iters, lr = 300, 30, 3, 3, 0.05
    say(f"[bootstrap] B={B} n={n} T={T} iters={iters}")
    xi, zeta = plummer_unit(n, 61)
    xt, zt = plummer_unit(n, 62)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    pot = engine.Potential()
    u_true = np.array([-0.9, 0.2, 0.0, 0.1])
    target = make_target(ctx, t3(xt), t3(zt), torch.tensor(BS.theta_rows(u_true[None])[0],
                                                           device="cuda"), T, pot=pot)
    noise = torch.tensor(np.random.default_rng(63).normal(size=(B, 3, n)), device="cuda")
    targets = BS.resample(target, 0.005, noise)
    u0 = u_true[None] + np.array([[0.05, -0.1, 0.1, 0.0], [0.0, 0.1, -0.05, 0.05],
                                  [-0.05, 0.0, 0.05, -0.1]])
    u_fin, L_fin, hist, acc = BS.refine(ctx, u0, t3(xi), t3(zeta), targets, T, lr, iters,
                                        pot=pot)
    assert hist.shape == (iters + 1, B) and acc.shape == (iters, B)
    for b in range(B):
        model = StreamModel(ctx, t3(xi), t3(zeta), targets[b].contiguous(), T, pot=pot,
                            ckpt_every=1)

        def ev(u):
            L, g = model.loss_and_grad(torch.tensor(BS.theta_rows(u[None])[0], device="cuda"))
            return L.item(), g.cpu().numpy() * BS.dtheta_du_rows(u[None])[0]

        u = u0[b].copy()
        L, gu = ev(u)
        assert abs(hist[0, b] / L - 1) <= 1e-12
        step = lr
        for it in range(iters):
            cand = np.clip(u - step * gu / np.sqrt((gu * gu).sum()), -1, 1)
            Lc, gc = ev(cand)
            assert abs(hist[it + 1, b] / Lc - 1) <= 1e-6, (b, it, hist[it + 1, b], Lc)
            assert acc[it, b] == (Lc <= L)
            if Lc <= L:
                u, L, gu = cand, Lc, gc
            else:
                step *= 0.5
        np.testing.assert_allclose(u_fin[b], u, rtol=0, atol=1e-6)
        assert L_fin[b] <= hist[0, b] and L_fin[b] == hist[:, b][np.r_[True, acc[:, b]]].min()


def test_batched_adjoint_of_single_particle_members(eng):
    """n = 1: every member is a test particle (the self term vanishes), so the
    batched adjoint is the oracle's adjoint of an orbit in the member's own
    potential, including dL/dm_nfw, dL/dm_mn and dL/ddt."""
    pk, engine, ctx = eng
    from oracle import adjoint as oadj
    B, T = 3, 50
    rng = np.random.default_rng(96)
    x = W_X + rng.normal(0, 1, (B, 1, 3))
    v = W_V + rng.normal(0, 10, (B, 1, 3))
    ops = [member_pot(b) for b in range(B)]
    dts = [pk.myr(1.0) * (1 + 0.3 * b) for b in range(B)]
    m1 = np.array([5e3])
    px, pv, pm = stack([(x[b], v[b], m1) for b in range(B)])
    tape = ctx.simulate_batch(px, pv, pm, [gpu_pot(engine, o) for o in ops], dts, T, tape=True)
    gx = torch.tensor(rng.normal(size=(B, 3, 1)), device="cuda")
    gv = torch.tensor(rng.normal(size=(B, 3, 1)), device="cuda")
    g0, gv0, gpar = ctx.simulate_batch_vjp(pm, [gpu_pot(engine, o) for o in ops], dts, T, tape,
                                           px, gx, gv)
    for b in range(B):
        _, _, traj = oint.simulate(x[b], v[b], m1, ops[b], dts[b], T, keep=True,
                                   self_gravity=False)
        ref = oadj.simulate_vjp(traj, m1, ops[b], dts[b], gx[b].cpu().numpy().T,
                                gv[b].cpu().numpy().T, self_gravity=False)
        rel = lambda a, r: np.sqrt(((a - r) ** 2).sum()) / np.sqrt((r ** 2).sum())
        assert rel(g0[b].cpu().numpy().T, ref["x0"]) <= 1e-10, b
        assert rel(gv0[b].cpu().numpy().T, ref["v0"]) <= 1e-10, b
        got = gpar[b].cpu().numpy()
        np.testing.assert_allclose(got[:3], [ref["m_nfw"], ref["m_mn"], ref["dt"]], rtol=1e-9)


def test_batched_pipeline_gradient_with_a_centre_per_row(eng):
    """Rows with their own present-day centre (a bootstrap realisation's centre
    of mass, Fig. 2 step 1) equal StreamModel built on that centre."""
    pk, engine, ctx = eng
    from paper_2511_22468_amd.pipeline import StreamModel, batch_loss_and_grad
    n, T = 300, 20
    say(f"[batch-grad-centres] n={n} T={T}")
    xi, zeta = plummer_unit(n, 33)
    Y = W_X + 0.05 * np.random.default_rng(34).normal(size=(100, 3))
    op = OPot()
    theta = np.array([pk.myr(20.0), 3e4, 1.1e12, 6.0e10])
    w_rows = np.array([[12.0, 0.0, 0.0, 0.0, -180.0, 60.0], [12.05, 0.02, -0.01, 1.0, -179.0, 60.5]])
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    losses, grads = batch_loss_and_grad(ctx, np.repeat(theta[None], 2, 0), t3(xi), t3(zeta), t3(Y),
                                        T, gpu_pot(engine, op), w_now=w_rows)
    assert abs(losses[0] - losses[1]) > 1e-6 * abs(losses[0])
    for b in range(2):
        model = StreamModel(ctx, t3(xi), t3(zeta), t3(Y), T, pot=gpu_pot(engine, op),
                            ckpt_every=1, w_now=tuple(w_rows[b]))
        L, g = model.loss_and_grad(torch.tensor(theta, device="cuda"))
        assert abs(losses[b] / L.item() - 1) <= 1e-12, b
        sg, sr = grads[b] * theta, g.cpu().numpy() * theta
        assert np.abs(sg - sr).max() <= 1e-6 * np.abs(sr).max(), (b, sg, sr)


def test_inference_pipeline_end_to_end(eng):
    """infer.run: the grid losses of every realisation equal grid_search against
    that realisation's target, each refinement starts at its realisation's best
    grid point and ends no worse than it."""
    pk, engine, ctx = eng
    from paper_2511_22468_amd import bootstrap as BS, infer
    from paper_2511_22468_amd.pipeline import grid_search
    n, T, B, per_axis, iters = 300, 30, 3, 3, 2
    say(f"[infer] n={n} T={T} B={B} grid={per_axis}^4")
    xi, zeta = plummer_unit(n, 91)
    xt, zt = plummer_unit(n, 92)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    pot = engine.Potential()
    noise = torch.tensor(np.random.default_rng(93).normal(size=(B, 3, n)), device="cuda")
    u_true = np.array([-0.9, 0.1, 0.0, 0.2])
    res = infer.run(ctx, u_true, t3(xi), t3(zeta), t3(xt), t3(zt), T, noise, 0.005, per_axis,
                    iters, 0.05, pot)
    L = res["grid_losses"]
    assert L.shape == (per_axis ** 4, B)
    th = BS.theta_rows(infer.grid_points(per_axis))
    target = infer.make_target(ctx, t3(xt), t3(zt), torch.tensor(BS.theta_rows(u_true[None])[0],
                                                                  device="cuda"), T, pot=pot)
    targets = BS.resample(target, 0.005, noise)
    for b in range(B):
        ref = grid_search(ctx, th, t3(xi), t3(zeta), targets[b].contiguous(), T, pot)
        # same runs; the target's own kernel sum is reduced in another order
        np.testing.assert_allclose(L[:, b], ref, rtol=1e-12, atol=0)
        k = int(np.argmin(L[:, b]))
        np.testing.assert_array_equal(res["u_grid_best"][b], infer.grid_points(per_axis)[k])
        assert res["L_fit"][b] <= L[k, b] * (1 + 1e-6), b
    s = infer.summary(res, u_true)
    assert len(s["fit_mean"]) == 4 and np.all(np.isfinite(s["fit_std"]))


def test_batched_gradient_is_independent_of_the_chunking(eng):
    """Members do not interact: the batched pipeline gradient of four rows is the
    same bit for bit whether they run as one ensemble, in chunks of 3 or one at a
    time (n = 300 keeps the same source slicing for all three ensemble sizes)."""
    pk, engine, ctx = eng
    from paper_2511_22468_amd.pipeline import batch_loss_and_grad
    n, T, B = 300, 15, 4
    say(f"[batch-chunks] B={B} n={n} T={T}")
    xi, zeta = plummer_unit(n, 35)
    Y = W_X + 0.05 * np.random.default_rng(36).normal(size=(90, 3))
    thetas = np.array([[pk.myr(15.0 * (1 + 0.2 * b)), 2e4 * (1 + 0.3 * b), 1e12, 6.5e10]
                       for b in range(B)])
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    runs = [batch_loss_and_grad(ctx, thetas, t3(xi), t3(zeta), t3(Y), T, engine.Potential(),
                                chunk=c) for c in (None, 3, 1)]
    for L, g in runs[1:]:
        assert np.array_equal(L, runs[0][0]) and np.array_equal(g, runs[0][1])


def test_mmd_batch_against_several_targets(eng):
    """dnb_mmd_batch_targets: loss[b][t] equals the per-member-target call with
    every member's target tgts[t] bit for bit, and dnb_mmd (sums ordered
    otherwise; the loss is a difference of three kernel sums) to 1e-12."""
    pk, engine, ctx = eng
    B, n, T, m = 5, 300, 4, 260
    say(f"[mmd-targets] B={B} n={n} T={T} m={m}")
    rng = np.random.default_rng(97)
    pos = torch.tensor(W_X[None, :, None] + 0.1 * rng.normal(size=(B, 3, n)), device="cuda")
    tgts = torch.tensor(W_X[None, :, None] + 0.1 * rng.normal(size=(T, 3, m)), device="cuda")
    L = ctx.mmd_batch_targets(pos, tgts, 0.2)
    assert L.shape == (B, T)
    for t in range(T):
        same = tgts[t:t + 1].expand(B, 3, m).contiguous()
        assert torch.equal(L[:, t].contiguous(), ctx.mmd_batch(pos, same, 0.2)), t
        for b in range(B):
            sl, _ = ctx.mmd(pos[b].contiguous(), tgts[t].contiguous(), 0.2, grad=False)
            assert abs(L[b, t].item() / sl.item() - 1) <= 1e-12, (b, t)
