"""Restart of a forward run from a tape checkpoint, and the debug scan of an
initial state (run on an MI355X).

The fixed-step kick-drift-kick map (Sec. 2.2.1) is a deterministic function of
the state, so a run continued from a stored checkpoint must reach the state of
the uninterrupted run bit for bit, in FP64 and in FP32C (where the checkpoint
also supplies the two staging centres the run used there).  The oracle's
integrator satisfies the same identity (tests/test_oracle_dynamics.py).
"""
import numpy as np
import pytest
import torch

from oracle.forces import Potential as OPot
from synth import plummer_unit

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

G = 4.3009e-6
W_X = np.array([12.0, 0.0, 0.0])
W_V = np.array([0.0, -180.0, 60.0])


@pytest.fixture(scope="module")
def dnb():
    import paper_2511_22468_amd as pk
    from paper_2511_22468_amd import engine
    ctx = {p: engine.Context(8192, p) for p in ("fp64", "fp32c")}
    yield pk, engine, ctx
    for c in ctx.values():
        c.close()


def plummer_state(n, seed, unequal=False, m_tot=2e4, a_p=0.01):
    xi, zeta = plummer_unit(n, seed)
    m = np.full(n, m_tot / n)
    if unequal:
        m = m * np.random.default_rng(seed + 1).uniform(0.5, 1.5, n)
    return W_X + a_p * xi, W_V + np.sqrt(G * m_tot / a_p) * zeta, m


def gpu_pot(engine, op):
    return engine.Potential(G=op.G, eps=op.eps, m_nfw=op.m_nfw, rs_nfw=op.rs_nfw, m_mn=op.m_mn,
                            a_mn=op.a_mn, b_mn=op.b_mn)


def tape_sections(t, n, n_ckpt):
    """The tape's sections: states [n_ckpt][6n], centres [n_ckpt][8], internal
    accelerations at the checkpoints [n_ckpt][3n] and at the final positions [3n]."""
    a = 6 * n * n_ckpt
    b = a + 8 * n_ckpt
    c = b + 3 * n * n_ckpt
    return (t[:a].view(n_ckpt, 6 * n), t[a:b].view(n_ckpt, 8), t[b:c].view(n_ckpt, 3 * n),
            t[c:c + 3 * n])


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("masses", ["equal", "unequal"])
def test_resume_continues_the_run_bitwise(dnb, prec, masses):
    pk, engine, ctx = dnb
    n, T, K = 1300, 30, 10
    say(f"[resume] n={n} T={T} K={K} prec={prec} masses={masses}")
    x, v, m = plummer_state(n, 21, unequal=masses == "unequal")
    c = ctx[prec]
    pot = gpu_pot(engine, OPot())
    dt = pk.myr(0.5)
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    tape = c.simulate(px, pv, pm, pot, dt, T, ckpt_every=K)
    for ck in range(T // K):
        qx, qv = torch.empty_like(px), torch.empty_like(pv)
        c.simulate_resume(tape, T, K, ck, qx, qv, pm, pot, dt, T - ck * K)
        assert torch.equal(qx, px), (ck, (qx - px).abs().max().item())
        assert torch.equal(qv, pv), (ck, (qv - pv).abs().max().item())
    # n_steps = 0: the checkpoint's state itself
    qx, qv = torch.empty_like(px), torch.empty_like(pv)
    c.simulate_resume(tape, T, K, 1, qx, qv, pm, pot, dt, 0)
    st = tape_sections(tape, n, T // K)[0]
    assert torch.equal(qx.reshape(-1), st[1, :3 * n]) and torch.equal(qv.reshape(-1), st[1, 3 * n:])
    # the continuation's own tape is the tail of the source tape
    qx, qv = torch.empty_like(px), torch.empty_like(pv)
    t2 = c.simulate_resume(tape, T, K, 1, qx, qv, pm, pot, dt, T - K, ckpt_every=K)
    src, out = tape_sections(tape, n, 3), tape_sections(t2, n, 2)
    assert torch.equal(out[0], src[0][1:])
    assert torch.equal(out[2], src[2][1:])
    assert torch.equal(out[3], src[3])
    if prec == "fp32c":   # the FP64 path stages without a centre
        assert torch.equal(out[1], src[1][1:])
    # the reverse sweep accepts the continuation's tape; in FP64 its gradient is
    # that of a fresh run from the checkpoint's state, bit for bit
    w = to_dev(np.random.default_rng(22).normal(size=x.shape))
    g2 = c.simulate_vjp(pm, pot, dt, T - K, K, t2, qx, w)
    assert all(torch.isfinite(g).all() for g in (g2[0], g2[1], g2[3]))
    if prec == "fp64":
        fx, fv = st[1, :3 * n].view(3, n).clone(), st[1, 3 * n:].view(3, n).clone()
        t3 = c.simulate(fx, fv, pm, pot, dt, T - K, ckpt_every=K)
        g3 = c.simulate_vjp(pm, pot, dt, T - K, K, t3, fx, w)
        assert torch.equal(fx, qx)
        for a, b in zip((g2[0], g2[1], g2[3]), (g3[0], g3[1], g3[3])):
            assert torch.equal(a, b)


def test_resume_refusals(dnb):
    pk, engine, ctx = dnb
    from paper_2511_22468_amd._lib import DnbError
    n, T, K = 300, 12, 4
    say(f"[resume] refusals n={n}")
    x, v, m = plummer_state(n, 23)
    c = ctx["fp32c"]
    pot = gpu_pot(engine, OPot())
    dt = pk.myr(0.5)
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    tape = c.simulate(px, pv, pm, pot, dt, T, ckpt_every=K)
    qx, qv = torch.empty_like(px), torch.empty_like(pv)
    with pytest.raises(DnbError, match="outside"):
        c.simulate_resume(tape, T, K, 3, qx, qv, pm, pot, dt, 4)
    with pytest.raises(DnbError, match="outside"):
        c.simulate_resume(tape, T, K, -1, qx, qv, pm, pot, dt, 4)
    with pytest.raises(DnbError, match="overlap"):
        c.simulate_resume(tape, T, K, 1, tape[:3 * n].view(3, n), qv, pm, pot, dt, 4)
    with pytest.raises(ValueError):   # the binding checks the stated tape length
        c.simulate_resume(tape[:100], T, K, 1, qx, qv, pm, pot, dt, 4)
    # nothing was integrated by the refused calls: a valid call still continues bitwise
    c.simulate_resume(tape, T, K, 2, qx, qv, pm, pot, dt, T - 2 * K)
    assert torch.equal(qx, px) and torch.equal(qv, pv)


@pytest.mark.parametrize("n", [1, 255, 1300, 5000])
def test_check_state_finds_the_first_non_finite_particle(dnb, n):
    pk, engine, ctx = dnb
    say(f"[scan] n={n}")
    x, v, m = plummer_state(n, 24)
    c = ctx["fp64"]
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    assert c.check_state(px, pv, pm) == -1
    assert c.check_state(px) == -1
    rng = np.random.default_rng(25)
    for trial in range(6):
        ks = sorted(rng.choice(n, size=min(3, n), replace=False))
        qx, qv, qm = px.clone(), pv.clone(), pm.clone()
        bad = [np.nan, np.inf, -np.inf]
        for j, k in enumerate(ks):
            where = (trial + j) % 3
            val = bad[(trial + 2 * j) % 3]
            if where == 0:
                qx[(trial + j) % 3, k] = val
            elif where == 1:
                qv[(trial + j) % 3, k] = val
            else:
                qm[k] = val
        assert c.check_state(qx, qv, qm) == ks[0], (trial, ks)
        # a field that is not scanned does not count
        only_x = [k for j, k in enumerate(ks) if (trial + j) % 3 == 0]
        assert c.check_state(qx) == (only_x[0] if only_x else -1)


def test_checks_refuse_a_non_finite_initial_state(dnb):
    pk, engine, ctx = dnb
    from paper_2511_22468_amd._lib import DnbError
    n = 700
    say(f"[scan] integrator checks n={n}")
    x, v, m = plummer_state(n, 26)
    c = ctx["fp32c"]
    pot = gpu_pot(engine, OPot())
    dt = pk.myr(0.5)
    px, pv, pm = to_dev(x), to_dev(v), to_dev(m)
    pv[1, 433] = float("nan")
    keep = px.clone()
    c.set_checks(True)
    try:
        with pytest.raises(DnbError, match="particle 433"):
            c.simulate(px, pv, pm, pot, dt, 5)
        assert torch.equal(px, keep)   # refused before any step
        # a batch names the member and the particle
        B = 3
        bx = torch.stack([to_dev(x)] * B).contiguous()
        bv = torch.stack([to_dev(v)] * B).contiguous()
        bm = torch.stack([pm] * B).contiguous()
        bm[2, 17] = float("inf")
        with pytest.raises(DnbError, match="member 2, particle 17"):
            c.simulate_batch(bx, bv, bm, [pot] * B, [dt] * B, 5)
        bm[2, 17] = pm[17]
        c.simulate_batch(bx, bv, bm, [pot] * B, [dt] * B, 5)   # a finite state runs
        assert torch.isfinite(bx).all()
    finally:
        c.set_checks(False)
