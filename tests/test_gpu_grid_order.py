"""The pair grids' block order changes which compute unit runs which block, not
what a block computes: the (slices, target blocks) order of the single-system
kernels and the remapped linear index of the batched kernels give the same bits
as the plain (target blocks, slices[, members]) order (DNB_SLICE_MAJOR=0, read
when a context is created).  Sizes where the launch carries no external-field
row (which keeps the plain order) and a ragged tail; a batch whose (member,
slice) pairs are not a multiple of 256, so that both parts of the remap run.
"""
import os

import numpy as np
import pytest
import torch

from synth import plummer_unit

from gpu_util import say

pytestmark = pytest.mark.gpu


def contexts(engine, n, prec):
    old = os.environ.get("DNB_SLICE_MAJOR")
    try:
        os.environ["DNB_SLICE_MAJOR"] = "0"
        plain = engine.Context(n, prec)
    finally:
        if old is None:
            del os.environ["DNB_SLICE_MAJOR"]
        else:
            os.environ["DNB_SLICE_MAJOR"] = old
    return engine.Context(n, prec), plain


def state(n, seed):
    xi, zeta = plummer_unit(n, seed)
    t = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    x = t(np.array([12.0, 0.0, 0.0]) + 0.01 * xi)
    v = t(np.array([0.0, -180.0, 60.0]) + 4.0 * zeta)
    m = torch.full((n,), 1e5 / n, dtype=torch.float64, device="cuda")
    return x, v, m


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("n", [8192, 20000])
def test_single_system_orders_give_the_same_bits(prec, n):
    from paper_2511_22468_amd import engine, myr
    say(f"[grid order] n={n} prec={prec}")
    x, v, m = state(n, 21)
    m = m * torch.linspace(0.5, 1.5, n, dtype=torch.float64, device="cuda")
    w = torch.randn(3, n, dtype=torch.float64, device="cuda", generator=torch.Generator(
        device="cuda").manual_seed(5))
    pot = engine.Potential(eps=1e-3)
    out = []
    for c in contexts(engine, n, prec):
        a = c.accelerations(x, m, pot)
        rows = c.accelerations_rows(x, m, pot, 1000, 3000)
        g, gm = c.accelerations_vjp(x, m, pot, w, with_mass=True)
        xx, vv = x.clone(), v.clone()
        tape = c.simulate(xx, vv, m, pot, myr(0.5), 6, ckpt_every=3)
        r = c.simulate_vjp(m, pot, myr(0.5), 6, 3, tape, xx, w, with_mass=True)
        rr = c.simulate_vjp(m, pot, myr(0.5), 6, 3, tape, xx, w, with_mass=True, vel_T=vv)
        out.append([a, rows, g, gm, xx, vv, *r, *rr])
        c.close()
    names = ["acc", "rows", "vjp", "vjp_mass", "pos_T", "vel_T", "gpos0", "gvel0", "gmass",
             "gpar", "rev_gpos0", "rev_gvel0", "rev_gmass", "rev_gpar"]
    bad = [k for k, p, q in zip(names, *out) if not torch.equal(p, q)]
    assert not bad, bad


def test_batched_orders_give_the_same_bits():
    from paper_2511_22468_amd import engine, myr
    B, n = 40, 1000   # 40 members x 8 slices = 320 (member, slice) pairs: head and tail
    say(f"[grid order] batch B={B} n={n}")
    xs, vs, ms = zip(*(state(n, 30 + b) for b in range(B)))
    pots = [engine.Potential(eps=1e-3, m_nfw=1e12 * (1 + 0.01 * b)) for b in range(B)]
    dts = [myr(0.5)] * B
    out = []
    for c in contexts(engine, 1024 * B, "fp32c"):   # members padded to 1024 sources
        assert c.batch_capacity(n) >= B
        x, v, m = torch.stack(xs), torch.stack(vs), torch.stack(ms)
        tape = c.simulate_batch(x, v, m, pots, dts, 5, tape=True)
        w = torch.ones_like(x)
        g = c.simulate_batch_vjp(m, pots, dts, 5, tape, x, w)
        out.append([x, v, *g])
        c.close()
    bad = [k for k, (p, q) in enumerate(zip(*out)) if not torch.equal(p, q)]
    assert not bad, bad
