"""Call-sequence and buffer-size refusals of the reverse sweeps (DNB_ERR_STATE).

dnb_simulate_vjp differentiates the tape that a dnb_simulate call wrote; the
context keeps a descriptor of every tape it wrote (address, final-position
array, mass array, sizes, step and potential) and refuses a reverse sweep that
does not match one, before anything is enqueued.  The batched sweep is checked
the same way.  Each refusal is followed by a matching call, which must still
give the gradient of a fresh forward/reverse pair bit for bit.
"""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu

N, T = 300, 6


@pytest.fixture(scope="module")
def mods():
    from paper_2511_22468_amd import _lib, engine
    from synth import plummer_unit
    return _lib, engine, plummer_unit


def system(mods, seed=3):
    _, _, plummer_unit = mods
    xi, zeta = plummer_unit(N, seed)
    x = np.array([12.0, 0.0, 0.0]) + 0.01 * xi
    v = np.array([0.0, -180.0, 60.0]) + 2.0 * zeta
    t = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    m = torch.full((N,), 3e4 / N, dtype=torch.float64, device="cuda")
    return t(x), t(v), m


def raw_vjp(lib, ctx, mass, pot, dt, n_steps, K, tape, pos_T, g, work, outs):
    g0, gv0, gpar = outs
    return lib.dnb_simulate_vjp(ctx._h, N, ctypes.c_void_p(mass.data_ptr()), pot.c(), dt,
                                n_steps, K, ctypes.c_void_p(tape.data_ptr()),
                                ctypes.c_void_p(pos_T.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                None, ctypes.c_void_p(work.data_ptr()),
                                ctypes.c_void_p(g0.data_ptr()), ctypes.c_void_p(gv0.data_ptr()),
                                None, ctypes.c_void_p(gpar.data_ptr()), None)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_vjp_refuses_a_tape_it_did_not_write(mods, prec):
    _lib, engine, _ = mods
    lib = _lib.lib()
    say(f"boundary: tape refusals, {prec}, n = {N}, T = {T}")
    ctx = engine.Context(N, prec)
    pot = engine.Potential()
    dt = 5e-4
    x, v, m = system(mods)
    g = torch.ones(3, N, dtype=torch.float64, device="cuda")
    K = 2
    tape = torch.zeros(ctx.tape_len(N, T, K), dtype=torch.float64, device="cuda")
    work = torch.zeros(int(lib.dnb_vjp_workspace_doubles(N, K)), dtype=torch.float64,
                       device="cuda")
    outs = (torch.zeros(3, N, dtype=torch.float64, device="cuda"),
            torch.zeros(3, N, dtype=torch.float64, device="cuda"),
            torch.zeros(7, dtype=torch.float64, device="cuda"))

    # no dnb_simulate has written this tape
    assert raw_vjp(lib, ctx, m, pot, dt, T, K, tape, x, g, work, outs) == _lib.DNB_ERR_STATE
    assert b"no current tape" in lib.dnb_last_error()

    x0, v0 = x.clone(), v.clone()
    ctx.simulate(x, v, m, pot, dt, T, ckpt_every=K, tape=tape)
    # other step count, other checkpoint spacing
    assert raw_vjp(lib, ctx, m, pot, dt, T - 1, K, tape, x, g, work, outs) == _lib.DNB_ERR_STATE
    assert b"written for n" in lib.dnb_last_error()
    assert raw_vjp(lib, ctx, m, pot, dt, T, K + 1, tape, x, g, work, outs) == _lib.DNB_ERR_STATE
    # final positions that are not the forward run's
    assert raw_vjp(lib, ctx, m, pot, dt, T, K, tape, x.clone(), g, work,
                   outs) == _lib.DNB_ERR_STATE
    assert b"pos_T" in lib.dnb_last_error()
    # another step, another potential, another mass array
    assert raw_vjp(lib, ctx, m, pot, 2 * dt, T, K, tape, x, g, work, outs) == _lib.DNB_ERR_STATE
    assert raw_vjp(lib, ctx, m, pot.replace(m_nfw=2e12), dt, T, K, tape, x, g, work,
                   outs) == _lib.DNB_ERR_STATE
    assert raw_vjp(lib, ctx, m.clone(), pot, dt, T, K, tape, x, g, work,
                   outs) == _lib.DNB_ERR_STATE
    assert b"mass, dt or pot" in lib.dnb_last_error()
    # the binding checks buffer lengths before the call
    with pytest.raises(ValueError):
        ctx.simulate_vjp(m, pot, dt, T, K, tape[:-1], x, g)
    with pytest.raises(ValueError):
        ctx.simulate_vjp(m, pot, dt, T, K, tape, x, g, workspace=work[:-1])
    # nothing above was enqueued: the matching call gives the gradient of a
    # fresh forward and reverse pass bit for bit
    assert raw_vjp(lib, ctx, m, pot, dt, T, K, tape, x, g, work, outs) == _lib.DNB_OK
    xr, vr = x0.clone(), v0.clone()
    tape_r = ctx.simulate(xr, vr, m, pot, dt, T, ckpt_every=K)
    r0, rv0, _, rpar = ctx.simulate_vjp(m, pot, dt, T, K, tape_r, xr, g)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], r0) and torch.equal(outs[1], rv0) and torch.equal(outs[2], rpar)

    # a later step moves the final positions: the tape is stale
    ctx.step(x, v, m, pot, dt)
    assert raw_vjp(lib, ctx, m, pot, dt, T, K, tape, x, g, work, outs) == _lib.DNB_ERR_STATE
    assert b"no current tape" in lib.dnb_last_error()
    # a new tape written over the old one replaces its descriptor
    x2, v2 = x0.clone(), v0.clone()
    ctx.simulate(x2, v2, m, pot, dt, T, ckpt_every=K, tape=tape)
    assert raw_vjp(lib, ctx, m, pot, dt, T, K, tape, x2, g, work, outs) == _lib.DNB_OK
    ctx.close()


def test_vjp_refuses_a_short_device_buffer(mods):
    """A workspace allocation shorter than dnb_vjp_workspace_doubles is refused
    by the library itself (the allocation's extent is known to the runtime)."""
    _lib, engine, _ = mods
    lib = _lib.lib()
    # the HIP runtime already loaded by torch and the library (same instance)
    hip = ctypes.CDLL(next(l.split()[-1] for l in open("/proc/self/maps")
                           if "libamdhip64" in l))
    say("boundary: short workspace allocation")
    ctx = engine.Context(N, "fp32c")
    pot = engine.Potential()
    x, v, m = system(mods)
    g = torch.ones(3, N, dtype=torch.float64, device="cuda")
    K = 2
    tape = ctx.simulate(x, v, m, pot, 5e-4, T, ckpt_every=K)
    need = int(lib.dnb_vjp_workspace_doubles(N, K))
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(8 * (need - 1))) == 0
    try:
        outs = [ctypes.c_void_p(t.data_ptr()) for t in
                (torch.zeros(3, N, dtype=torch.float64, device="cuda"),
                 torch.zeros(3, N, dtype=torch.float64, device="cuda"),
                 torch.zeros(7, dtype=torch.float64, device="cuda"))]
        st = lib.dnb_simulate_vjp(ctx._h, N, ctypes.c_void_p(m.data_ptr()), pot.c(), 5e-4, T, K,
                                  ctypes.c_void_p(tape.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                  None, p, outs[0], outs[1], None, outs[2], None)
        assert st == _lib.DNB_ERR_STATE
        assert b"workspace needs" in lib.dnb_last_error()
    finally:
        torch.cuda.synchronize()
        hip.hipFree(p)
    ctx.close()


def test_batch_vjp_refuses_a_mismatched_tape(mods):
    _lib, engine, plummer_unit = mods
    say("boundary: batched tape refusals")
    B, n, Tb = 3, 200, 5
    ctx = engine.Context(B * n, "fp32c")
    xi, zeta = plummer_unit(n, 7)
    t = lambda a: torch.tensor(np.ascontiguousarray(a.T), device="cuda")
    x = torch.stack([t(np.array([12.0, 0.0, 0.0]) + 0.01 * xi)] * B).contiguous()
    v = torch.stack([t(np.array([0.0, -180.0, 60.0]) + 2.0 * zeta)] * B).contiguous()
    m = torch.full((B, n), 1e2, dtype=torch.float64, device="cuda")
    pots = [engine.Potential(m_nfw=1e12 * (1 + 0.1 * b)) for b in range(B)]
    dts = [5e-4] * B
    g = torch.ones(B, 3, n, dtype=torch.float64, device="cuda")
    tape = ctx.simulate_batch(x, v, m, pots, dts, Tb, tape=True)
    with pytest.raises(_lib.DnbError) as e:
        ctx.simulate_batch_vjp(m, pots, [6e-4] * B, Tb, tape, x, g)
    assert e.value.status == _lib.DNB_ERR_STATE
    with pytest.raises(_lib.DnbError) as e:
        ctx.simulate_batch_vjp(m, pots, dts, Tb, tape, x.clone(), g)
    assert e.value.status == _lib.DNB_ERR_STATE
    with pytest.raises(ValueError):
        ctx.simulate_batch_vjp(m, pots, dts, Tb + 1, tape, x, g)
    a = ctx.simulate_batch_vjp(m, pots, dts, Tb, tape, x, g)
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(z).all()) for z in a)
    ctx.close()
