"""dnb_accelerations_noalloc (no context, no allocation; the kernels' scratch is a
static device array) against dnb_accelerations, through the C ABI: two calls in
a row, the second with a smaller system, in both precisions.  The no-alloc path
splits the sources into fewer slices, so FP32C agrees with the context path to
FP32 rounding (per particle <= 2e-7 relative) and FP64 to FP64 rounding; both are
also checked against the oracle on sampled rows (FP32C <= 1e-5, FP64 <= 1e-12)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import forces as of
from oracle.forces import Potential as OPot
from synth import plummer_unit, sample_rows

from gpu_util import rel_rows, say, to_dev, to_host

pytestmark = pytest.mark.gpu

G = 4.3009e-6
W_X = np.array([12.0, 0.0, 0.0])


def system(n, seed, m_tot=1e5, a_p=0.01):
    xi, _ = plummer_unit(n, seed)
    return W_X + a_p * xi, np.full(n, m_tot / n)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_noalloc_accelerations_match_the_context_path(prec):
    from paper_2511_22468_amd import _lib, engine
    lib = _lib.lib()
    op = OPot(eps=5e-4)
    pot = engine.Potential(eps=op.eps)
    ctx = engine.Context(65536, prec)
    tol_ctx = 2e-7 if prec == "fp32c" else 1e-13
    tol_ref = 1e-5 if prec == "fp32c" else 1e-12
    for n, seed in ((65536, 70), (3001, 71)):
        say(f"[noalloc] {prec} n = {n}")
        x, m = system(n, seed)
        px, pm = to_dev(x), to_dev(m)
        ref_ctx = to_host(ctx.accelerations(px, pm, pot))
        out = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda")
        st = lib.dnb_accelerations_noalloc(n, _lib.ptr(px), _lib.ptr(pm), pot.c(), 1,
                                           _lib.PRECISIONS[prec], _lib.ptr(out),
                                           _lib.stream_handle())
        assert st == _lib.DNB_OK, lib.dnb_last_error()
        got = to_host(out)
        assert np.isfinite(got).all()
        d = rel_rows(got, ref_ctx)
        rows = sample_rows(n, 256, seed + 10)
        ref = of.pair_accel(x, m, G, op.eps, rows=rows) + of.ext_accel(x[rows], op)
        e = rel_rows(got[rows], ref)
        say(f"  vs dnb_accelerations: max {d.max():.2e}; vs oracle (256 rows): max {e.max():.2e}")
        assert d.max() <= tol_ctx
        assert e.max() <= tol_ref
    ctx.close()


def test_noalloc_refuses_sizes_beyond_its_array():
    from paper_2511_22468_amd import _lib, engine
    lib = _lib.lib()
    n = 65537
    x = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    m = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty(3, n, dtype=torch.float64, device="cuda")
    pot = engine.Potential()
    st = lib.dnb_accelerations_noalloc(n, _lib.ptr(x), _lib.ptr(m), pot.c(), 1, 1,
                                       _lib.ptr(out), _lib.stream_handle())
    assert st == _lib.DNB_ERR_ARG
    assert b"DNB_NOALLOC_MAX_N" in lib.dnb_last_error()
    with pytest.raises(_lib.DnbError):
        engine.accelerations_noalloc(x, m, pot)
