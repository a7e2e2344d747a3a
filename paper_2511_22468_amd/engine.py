"""Python face of libdnb: one method per C entry point, same names and meaning.

Particle arrays are torch float64 CUDA tensors of shape (3, n) (structure of
arrays: row 0 holds x, row 1 y, row 2 z) or (n,); see include/dnb.h for the
definition of every operation.  All calls are asynchronous on the current torch
stream.
"""
import ctypes
from dataclasses import dataclass, replace as _dc_replace

import numpy as np
import torch

from . import _lib
from .units import G as G_DEFAULT


@dataclass(frozen=True)
class Potential:
    """Softening and host potential (NFW halo + Miyamoto-Nagai disk)."""
    G: float = G_DEFAULT
    eps: float = 1.0e-3
    m_nfw: float = 1.0e12
    rs_nfw: float = 16.0
    m_mn: float = 6.5e10
    a_mn: float = 3.0
    b_mn: float = 0.28

    def replace(self, **kw):
        return _dc_replace(self, **kw)

    def c(self):
        return _lib.dnb_pot(self.G, self.eps, self.m_nfw, self.rs_nfw, self.m_mn, self.a_mn,
                            self.b_mn)


def batch_table(pots, dts, B):
    """Host parameter table [B][8] = (G, eps, m_nfw, rs_nfw, m_mn, a_mn, b_mn, dt)."""
    pots, dts = list(pots), list(dts)
    if len(pots) != B or len(dts) != B:
        raise ValueError(f"need {B} potentials and {B} step sizes")
    return np.ascontiguousarray(
        [[p.G, p.eps, p.m_nfw, p.rs_nfw, p.m_mn, p.a_mn, p.b_mn, float(dt)]
         for p, dt in zip(pots, dts)], dtype=np.float64)


def _vec(t, n, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and tuple(t.shape) == (3, n)):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (3, {n})")
    return t


def _arr(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")
    return t


NOALLOC_MAX_N = 65536


def accelerations_noalloc(pos, mass, pot, with_ext=True, prec="fp32c", out=None):
    """dnb_accelerations_noalloc: the accelerations without a context or any
    device allocation in the library (n <= 65536; calls on one device must not
    overlap).  out (optional) receives them in place."""
    if prec not in _lib.PRECISIONS:
        raise ValueError(f"prec must be one of {list(_lib.PRECISIONS)}")
    n = mass.shape[0]
    _vec(pos, n, "pos"); _arr(mass, (n,), "mass")
    acc = torch.empty(3, n, dtype=torch.float64, device=pos.device) if out is None \
        else _vec(out, n, "out")
    _lib.check(_lib.lib().dnb_accelerations_noalloc(
        n, _lib.ptr(pos), _lib.ptr(mass), pot.c(), int(bool(with_ext)), _lib.PRECISIONS[prec],
        _lib.ptr(acc), _lib.stream_handle()))
    return acc


def _buffer(t, length, name):
    """A flat float64 CUDA buffer of at least `length` elements."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() < length:
        raise ValueError(f"{name} holds {t.numel()} doubles, {length} needed")
    return t


class Context:
    """Owns a dnb_ctx: device workspace for up to max_n particles."""

    def __init__(self, max_n, prec="fp32c", device=None):
        if prec not in _lib.PRECISIONS:
            raise ValueError(f"prec must be one of {list(_lib.PRECISIONS)}")
        self.prec = prec
        self.max_n = int(max_n)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = _lib.ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().dnb_create(_lib.ctypes.byref(self._h), self.max_n,
                                             _lib.PRECISIONS[prec]))

    def close(self):
        if self._h:
            _lib.lib().dnb_destroy(self._h)
            self._h = _lib.ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    # --------------------------------------------------- instrumentation --
    def profile(self, enable=True):
        """Bracket every O(N^2) kernel launch with HIP events (see dnb_profile)."""
        _lib.check(_lib.lib().dnb_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{'fwd_ms', 'fwd_launches', 'vjp_ms', 'vjp_launches'} since the last read."""
        out = (_lib.ctypes.c_double * 4)()
        _lib.check(_lib.lib().dnb_profile_read(self._h, out))
        return dict(fwd_ms=out[0], fwd_launches=int(out[1]), vjp_ms=out[2],
                    vjp_launches=int(out[3]))

    # ------------------------------------------------------------ forward --
    def accelerations(self, pos, mass, pot, with_ext=True, out=None):
        n = mass.shape[0]
        _vec(pos, n, "pos"); _arr(mass, (n,), "mass")
        acc = self._new(3, n) if out is None else _vec(out, n, "out")
        _lib.check(_lib.lib().dnb_accelerations(self._h, n, _lib.ptr(pos), _lib.ptr(mass),
                                                pot.c(), int(bool(with_ext)), _lib.ptr(acc),
                                                _lib.stream_handle()))
        return acc

    def accelerations_rows(self, pos, mass, pot, i_begin, i_count, with_ext=True):
        """Accelerations (3, i_count) of targets i_begin .. i_begin + i_count - 1
        against all n sources (one device's block of a target-split system)."""
        n = mass.shape[0]
        _vec(pos, n, "pos"); _arr(mass, (n,), "mass")
        acc = self._new(3, int(i_count))
        _lib.check(_lib.lib().dnb_accelerations_rows(
            self._h, n, _lib.ptr(pos), _lib.ptr(mass), pot.c(), int(bool(with_ext)),
            int(i_begin), int(i_count), _lib.ptr(acc), _lib.stream_handle()))
        return acc

    def accelerations_vjp(self, pos, mass, pot, w, with_ext=True, i_begin=0, i_count=None,
                          with_mass=True):
        """(gpos (3, i_count), gmass (i_count,) or None): the derivatives of
        sum_j w_j . a_j with respect to the positions and masses of targets
        i_begin .. i_begin + i_count - 1 (all n by default)."""
        n = mass.shape[0]
        _vec(pos, n, "pos"); _arr(mass, (n,), "mass"); _vec(w, n, "w")
        ni = n - int(i_begin) if i_count is None else int(i_count)
        g = self._new(3, ni)
        gm = self._new(ni) if with_mass else None
        _lib.check(_lib.lib().dnb_accelerations_vjp(
            self._h, n, _lib.ptr(pos), _lib.ptr(mass), pot.c(), int(bool(with_ext)),
            _lib.ptr(w), int(i_begin), ni, _lib.ptr(g), _lib.ptr(gm), _lib.stream_handle()))
        return g, gm

    def step(self, pos, vel, mass, pot, dt):
        n = mass.shape[0]
        _vec(pos, n, "pos"); _vec(vel, n, "vel"); _arr(mass, (n,), "mass")
        _lib.check(_lib.lib().dnb_step(self._h, n, _lib.ptr(pos), _lib.ptr(vel), _lib.ptr(mass),
                                       pot.c(), float(dt), _lib.stream_handle()))

    def tape_len(self, n, n_steps, ckpt_every):
        return int(_lib.lib().dnb_tape_doubles(n, n_steps, ckpt_every))

    def simulate(self, pos, vel, mass, pot, dt, n_steps, ckpt_every=0, tape=None):
        """In-place integration.  With ckpt_every > 0 a tape is written (and returned)."""
        n = mass.shape[0]
        _vec(pos, n, "pos"); _vec(vel, n, "vel"); _arr(mass, (n,), "mass")
        K = int(ckpt_every)
        if K > 0 and tape is None:
            tape = self._new(max(1, self.tape_len(n, n_steps, K)))
        _lib.check(_lib.lib().dnb_simulate(self._h, n, _lib.ptr(pos), _lib.ptr(vel),
                                           _lib.ptr(mass), pot.c(), float(dt), int(n_steps),
                                           max(K, 1), _lib.ptr(tape) if K > 0 else None,
                                           _lib.stream_handle()))
        return tape

    def check_state(self, pos, vel=None, mass=None):
        """Index of the first particle with a NaN or infinite position, velocity
        or mass, or -1 (waits for the stream)."""
        n = pos.shape[1]
        _vec(pos, n, "pos")
        if vel is not None:
            _vec(vel, n, "vel")
        if mass is not None:
            _arr(mass, (n,), "mass")
        out = ctypes.c_int64(-2)
        _lib.check(_lib.lib().dnb_check_state(
            self._h, n, _lib.ptr(pos), _lib.ptr(vel) if vel is not None else None,
            _lib.ptr(mass) if mass is not None else None, ctypes.byref(out),
            _lib.stream_handle()))
        return int(out.value)

    def set_checks(self, on=True):
        """With checks on, the integrators refuse a non-finite initial state."""
        _lib.check(_lib.lib().dnb_set_checks(self._h, 1 if on else 0))

    def simulate_resume(self, tape, tape_steps, tape_ckpt_every, ckpt, pos, vel, mass, pot, dt,
                        n_steps, ckpt_every=0, tape_out=None):
        """pos, vel <- checkpoint ckpt of tape (written for tape_steps, tape_ckpt_every),
        then n_steps further steps, continuing the source run bit for bit.  With
        ckpt_every > 0 the continuation's tape is written (and returned)."""
        n = mass.shape[0]
        _vec(pos, n, "pos"); _vec(vel, n, "vel"); _arr(mass, (n,), "mass")
        _buffer(tape, self.tape_len(n, tape_steps, tape_ckpt_every), "tape")
        K = int(ckpt_every)
        if K > 0 and tape_out is None:
            tape_out = self._new(max(1, self.tape_len(n, n_steps, K)))
        if K > 0:
            _buffer(tape_out, self.tape_len(n, n_steps, K), "tape_out")
        _lib.check(_lib.lib().dnb_simulate_resume(
            self._h, n, _lib.ptr(tape), int(tape_steps), int(tape_ckpt_every), int(ckpt),
            _lib.ptr(pos), _lib.ptr(vel), _lib.ptr(mass), pot.c(), float(dt), int(n_steps),
            max(K, 1), _lib.ptr(tape_out) if K > 0 else None, _lib.stream_handle()))
        return tape_out

    def simulate_vjp(self, mass, pot, dt, n_steps, ckpt_every, tape, pos_T, gpos_T, gvel_T=None,
                     with_mass=False, workspace=None, vel_T=None):
        """Returns (gpos_0, gvel_0, gmass or None, gparams[7]) with gparams =
        (dL/dm_nfw, dL/dm_mn, dL/ddt, sum_k m_k dL/dm_k, dL/drs_nfw, dL/da_mn,
        dL/db_mn).  With vel_T (the final velocities of the forward run) the
        sweep rebuilds the trajectory between checkpoints by stepping it backward
        (dnb_simulate_vjp_reversed); without, it recomputes it forward
        (dnb_simulate_vjp)."""
        n = mass.shape[0]
        _arr(mass, (n,), "mass"); _vec(pos_T, n, "pos_T"); _vec(gpos_T, n, "gpos_T")
        if gvel_T is not None:
            _vec(gvel_T, n, "gvel_T")
        if vel_T is not None:
            _vec(vel_T, n, "vel_T")
        K = int(ckpt_every)
        if vel_T is None:
            ws_len = int(_lib.lib().dnb_vjp_workspace_doubles(n, K))
        else:
            ws_len = int(_lib.lib().dnb_vjp_reversed_workspace_doubles(n))
        if workspace is None:
            workspace = self._new(ws_len)
        _buffer(workspace, ws_len, "workspace")
        if int(n_steps) > 0:
            _buffer(tape, self.tape_len(n, n_steps, K), "tape")
        gpos0, gvel0 = self._new(3, n), self._new(3, n)
        gmass = self._new(n) if with_mass else None
        gpar = self._new(7)
        head = (self._h, n, _lib.ptr(mass), pot.c(), float(dt), int(n_steps), K, _lib.ptr(tape),
                _lib.ptr(pos_T))
        tail = (_lib.ptr(gpos_T), _lib.ptr(gvel_T), _lib.ptr(workspace), _lib.ptr(gpos0),
                _lib.ptr(gvel0), _lib.ptr(gmass), _lib.ptr(gpar), _lib.stream_handle())
        if vel_T is None:
            _lib.check(_lib.lib().dnb_simulate_vjp(*head, *tail))
        else:
            _lib.check(_lib.lib().dnb_simulate_vjp_reversed(*head, _lib.ptr(vel_T), *tail))
        return gpos0, gvel0, gmass, gpar

    # --------------------------------------------------------------- loss --
    def mmd(self, pos, tgt, h, grad=True):
        n, m = pos.shape[1], tgt.shape[1]
        _vec(pos, n, "pos"); _vec(tgt, m, "tgt")
        loss = self._new(1)
        g = self._new(3, n) if grad else None
        _lib.check(_lib.lib().dnb_mmd(self._h, n, _lib.ptr(pos), m, _lib.ptr(tgt), float(h),
                                      _lib.ptr(loss), _lib.ptr(g), _lib.stream_handle()))
        return loss, g

    def energy(self, pos, vel, mass, pot):
        n = mass.shape[0]
        _vec(pos, n, "pos"); _vec(vel, n, "vel"); _arr(mass, (n,), "mass")
        out = self._new(3)
        _lib.check(_lib.lib().dnb_energy(self._h, n, _lib.ptr(pos), _lib.ptr(vel), _lib.ptr(mass),
                                         pot.c(), _lib.ptr(out), _lib.stream_handle()))
        return out

    # -------------------------------------------------------- progenitor --
    def orbit(self, w0, pot, dt, n_steps, keep=True):
        _arr(w0, (6,), "w0")
        w_out = self._new(6)
        traj = self._new(n_steps + 1, 3) if keep else None
        _lib.check(_lib.lib().dnb_orbit(self._h, _lib.ptr(w0), pot.c(), float(dt), int(n_steps),
                                        _lib.ptr(w_out), _lib.ptr(traj), _lib.stream_handle()))
        return w_out, traj

    def orbit_vjp(self, traj, pot, dt, n_steps, gw_out):
        _arr(traj, (n_steps + 1, 3), "traj"); _arr(gw_out, (6,), "gw_out")
        gw0, gpar = self._new(6), self._new(3)
        _lib.check(_lib.lib().dnb_orbit_vjp(self._h, _lib.ptr(traj), pot.c(), float(dt),
                                            int(n_steps), _lib.ptr(gw_out), _lib.ptr(gw0),
                                            _lib.ptr(gpar), _lib.stream_handle()))
        return gw0, gpar

    def simulate_batch(self, pos, vel, mass, pots, dts, n_steps, tape=False):
        """In-place integration of an ensemble: pos, vel (B, 3, n), mass (B, n),
        pots a sequence of B Potential, dts a sequence of B step sizes.  With
        tape=True every step is recorded and the tape returned (for
        simulate_batch_vjp)."""
        B, n = mass.shape
        _arr(pos, (B, 3, n), "pos"); _arr(vel, (B, 3, n), "vel"); _arr(mass, (B, n), "mass")
        table = batch_table(pots, dts, B)
        t = None
        if tape and n_steps > 0:
            t = self._new(int(_lib.lib().dnb_batch_tape_doubles(B, n, int(n_steps))))
        _lib.check(_lib.lib().dnb_simulate_batch(
            self._h, B, n, _lib.ptr(pos), _lib.ptr(vel), _lib.ptr(mass),
            table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n_steps), _lib.ptr(t),
            _lib.stream_handle()))
        return t

    def simulate_batch_vjp(self, mass, pots, dts, n_steps, tape, pos_T, gpos_T, gvel_T=None):
        """Returns (gpos_0 (B, 3, n), gvel_0 (B, 3, n), gparams (B, 4)) with gparams[b] =
        (dL/dm_nfw, dL/dm_mn, dL/ddt, sum_k m_k dL/dm_k) of member b."""
        B, n = mass.shape
        _arr(mass, (B, n), "mass"); _arr(pos_T, (B, 3, n), "pos_T")
        _arr(gpos_T, (B, 3, n), "gpos_T")
        if gvel_T is not None:
            _arr(gvel_T, (B, 3, n), "gvel_T")
        table = batch_table(pots, dts, B)
        _buffer(tape, int(_lib.lib().dnb_batch_tape_doubles(B, n, int(n_steps))), "tape")
        work = self._new(4 * B * n)
        g0, gv0, gpar = self._new(B, 3, n), self._new(B, 3, n), self._new(B, 4)
        _lib.check(_lib.lib().dnb_simulate_batch_vjp(
            self._h, B, n, _lib.ptr(mass), table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            int(n_steps), _lib.ptr(tape), _lib.ptr(pos_T), _lib.ptr(gpos_T), _lib.ptr(gvel_T),
            _lib.ptr(work), _lib.ptr(g0), _lib.ptr(gv0), _lib.ptr(gpar), _lib.stream_handle()))
        return g0, gv0, gpar

    def _mmd_batch(self, pos, tgt, h, grad):
        B, n, m = pos.shape[0], pos.shape[2], tgt.shape[-1]
        _arr(pos, (B, 3, n), "pos")
        per = tgt.dim() == 3
        if per:
            _arr(tgt, (B, 3, m), "tgt")
        else:
            _vec(tgt, m, "tgt")
        loss = self._new(B)
        g = self._new(B, 3, n) if grad else None
        _lib.check(_lib.lib().dnb_mmd_batch(self._h, B, n, _lib.ptr(pos), m, _lib.ptr(tgt),
                                            int(per), float(h), _lib.ptr(loss), _lib.ptr(g),
                                            _lib.stream_handle()))
        return loss, g

    def mmd_batch(self, pos, tgt, h):
        """Loss of each member pos[b] (B, 3, n) against tgt: one target (3, m) for
        all members, or tgt[b] (B, 3, m) for member b.  A (B,) tensor."""
        return self._mmd_batch(pos, tgt, h, False)[0]

    def mmd_batch_targets(self, pos, tgts, h):
        """Loss of every member pos[b] (B, 3, n) against every target tgts[t]
        (T, 3, m): a (B, T) tensor."""
        B, n, T, m = pos.shape[0], pos.shape[2], tgts.shape[0], tgts.shape[2]
        _arr(pos, (B, 3, n), "pos"); _arr(tgts, (T, 3, m), "tgts")
        loss = self._new(B, T)
        _lib.check(_lib.lib().dnb_mmd_batch_targets(self._h, B, n, _lib.ptr(pos), T, m,
                                                    _lib.ptr(tgts), float(h), _lib.ptr(loss),
                                                    _lib.stream_handle()))
        return loss

    def mmd_batch_grad(self, pos, tgt, h):
        """Losses (B,) and their gradients (B, 3, n) for every member pos[b]
        (targets as in mmd_batch)."""
        return self._mmd_batch(pos, tgt, h, True)

    def place_plummer_batch(self, w, xi, zeta, m_tot, a_p, G=G_DEFAULT):
        """Plummer spheres at w (B, 6) with masses m_tot (B,), shared unit samples
        xi, zeta (3, n): (pos (B, 3, n), vel (B, 3, n), mass (B, n))."""
        B, n = w.shape[0], xi.shape[1]
        _arr(w, (B, 6), "w"); _vec(xi, n, "xi"); _vec(zeta, n, "zeta"); _arr(m_tot, (B,), "m_tot")
        pos, vel, mass = self._new(B, 3, n), self._new(B, 3, n), self._new(B, n)
        _lib.check(_lib.lib().dnb_place_plummer_batch(
            self._h, B, n, _lib.ptr(w), _lib.ptr(xi), _lib.ptr(zeta), _lib.ptr(m_tot),
            float(a_p), float(G), _lib.ptr(pos), _lib.ptr(vel), _lib.ptr(mass),
            _lib.stream_handle()))
        return pos, vel, mass

    def batch_capacity(self, n):
        """Largest ensemble of n-particle systems that simulate_batch accepts."""
        return int(_lib.lib().dnb_batch_capacity(self._h, int(n)))

    def orbit_batch(self, w0, pots, dts, n_steps, keep=False):
        """Test-particle orbits w0 (B, 6) -> w_out (B, 6), member b in pots[b] with
        dts[b]; with keep=True also the positions (B, n_steps + 1, 3) for orbit_batch_vjp."""
        B = w0.shape[0]
        _arr(w0, (B, 6), "w0")
        table = batch_table(pots, dts, B)
        w_out = self._new(B, 6)
        traj = self._new(B, int(n_steps) + 1, 3) if keep else None
        _lib.check(_lib.lib().dnb_orbit_batch(
            self._h, B, _lib.ptr(w0), table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            int(n_steps), _lib.ptr(w_out), _lib.ptr(traj), _lib.stream_handle()))
        return (w_out, traj) if keep else w_out

    def orbit_batch_vjp(self, traj, pots, dts, n_steps, gw_out):
        """(gw0 (B, 6), gparams (B, 3) = dL/dm_nfw, dL/dm_mn, dL/ddt) per member."""
        B = traj.shape[0]
        _arr(traj, (B, int(n_steps) + 1, 3), "traj"); _arr(gw_out, (B, 6), "gw_out")
        table = batch_table(pots, dts, B)
        gw0, gpar = self._new(B, 6), self._new(B, 3)
        _lib.check(_lib.lib().dnb_orbit_batch_vjp(
            self._h, B, _lib.ptr(traj), table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            int(n_steps), _lib.ptr(gw_out), _lib.ptr(gw0), _lib.ptr(gpar), _lib.stream_handle()))
        return gw0, gpar

    def place_plummer_batch_vjp(self, zeta, m_tot, a_p, gpos, gvel, G=G_DEFAULT):
        """(gw (B, 6), gm_tot (B,)) of the batched placement."""
        B, n = gpos.shape[0], zeta.shape[1]
        _vec(zeta, n, "zeta"); _arr(m_tot, (B,), "m_tot")
        _arr(gpos, (B, 3, n), "gpos"); _arr(gvel, (B, 3, n), "gvel")
        gw, gm = self._new(B, 6), self._new(B)
        _lib.check(_lib.lib().dnb_place_plummer_batch_vjp(
            self._h, B, n, _lib.ptr(zeta), _lib.ptr(m_tot), float(a_p), float(G), _lib.ptr(gpos),
            _lib.ptr(gvel), _lib.ptr(gw), _lib.ptr(gm), _lib.stream_handle()))
        return gw, gm

    def place_plummer(self, w, xi, zeta, m_tot, a_p, G=G_DEFAULT):
        n = xi.shape[1]
        _arr(w, (6,), "w"); _vec(xi, n, "xi"); _vec(zeta, n, "zeta")
        pos, vel, mass = self._new(3, n), self._new(3, n), self._new(n)
        _lib.check(_lib.lib().dnb_place_plummer(self._h, n, _lib.ptr(w), _lib.ptr(xi),
                                                _lib.ptr(zeta), float(m_tot), float(a_p), float(G),
                                                _lib.ptr(pos), _lib.ptr(vel), _lib.ptr(mass),
                                                _lib.stream_handle()))
        return pos, vel, mass

    def place_plummer_vjp(self, zeta, m_tot, a_p, gpos, gvel, gmass=None, G=G_DEFAULT):
        n = zeta.shape[1]
        _vec(zeta, n, "zeta"); _vec(gpos, n, "gpos"); _vec(gvel, n, "gvel")
        if gmass is not None:
            _arr(gmass, (n,), "gmass")
        gw, gm = self._new(6), self._new(1)
        _lib.check(_lib.lib().dnb_place_plummer_vjp(self._h, n, _lib.ptr(zeta), float(m_tot),
                                                    float(a_p), float(G), _lib.ptr(gpos),
                                                    _lib.ptr(gvel), _lib.ptr(gmass), _lib.ptr(gw),
                                                    _lib.ptr(gm), _lib.stream_handle()))
        return gw, gm
