"""Accelerations and potentials of the oracle (test infrastructure only).

Sec. 1 ("N-body codes") states that the method sums pairwise forces directly,
with softening and without a tree or multipole expansion, so that forces are
exact up to the softening scale.  The paper does not print the softening
kernel; the reading taken is Plummer softening:

    a_i = G sum_{j != i} m_j d_ij (|d_ij|^2 + eps^2)^(-3/2),   d_ij = x_j - x_i.

The host galaxy (Sec. 2.2.1) is an NFW halo plus a Miyamoto-Nagai disk.  The
paper gives only the masses as inference parameters; the potentials are the
textbook ones:

    NFW:  Phi = -G M ln(1 + r/rs) / r, with M the scale mass 4 pi rho0 rs^3,
    MN:   Phi = -G M / sqrt(R^2 + (a + sqrt(z^2 + b^2))^2).

All functions accept arrays of any floating or complex dtype and never take
absolute values, so complex-step differentiation goes through them.
Positions are arrays of shape (N, 3).
"""
from dataclasses import dataclass

import numpy as np

from . import constants as C


@dataclass(frozen=True)
class Potential:
    """Softening and host-potential parameters.  A zero mass disables a term."""
    G: float = C.G
    eps: float = 1.0e-3
    m_nfw: float = C.M_NFW
    rs_nfw: float = C.RS_NFW
    m_mn: float = C.M_MN
    a_mn: float = C.A_MN
    b_mn: float = C.B_MN

    def replace(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Potential(**d)


def _real(x):
    return np.real(x) if np.iscomplexobj(x) else x


# ---------------------------------------------------------------- pair sum --

def pair_accel(pos, mass, G, eps, rows=None, block=256):
    """Softened direct-sum acceleration (Sec. 1, direct pairwise forces).

    pos: (N, 3); mass: (N,).  rows: optional index array; if given only those
    particles' accelerations are returned (still summed over all N sources).
    The sum runs over j in index order for blocks of 256 targets.  With
    eps == 0 the self term j == i is masked out explicitly; with eps > 0 it is
    exactly zero because d_ii = 0.
    """
    pos = np.asarray(pos)
    mass = np.asarray(mass)
    n = pos.shape[0]
    idx = np.arange(n) if rows is None else np.asarray(rows)
    out = np.zeros((idx.shape[0], 3), dtype=np.result_type(pos, mass, float))
    eps2 = eps * eps
    for b0 in range(0, idx.shape[0], block):
        ii = idx[b0:b0 + block]
        d = pos[None, :, :] - pos[ii, None, :]          # (B, N, 3) = x_j - x_i
        s = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2] + eps2
        if eps2 == 0:
            s = s.copy()
            s[np.arange(ii.shape[0]), ii] = 1.0          # masked below
        w = mass[None, :] * s ** -1.5
        if eps2 == 0:
            w[np.arange(ii.shape[0]), ii] = 0.0
        out[b0:b0 + block] = G * np.einsum("bj,bjk->bk", w, d)
    return out


def pair_potential_energy(pos, mass, G, eps, block=256):
    """W_int = -G sum_{i<j} m_i m_j (r_ij^2 + eps^2)^(-1/2)."""
    pos = np.asarray(pos)
    mass = np.asarray(mass)
    n = pos.shape[0]
    total = np.zeros((), dtype=np.result_type(pos, mass, float))
    for b0 in range(0, n, block):
        ii = np.arange(b0, min(n, b0 + block))
        d = pos[None, :, :] - pos[ii, None, :]
        s = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2] + eps * eps
        s = np.where(np.arange(n)[None, :] > ii[:, None], s, 1.0)
        inv = np.where(np.arange(n)[None, :] > ii[:, None], s ** -0.5, 0.0)
        total = total + np.sum(mass[ii, None] * mass[None, :] * inv)
    return -G * total


# ---------------------------------------------------------------- NFW halo --

def _nfw_mu(x):
    """mu(x) = ln(1+x) - x/(1+x), with its Taylor series for x < 1e-4."""
    x = np.asarray(x)
    small = _real(x) < 1e-4
    xs = np.where(small, x, 0.0)
    series = xs * xs * (0.5 + xs * (-2.0 / 3.0 + xs * (0.75 - xs * 0.8)))
    xl = np.where(small, 1.0, x)
    closed = np.log1p(xl) - xl / (1.0 + xl)
    return np.where(small, series, closed)


def nfw_potential(pos, G, M, rs):
    pos = np.asarray(pos)
    r = np.sqrt(pos[:, 0] ** 2 + pos[:, 1] ** 2 + pos[:, 2] ** 2)
    x = r / rs
    small = _real(x) < 1e-8
    rr = np.where(small, 1.0, r)
    return np.where(small, -G * M / rs, -G * M * np.log1p(rr / rs) / rr)


def nfw_accel(pos, G, M, rs):
    """a = -G M mu(r/rs) r_vec / r^3; zero at r = 0."""
    pos = np.asarray(pos)
    r2 = pos[:, 0] ** 2 + pos[:, 1] ** 2 + pos[:, 2] ** 2
    zero = _real(r2) == 0
    r = np.sqrt(np.where(zero, 1.0, r2))
    g = np.where(zero, 0.0, G * M * _nfw_mu(r / rs) / (r * r * r))
    return -g[:, None] * pos


def nfw_hvp(pos, w, G, M, rs):
    """Jacobian of the NFW acceleration applied to w (the Hessian is symmetric).

    With a = -g(r) r_vec, g = G M mu(r/rs)/r^3:
        da/dx = -g I - (g'(r)/r) r_vec r_vec^T,
        g'(r) = G M [1/(r^2 (r+rs)^2) - 3 mu/r^4].
    """
    pos = np.asarray(pos)
    w = np.asarray(w)
    r2 = pos[:, 0] ** 2 + pos[:, 1] ** 2 + pos[:, 2] ** 2
    r = np.sqrt(r2)
    mu = _nfw_mu(r / rs)
    g = G * M * mu / (r2 * r)
    gp = G * M * (1.0 / (r2 * (r + rs) ** 2) - 3.0 * mu / (r2 * r2))
    xw = pos[:, 0] * w[:, 0] + pos[:, 1] * w[:, 1] + pos[:, 2] * w[:, 2]
    return -g[:, None] * w - (gp / r * xw)[:, None] * pos


def nfw_accel_drs(pos, G, M, rs):
    """Derivative of the NFW acceleration with respect to the scale radius.

    With x = r/rs, mu'(x) = x/(1+x)^2 and dx/drs = -x/rs,
        da/drs = -G M mu'(x) (-x/rs) r_vec / r^3 = G M x^2 / ((1+x)^2 rs) r_vec / r^3;
    zero at r = 0.
    """
    pos = np.asarray(pos)
    r2 = pos[:, 0] ** 2 + pos[:, 1] ** 2 + pos[:, 2] ** 2
    zero = _real(r2) == 0
    r = np.sqrt(np.where(zero, 1.0, r2))
    x = r / rs
    f = np.where(zero, 0.0, G * M * x * x / ((1.0 + x) ** 2 * rs) / (r * r * r))
    return f[:, None] * pos


# ------------------------------------------------------- Miyamoto-Nagai ----

def mn_potential(pos, G, M, a, b):
    pos = np.asarray(pos)
    S = np.sqrt(pos[:, 2] ** 2 + b * b)
    D = np.sqrt(pos[:, 0] ** 2 + pos[:, 1] ** 2 + (a + S) ** 2)
    return -G * M / D


def mn_accel(pos, G, M, a, b):
    """a = -grad Phi_MN.  With S = sqrt(z^2+b^2), D^2 = R^2 + (a+S)^2:
    a_x = -G M x/D^3, a_y = -G M y/D^3, a_z = -G M z (a+S)/(S D^3).
    For b = 0 the z-component is set to zero on the plane z = 0."""
    pos = np.asarray(pos)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    S = np.sqrt(z * z + b * b)
    D2 = x * x + y * y + (a + S) ** 2
    D3 = D2 * np.sqrt(D2)
    k = G * M / D3
    Ssafe = np.where(_real(S) == 0, 1.0, S)
    az = np.where(_real(S) == 0, 0.0, -k * z * (a + S) / Ssafe)
    return np.stack([-k * x, -k * y, az], axis=1)


def mn_accel_dab(pos, G, M, a, b):
    """Derivatives of the MN acceleration with respect to the scale lengths a and b.

    With S = sqrt(z^2+b^2), A = a+S, D^2 = R^2 + A^2, so that dD^2/da = 2A and
    dS/db = dA/db = b/S:
        da_x/da = 3 G M x A / D^5 (likewise y),
        da_z/da = -G M (z/S) (1/D^3 - 3 A^2/D^5),
        da_x/db = (b/S) da_x/da,
        da_z/db = -G M z [d(A/S)/db / D^3 - 3 (A/S) A (b/S) / D^5]
                = G M z b [a/(S^3 D^3) + 3 A^2/(S^2 D^5)]      (d(A/S)/db = -a b/S^3).
    Where S = 0 the z-derivatives and b/S are taken as zero, as mn_accel takes a_z.
    Returns (da/da, da/db), each (N, 3).
    """
    pos = np.asarray(pos)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    S = np.sqrt(z * z + b * b)
    A = a + S
    D2 = x * x + y * y + A * A
    D = np.sqrt(D2)
    D3 = D2 * D
    D5 = D3 * D2
    GM = G * M
    flat = _real(S) == 0
    Ss = np.where(flat, 1.0, S)
    dxa = 3.0 * GM * A / D5
    dza = np.where(flat, 0.0, -GM * (z / Ss) * (1.0 / D3 - 3.0 * A * A / D5))
    bS = np.where(flat, 0.0, b / Ss)
    dzb = np.where(flat, 0.0, GM * z * b * (a / (Ss ** 3 * D3) + 3.0 * A * A / (Ss * Ss * D5)))
    da = np.stack([dxa * x, dxa * y, dza], axis=1)
    db = np.stack([bS * dxa * x, bS * dxa * y, dzb], axis=1)
    return da, db


def mn_hvp(pos, w, G, M, a, b):
    """Jacobian of the MN acceleration applied to w (symmetric Hessian).

    With A = a + S:
      da_x/dx = -GM (1/D^3 - 3x^2/D^5), da_x/dy = 3GM xy/D^5,
      da_x/dz = 3GM x z A/(S D^5), da_y/dz = 3GM y z A/(S D^5),
      da_z/dz = -GM ((1 + a b^2/S^3)/D^3 - 3 z^2 A^2/(S^2 D^5)).
    """
    pos = np.asarray(pos)
    w = np.asarray(w)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    S = np.sqrt(z * z + b * b)
    A = a + S
    D2 = x * x + y * y + A * A
    D = np.sqrt(D2)
    D3 = D2 * D
    D5 = D3 * D2
    GM = G * M
    hxx = -GM * (1.0 / D3 - 3.0 * x * x / D5)
    hyy = -GM * (1.0 / D3 - 3.0 * y * y / D5)
    hxy = 3.0 * GM * x * y / D5
    hxz = 3.0 * GM * x * z * A / (S * D5)
    hyz = 3.0 * GM * y * z * A / (S * D5)
    hzz = -GM * ((1.0 + a * b * b / (S * S * S)) / D3 - 3.0 * z * z * A * A / (S * S * D5))
    wx, wy, wz = w[:, 0], w[:, 1], w[:, 2]
    return np.stack([hxx * wx + hxy * wy + hxz * wz,
                     hxy * wx + hyy * wy + hyz * wz,
                     hxz * wx + hyz * wy + hzz * wz], axis=1)


# ---------------------------------------------------------------- totals ----

def ext_accel(pos, pot):
    pos = np.asarray(pos)
    a = np.zeros(pos.shape, dtype=np.result_type(pos, float))
    if pot.m_nfw != 0:
        a = a + nfw_accel(pos, pot.G, pot.m_nfw, pot.rs_nfw)
    if pot.m_mn != 0:
        a = a + mn_accel(pos, pot.G, pot.m_mn, pot.a_mn, pot.b_mn)
    return a


def ext_potential(pos, pot):
    pos = np.asarray(pos)
    phi = np.zeros(pos.shape[0], dtype=np.result_type(pos, float))
    if pot.m_nfw != 0:
        phi = phi + nfw_potential(pos, pot.G, pot.m_nfw, pot.rs_nfw)
    if pot.m_mn != 0:
        phi = phi + mn_potential(pos, pot.G, pot.m_mn, pot.a_mn, pot.b_mn)
    return phi


def ext_hvp(pos, w, pot):
    pos = np.asarray(pos)
    out = np.zeros(pos.shape, dtype=np.result_type(pos, w, float))
    if pot.m_nfw != 0:
        out = out + nfw_hvp(pos, w, pot.G, pot.m_nfw, pot.rs_nfw)
    if pot.m_mn != 0:
        out = out + mn_hvp(pos, w, pot.G, pot.m_mn, pot.a_mn, pot.b_mn)
    return out


def accel(pos, mass, pot, with_ext=True, self_gravity=True):
    """Total acceleration a = a_int + a_ext."""
    a = pair_accel(pos, mass, pot.G, pot.eps) if self_gravity else 0.0
    if with_ext:
        a = a + ext_accel(pos, pot)
    return a


def energies(pos, vel, mass, pot):
    """(K, W_int, W_ext): kinetic, pair and external potential energy."""
    pos = np.asarray(pos)
    vel = np.asarray(vel)
    K = 0.5 * np.sum(mass * (vel[:, 0] ** 2 + vel[:, 1] ** 2 + vel[:, 2] ** 2))
    W = pair_potential_energy(pos, mass, pot.G, pot.eps)
    X = np.sum(mass * ext_potential(pos, pot))
    return K, W, X
