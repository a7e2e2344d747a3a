"""Orbit fit of the progenitor with a chi-squared track likelihood, its
Levenberg-Marquardt minimisation and the Fisher matrix (Sec. 2.2.2) -- oracle.

Test infrastructure only: the product path never imports this module.

Model (Sec. 2.2.2).  Only the progenitor is evolved, as one test particle: it
starts at the present-day point w_now and is integrated forward and backward in
time for dt_total each way in the host potential (kick-drift-kick, n steps of
+-dt_total/n).  The free parameters are the five host-potential parameters
theta = (M_NFW, rs_NFW, M_MN, a_MN, b_MN), handled in dex: p = log10(theta).
M_NFW is the NFW scale mass, as everywhere in this code.

Observables.  The GD-1 frame and data of the paper are not available; the
orbit is projected onto the orbit-aligned frame fixed by w_now (e1 along x_now,
n along x_now x v_now, e2 = n x e1) and described by
    phi1 = longitude in the (e1, e2) plane, continuous along the orbit,
           phi1(t = 0) = 0 (x_now lies on e1),
    phi2 = asin(x . n / |x|)  [rad],
    d    = |x|                [kpc],
    v_r  = x . v / |x|        [km/s].
phi1 is accumulated step by step as the sum of the turning angles
atan(cross / dot) of consecutive projected positions, which equals the
unwrapped atan2 longitude while a step turns by less than 90 degrees.

Track.  Observed points (phi1_k; phi2_k, d_k, v_r,k) with fixed errors
(s_phi2, s_d, s_vr).  The model value at phi1_k is the linear interpolation
along phi1 between the two consecutive orbit points of the first segment, in
time order from t = 0, whose phi1 interval contains phi1_k: on the forward
branch for phi1_k >= 0, on the backward branch otherwise.  A point that no
segment reaches makes chi2 infinite.

    chi2(p) = sum_k sum_c ((y_c(phi1_k; p) - y_c,k) / s_c)^2.

Fisher matrix F = 1/2 d2 chi2 / dp dp (Sec. 2.2.2), covariance C = F^-1, both in
dex.  The chi2 is piecewise smooth in p (the bracketing segment of a track
point changes at isolated p); the Hessian here is the one within the current
segments.

All arithmetic accepts complex dtypes (no abs, no atan2 on the differentiated
path), so derivatives come from complex steps.
"""
import numpy as np

from . import forces
from .forces import Potential

PARAMS = ("m_nfw", "rs_nfw", "m_mn", "a_mn", "b_mn")
LN10 = np.log(10.0)


def frame(w_now):
    """Unit vectors (e1, e2, n) of the orbit-aligned frame of w_now."""
    x = np.asarray(w_now[:3], float)
    v = np.asarray(w_now[3:], float)
    n = np.cross(x, v)
    n = n / np.sqrt(n @ n)
    e1 = x / np.sqrt(x @ x)
    e2 = np.cross(n, e1)
    return e1, e2, n


def potential(p, G):
    """Host potential at p = log10(M_NFW, rs_NFW, M_MN, a_MN, b_MN)."""
    th = 10.0 ** np.asarray(p)
    return Potential(G=G, eps=0.0, m_nfw=th[0], rs_nfw=th[1], m_mn=th[2], a_mn=th[3],
                     b_mn=th[4])


def branch(w_now, pot, dt, n_steps):
    """Positions and velocities (n_steps + 1, 3) of one kick-drift-kick branch."""
    dtype = np.result_type(pot.m_nfw, pot.rs_nfw, pot.m_mn, pot.a_mn, pot.b_mn, float)
    x = np.array(w_now[:3], dtype=dtype)[None, :]
    v = np.array(w_now[3:], dtype=dtype)[None, :]
    X, V = [x[0].copy()], [v[0].copy()]
    a = forces.ext_accel(x, pot)
    for _ in range(n_steps):
        vh = v + (0.5 * dt) * a
        x = x + dt * vh
        a = forces.ext_accel(x, pot)
        v = vh + (0.5 * dt) * a
        X.append(x[0].copy())
        V.append(v[0].copy())
    return np.array(X), np.array(V)


def observables(X, V, fr):
    """(phi1, phi2, d, v_r) along a branch; phi1 accumulated from 0."""
    e1, e2, n = fr
    u, w = X @ e1, X @ e2
    cross = u[:-1] * w[1:] - w[:-1] * u[1:]
    dot = u[:-1] * u[1:] + w[:-1] * w[1:]
    phi1 = np.concatenate([np.zeros(1, dtype=cross.dtype), np.cumsum(np.arctan(cross / dot))])
    d = np.sqrt((X * X).sum(1))
    phi2 = np.arcsin((X @ n) / d)
    vr = (X * V).sum(1) / d
    return phi1, np.stack([phi2, d, vr], 1)


def bracket(phi1, target):
    """First s with target between phi1[s] and phi1[s+1] (real parts), or -1."""
    a, b = np.real(phi1[:-1]), np.real(phi1[1:])
    hit = (np.minimum(a, b) <= target) & (target <= np.maximum(a, b)) & (a != b)
    idx = np.flatnonzero(hit)
    return int(idx[0]) if idx.size else -1


def model_track(p, w_now, G, dt_total, n_steps, phi1_obs):
    """Model observables (K, 3) at the track longitudes and the bracketing
    segment of each point (its index, and the branch: +1 forward, -1 backward)."""
    pot = potential(p, G)
    dt = dt_total / n_steps
    fr = frame(w_now)
    out, seg = [], []
    cache = {}
    for phk in np.asarray(phi1_obs, float):
        sgn = 1 if phk >= 0 else -1
        if sgn not in cache:
            X, V = branch(w_now, pot, sgn * dt, n_steps)
            cache[sgn] = observables(X, V, fr)
        ph, Y = cache[sgn]
        s = bracket(ph, phk)
        seg.append((sgn, s))
        if s < 0:
            out.append(np.full(3, np.inf, dtype=Y.dtype))
            continue
        wgt = (phk - ph[s]) / (ph[s + 1] - ph[s])
        out.append(Y[s] + wgt * (Y[s + 1] - Y[s]))
    return np.array(out), seg


def residuals(p, track, sigma, w_now, G, dt_total, n_steps):
    """r_kc = (y_c(phi1_k) - y_c,k) / s_c, flattened (3K,); track is (K, 4)."""
    track = np.asarray(track, float)
    Y, _ = model_track(p, w_now, G, dt_total, n_steps, track[:, 0])
    return ((Y - track[:, 1:]) / np.asarray(sigma, float)).reshape(-1)


def chi2(p, track, sigma, w_now, G, dt_total, n_steps):
    r = residuals(p, track, sigma, w_now, G, dt_total, n_steps)
    return np.sum(r * r)


def jacobian(p, track, sigma, w_now, G, dt_total, n_steps, h=1e-20):
    """(r, J): residuals and dr/dp by complex steps (exact to rounding)."""
    p = np.asarray(p, float)
    r = residuals(p, track, sigma, w_now, G, dt_total, n_steps)
    J = np.empty((r.size, p.size))
    for i in range(p.size):
        pc = p.astype(complex)
        pc[i] += 1j * h
        J[:, i] = np.imag(residuals(pc, track, sigma, w_now, G, dt_total, n_steps)) / h
    return r, J


def gradient(p, *args):
    r, J = jacobian(p, *args)
    return 2.0 * J.T @ r


def hessian(p, track, sigma, w_now, G, dt_total, n_steps, h=2e-5):
    """d2 chi2 / dp dp within the current segments: central differences of the
    complex-step gradient with one Richardson extrapolation (steps h and h/2).
    Raises if a track point changes segment inside the stencil."""
    p = np.asarray(p, float)
    args = (track, sigma, w_now, G, dt_total, n_steps)
    seg0 = model_track(p, w_now, G, dt_total, n_steps, np.asarray(track)[:, 0])[1]
    H = np.empty((p.size, p.size))
    for j in range(p.size):
        cols = []
        for hh in (h, 0.5 * h):
            e = np.zeros(p.size)
            e[j] = hh
            for q in (p + e, p - e):
                if model_track(q, w_now, G, dt_total, n_steps, np.asarray(track)[:, 0])[1] != seg0:
                    raise ValueError("a track point changes segment inside the stencil")
            cols.append((gradient(p + e, *args) - gradient(p - e, *args)) / (2.0 * hh))
        H[:, j] = (4.0 * cols[1] - cols[0]) / 3.0
    return 0.5 * (H + H.T)


def fisher(H):
    """F = H / 2 and its inverse, the covariance (dex^2)."""
    F = 0.5 * np.asarray(H)
    return F, np.linalg.inv(F)


def levenberg_marquardt(p0, track, sigma, w_now, G, dt_total, n_steps, n_iter=20, lam0=1e-3):
    """Textbook Levenberg-Marquardt on chi2 = |r|^2 with Marquardt's diagonal
    scaling: solve (J^T J + lam diag(J^T J)) delta = -J^T r, accept the step if
    chi2 decreases (lam /= 10), else reject it (lam *= 10).  Returns (p, chi2)."""
    args = (track, sigma, w_now, G, dt_total, n_steps)
    p = np.asarray(p0, float).copy()
    r, J = jacobian(p, *args)
    c = float(np.sum(r * r))
    lam = lam0
    for _ in range(n_iter):
        A = J.T @ J
        A = A + lam * np.diag(np.diag(A))
        try:
            delta = np.linalg.solve(A, -(J.T @ r))
        except np.linalg.LinAlgError:
            lam *= 10.0
            continue
        pt = p + delta
        rt, Jt = jacobian(pt, *args)
        ct = float(np.sum(rt * rt))
        if ct < c:
            p, r, J, c = pt, rt, Jt, ct
            lam = max(lam / 10.0, 1e-12)
        else:
            lam = min(lam * 10.0, 1e16)
    return p, c
