#!/usr/bin/env python3
"""Benchmark of the differentiable direct N-body hot path on one MI355X.

One step is one full pass of the method at the large-N workload: back-integrate
the progenitor's centre of mass for t_end in the NFW + Miyamoto-Nagai host,
place an N = 65536 Plummer sphere (1e5 Msun, scale 0.01 kpc) there, run 1000
kick-drift-kick steps of 0.5 Myr with softening 5e-4 kpc (FP32 compensated pair
terms, FP64 drift) while recording the tape, evaluate the MMD against a
4096-point target stream, and run the full reverse sweep back to the four
parameters (t_end, M_Plummer, M_NFW, M_MN).

value = (forward pair interactions + adjoint pair interactions) / step time,
with (T + 1) N^2 pairs each per step.  The roofline object reports the
dominant kernel (the pair VJP) and its forward sibling, timed with HIP events
around every launch inside the timed region; cpu_baseline times the FP64 NumPy
oracle on a bounded subsample of the same pair work on the host's cores.
time_to_fit carries the metric's second half, outside the timed region: the
surrogate-warm-started fit against plain N-body gradient descent on five held-out
targets (fit N = 8192, 4000 steps; one surrogate per training set of 512 runs of
N = 4096 with 4000 or 1000 steps, trained once for all targets), both arms
descending to convergence; the plain fit's duration against the time the warm
arm takes to reach the plain fit's final loss.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline]
                       [--no-time-to-fit]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s fwd & adjoint at N=65536; time-to-fit vs plain N-body"
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak
FLOPS_FWD = 20                    # per pair interaction, conventional count
FLOPS_VJP = 41                    # per pair of the vector-Jacobian product
# What the equal-mass path the benchmark takes executes per pair, by the same
# counting (the mass is applied once per target instead of once per pair), and
# what the hardware's FP32 instruction counters count per pair for that path
# (profiles/pair_kernels_n65536_flops.md, same kernel sources as the traffic key).
FLOPS_FWD_EXEC, FLOPS_VJP_EXEC = 18, 35
FLOPS_COUNTED = {"k_pair_fwd_f32c": 18.2, "k_pair_vjp_f32c": 34.2,
                 "k_pair_vjp_f32c+force": 40.4}
# The pair launch of the sweep that steps the trajectory backward sums the VJP
# and the acceleration together: the VJP's count plus three FMA per pair.
FLOPS_VJP_FORCE, FLOPS_VJP_FORCE_EXEC = FLOPS_VJP + 6, FLOPS_VJP_EXEC + 6

# HBM bytes per launch from the two rocprofv3 counter passes recorded in
# profiles/pair_kernels_n65536_traffic.md (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, the
# factors measured on a 256 MiB copy), valid only for the kernel source they were
# measured on (sha256 prefix of pair.hip, pair_common.h and host_logic.h) and for
# N = 65536.
TRAFFIC_SRC_SHA = "6365a8ba9647dfaf"
TRAFFIC_N = 65536
TRAFFIC_KIB = {"k_pair_fwd_f32c": (4565.6, 98304.0), "k_pair_vjp_f32c": (9116.7, 98304.0),
               "k_pair_vjp_f32c+force": (9135.6, 196608.0)}
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


class ClockSampler:
    """Samples the GPU's current shader clock from sysfs (the level marked '*'
    in pp_dpm_sclk of the first card that has one) every `period` seconds in a
    background thread, so that the timed region's clock is recorded beside its
    result.  Reads a file only; reports None where the file is not readable."""

    def __init__(self, period=0.2):
        import glob
        import threading
        paths = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
        self.path = paths[0] if paths else None
        self.period, self.samples = period, []
        self._stop = threading.Event()
        self._thread = threading.Thread(target=self._run, daemon=True)

    def _read(self):
        try:
            with open(self.path) as f:
                for line in f:
                    if line.rstrip().endswith("*"):
                        return float(line.split(":")[1].strip().split("Mhz")[0].split("MHz")[0])
        except (OSError, ValueError, IndexError):
            return None
        return None

    def __enter__(self):
        if self.path:
            self._thread.start()
        return self

    def _run(self):
        while not self._stop.is_set():
            v = self._read()
            if v is not None:
                self.samples.append(v)
            self._stop.wait(self.period)

    def __exit__(self, *exc):
        self._stop.set()
        if self.path:
            self._thread.join()

    def summary(self):
        if not self.samples:
            return None
        v = sorted(self.samples)
        return {"source": self.path, "samples": len(v), "min": v[0], "median": v[len(v) // 2],
                "max": v[-1]}


def kernel_source_sha():
    """sha256 prefix of the pair-kernel sources and their launch geometry (pair.hip,
    pair_common.h, then host_logic.h)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("pair.hip", "pair_common.h", "host_logic.h"):
        with open(os.path.join(ROOT, "paper_2511_22468_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n):
    sha = kernel_source_sha()
    if sha != TRAFFIC_SRC_SHA or n != TRAFFIC_N or kernel not in TRAFFIC_KIB:
        return None
    fetch, write = TRAFFIC_KIB[kernel]
    return (fetch * FETCH_FACTOR + write * WRITE_FACTOR) * 1024.0


def cpu_baseline(n, t_end_steps, seed):
    """Time the oracle's pair sum (every target row) and pair VJP (a sample of
    24576 target rows) against all n sources on the host's cores (at most 16, the
    CPU share of one GPU's host): about 10-12 s at n = 65536.  Then the same on one
    thread for a smaller sample (2048 and 512 rows, about 4 s)."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from oracle import adjoint as oadj, forces as of
    from synth import plummer_unit, random_directions, sample_rows

    G = 4.3009e-6
    xi, _ = plummer_unit(n, seed)
    x = np.array([12.0, 0.0, 0.0]) + 0.01 * xi
    m = np.full(n, 1e5 / n)
    w = random_directions(n, seed + 1)
    cores = min(len(os.sched_getaffinity(0)), 16)
    rows_f = np.arange(n)
    rows_v = sample_rows(n, min(n, 24576), seed + 3)

    def run(fn, rows):
        chunks = np.array_split(rows, cores * 2)
        with threadpool_limits(1), ThreadPoolExecutor(cores) as ex:
            t0 = time.perf_counter()
            list(ex.map(fn, chunks))
            return time.perf_counter() - t0

    tf = run(lambda r: of.pair_accel(x, m, G, 5e-4, rows=r), rows_f)
    tv = run(lambda r: oadj.pair_vjp(x, m, G, 5e-4, w, rows=r), rows_v)
    pairs = (rows_f.size + rows_v.size) * n
    # rate for the same fwd:adjoint mix as the GPU step (one forward and one VJP per pair)
    rate = 2.0 / (tf / (rows_f.size * n) + tv / (rows_v.size * n))
    r1f, r1v = sample_rows(n, 2048, seed + 4), sample_rows(n, 512, seed + 5)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        of.pair_accel(x, m, G, 5e-4, rows=r1f)
        t1f = time.perf_counter() - t0
        t0 = time.perf_counter()
        oadj.pair_vjp(x, m, G, 5e-4, w, rows=r1v)
        t1v = time.perf_counter() - t0
    rate1 = 2.0 / (t1f / (r1f.size * n) + t1v / (r1v.size * n))
    return {
        "value": rate, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
        "one_core": {"value": rate1, "sample": f"{r1f.size} pair-sum and {r1v.size} pair-VJP "
                     f"target rows x {n} sources on one thread ({t1f:.2f} + {t1v:.2f} s)"},
        "sample": (f"FP64 NumPy oracle on the N={n} initial Plummer state: pair sum for "
                   f"all {rows_f.size} targets x {n} sources ({tf:.2f} s) and pair VJP for "
                   f"{rows_v.size} targets x {n} sources ({tv:.2f} s), {pairs:.3g} pairs in "
                   f"{cores} threads; rate is the harmonic mix of one forward and one adjoint "
                   f"pair per interaction pair"),
    }


def sweep(prec, sizes=(1024, 4096, 8192, 16384, 65536), reps=20):
    """Average launch time of the two O(N^2) kernels at each size (HIP events around
    every launch), on a Plummer sphere placed at the present-day point."""
    import torch

    from paper_2511_22468_amd import engine, myr
    from synth import plummer_unit, random_directions

    dev = torch.device("cuda", 0)
    G = 4.3009e-6
    rows = []
    for n in sizes:
        xi, zeta = plummer_unit(n, 7)
        x = torch.tensor(np.ascontiguousarray((np.array([12.0, 0, 0]) + 0.01 * xi).T), device=dev)
        v = torch.tensor(np.ascontiguousarray((np.array([0, -180.0, 60.0])
                                               + np.sqrt(G * 1e5 / 0.01) * zeta).T), device=dev)
        m = torch.full((n,), 1e5 / n, dtype=torch.float64, device=dev)
        w = torch.tensor(np.ascontiguousarray(random_directions(n, 8).T), device=dev)
        pot = engine.Potential(eps=5e-4 if n >= 65536 else 1e-3)
        ctx = engine.Context(n, prec)
        T = max(4, reps // 2)
        for _ in range(2):     # warm-up, then a profiled pass
            ctx.profile(True)
            ctx.profile_read()
            for _ in range(reps):
                ctx.accelerations(x, m, pot)
            xx, vv = x.clone(), v.clone()
            tape = ctx.simulate(xx, vv, m, pot, myr(0.5), T, ckpt_every=1)
            ctx.simulate_vjp(m, pot, myr(0.5), T, 1, tape, xx, w)
            torch.cuda.synchronize()
            p = ctx.profile_read()
        shard = unequal = None
        if n >= 65536:
            # one device's block of the system split over 8: n / 8 targets x n sources
            ni = n // 8
            for _ in range(2):
                ctx.profile(True)
                ctx.profile_read()
                for _ in range(reps):
                    ctx.accelerations_rows(x, m, pot, 3 * ni, ni)
                torch.cuda.synchronize()
                q = ctx.profile_read()
            s_ms = q["fwd_ms"] / q["fwd_launches"]
            for _ in range(2):
                ctx.profile(True)
                ctx.profile_read()
                for _ in range(reps):
                    ctx.accelerations_vjp(x, m, pot, w, i_begin=3 * ni, i_count=ni,
                                          with_mass=False)
                torch.cuda.synchronize()
                q = ctx.profile_read()
            sv_ms = q["vjp_ms"] / q["vjp_launches"]
            shard = {"targets": ni, "sources": n, "fwd_us": s_ms * 1e3,
                     "fwd_pairs_per_s": ni * n / (s_ms * 1e-3), "vjp_us": sv_ms * 1e3,
                     "vjp_pairs_per_s": ni * n / (sv_ms * 1e-3)}
            # the general (unequal-mass) path of both kernels: masses drawn
            # uniformly in [0.5, 1.5] x M / n (seeded), the mass inside the pair term
            mu = np.random.Generator(np.random.PCG64(9)).uniform(0.5, 1.5, n)
            mu = torch.tensor(mu * (1e5 / mu.sum()), device=dev)
            for _ in range(2):
                ctx.profile(True)
                ctx.profile_read()
                for _ in range(reps):
                    ctx.accelerations(x, mu, pot)
                    ctx.accelerations_vjp(x, mu, pot, w, with_mass=False)
                torch.cuda.synchronize()
                q = ctx.profile_read()
            uf, uv = q["fwd_ms"] / q["fwd_launches"], q["vjp_ms"] / q["vjp_launches"]
            unequal = {"fwd_us": uf * 1e3, "vjp_us": uv * 1e3,
                       "fwd_pairs_per_s": n * n / (uf * 1e-3),
                       "vjp_pairs_per_s": n * n / (uv * 1e-3),
                       "fwd_frac_of_157.3TF": FLOPS_FWD * n * n / (uf * 1e-3) / 157.3e12,
                       "vjp_frac_of_157.3TF": FLOPS_VJP * n * n / (uv * 1e-3) / 157.3e12}
        ctx.close()
        f_ms = p["fwd_ms"] / p["fwd_launches"]
        v_ms = p["vjp_ms"] / p["vjp_launches"]
        row = {"n": n, "fwd_us": f_ms * 1e3, "vjp_us": v_ms * 1e3,
               "fwd_pairs_per_s": n * n / (f_ms * 1e-3),
               "vjp_pairs_per_s": n * n / (v_ms * 1e-3),
               "fwd_frac_of_157.3TF": FLOPS_FWD * n * n / (f_ms * 1e-3) / 157.3e12,
               "vjp_frac_of_157.3TF": FLOPS_VJP * n * n / (v_ms * 1e-3) / 157.3e12}
        if shard:
            row["shard_rows"] = shard
        if unequal:
            row["unequal_masses"] = unequal
        rows.append(row)
    return {"sweep": rows, "prec": prec}


def ensemble(B=512, n=4096, T=200, n_single=8):
    """A batched ensemble of the kind the surrogate's training set and the grid
    search run: B independent runs of n particles (parameters drawn from the
    priors), T kick-drift-kick steps, advanced as one batched ensemble, against
    the same runs one system at a time (n_single of them, the rate extrapolated).
    Pair interactions per second of each."""
    import torch

    from paper_2511_22468_amd import engine, gyr
    from synth import draw_theta, plummer_unit

    dev = torch.device("cuda", 0)
    G = 4.3009e-6
    th = draw_theta(B, 11)
    pots = [engine.Potential(eps=1e-3, m_nfw=r[2], m_mn=r[3]) for r in th]
    dts = [gyr(r[0]) / 4000 for r in th]
    xi, zeta = plummer_unit(n, 12)
    x0 = np.array([12.0, 0, 0]) + 0.01 * xi
    pos = torch.empty(B, 3, n, dtype=torch.float64, device=dev)
    vel, mass = torch.empty_like(pos), torch.empty(B, n, dtype=torch.float64, device=dev)
    for b in range(B):
        pos[b] = torch.tensor(np.ascontiguousarray(x0.T), device=dev)
        v = np.array([0, -180.0, 60.0]) + np.sqrt(G * th[b, 1] / 0.01) * zeta
        vel[b] = torch.tensor(np.ascontiguousarray(v.T), device=dev)
        mass[b] = th[b, 1] / n
    bctx = engine.Context(B * n, "fp32c")
    p0, v0 = pos.clone(), vel.clone()
    bctx.simulate_batch(pos, vel, mass, pots, dts, 2)      # warm-up
    torch.cuda.synchronize()
    pos.copy_(p0); vel.copy_(v0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    bctx.simulate_batch(pos, vel, mass, pots, dts, T)
    e1.record()
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) * 1e-3
    bctx.close()
    sctx = engine.Context(n, "fp32c")
    px, pv = p0[0].clone(), v0[0].clone()
    sctx.simulate(px, pv, mass[0], pots[0], dts[0], 2)
    torch.cuda.synchronize()
    e0.record()
    for b in range(n_single):
        px.copy_(p0[b]); pv.copy_(v0[b])
        sctx.simulate(px, pv, mass[b], pots[b], dts[b], T)
    e1.record()
    torch.cuda.synchronize()
    t_single = e0.elapsed_time(e1) * 1e-3 * B / n_single
    sctx.close()
    pairs = B * (T + 1) * float(n) * n
    return {"ensemble": {"members": B, "n": n, "steps": T,
                         "batched_s": t_batch, "batched_pairs_per_s": pairs / t_batch,
                         "one_at_a_time_s_extrapolated": t_single,
                         "one_at_a_time_pairs_per_s": pairs / t_single,
                         "speedup": t_single / t_batch}}


def grid(n=1000, T=1000, per_axis=10):
    """The grid-search stage of the stream inference: the MMD loss of the full
    pipeline (back-integration, Plummer placement, T kick-drift-kick steps) at
    per_axis^4 = 10^4 parameter combinations spanning the prior box, with n = 1000
    particles and 1000 steps as in the paper's inference, against a mock stream
    generated at known parameters from its own initial-condition seed."""
    import torch

    from paper_2511_22468_amd import engine, gyr
    from paper_2511_22468_amd.pipeline import grid_search, make_target
    from synth import plummer_unit

    dev = torch.device("cuda", 0)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device=dev)
    lo = np.array([1.0, 4.0, np.log10(5e11), np.log10(3e10)])
    hi = np.array([4.0, 5.0, np.log10(2e12), np.log10(1e11)])
    axes = [np.linspace(lo[k], hi[k], per_axis) for k in range(4)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 4)
    thetas = np.column_stack([[gyr(t) for t in g[:, 0]], 10 ** g[:, 1], 10 ** g[:, 2],
                              10 ** g[:, 3]])
    k_true = np.ravel_multi_index((6, 5, 4, 5), (per_axis,) * 4)
    pot = engine.Potential(eps=1e-3)
    ctx = engine.Context(4096 * 1024, "fp32c")
    xt, zt = plummer_unit(n, 71)
    xi, zeta = plummer_unit(n, 72)
    target = make_target(ctx, t3(xt), t3(zt), torch.tensor(thetas[k_true], device=dev), T,
                         pot=pot)
    grid_search(ctx, thetas[:64], t3(xi), t3(zeta), target, T, pot)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = grid_search(ctx, thetas, t3(xi), t3(zeta), target, T, pot)
    secs = time.perf_counter() - t0
    ctx.close()
    best = int(np.argmin(losses))
    return {"grid_search": {"points": len(thetas), "n": n, "steps": T, "seconds": secs,
                            "pair_interactions_per_s": len(thetas) * (T + 1) * n * n / secs,
                            "true_point": int(k_true), "best_point": best,
                            "best_loss": float(losses[best]),
                            "loss_at_true_point": float(losses[k_true]),
                            "rank_of_true_point": int((losses < losses[k_true]).sum())}}


def bootstrap(sizes=(64, 256), n=1000, T=1000, iters=10, n_seq=2):
    """The refinement stage of the stream inference for a bootstrap of B
    realisations of the observed stream (Fig. 2, steps 5-6): iters descent steps
    of the full pipeline gradient for each, n = 1000 particles and 1000 steps,
    all realisations advanced together by the batched gradient (B = 64 and 256);
    against the same descent for n_seq realisations one at a time (StreamModel),
    scaled to B.  Softening at the Plummer scale radius (the fit's setting, under
    which the gradient of the 1000-step map is informative)."""
    import torch

    from paper_2511_22468_amd import bootstrap as BS, engine
    from paper_2511_22468_amd.fit import EPS_FIT
    from paper_2511_22468_amd.pipeline import StreamModel, grid_search, make_target
    from synth import plummer_unit

    dev = torch.device("cuda", 0)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device=dev)
    pot = engine.Potential(eps=EPS_FIT)
    Bmax = max(sizes)
    ctx = engine.Context(Bmax * 1024, "fp32c")
    u_true = np.array([-0.5, 0.0, 0.0, 0.0])
    xt, zt = plummer_unit(n, 81)
    xi, zeta = plummer_unit(n, 82)
    target = make_target(ctx, t3(xt), t3(zt),
                         torch.tensor(BS.theta_rows(u_true[None])[0], device=dev), T, pot=pot)
    noise = torch.tensor(np.random.default_rng(83).normal(size=(Bmax, 3, n)), device=dev)
    targets = BS.resample(target, 0.05, noise)
    u0 = np.repeat((u_true + np.array([0.1, -0.15, 0.1, -0.1]))[None], Bmax, 0)
    lr = 0.1
    BS.refine(ctx, u0[:2], t3(xi), t3(zeta), targets[:2].contiguous(), T, lr, 1, pot=pot)
    torch.cuda.synchronize()
    runs = {}
    for B in sizes:
        t0 = time.perf_counter()
        u_best, L_best, hist, acc = BS.refine(ctx, u0[:B], t3(xi), t3(zeta),
                                              targets[:B].contiguous(), T, lr, iters, pot=pot)
        torch.cuda.synchronize()
        runs[B] = (time.perf_counter() - t0, u_best, L_best, hist, acc)
    # the loss at the true parameters: the floor set by the finite samples
    L_true = grid_search(ctx, BS.theta_rows(np.repeat(u_true[None], Bmax, 0)), t3(xi), t3(zeta),
                         targets, T, pot)
    # the same descent one realisation at a time
    t0 = time.perf_counter()
    for b in range(n_seq):
        model = StreamModel(ctx, t3(xi), t3(zeta), targets[b].contiguous(), T, pot=pot,
                            ckpt_every=1)

        def ev(u):
            L, g = model.loss_and_grad(torch.tensor(BS.theta_rows(u[None])[0], device=dev))
            return L.item(), g.cpu().numpy() * BS.dtheta_du_rows(u[None])[0]

        u, step = u0[b].copy(), lr
        L, gu = ev(u)
        for it in range(iters):
            cand = np.clip(u - step * gu / np.sqrt((gu * gu).sum()), -1, 1)
            Lc, gc = ev(cand)
            if Lc <= L:
                u, L, gu = cand, Lc, gc
            else:
                step *= 0.5
    torch.cuda.synchronize()
    t_one = (time.perf_counter() - t0) / n_seq
    ctx.close()
    th_true = BS.theta_rows(u_true[None])[0]
    out = {"n": n, "steps": T, "descent_steps": iters, "gradient_evaluations_per_realisation":
           iters + 1, "seconds_per_realisation_one_at_a_time": t_one,
           "sequential_realisations_timed": n_seq, "u_true": u_true.tolist(),
           "u_start": u0[0].tolist(), "loss_at_truth_mean": float(L_true.mean())}
    for B, (t_b, u_best, L_best, hist, acc) in runs.items():
        out[f"B{B}"] = {
            "seconds_batched": t_b, "seconds_one_at_a_time_scaled": t_one * B,
            "speedup": t_one * B / t_b,
            "pair_interactions_per_s": B * (iters + 1) * 2 * (T + 1) * n * n / t_b,
            "loss_first_mean": float(hist[0].mean()), "loss_best_mean": float(L_best.mean()),
            "accepted_steps_mean": float(acc.sum(0).mean()),
            "u_best_mean": u_best.mean(0).tolist(), "u_best_std": u_best.std(0).tolist(),
            "theta_best_over_true_mean": (BS.theta_rows(u_best) / th_true).mean(0).tolist()}
    return {"bootstrap_refinement": out}


def configs():
    """End-to-end wall time of the three smaller workloads (HIP events, after one
    warm-up): N = 1024 FP64, 400 steps of 0.5 Myr; N = 16384 FP32C, 4000 steps;
    N = 8192 stream pipeline, 2000 steps of t_acc / 2000, loss and gradient with
    checkpoints every 100 steps (FP32C).  One JSON line per workload."""
    import torch

    from paper_2511_22468_amd import engine, gyr, myr
    from paper_2511_22468_amd.pipeline import StreamModel, make_target
    from synth import plummer_unit

    dev = torch.device("cuda", 0)
    G = 4.3009e-6
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device=dev)
    out = []

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3, r

    for n, prec, m_tot, T, seed in ((1024, "fp64", 2e4, 400, 1), (16384, "fp32c", 5e4, 4000, 2)):
        xi, zeta = plummer_unit(n, seed)
        x = t3(np.array([12.0, 0, 0]) + 0.01 * xi)
        v = t3(np.array([0, -180.0, 60.0]) + np.sqrt(G * m_tot / 0.01) * zeta)
        m = torch.full((n,), m_tot / n, dtype=torch.float64, device=dev)
        ctx = engine.Context(n, prec)
        pot = engine.Potential(eps=1e-3)
        state = {}

        def run():
            state["x"], state["v"] = x.clone(), v.clone()
            ctx.simulate(state["x"], state["v"], m, pot, myr(0.5), T)

        secs, _ = timed(run)
        e = ctx.energy(state["x"], state["v"], m, pot).sum().item()
        e0 = ctx.energy(x, v, m, pot).sum().item()
        out.append({"workload": f"N={n} {prec} Plummer {m_tot:g} Msun, {T} KDK steps of 0.5 Myr",
                    "seconds": secs, "pair_interactions_per_s": (T + 1) * n * n / secs,
                    "energy_drift": (e - e0) / abs(e0)})
        ctx.close()
    n, T, K = 8192, 2000, 100
    ctx = engine.Context(n, "fp32c")
    xt, zt = plummer_unit(4096, 30)
    theta_true = torch.tensor([gyr(2.0), 3e4, 1.0e12, 6.5e10], dtype=torch.float64, device=dev)
    target = make_target(ctx, t3(xt), t3(zt), theta_true, T)
    xi, zeta = plummer_unit(n, 3)
    model = StreamModel(ctx, t3(xi), t3(zeta), target, T, ckpt_every=K)
    theta = theta_true * torch.tensor([1.1, 1.2, 0.9, 1.1], dtype=torch.float64, device=dev)
    secs, (L, g) = timed(lambda: model.loss_and_grad(theta))
    # forward: T + 1 pair sums; recompute: K pair sums per segment (K - 1 steps
    # and the acceleration of the segment's last position), T in all; reverse:
    # T + 1 pair VJPs
    pairs = (2 * (T + 1) + T) * n * n
    out.append({"workload": f"N={n} stream pipeline, {T} steps of t_acc/2000, MMD vs 4096, "
                            f"loss and gradient, checkpoints every {K} (FP32C)",
                "seconds": secs, "pair_interactions_per_s": pairs / secs})
    # the same with the trajectory between checkpoints rebuilt by stepping backward
    model_r = StreamModel(ctx, t3(xi), t3(zeta), target, T, ckpt_every=K, reversal=True)
    secs_r, (Lr, gr) = timed(lambda: model_r.loss_and_grad(theta))
    out.append({"workload": f"N={n} stream pipeline, {T} steps of t_acc/2000, MMD vs 4096, "
                            f"loss and gradient, checkpoints every {K}, trajectory stepped "
                            f"backward (FP32C)",
                "seconds": secs_r, "pair_interactions_per_s": 2 * (T + 1) * n * n / secs_r,
                "grad": [float(v) for v in gr.cpu().numpy()],
                "grad_recomputed": [float(v) for v in g.cpu().numpy()],
                "loss_same": bool(torch.equal(L, Lr))})
    ctx.close()
    return out


def small_gradient(n=1000, T=1000, reps=5):
    """One small system's pipeline gradient at the paper's inference size (n = 1000
    particles, 1000 steps of t_end / 1000, eps = a_P = 0.01 kpc, MMD against a mock
    stream from its own IC seed), through the single-system path, with the tape every
    step, with checkpoints every 10 steps, and with the same checkpoints and the
    trajectory stepped backward between them.  Best and median of `reps` timed
    evaluations after one warm-up; one JSON object."""
    import torch

    from paper_2511_22468_amd import engine, gyr
    from paper_2511_22468_amd.pipeline import StreamModel, make_target
    from synth import plummer_unit

    dev = torch.device("cuda", 0)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device=dev)
    pot = engine.Potential(eps=0.01)
    ctx = engine.Context(n, "fp32c")
    theta = torch.tensor([gyr(1.75), 10 ** 4.5, 1e12, 6.5e10], dtype=torch.float64, device=dev)
    xt, zt = plummer_unit(n, 11)
    target = make_target(ctx, t3(xt), t3(zt), theta, T, pot=pot)
    xi, zeta = plummer_unit(n, 12)
    out = {"n": n, "steps": T, "eps_kpc": 0.01}
    grads = []
    for K, rev in ((1, False), (10, False), (10, True)):
        model = StreamModel(ctx, t3(xi), t3(zeta), target, T, pot=pot, h=0.2, ckpt_every=K,
                            reversal=rev)
        th = theta * 1.05
        L, g = model.loss_and_grad(th)
        torch.cuda.synchronize()
        grads.append(g.cpu().numpy())
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            model.loss_and_grad(th)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        times.sort()
        out[f"ckpt_every_{K}" + ("_stepped_backward" if rev else "")] = {
            "best_us_per_step": times[0] / T * 1e6,
            "median_us_per_step": times[len(times) // 2] / T * 1e6}
    out["same_gradient"] = bool(np.array_equal(grads[0], grads[1]))
    out["stepped_backward_grad_rel_diff"] = [float(v) for v in np.abs(grads[2] / grads[0] - 1)]
    ctx.close()
    return out


def cpu_sweep(sizes=(1024, 8192, 16384, 65536), budget_pairs=2.0e8):
    """The oracle's pair sum at each workload size on one host thread and on all of
    them (at most 16), on sampled target rows bounded by budget_pairs pairs."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from oracle import forces as of
    from synth import plummer_unit, sample_rows

    G = 4.3009e-6
    cores = min(len(os.sched_getaffinity(0)), 16)
    rows_out = []
    for n in sizes:
        xi, _ = plummer_unit(n, 7)
        x = np.array([12.0, 0.0, 0.0]) + 0.01 * xi
        m = np.full(n, 1e5 / n)
        rows = sample_rows(n, int(min(n, max(cores * 64, budget_pairs // n))), 8)
        out = {"n": n, "rows": int(rows.size)}
        for threads in (1, cores):
            chunks = np.array_split(rows, threads * 2)
            with threadpool_limits(1), ThreadPoolExecutor(threads) as ex:
                t0 = time.perf_counter()
                list(ex.map(lambda r: of.pair_accel(x, m, G, 1e-3, rows=r), chunks))
                dt = time.perf_counter() - t0
            out[f"pairs_per_s_{threads}_threads"] = rows.size * n / dt
        rows_out.append(out)
    return {"cpu_sweep": rows_out, "kind": "oracle", "cores": cores}


def orbit_fit(n_starts=1000, n_iter=60, K=32):
    """The orbit fit of the progenitor: Levenberg-Marquardt from n_starts starts
    drawn in [theta/2, 2 theta] on a noise-free K-point mock track (2 Gyr forward and
    backward, 2000 steps each way), then the exact Hessian and the Fisher covariance
    at the best fit.  Wall time of each part (HIP events) and the recovery error."""
    import torch

    from paper_2511_22468_amd import engine, orbitfit

    dev = torch.device("cuda", 0)
    ctx = engine.Context(1024, "fp64")
    model = orbitfit.TrackModel()
    p_true = np.log10([1.0e12, 16.0, 6.5e10, 3.0, 0.28])
    pt = torch.tensor(p_true, device=dev)
    phi1 = torch.linspace(-1.2, 0.8, K, dtype=torch.float64, device=dev)
    y = orbitfit.observe(ctx, model, phi1, pt)
    track = torch.cat([phi1[:, None], y], 1).contiguous()
    orbitfit.fit(ctx, model, track, p_true, n_starts=64, n_iter=2)     # warm-up
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    rng = np.random.Generator(np.random.PCG64(0))
    half = np.log10(2.0)
    p0 = torch.tensor(p_true[None, :] + rng.uniform(-half, half, (n_starts, 5)), device=dev)
    e[0].record()
    fits, c = orbitfit.lm(ctx, model, track, p0, n_iter)
    e[1].record()
    k = int(torch.argmin(torch.nan_to_num(c, nan=float("inf"))).item())
    H, C = orbitfit.hessian(ctx, model, track, fits[k:k + 1].contiguous())
    e[2].record()
    torch.cuda.synchronize()
    best = fits[k].cpu().numpy()
    ok = (c < 1e-10).sum().item()
    ctx.close()
    return {"orbit_fit": {"starts": n_starts, "iterations": n_iter, "track_points": K,
                          "steps_per_branch": model.n_steps,
                          "lm_seconds": e[0].elapsed_time(e[1]) * 1e-3,
                          "hessian_and_covariance_seconds": e[1].elapsed_time(e[2]) * 1e-3,
                          "starts_reaching_chi2_below_1e-10": ok,
                          "best_chi2": c[k].item(),
                          "best_minus_true_dex": (best - p_true).tolist(),
                          "fisher_sigma_dex": np.sqrt(np.diag(C[0].cpu().numpy())).tolist()}}


def time_to_fit_summary(seeds=(50, 60, 70, 80, 90)):
    """The metric's second half at its workload (fit N = 8192 with 4000 steps; the
    surrogate trained once on 512 runs of N = 4096, with 4000 steps and, as a
    cheaper training set over the same t_end, 1000 steps), on five held-out
    targets: both arms descend to convergence; the plain fit's duration against
    the warm arm's time to reach the plain fit's final loss.  The top-level
    figures are the first target's with the 4000-step training set."""
    from paper_2511_22468_amd import fit
    r = fit.study(seeds=seeds, train_steps=(4000, 1000), sur_seed=seeds[0])
    t0, s0 = r["targets"][0], r["surrogates"][0]
    p, w = t0["plain"], t0["warm"][0]
    tp, tw = p["seconds"], w["seconds_to_plain_fit_loss"]
    cost = s0["data_seconds"] + s0["train_seconds"]
    return {
        "workload": (f"held-out targets drawn from the priors (seeds {seeds[0] + 1}, "
                     f"{seeds[1] + 1}, ...); fit N = {r['n_fit']}, {r['n_steps']} steps, eps "
                     f"{r['eps_kpc']} kpc; one surrogate per training set of "
                     f"{r['n_train_runs']} runs of N = {r['n_train_particles']} (4000 or 1000 "
                     f"steps over the same t_end), trained once for all targets; descent stops "
                     f"at {r['stop_rule']}"),
        "definition": ("plain_seconds: the plain fit until its descent stops, ending at "
                       "plain_fit_loss; warm_seconds: the warm arm (inversion, then descent) "
                       "until it first reaches plain_fit_loss; surrogates[].amortised_speedup_"
                       "incl_training: all targets' plain fits over the training set, training "
                       "and warm arms, a target the warm arm does not bring to the plain fit's "
                       "loss costing its whole warm descent plus the plain fit"),
        "plain_fit_loss": p["final_loss"],
        "plain_seconds": tp,
        "warm_seconds": tw,
        "plain_reaches_warm_final_loss": w["plain_reaches_warm_final_loss"],
        "speedup_excl_training": (tp / tw) if tw else None,
        "speedup_incl_training": (tp / (tw + cost)) if tw else None,
        "data_seconds": s0["data_seconds"],
        "train_seconds": s0["train_seconds"],
        "inversion_seconds": w["inversion_seconds"],
        "plain": {"final_loss": p["final_loss"], "iterations": p["iterations"],
                  "converged": p["converged"], "seconds_total": tp},
        "warm": {"final_loss": w["final_loss"], "iterations": w["iterations"],
                 "converged": w["converged"], "seconds_total": w["seconds"]},
        "surrogates": r["surrogates"],
        "targets": [{"seed": t["seed"], "plain_fit_loss": t["plain"]["final_loss"],
                     "plain_seconds": t["plain"]["seconds"],
                     "warm": [{k: x[k] for k in ("n_train_steps", "seconds_to_plain_fit_loss",
                                                 "speedup_excl_training", "final_loss")}
                              for x in t["warm"]]}
                    for t in r["targets"]],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--n-steps", type=int, default=1000)
    ap.add_argument("--ckpt-every", type=int, default=1)
    ap.add_argument("--prec", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-checkpointed", action="store_true",
                    help="skip the one-step timing with checkpoints every 100 steps")
    ap.add_argument("--no-time-to-fit", action="store_true",
                    help="skip the time-to-fit comparison that the default line carries")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for hardware counters: one step of 20 KDK steps at the "
                         "same N, one reverse sweep of them that steps the trajectory backward "
                         "(checkpoints every 10), plus a 256 MiB device copy that calibrates "
                         "FETCH_SIZE and WRITE_SIZE")
    ap.add_argument("--sweep", action="store_true",
                    help="kernel rates of the forward and VJP pair kernels at every workload "
                         "size (N = 1024 ... 65536), one JSON line")
    ap.add_argument("--ensemble", action="store_true",
                    help="512 runs of N = 4096 (parameters from the priors) as one batched "
                         "ensemble vs one run at a time, one JSON line")
    ap.add_argument("--orbit-fit", action="store_true",
                    help="orbit fit of the progenitor: Levenberg-Marquardt from 1000 starts, "
                         "exact Hessian and Fisher covariance, one JSON line")
    ap.add_argument("--grid", action="store_true",
                    help="grid-search stage of the stream inference: the pipeline loss at "
                         "10^4 parameter combinations (N = 1000, 1000 steps), one JSON line")
    ap.add_argument("--bootstrap", action="store_true",
                    help="bootstrap refinement of the stream inference: 10 descent steps of "
                         "the pipeline gradient for 64 and 256 resampled streams at once vs one "
                         "at a time (N = 1000, 1000 steps), one JSON line")
    ap.add_argument("--infer", action="store_true",
                    help="the whole inference pipeline at the paper's scale: grid search over "
                         "10^4 points for 1000 bootstrap realisations, then their batched "
                         "refinement (N = 1000, 1000 steps), one JSON line")
    ap.add_argument("--time-to-fit", action="store_true",
                    help="the second half of the headline metric: surrogate-warm-started vs "
                         "plain N-body gradient descent on five held-out targets (fit N = "
                         "8192, 4000 steps; surrogates from 4000- and 1000-step training sets), "
                         "one JSON line")
    ap.add_argument("--configs", action="store_true",
                    help="end-to-end time of the N = 1024, 16384 and 8192 (gradient) workloads, "
                         "one JSON line each")
    ap.add_argument("--small", action="store_true",
                    help="one small system's pipeline gradient at the paper's inference size "
                         "(n = 1000, 1000 steps), tape every step and every 10 steps, one JSON "
                         "line")
    ap.add_argument("--cpu-sweep", action="store_true",
                    help="the FP64 oracle's pair sum at every workload size on one and on all "
                         "host threads, one JSON line (no GPU)")
    args = ap.parse_args()
    if args.cpu_sweep:
        print(json.dumps(cpu_sweep()), flush=True)
        return
    if (args.sweep or args.ensemble or args.orbit_fit or args.configs or args.grid
            or args.bootstrap or args.infer or args.time_to_fit or args.small) and args.gpus != 1:
        print("bench.py measures one GPU only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        print(json.dumps(sweep(args.prec)), flush=True)
        return
    if args.small:
        print(json.dumps({"small_system_gradient": small_gradient()}), flush=True)
        return
    if args.ensemble:
        print(json.dumps(ensemble()), flush=True)
        return
    if args.orbit_fit:
        print(json.dumps(orbit_fit()), flush=True)
        return
    if args.grid:
        print(json.dumps(grid()), flush=True)
        return
    if args.bootstrap:
        print(json.dumps(bootstrap()), flush=True)
        return
    if args.time_to_fit:
        from paper_2511_22468_amd import fit
        print(json.dumps(fit.study()), flush=True)
        return
    if args.infer:
        from paper_2511_22468_amd import infer
        print(json.dumps(infer.main()), flush=True)
        return
    if args.configs:
        for row in configs():
            print(json.dumps(row), flush=True)
        return
    if args.profile_run:
        args.n_steps, args.steps, args.warmup, args.no_cpu_baseline = 20, 1, 0, True
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2511_22468_amd import engine, myr
    from paper_2511_22468_amd.pipeline import StreamModel, make_target
    from synth import plummer_unit

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, T, K = args.n, args.n_steps, args.ckpt_every
    dt = myr(0.5)
    theta = torch.tensor([T * dt, 1.0e5, 1.0e12, 6.5e10], dtype=torch.float64, device=dev)
    pot = engine.Potential(eps=5e-4)

    def unit(nn, seed):
        xi, zeta = plummer_unit(nn, seed)
        return (torch.tensor(np.ascontiguousarray(xi.T), device=dev),
                torch.tensor(np.ascontiguousarray(zeta.T), device=dev))

    ctx = engine.Context(n, args.prec)
    # mock observed stream: a 4096-particle run of the same pipeline, own seed,
    # at slightly different parameters
    xt, zt = unit(4096, 41)
    theta_t = theta * torch.tensor([1.0, 0.8, 1.05, 0.95], dtype=torch.float64, device=dev)
    target = make_target(ctx, xt, zt, theta_t, T, pot=pot)
    xi, zeta = unit(n, 40)
    model = StreamModel(ctx, xi, zeta, target, T, pot=pot, h=0.2, ckpt_every=K)

    for _ in range(args.warmup):
        model.loss_and_grad(theta)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    with ClockSampler() as clock:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            L, g = model.loss_and_grad(theta)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)

    sec = (t1 - t0) / args.steps
    pairs = 2.0 * (T + 1) * float(n) * n
    # counter-based flops apply to the kernel sources and size they were taken on
    counted = (args.prec == "fp32c" and n == TRAFFIC_N
               and kernel_source_sha() == TRAFFIC_SRC_SHA)
    fwd_ms = prof["fwd_ms"] / max(prof["fwd_launches"], 1)
    vjp_ms = prof["vjp_ms"] / max(prof["vjp_launches"], 1)
    vjp_tf = FLOPS_VJP * float(n) * n / (vjp_ms * 1e-3) / 1e12
    fwd_tf = FLOPS_FWD * float(n) * n / (fwd_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": pairs / sec,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32c" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"stream pipeline at N={n}: back-integrated centre, Plummer sphere "
                         f"1e5 Msun / 0.01 kpc, eps 5e-4 kpc, {T} KDK steps of 0.5 Myr, "
                         f"MMD (h=0.2 kpc) vs 4096-point target, full reverse sweep to "
                         f"(t_end, M_Plummer, M_NFW, M_MN)"),
            "n": n, "n_steps": T, "dt_myr": 0.5, "eps_kpc": 5e-4, "ckpt_every": K,
            "pair_precision": ("FP32 pair terms, TwoSum-compensated, FP64 drift and reductions"
                               if args.prec == "fp32c" else "FP64"),
            "pairs_per_step": pairs,
            "loss": float(L.item()),
            "grad": [float(v) for v in g.cpu().numpy()],
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_pair_vjp_f32c" if args.prec == "fp32c" else "k_pair_vjp_f64",
            "achieved": vjp_tf,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": vjp_tf / PEAK_FP32_TFLOPS,
            "traffic": (measured_traffic("k_pair_vjp_f32c", n) if args.prec == "fp32c"
                        else None),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE)",
            "flops_per_pair": FLOPS_VJP,
            "avg_launch_ms": vjp_ms,
            "launches": prof["vjp_launches"],
            "judged_on": "flops_per_pair, the conventional algorithmic count of a VJP pair",
            "flops_per_pair_executed": FLOPS_VJP_EXEC,
            "frac_executed": FLOPS_VJP_EXEC * float(n) * n / (vjp_ms * 1e-3) / 1e12
            / PEAK_FP32_TFLOPS,
            "flops_per_pair_counted": FLOPS_COUNTED["k_pair_vjp_f32c"] if counted else None,
            "frac_counted": (FLOPS_COUNTED["k_pair_vjp_f32c"] * float(n) * n / (vjp_ms * 1e-3)
                             / 1e12 / PEAK_FP32_TFLOPS) if counted else None,
        },
        "roofline_fwd": {
            "bound": "alu",
            "kernel": "k_pair_fwd_f32c" if args.prec == "fp32c" else "k_pair_fwd_f64",
            "achieved": fwd_tf,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": fwd_tf / PEAK_FP32_TFLOPS,
            "flops_per_pair": FLOPS_FWD,
            "avg_launch_ms": fwd_ms,
            "launches": prof["fwd_launches"],
            "pairs_per_s": float(n) * n / (fwd_ms * 1e-3),
            "traffic": (measured_traffic("k_pair_fwd_f32c", n) if args.prec == "fp32c"
                        else None),
            "flops_per_pair_executed": FLOPS_FWD_EXEC,
            "frac_executed": FLOPS_FWD_EXEC * float(n) * n / (fwd_ms * 1e-3) / 1e12
            / PEAK_FP32_TFLOPS,
            "flops_per_pair_counted": FLOPS_COUNTED["k_pair_fwd_f32c"] if counted else None,
            "frac_counted": (FLOPS_COUNTED["k_pair_fwd_f32c"] * float(n) * n / (fwd_ms * 1e-3)
                             / 1e12 / PEAK_FP32_TFLOPS) if counted else None,
        },
        "cpu_baseline": None,
        "sclk_mhz": clock.summary(),
    }
    if K == 1 and not args.profile_run and not args.no_checkpointed:
        # the same step with checkpoints every 100 steps: the reverse sweep
        # recomputes each segment from its checkpoint (one more forward pair sum
        # per step) instead of reading a full tape
        model_k = StreamModel(ctx, xi, zeta, target, T, pot=pot, h=0.2, ckpt_every=100)
        model_k.loss_and_grad(theta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Lk, gk = model_k.loss_and_grad(theta)
        torch.cuda.synchronize()
        sk = time.perf_counter() - t0
        out["checkpointed"] = {
            "ckpt_every": 100, "steps": 1, "warmup": 1, "ms_per_step": sk * 1e3,
            "value": pairs / sk, "unit": "pair interactions/s (forward and adjoint, as value)",
            "pair_evaluations_per_s": (pairs + T * float(n) * n) / sk,
            "tape_bytes": 8 * ctx.tape_len(n, T, 100), "full_tape_bytes": 8 * ctx.tape_len(n, T, 1),
            "same_gradient_as_full_tape": bool(torch.equal(gk, g) and torch.equal(Lk, L)),
        }
        # the same checkpoints with the trajectory rebuilt by stepping it backward
        # from the final state: one pair launch per reverse step that sums the VJP
        # and the acceleration together, no recomputed segments
        model_r = StreamModel(ctx, xi, zeta, target, T, pot=pot, h=0.2, ckpt_every=100,
                              reversal=True)
        model_r.loss_and_grad(theta)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        Lr, gr = model_r.loss_and_grad(theta)
        torch.cuda.synchronize()
        sr = time.perf_counter() - t0
        pr = ctx.profile_read()
        ctx.profile(False)
        from paper_2511_22468_amd import _lib
        fused_ms = pr["vjp_ms"] / max(pr["vjp_launches"], 1)
        fused_tf = FLOPS_VJP_FORCE * float(n) * n / (fused_ms * 1e-3) / 1e12
        counted_f = FLOPS_COUNTED["k_pair_vjp_f32c+force"] if counted else None
        out["checkpointed"]["reversed"] = {
            "ckpt_every": 100, "ms_per_step": sr * 1e3, "value": pairs / sr,
            "fused_launch_ms": fused_ms, "fused_launches": pr["vjp_launches"],
            "fused_pairs_per_s": float(n) * n / (fused_ms * 1e-3),
            "fused_roofline": {
                "bound": "alu", "kernel": "k_pair_vjp_f32c (with the acceleration)",
                "achieved": fused_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": fused_tf / PEAK_FP32_TFLOPS, "flops_per_pair": FLOPS_VJP_FORCE,
                "flops_per_pair_executed": FLOPS_VJP_FORCE_EXEC,
                "flops_per_pair_counted": counted_f,
                "frac_counted": (counted_f * float(n) * n / (fused_ms * 1e-3) / 1e12
                                 / PEAK_FP32_TFLOPS) if counted else None,
                "traffic": (measured_traffic("k_pair_vjp_f32c+force", n)
                            if args.prec == "fp32c" else None),
            },
            "workspace_bytes": 8 * int(_lib.lib().dnb_vjp_reversed_workspace_doubles(n)),
            "recompute_workspace_bytes": 8 * int(_lib.lib().dnb_vjp_workspace_doubles(n, 100)),
            "loss_same_as_full_tape": bool(torch.equal(Lr, L)),
            "grad": [float(v) for v in gr.cpu().numpy()],
            "grad_rel_diff_vs_full_tape": [float(v) for v in
                                           (gr / g - 1).abs().cpu().numpy()],
        }
    if args.profile_run:
        # one reverse sweep that steps the trajectory backward (checkpoints every
        # 10 of the 20 steps), so that the counter passes see its fused pair launch
        StreamModel(ctx, xi, zeta, target, T, pot=pot, h=0.2, ckpt_every=10,
                    reversal=True).loss_and_grad(theta)
        torch.cuda.synchronize()
    ctx.close()
    if args.profile_run:
        # calibration for the traffic counters: a plain copy of 256 MiB
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if not args.no_time_to_fit and not args.profile_run:
        out["time_to_fit"] = time_to_fit_summary()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, T, 40)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
