"""The stream-inference pipeline of the paper end to end (Fig. 2; Sec. 2.2.1).

1. A mock observed stream: the pipeline's final positions at theta_true, from an
   initial-condition seed of its own.
2. B bootstrap realisations of it, every position displaced by the
   observational error (Fig. 2, step 6).
3. Grid search (stage one of Sec. 2.2.1): the pipeline at every point of a
   regular grid over the prior box.  The runs do not depend on the realisation,
   so they are made once, as batched ensembles, and every realisation's MMD is
   taken against each run (dnb_mmd_batch_targets: the run-run kernel sums once
   per run, the run-realisation sums per realisation).
4. Refinement (stage two, Fig. 2 step 5): from each realisation's best grid
   point, descent steps on the batched pipeline gradient, all realisations
   together (bootstrap.refine).
5. The spread of the refined estimates over the realisations.

Usage: python -m paper_2511_22468_amd.infer [--quick] [--realisations B]
(prints one JSON line)
"""
import argparse
import json
import time

import numpy as np
import torch

from . import bootstrap as BS
from .pipeline import W_NOW, make_target, run_ensemble
from .surrogate import denormalise, normalise


# The paper's inference setup (Sec. 2.2.1; Fig. 2): 1000 Plummer particles,
# 1000 fixed steps, 1000 bootstrap realisations of the observed stream, a grid of
# 10^4 parameter points, then 10 gradient refinement steps.
FULL = {"n": 1000, "steps": 1000, "realisations": 1000, "per_axis": 10, "iters": 10}
QUICK = {"n": 300, "steps": 200, "realisations": 8, "per_axis": 5, "iters": 4}


def grid_points(per_axis):
    """Regular grid over the prior box in the normalised coordinates u, (G, 4)."""
    ax = np.linspace(-1.0, 1.0, per_axis)
    return np.stack(np.meshgrid(ax, ax, ax, ax, indexing="ij"), -1).reshape(-1, 4)


def grid_losses(engine_ctx, u_grid, xi, zeta, targets, n_steps, pot, h=0.2, a_p=0.01,
                w_now=W_NOW):
    """MMD of every grid run against every realisation: (G, B) host array."""
    th = BS.theta_rows(u_grid)
    G, B = th.shape[0], targets.shape[0]
    out = torch.empty(G, B, dtype=torch.float64, device=xi.device)
    for s, pos in run_ensemble(engine_ctx, th, xi, zeta, n_steps, pot, a_p, w_now):
        out[s:s + pos.shape[0]] = engine_ctx.mmd_batch_targets(pos, targets, h)
    return out.cpu().numpy()


def run(engine_ctx, u_true, xi, zeta, xt, zt, n_steps, noise, sigma, per_axis, iters, lr, pot,
        h=0.2, a_p=0.01):
    """The pipeline for B = noise.shape[0] realisations.  xi, zeta: the model's
    unit Plummer samples; xt, zt: the mock stream's own.  noise (B, 3, m)
    standard normal draws.  Returns a dict of host arrays and stage timings."""
    dev = xi.device
    sync = torch.cuda.synchronize
    th_true = torch.tensor(BS.theta_rows(np.asarray(u_true, float)[None])[0], device=dev)
    t0 = time.perf_counter()
    target = make_target(engine_ctx, xt, zt, th_true, n_steps, pot=pot, a_p=a_p)
    targets = BS.resample(target, sigma, noise)
    sync()
    t1 = time.perf_counter()
    u_grid = grid_points(per_axis)
    L = grid_losses(engine_ctx, u_grid, xi, zeta, targets, n_steps, pot, h, a_p)
    best = np.argmin(L, axis=0)
    u0 = u_grid[best]
    sync()
    t2 = time.perf_counter()
    u_fit, L_fit, hist, acc = BS.refine(engine_ctx, u0, xi, zeta, targets, n_steps, lr, iters,
                                        pot, h, a_p)
    sync()
    t3 = time.perf_counter()
    return {"u_grid_best": u0, "L_grid_best": L[best, np.arange(L.shape[1])], "grid_losses": L,
            "u_fit": u_fit, "L_fit": L_fit, "history": hist, "accepted": acc,
            "seconds": {"target": t1 - t0, "grid": t2 - t1, "refine": t3 - t2}}


def summary(res, u_true):
    """Estimates in (t_end [Gyr], log10 M_Plummer, log10 M_NFW, log10 M_MN)."""
    def phys(u):
        th = denormalise(u)
        return np.column_stack([th[:, 0], np.log10(th[:, 1:])])
    truth = phys(np.asarray(u_true, float)[None])[0]
    g, f = phys(res["u_grid_best"]), phys(res["u_fit"])
    return {"truth": truth.tolist(),
            "grid_mean": g.mean(0).tolist(), "grid_std": g.std(0).tolist(),
            "fit_mean": f.mean(0).tolist(), "fit_std": f.std(0).tolist(),
            "loss_grid_mean": float(res["L_grid_best"].mean()),
            "loss_fit_mean": float(res["L_fit"].mean()),
            "accepted_steps_mean": float(res["accepted"].sum(0).mean())}


def main(quick=False, seed=90, realisations=None):
    from . import engine
    from .fit import EPS_FIT
    from synth import plummer_unit

    dev = torch.device("cuda", 0)
    t3 = lambda a: torch.tensor(np.ascontiguousarray(a.T), device=dev)
    cfg = QUICK if quick else FULL
    n, T, per_axis, iters = cfg["n"], cfg["steps"], cfg["per_axis"], cfg["iters"]
    B = int(realisations) if realisations else cfg["realisations"]
    pot = engine.Potential(eps=EPS_FIT)
    ctx = engine.Context(4096 * 1024, "fp32c")
    u_true = normalise(np.array([[1.75, 10 ** 4.5, 1.0e12, 6.5e10]]))[0]
    xi, zeta = plummer_unit(n, seed)
    xt, zt = plummer_unit(n, seed + 1)
    noise = torch.tensor(np.random.Generator(np.random.PCG64(seed + 2)).normal(size=(B, 3, n)),
                         device=dev)
    res = run(ctx, u_true, t3(xi), t3(zeta), t3(xt), t3(zt), T, noise, 0.05, per_axis, iters,
              0.1, pot)
    ctx.close()
    out = {"pipeline": "grid search + bootstrap refinement (Fig. 2)", "n": n, "steps": T,
           "realisations": B, "grid_points": per_axis ** 4, "descent_steps": iters,
           "softening_kpc": EPS_FIT, "seconds": res["seconds"],
           "estimate": summary(res, u_true)}
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--seed", type=int, default=90)
    ap.add_argument("--realisations", type=int, default=None,
                    help="bootstrap realisations (default: the paper's 1000; 8 with --quick)")
    a = ap.parse_args()
    print(json.dumps(main(a.quick, a.seed, a.realisations)), flush=True)
