"""The defaults of the code against the experiment setup the paper states
(tests/golden/paper_setup.txt, each value with its passage).  CPU only."""
import inspect
import os

import numpy as np

import bench
import oracle.orbitfit as OF
from paper_2511_22468_amd import infer, orbitfit
from paper_2511_22468_amd.units import gyr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_setup.txt")


def load_setup():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, value = line.split()[:2]
            vals[key] = float(value)
    return vals


def defaults(fn):
    return {k: p.default for k, p in inspect.signature(fn).parameters.items()
            if p.default is not inspect.Parameter.empty}


def test_fixture_lists_every_checked_value():
    assert set(load_setup()) == {
        "inference.plummer_particles", "inference.time_steps",
        "inference.bootstrap_realisations", "inference.grid_points",
        "inference.refinement_steps", "orbitfit.starts", "orbitfit.start_low_factor",
        "orbitfit.start_high_factor", "orbitfit.horizon_gyr", "orbitfit.fisher_factor"}


def test_inference_defaults_follow_the_paper():
    s = load_setup()
    full, grid, boot = infer.FULL, defaults(bench.grid), defaults(bench.bootstrap)
    for n in (full["n"], grid["n"], boot["n"]):
        assert n == s["inference.plummer_particles"]
    for T in (full["steps"], grid["T"], boot["T"]):
        assert T == s["inference.time_steps"]
    assert full["realisations"] == s["inference.bootstrap_realisations"]
    for per_axis in (full["per_axis"], grid["per_axis"]):
        assert per_axis ** 4 == s["inference.grid_points"]
    assert len(infer.grid_points(full["per_axis"])) == s["inference.grid_points"]
    for iters in (full["iters"], boot["iters"]):
        assert iters == s["inference.refinement_steps"]


def test_orbit_fit_defaults_follow_the_paper():
    s = load_setup()
    assert defaults(orbitfit.fit)["n_starts"] == s["orbitfit.starts"]
    assert orbitfit.START_FACTOR == s["orbitfit.start_high_factor"]
    assert 1.0 / orbitfit.START_FACTOR == s["orbitfit.start_low_factor"]
    assert orbitfit.TrackModel().dt_total == gyr(s["orbitfit.horizon_gyr"])
    H = np.diag([2.0, 4.0, 8.0, 16.0, 32.0])
    F, C = OF.fisher(H)
    assert np.allclose(F, s["orbitfit.fisher_factor"] * H, rtol=0, atol=0)
    assert np.allclose(C @ F, np.eye(5), rtol=0, atol=1e-15)
