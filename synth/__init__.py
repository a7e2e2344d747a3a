"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds input generators only: random draws and their
transformation into unit-scaled samples.  It contains none of the N-body
method's arithmetic (no forces, integrator, loss or gradients), so both the
HIP path and the oracle can take their inputs from here without sharing any
of the computation they are compared on.
"""
from .plummer import plummer_unit, random_directions, sample_rows  # noqa: F401
from .priors import draw_theta, PRIOR_BOUNDS  # noqa: F401
from .weights import mlp_init, flatten, unflatten  # noqa: F401
