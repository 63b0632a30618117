"""Seeded synthetic inputs for leading-order reweighting.

This package generates the event samples (momenta, input weights), the model
parameter points and the other random draws that both the HIP path and the
oracle consume.  It holds none of the amplitude arithmetic: it only produces
on-shell, momentum-conserving partonic configurations in the centre-of-mass
frame, as a Monte Carlo event generator would hand them to a reweighting
library (the events "parsed" in step 2 of the reweighting procedure, Sec. 3.2).
"""
from .rng import uniform, splitmix64  # noqa: F401
from .phase_space import (  # noqa: F401
    PROCESSES,
    ProcessSpec,
    generate_events,
    kappa_points,
    uneven_batches,
    alpha_points,
    ee_mumu,
    gg_tt,
    rambo_massive,
)
