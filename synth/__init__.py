"""Seeded synthetic inputs for the differentiable agent-based epidemic model.

This package is the one place that both the GPU library's callers and the
FP64 oracle take their inputs from.  It holds no arithmetic of the method
itself (no transmission rates, no sampling, no disease progression): it only
draws populations, contact layers and parameter values with numpy, so that
the two implementations can be compared on identical inputs.
"""

from .graphs import (  # noqa: F401
    Population,
    households,
    workplaces,
    chung_lu,
    complete_pairs,
    to_symmetric_coo,
    quantized_unit_weights,
    location_visits,
    location_degree,
)
from .workloads import Workload, make_workload, CONFIG_NAMES  # noqa: F401
