"""Seeded synthetic C-RAN scenarios (device and RRH positions, traffic, marginals).

This package draws inputs only. It holds none of the association method's
arithmetic: no path loss, no rates, no costs and no Sinkhorn step. Both the
HIP library's tests and the CPU oracle take their inputs from here.
"""

from .generator import (  # noqa: F401
    RADIO,
    PRESETS,
    Layout,
    grid_shape,
    make_layout,
    preset_layout,
    batch_sizes,
    batch_layouts,
    snapshot_marginals,
    drift_positions,
    poisson_arrivals,
    with_positions,
)
