"""Seeded synthetic inputs for the commute-time anomaly-detection hot path.

This package only draws random inputs (node time series, anomaly patches,
node subsets, and the paper's Gaussian-mixture graph pair, whose input graphs
are defined by a kernel of point distances).  It contains none of the method's
arithmetic (no graph construction from series, Laplacians, projections, solves
or scores), so both the GPU path and the CPU oracle can take their inputs from
here without sharing any code of the method itself.

The inputs stand in for the gridded precipitation fields the paper analyses
(Section "Climate Data"): one node per lat/lon grid cell, each node carrying a
time series; a graph snapshot is built from one time window of the series.
"""

from .grid import (  # noqa: F401
    GridPair,
    GridSequence,
    ar1_grid_series,
    place_patches,
    make_pair,
    make_sequence,
    CONFIGS,
)
from .gmm import GmmPair, make_gmm_pair  # noqa: F401
