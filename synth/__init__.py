"""Seeded synthetic inputs for enhanced MsRSB workloads.

This module only draws random fields and lays out geometry (grids, coarse
partitions, support regions).  It holds none of the method's arithmetic:
filtering, smoothing, coarse operators and solves live in the HIP library
and, independently, in the CPU oracle.  Both consume exactly what this
module produces.

Discretisations that are inputs to the method rather than part of it (the
MPFA-O flow matrix and the Q1 elasticity matrix) are generated in
``synth.mpfa`` and ``synth.q1``; the two-point flux matrix is assembled on
each side from the log-permeability given here.
"""
from .grids import (cell_supports, vertex_supports, vector_supports,
                    tensor_index)
from .fields import (lognormal_iid, channelised_logk, gaussian_smoothed,
                     observation_cells)
from .configs import CONFIGS, make_config

__all__ = ["cell_supports", "vertex_supports", "vector_supports", "tensor_index",
           "lognormal_iid", "channelised_logk", "gaussian_smoothed",
           "observation_cells", "CONFIGS", "make_config"]
