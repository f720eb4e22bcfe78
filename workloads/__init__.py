"""Seeded synthetic inputs for the SBFEM full-waveform-inversion hot path.

This package generates *inputs only*: polygon meshes (node coordinates and
counter-clockwise element loops), fine-grid density models, source wavelets
and source/receiver node choices.  It contains none of the method's
arithmetic (no coefficient matrices, no radial discretisation, no time
stepping), so both the CPU oracle and the GPU path can consume it without
sharing any computation.

Inputs stand in for the paper's specimens (Section "Numerical
implementation"): the specimen geometry, its finite-element data and its
meshes are not available, so plates of the same scale (centimetres, 500 kHz,
rho0 = 2700 kg/m^3) with seeded voids and smooth fields are used instead.
"""

from .meshes import Mesh, uniform_rect_mesh, quadtree_mesh, top_edge_nodes, nearest_top_node, cvt_mesh, edge_nodes
from .models import (fine_point_positions, homogeneous, smoothed_voids, sharp_voids,
                     smooth_random_field, seeded_ellipses, seeded_circle)
from .fem_grid import FemGrid, fem_grid, fem_nodes, fem_density
from .signals import ricker, sine_burst
from .configs import (config_tiny, config_paper, config_small, config_quadtree_tiny, config_quadtree, config_cvt,
                      Workload)

__all__ = [
    "Mesh", "uniform_rect_mesh", "quadtree_mesh", "top_edge_nodes", "nearest_top_node", "cvt_mesh", "edge_nodes",
    "fine_point_positions", "homogeneous", "smoothed_voids", "sharp_voids", "smooth_random_field",
    "FemGrid", "fem_grid", "fem_nodes", "fem_density",
    "seeded_ellipses", "seeded_circle", "ricker", "sine_burst",
    "config_tiny", "config_paper", "config_small", "config_quadtree_tiny", "config_quadtree", "config_cvt",
    "Workload",
]
