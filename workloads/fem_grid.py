"""Uniform rectangular grid of the finite element data model (inputs only).

The observed data of an inversion come from a finer, conventional finite
element model (Section "Numerical examples").  This module places that grid
over a workload's plate, samples a continuous model at its element centres
and maps scaled-boundary node ids (sources, receivers) to grid node ids.
Grid node (i, j) is j (nx + 1) + i; element (ie, je) is je nx + ie.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FemGrid:
    nx: int
    ny: int
    lx: float
    ly: float

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    def centres(self) -> np.ndarray:
        xs = (np.arange(self.nx) + 0.5) * self.lx / self.nx
        ys = (np.arange(self.ny) + 0.5) * self.ly / self.ny
        X, Y = np.meshgrid(xs, ys)
        return np.stack([X.ravel(), Y.ravel()], axis=1)

    def node_at(self, x: float, y: float) -> int:
        hx, hy = self.lx / self.nx, self.ly / self.ny
        i, j = int(round(x / hx)), int(round(y / hy))
        tol = 1e-9 * max(self.lx, self.ly)
        if not (0 <= i <= self.nx and 0 <= j <= self.ny) or abs(i * hx - x) > tol or abs(j * hy - y) > tol:
            raise ValueError(f"({x}, {y}) is not a grid node")
        return j * (self.nx + 1) + i


def fem_grid(w, cells: tuple | None = None) -> FemGrid:
    """The data grid of workload ``w`` (its ``fem_cells`` unless ``cells`` is given)."""
    nx, ny = cells if cells is not None else w.fem_cells
    xy = w.mesh.node_xy
    return FemGrid(int(nx), int(ny), float(xy[:, 0].max()), float(xy[:, 1].max()))


def fem_nodes(w, grid: FemGrid, node_ids) -> np.ndarray:
    """Grid node of each scaled-boundary node id (int64)."""
    xy = w.mesh.node_xy
    return np.asarray([grid.node_at(*xy[int(n)]) for n in node_ids], dtype=np.int64)


def fem_density(w, grid: FemGrid, name: str) -> np.ndarray:
    """Model ``name`` of workload ``w`` sampled at the grid's element centres."""
    return np.asarray(w.fields[name](grid.centres()), dtype=np.float64)
