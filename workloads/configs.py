"""Named synthetic workloads (inputs only).

* ``config_tiny``   -- 0.02 m square plate, 8 x 8 square elements, n_b = 8,
  N_r = 16, c = 3000 m/s, rho0 = 2700, dt = 5e-8 s, 200 steps, one Ricker
  source (500 kHz) at mid-top, 8 receivers at the odd top-edge nodes.
* ``config_paper``  -- 0.1 x 0.05 m plate, 128 x 64 elements, n_b = 16,
  N_r = 32, dt = 2e-8 s, 4000 steps, 4 sources and 32 receivers on the top
  edge.
* ``config_small``  -- a reduced plate used by parity tests at sizes that
  span several tiles and a ragged tail.
* ``config_cvt``    -- the workload shape of the paper's timing tables:
  centroidal Voronoi polygons (1000 .. 8000 cells) with 5 or 7 radial
  intervals, c = 6000 m/s, dt = 0.2 us, 200 steps, two 2-cycle 500 kHz sine
  bursts 30 mm apart at the middle of the top edge, receivers at a 1 mm pitch
  along all four edges (nearest boundary nodes); the plate is 0.1 x 0.05 m
  (the paper's specimen drawing is not available) with a central circular
  hole of 5 mm radius in its models.
* ``config_quadtree`` -- the 0.1 x 0.05 m plate as a quadtree refined from
  level 4 (3.125 mm cells) to level 8 around three seeded voids: about 6200
  elements with hanging nodes (n_b 8 .. 14), N_r proportional to the cell
  size (16 .. 64), 16 shots on the top edge, 32 receivers as in
  ``config_paper``.

Every model is sampled on the fine grid (one density per element, radial
level and boundary node).  ``fields`` holds the continuous models, so the
same model can also be sampled at the element centres of the finite element
data grid (``fem_cells`` cells per direction, a multiple of the boundary
segments per element edge, so that every scaled-boundary node is a grid
node).  Models whose name ends in ``_data`` are for observed data only.  Seeds are 1000 * config_index + item_index.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import Mesh, uniform_rect_mesh, quadtree_mesh, top_edge_nodes, nearest_top_node, cvt_mesh, edge_nodes
from .models import (fine_point_positions, homogeneous, smoothed_voids, smooth_random_field,
                     seeded_circle, seeded_ellipses, sharp_voids)
from .signals import ricker, sine_burst


@dataclass
class Workload:
    name: str
    mesh: Mesh
    c: float
    rho0: float
    dt: float
    n_steps: int
    src_nodes: np.ndarray          # [n_shots] int64
    wavelets: np.ndarray           # [n_shots, n_steps] float64
    rec_nodes: np.ndarray          # [n_rec] int64
    models: dict = field(default_factory=dict)   # name -> rho [n_params]
    fields: dict = field(default_factory=dict)   # name -> callable(points [P, 2]) -> rho [P]
    fem_cells: tuple | None = None                # (nx, ny) of the finite element data grid
    beta: float = 0.25
    gamma: float = 0.5
    xi0: float = 1e-3
    f0: float = 5e5

    @property
    def n_shots(self) -> int:
        return int(self.src_nodes.shape[0])

    def units_per_pass(self) -> int:
        """Element x radial-level x step x shot count of one forward pass."""
        return int(self.mesh.n_r.astype(np.int64).sum()) * self.n_steps * self.n_shots


def config_tiny(n_steps: int = 200) -> Workload:
    lx = ly = 0.02
    mesh = uniform_rect_mesh(lx, ly, 8, 8, segs=2, n_r=16)
    top = top_edge_nodes(mesh)
    src = np.asarray([nearest_top_node(mesh, 0.01)], dtype=np.int64)
    rec = top[1::2].astype(np.int64)
    dt, f0 = 5e-8, 5e5
    wav = ricker(n_steps, dt, f0)[None, :]
    pts = fine_point_positions(mesh)
    le = lx / 8
    void = seeded_circle(0 * 1000 + 0, [0.004, 0.004], [0.016, 0.016], 0.002)
    fields = {
        "homogeneous": lambda p: np.full(p.shape[0], 2700.0),
        "void_floor_half": lambda p: smoothed_voids(p, void, 2700.0, 0.5, le / 16),
        "random30": lambda p: smooth_random_field(p, 0 * 1000 + 1, 2700.0, 0.3),
        "void_data": lambda p: smoothed_voids(p, void, 2700.0, 1e-5, le / 16),
        "void_sharp_data": lambda p: sharp_voids(p, void, 2700.0, 1e-5),
    }
    models = {k: fields[k](pts) for k in ("homogeneous", "void_floor_half", "random30", "void_data")}
    return Workload("tiny-8x8-nb8-nr16", mesh, 3000.0, 2700.0, dt, n_steps, src, wav, rec, models,
                    fields=fields, fem_cells=(32, 32))


def config_paper(n_steps: int = 4000, n_shots: int = 4) -> Workload:
    lx, ly = 0.1, 0.05
    mesh = uniform_rect_mesh(lx, ly, 128, 64, segs=4, n_r=32)
    xs = [lx * (k + 0.5) / n_shots for k in range(n_shots)]
    src = np.asarray([nearest_top_node(mesh, x) for x in xs], dtype=np.int64)
    rec = np.asarray([nearest_top_node(mesh, lx * (k + 0.5) / 32) for k in range(32)], dtype=np.int64)
    dt, f0 = 2e-8, 5e5
    wav = np.repeat(ricker(n_steps, dt, f0)[None, :], n_shots, axis=0)
    pts = fine_point_positions(mesh)
    le = lx / 128
    ell = seeded_ellipses(1 * 1000 + 0, 2, (lx, ly), 0.002, 0.006, 2 * le)
    fields = {
        "homogeneous": lambda p: np.full(p.shape[0], 2700.0),
        "voids_floor_half": lambda p: smoothed_voids(p, ell, 2700.0, 0.5, le / 32),
        "random30": lambda p: smooth_random_field(p, 1 * 1000 + 1, 2700.0, 0.3),
        "voids_data": lambda p: sharp_voids(p, ell, 2700.0, 1e-5),
    }
    models = {k: fields[k](pts) for k in ("homogeneous", "voids_floor_half", "random30")}
    return Workload("paper-128x64-nb16-nr32", mesh, 3000.0, 2700.0, dt, n_steps, src, wav, rec, models,
                    fields=fields, fem_cells=(512, 256))


def config_small(nx: int = 12, ny: int = 6, segs: int = 3, n_r: int = 12, n_steps: int = 60,
                 n_shots: int = 3, dt: float = 2e-8) -> Workload:
    """Reduced plate: several element tiles, n_b = 4 * segs, a few shots."""
    lx, ly = 0.1 * nx / 128 * 4, 0.05 * ny / 64 * 4
    mesh = uniform_rect_mesh(lx, ly, nx, ny, segs=segs, n_r=n_r)
    xs = [lx * (k + 0.5) / n_shots for k in range(n_shots)]
    src = np.asarray([nearest_top_node(mesh, x) for x in xs], dtype=np.int64)
    top = top_edge_nodes(mesh)
    rec = top[1::3].astype(np.int64)
    f0 = 5e5
    wav = np.stack([ricker(n_steps, dt, f0, t0=(1.5 + 0.1 * s) / f0) for s in range(n_shots)])
    pts = fine_point_positions(mesh)
    fields = {
        "homogeneous": lambda p: np.full(p.shape[0], 2700.0),
        "random30": lambda p: smooth_random_field(p, 2 * 1000 + 1, 2700.0, 0.3, wavelength=lx / 3),
    }
    models = {k: f(pts) for k, f in fields.items()}
    return Workload(f"small-{nx}x{ny}-nb{4*segs}-nr{n_r}", mesh, 3000.0, 2700.0, dt, n_steps,
                    src, wav, rec, models, fields=fields, fem_cells=(nx * 2 * segs, ny * 2 * segs))


def config_cvt(n_cells: int = 8000, intervals: int = 7, n_steps: int = 200, lloyd_iters: int = 30,
               mesh: Mesh | None = None) -> Workload:
    """Polygon (CVT) plate in the shape of the paper's timing tables (``mesh``: reuse
    the cells of an earlier call, with ``intervals + 1`` levels)."""
    lx, ly = 0.1, 0.05
    if mesh is None:
        mesh = cvt_mesh(lx, ly, n_cells, intervals + 1, seed=4 * 1000 + n_cells, lloyd_iters=lloyd_iters)
    else:
        mesh = Mesh(mesh.node_xy, mesh.elem_ptr, mesh.elem_nodes, np.full(mesh.n_elem, intervals + 1, dtype=np.int32),
                    mesh.extent, dict(mesh.meta))
    src = np.asarray([nearest_top_node(mesh, 0.035), nearest_top_node(mesh, 0.065)], dtype=np.int64)
    dt, f0 = 2e-7, 5e5
    wav = np.repeat(sine_burst(n_steps, dt, f0, 2, 1e12)[None, :], 2, axis=0)
    bnd = edge_nodes(mesh)
    bxy = mesh.node_xy[bnd]
    marks = [(x, y) for x in np.arange(0.0005, lx, 0.001) for y in (0.0, ly)] + \
            [(x, y) for y in np.arange(0.0005, ly, 0.001) for x in (0.0, lx)]
    rec = np.unique([bnd[np.argmin(np.hypot(bxy[:, 0] - x, bxy[:, 1] - y))] for (x, y) in marks]).astype(np.int64)
    pts = fine_point_positions(mesh)
    hole = [(lx / 2, ly / 2, 0.005, 0.005, 0.0)]
    h = np.sqrt(lx * ly / n_cells)
    fields = {
        "homogeneous": lambda p: np.full(p.shape[0], 2700.0),
        "hole_floor_half": lambda p: smoothed_voids(p, hole, 2700.0, 0.5, h / 4),
        "hole_data": lambda p: sharp_voids(p, hole, 2700.0, 1e-5),
    }
    models = {k: fields[k](pts) for k in fields}
    return Workload(f"cvt-{n_cells}-{intervals}i", mesh, 6000.0, 2700.0, dt, n_steps, src, wav, rec, models,
                    fields=fields, f0=f0)


def config_quadtree_tiny(n_steps: int = 40) -> Workload:
    """A small ragged quadtree (n_b and N_r vary per element) for parity tests."""
    lx, ly = 0.02, 0.01
    mesh = quadtree_mesh(lx, ly, base_level=2, max_level=4, refine_centres=[(0.011, 0.004)],
                         refine_radius=0.003, n_b_max=24, n_r_max=12, n_r_min=4)
    src = np.asarray([nearest_top_node(mesh, 0.008)], dtype=np.int64)
    top = top_edge_nodes(mesh)
    rec = top[::2].astype(np.int64)
    dt, f0 = 2e-8, 5e5
    wav = ricker(n_steps, dt, f0)[None, :]
    pts = fine_point_positions(mesh)
    models = {
        "homogeneous": homogeneous(mesh, 2700.0),
        "random30": smooth_random_field(pts, 3 * 1000 + 1, 2700.0, 0.3, wavelength=0.006),
    }
    return Workload("quadtree-tiny", mesh, 3000.0, 2700.0, dt, n_steps, src, wav, rec, models)


def config_quadtree(n_steps: int = 4000, n_shots: int = 16) -> Workload:
    """Batching workload: ragged quadtree plate, many shots."""
    lx, ly = 0.1, 0.05
    voids = seeded_ellipses(2 * 1000 + 0, 3, (lx, ly), 0.002, 0.006, 0.004)
    centres = [(v[0], v[1]) for v in voids]
    mesh = quadtree_mesh(lx, ly, base_level=4, max_level=8, refine_centres=centres, refine_radius=0.01,
                         n_b_max=24, n_r_max=64, n_r_min=16)
    xs = [lx * (k + 0.5) / n_shots for k in range(n_shots)]
    src = np.asarray([nearest_top_node(mesh, x) for x in xs], dtype=np.int64)
    rec = np.asarray([nearest_top_node(mesh, lx * (k + 0.5) / 32) for k in range(32)], dtype=np.int64)
    dt, f0 = 2e-8, 5e5
    wav = np.repeat(ricker(n_steps, dt, f0)[None, :], n_shots, axis=0)
    pts = fine_point_positions(mesh)
    models = {
        "homogeneous": homogeneous(mesh, 2700.0),
        "voids_floor_half": smoothed_voids(pts, voids, 2700.0, 0.5, ly / 2 ** 8 / 16),
        "random30": smooth_random_field(pts, 2 * 1000 + 1, 2700.0, 0.3),
    }
    return Workload("quadtree-l4-l8-3voids", mesh, 3000.0, 2700.0, dt, n_steps, src, wav, rec, models)
