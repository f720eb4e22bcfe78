"""Seeded request streams for the serving pattern (inputs only).

Each request is one forward + adjoint shot: a model (mesh + densities), one
source node and wavelet, the receivers, observed traces, a step count and an
arrival time.  The recipe follows the serving workload of the benchmark
description: uniform plates of several sizes or quadtree plates, n_b = 4 s
boundary nodes (s segments per element edge), N_r levels, 1..4 seeded
voids, Poisson arrivals, and half of the requests reusing one of the last
eight models (so that factored models can be kept on the device).  The shots
of one model share its time window (step count), as the shots of one
experiment do.

``scale`` picks the size ranges:

* ``"full"``    -- uniform meshes 32x16 .. 256x128 or quadtrees, n_b 8..24,
  N_r 8..64, 1000..8000 steps (hours of device time for 256 requests);
* ``"reduced"`` -- uniform 16x8 .. 64x32 or small quadtrees, n_b 8..16,
  N_r 16..32, 200..800 steps (the size measured here; stated with results).

Observed traces are zero (the misfit is then half the trace energy): the
adjoint source and the device work have the same shape as with real data.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import Mesh, nearest_top_node, quadtree_mesh, top_edge_nodes, uniform_rect_mesh
from .models import fine_point_positions, seeded_ellipses, smoothed_voids
from .signals import ricker


@dataclass
class ModelRecipe:
    key: str
    kind: str                      # "uniform" or "quadtree"
    nx: int = 0
    ny: int = 0
    segs: int = 2
    n_r: int = 16
    n_voids: int = 1
    seed: int = 0
    quad_radius: float = 0.004
    c: float = 3000.0
    dt: float = 2e-8
    rho0: float = 2700.0
    n_steps: int = 400

    def build(self):
        """(mesh, rho) of this model."""
        lx, ly = 0.1, 0.05
        if self.kind == "uniform":
            mesh = uniform_rect_mesh(lx, ly, self.nx, self.ny, segs=self.segs, n_r=self.n_r)
        else:
            cen = [(v[0], v[1]) for v in seeded_ellipses(self.seed, self.n_voids, (lx, ly), 0.002, 0.006, 0.004)]
            mesh = quadtree_mesh(lx, ly, base_level=3, max_level=6, refine_centres=cen,
                                 refine_radius=self.quad_radius, n_b_max=24, n_r_max=self.n_r,
                                 n_r_min=max(16, self.n_r // 4))
        voids = seeded_ellipses(self.seed + 1, self.n_voids, (lx, ly), 0.002, 0.006, 0.004)
        pts = fine_point_positions(mesh)
        rho = smoothed_voids(pts, voids, self.rho0, 0.5, ly / 256)
        return mesh, rho


@dataclass
class ShotRequest:
    rid: int
    model: ModelRecipe
    src_x: float
    n_steps: int
    arrival: float                  # seconds after the stream starts
    f0: float = 5e5
    n_rec: int = 16
    _built: dict = field(default_factory=dict, repr=False)

    def inputs(self, mesh: Mesh):
        """Source node, wavelet [n_steps], receiver nodes [n_rec], observed [n_rec, n_steps]."""
        src = nearest_top_node(mesh, self.src_x)
        top = top_edge_nodes(mesh)
        rec = top[np.linspace(0, len(top) - 1, self.n_rec).round().astype(int)].astype(np.int64)
        wav = ricker(self.n_steps, self.model.dt, self.f0)
        obs = np.zeros((len(rec), self.n_steps))
        return int(src), wav, rec, obs


def serving_requests(n: int = 256, seed: int = 4 * 1000, rate: float = 10.0, scale: str = "reduced"):
    """n requests with Poisson arrivals at `rate` per second (seeded)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    recent = []
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        if recent and rng.random() < 0.5:
            model = recent[rng.integers(len(recent))]
        else:
            if scale == "full":
                kinds = [(32, 16), (64, 32), (128, 64), (256, 128), None]
                segs = int(rng.integers(2, 7))
                n_r = int(rng.integers(8, 65))
                steps_lo, steps_hi = 1000, 8000
            else:
                kinds = [(16, 8), (32, 16), (64, 32), None]
                segs = int(rng.integers(2, 5))
                n_r = int(rng.integers(16, 33))
                steps_lo, steps_hi = 200, 800
            pick = kinds[rng.integers(len(kinds))]
            mseed = seed + 10 * i + 1
            if pick is None:
                model = ModelRecipe(key=f"q{i}", kind="quadtree", n_r=n_r, n_voids=int(rng.integers(1, 5)),
                                    seed=mseed)
            else:
                model = ModelRecipe(key=f"u{i}", kind="uniform", nx=pick[0], ny=pick[1], segs=segs, n_r=n_r,
                                    n_voids=int(rng.integers(1, 5)), seed=mseed)
            model.n_steps = int(rng.integers(steps_lo // 100, steps_hi // 100 + 1)) * 100
            recent = (recent + [model])[-8:]
        out.append(ShotRequest(rid=i, model=model, src_x=float(rng.uniform(0.005, 0.095)), n_steps=model.n_steps,
                               arrival=t))
    return out
