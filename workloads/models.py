"""Fine-grid density models (inputs only).

The inversion parameters are one density per (element, radial level j,
boundary node k), the nodal points along the scaled-boundary rays (the
paper defines the density at nodal points and interpolates it along the
boundary with the shape functions; Section "weak formulation" and the
implementation notes of Section "Numerical implementation").  The array
layout is level-major per element: rho[off_e + j * n_b + k].

To sample a continuous model at those points this module needs their
*nominal* positions.  It places the scaling centre at the vertex mean of the
loop and the levels uniformly between xi0 and 1.  These positions only
decide where a synthetic field is sampled; the method itself never reads
them.
"""

from __future__ import annotations

import numpy as np

from .meshes import Mesh


def fine_point_positions(mesh: Mesh, xi0: float = 1e-3) -> np.ndarray:
    """Nominal (x, y) of every fine-grid point, shape [n_params, 2]."""
    out = np.empty((mesh.n_params, 2), dtype=np.float64)
    offs = mesh.param_offsets()
    for e in range(mesh.n_elem):
        loop = mesh.loop(e)
        xy = mesh.node_xy[loop]
        ctr = xy.mean(axis=0)
        nr = int(mesh.n_r[e])
        levels = xi0 + (1.0 - xi0) * np.arange(nr) / (nr - 1)
        pts = ctr[None, None, :] + levels[:, None, None] * (xy[None, :, :] - ctr[None, None, :])
        out[offs[e]:offs[e + 1]] = pts.reshape(-1, 2)
    return out


def homogeneous(mesh: Mesh, rho0: float = 2700.0) -> np.ndarray:
    return np.full(mesh.n_params, rho0, dtype=np.float64)


def seeded_circle(seed: int, lo, hi, radius: float):
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo, hi)
    return [(float(c[0]), float(c[1]), radius, radius, 0.0)]


def seeded_ellipses(seed: int, count: int, extent, semi_lo: float, semi_hi: float,
                    margin: float, max_tries: int = 10000):
    """Non-overlapping ellipses (cx, cy, a, b, angle) inside the plate."""
    rng = np.random.default_rng(seed)
    lx, ly = extent
    out = []
    tries = 0
    while len(out) < count and tries < max_tries:
        tries += 1
        a, b = rng.uniform(semi_lo, semi_hi, size=2)
        ang = rng.uniform(0.0, np.pi)
        r = max(a, b)
        cx = rng.uniform(margin + r, lx - margin - r)
        cy = rng.uniform(margin + r, ly - margin - r)
        if all(np.hypot(cx - o[0], cy - o[1]) > r + max(o[2], o[3]) for o in out):
            out.append((float(cx), float(cy), float(a), float(b), float(ang)))
    if len(out) < count:
        raise RuntimeError("could not place non-overlapping ellipses")
    return out


def smoothed_voids(points: np.ndarray, voids, rho0: float, floor: float, width: float) -> np.ndarray:
    """rho/rho0 = floor + (1 - floor) * clamp(d / width + 1/2, 0, 1).

    d is a signed distance proxy to each ellipse boundary (positive outside):
    ((x'/a)^2 + (y'/b)^2 - 1) * min(a, b) / 2 in the ellipse frame.  The
    smallest value over all voids is used.
    """
    scale = np.ones(points.shape[0], dtype=np.float64)
    for (cx, cy, a, b, ang) in voids:
        dx, dy = points[:, 0] - cx, points[:, 1] - cy
        ca, sa = np.cos(ang), np.sin(ang)
        xp, yp = ca * dx + sa * dy, -sa * dx + ca * dy
        d = ((xp / a) ** 2 + (yp / b) ** 2 - 1.0) * min(a, b) / 2.0
        s = floor + (1.0 - floor) * np.clip(d / width + 0.5, 0.0, 1.0)
        scale = np.minimum(scale, s)
    return rho0 * scale


def sharp_voids(points: np.ndarray, voids, rho0: float, floor: float) -> np.ndarray:
    """rho0 * floor inside any ellipse (cx, cy, a, b, angle), rho0 outside."""
    inside = np.zeros(points.shape[0], dtype=bool)
    for (cx, cy, a, b, ang) in voids:
        dx, dy = points[:, 0] - cx, points[:, 1] - cy
        ca, sa = np.cos(ang), np.sin(ang)
        xp, yp = ca * dx + sa * dy, -sa * dx + ca * dy
        inside |= (xp / a) ** 2 + (yp / b) ** 2 < 1.0
    return np.where(inside, rho0 * floor, rho0)


def smooth_random_field(points: np.ndarray, seed: int, rho0: float, amplitude: float = 0.3,
                        wavelength: float = 5e-3, n_modes: int = 12) -> np.ndarray:
    """rho0 * (1 + amplitude * g), g a sum of seeded plane waves scaled to [-1, 1]."""
    rng = np.random.default_rng(seed)
    k = 2 * np.pi / wavelength
    ang = rng.uniform(0, 2 * np.pi, n_modes)
    ph = rng.uniform(0, 2 * np.pi, n_modes)
    g = np.zeros(points.shape[0])
    for i in range(n_modes):
        g += np.cos(k * (np.cos(ang[i]) * points[:, 0] + np.sin(ang[i]) * points[:, 1]) + ph[i])
    g /= n_modes ** 0.5 * 3.0
    g = np.clip(g, -1.0, 1.0)
    return rho0 * (1.0 + amplitude * g)
