"""Spectrum of the discrete step map (stability gate).

The paper is silent on stability of its radial finite-difference scheme.
Undamped average-acceleration Newmark is unconditionally stable for a
symmetric, positive semi-definite pencil; the radial scheme differences
dE0/dxi and dE1/dxi in non-conservative form, so its operator is not
symmetric and strong radial density contrasts can give step-map
eigenvalues outside the unit circle.  This module forms the unforced step
map s^k = T s^{k-1} of the condensed scheme (s = (u, v, a) at every level
and node) column by column and returns its eigenvalues, so tests can keep
to models on which the scheme is stable over the simulated window.
"""

from __future__ import annotations

import numpy as np

from .stepper import Model, step


def _flatten(st):
    parts = [st["U"], st["V"], st["A"]]
    for gs in st["groups"]:
        parts += [gs["u"].ravel(), gs["v"].ravel(), gs["a"].ravel()]
    return np.concatenate(parts)


def _unflatten(model, x):
    n = model.mesh.n_nodes
    st = {"U": x[:n], "V": x[n:2 * n], "A": x[2 * n:3 * n], "groups": []}
    off = 3 * n
    for g in model.groups:
        shp = (len(g.elem_ids), g.n, g.n_b)
        sz = int(np.prod(shp))
        gs = {}
        for key in ("u", "v", "a"):
            gs[key] = x[off:off + sz].reshape(shp)
            off += sz
        st["groups"].append(gs)
    return st


def step_map_eigenvalues(model: Model):
    z = _flatten(model.zero_state(np.float64))
    dim = z.size
    Tm = np.empty((dim, dim))
    zero_force = np.zeros(model.mesh.n_nodes)
    for j in range(dim):
        e = np.zeros(dim)
        e[j] = 1.0
        Tm[:, j] = _flatten(step(model, _unflatten(model, e), zero_force))
    return np.linalg.eigvals(Tm)


def gate(mu, dt, n_steps, f0, band_factor=3.0):
    """(in-band growth, worst growth) over n_steps; in-band = |arg mu| / (2 pi dt) < band_factor f0."""
    mag = np.abs(mu)
    freq = np.abs(np.angle(mu)) / (2 * np.pi * dt)
    grow = mag ** n_steps
    inband = grow[freq < band_factor * f0]
    return (float(inband.max()) if inband.size else 1.0), float(grow.max())
