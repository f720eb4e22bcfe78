"""Bilinear finite elements for the observed data of the inversion.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper inverts data computed by a finer, conventional finite element
model, not by its own scaled boundary discretisation (Section "Numerical
examples").  This module is the plain statement of the data model used here:

* the scalar wave equation of the paper's governing equations,
  rho u_tt - div(rho c^2 grad u) = f, with a free (natural) outer boundary
  and zero initial conditions;
* a uniform grid of nx x ny bilinear (Q1) rectangles on [0, lx] x [0, ly],
  nodes numbered row by row (node (i, j) = j (nx + 1) + i), one density per
  element;
* element stiffness kappa_e * integral of grad N_a . grad N_b over the
  rectangle (kappa_e = rho_e c^2), lumped (row-sum) mass rho_e hx hy / 4 at
  each element node;
* explicit central differences in time,
  M (u_{n+1} - 2 u_n + u_{n-1}) / dt^2 + K u_n = f_n, u_0 = u_1 = 0, with
  f_n the point source sampled at t_n = n dt (wavelet index n - 1) and
  traces u_n at the receiver nodes for n = 1 .. N.

Lumped mass and the explicit scheme (instead of a consistent mass with an
implicit Newmark step) keep the generator free of linear solves; it is
stable for dt below 1 / (c sqrt(1/hx^2 + 1/hy^2)).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def grid_nodes(nx: int, ny: int, lx: float, ly: float) -> np.ndarray:
    """Node coordinates [(nx+1)(ny+1), 2], row by row."""
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def element_centres(nx: int, ny: int, lx: float, ly: float) -> np.ndarray:
    """Element centres [nx ny, 2], element (ie, je) at index je nx + ie."""
    xs = (np.arange(nx) + 0.5) * lx / nx
    ys = (np.arange(ny) + 0.5) * ly / ny
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def unit_stiffness(hx: float, hy: float) -> np.ndarray:
    """Integral of grad N_a . grad N_b over an hx x hy rectangle (local nodes
    (0,0), (1,0), (1,1), (0,1)), by the closed form of the bilinear shape
    functions."""
    kx = np.array([[2, -2, -1, 1], [-2, 2, 1, -1], [-1, 1, 2, -2], [1, -1, -2, 2]], dtype=np.float64) / 6.0
    ky = np.array([[2, 1, -1, -2], [1, 2, -2, -1], [-1, -2, 2, 1], [-2, -1, 1, 2]], dtype=np.float64) / 6.0
    return (hy / hx) * kx + (hx / hy) * ky


def element_nodes(nx: int, ny: int) -> np.ndarray:
    """Global nodes of every element [nx ny, 4] in local order (0,0), (1,0), (1,1), (0,1)."""
    ie, je = np.meshgrid(np.arange(nx), np.arange(ny))
    ie, je = ie.ravel(), je.ravel()
    n0 = je * (nx + 1) + ie
    return np.stack([n0, n0 + 1, n0 + nx + 2, n0 + nx + 1], axis=1)


def assemble(nx: int, ny: int, lx: float, ly: float, rho_e: np.ndarray, c: float):
    """Global stiffness K (sparse CSR) and lumped mass m (per node)."""
    hx, hy = lx / nx, ly / ny
    ke = unit_stiffness(hx, hy)
    conn = element_nodes(nx, ny)
    kappa = np.asarray(rho_e, dtype=np.float64) * c * c
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    vals = (kappa[:, None, None] * ke[None, :, :]).ravel()
    n = (nx + 1) * (ny + 1)
    K = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    m = np.zeros(n)
    np.add.at(m, conn.ravel(), np.repeat(np.asarray(rho_e, dtype=np.float64) * hx * hy / 4.0, 4))
    return K, m


def stable_dt(nx: int, ny: int, lx: float, ly: float, c: float) -> float:
    """Step below which the explicit scheme is stable (bound of the largest
    eigenvalue of M^-1 K by its row sums: 4 c^2 (1/hx^2 + 1/hy^2))."""
    hx, hy = lx / nx, ly / ny
    return 1.0 / (c * np.sqrt(1.0 / hx ** 2 + 1.0 / hy ** 2))


def step(K, m, u, u_prev, f, dt):
    """u_{n+1} = 2 u_n - u_{n-1} + dt^2 M^-1 (f_n - K u_n)."""
    return 2.0 * u - u_prev + dt * dt * (f - K @ u) / m


def forward(nx: int, ny: int, lx: float, ly: float, rho_e, c: float, dt: float, src_nodes, wavelets,
            rec_nodes, n_steps: int) -> np.ndarray:
    """Receiver traces [S, R, N]: trace k - 1 is u_k = u(t_k), k = 1 .. N.

    The point force at t_k is wavelet sample k - 1 (the time convention of
    the scaled boundary stepper, whose step k solves for u at t_k under
    wavelet sample k - 1); u_0 = 0 and, with no force at t_0, u_1 = 0.
    """
    K, m = assemble(nx, ny, lx, ly, rho_e, c)
    src_nodes = np.asarray(src_nodes)
    rec_nodes = np.asarray(rec_nodes)
    wavelets = np.asarray(wavelets, dtype=np.float64)
    S, R = len(src_nodes), len(rec_nodes)
    n = m.shape[0]
    out = np.zeros((S, R, n_steps))
    for s in range(S):
        u_prev = np.zeros(n)
        u = np.zeros(n)
        out[s, :, 0] = u[rec_nodes]
        for k in range(1, n_steps):
            f = np.zeros(n)
            f[src_nodes[s]] += wavelets[s, k - 1]
            u_prev, u = u, step(K, m, u, u_prev, f, dt)
            out[s, :, k] = u[rec_nodes]
    return out
