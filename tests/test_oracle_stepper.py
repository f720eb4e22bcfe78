"""Pins of the oracle's time loop.

* brute force: every step of the condensed scheme (condense, coarse solve,
  recover, ghosts) equals a dense solve of the whole uncondensed system
  (all element rows of eq. system plus the assembled flux rows);
* undamped average-acceleration Newmark maps a real spectrum onto the unit
  circle: on a homogeneous element every step-map eigenvalue has |mu| = 1,
  apart from the rigid-body pair at mu = 1;
* the stability gate separates a stable homogeneous plate (17 levels) from
  a coarse one (9 levels) whose step map grows over a 4000-step window;
* the misfit is 1/2 sum dt (u - d)^2.
"""

import numpy as np
import pytest

import workloads as W
from oracle import stepper as stp
from oracle import stability as stab

from ._dense import DenseSystem


def _tiny(n_r=6, nx=2, seed=5):
    mesh = W.uniform_rect_mesh(0.005, 0.0025 * nx / 2 * 2, nx, 2, segs=2, n_r=n_r)
    pts = W.fine_point_positions(mesh)
    rho = W.smooth_random_field(pts, seed, 2700.0, 0.3, wavelength=0.004)
    return mesh, rho


def test_condensed_step_equals_dense_uncondensed_solve():
    mesh, rho = _tiny()
    dt, nt = 5e-8, 10
    src = np.array([W.nearest_top_node(mesh, 0.0025)])
    rec = W.top_edge_nodes(mesh)
    wav = W.ricker(nt, dt, 5e5, t0=2e-7)[None]
    m = stp.Model(mesh, rho, 3000.0, dt)
    _, trajs = stp.forward(m, src, wav, rec, nt, keep=True)
    dense = DenseSystem(m).run(src, wav, nt)
    for k in range(1, nt + 1):
        Xd = dense[k - 1]["X"]
        Xc = trajs[0][k - 1]["full"][0]["X"]
        assert np.abs(Xd - Xc).max() <= 1e-9 * np.abs(Xd).max()


def test_newmark_unit_modulus_on_homogeneous_element():
    mesh = W.uniform_rect_mesh(0.0025, 0.0025, 1, 1, segs=2, n_r=6)
    m = stp.Model(mesh, W.homogeneous(mesh), 3000.0, 5e-8)
    mu = stab.step_map_eigenvalues(m)
    mu = mu[np.abs(mu) > 1e-9]                    # a^k is a function of (u, v): zero modes
    mu = mu[np.abs(mu - 1.0) > 1e-5]              # rigid-body Jordan pair
    assert mu.size > 0
    assert np.abs(np.abs(mu) - 1.0).max() < 1e-10


def test_stability_gate_separates_models():
    mesh17 = W.uniform_rect_mesh(0.005, 0.005, 2, 2, segs=2, n_r=17)
    mesh9 = W.uniform_rect_mesh(0.005, 0.005, 2, 2, segs=2, n_r=9)
    mu17 = stab.step_map_eigenvalues(stp.Model(mesh17, W.homogeneous(mesh17), 3000.0, 2e-8))
    mu9 = stab.step_map_eigenvalues(stp.Model(mesh9, W.homogeneous(mesh9), 3000.0, 2e-8))
    inband17, worst17 = stab.gate(mu17[np.abs(mu17 - 1) > 1e-5], 2e-8, 4000, 5e5)
    _, worst9 = stab.gate(mu9[np.abs(mu9 - 1) > 1e-5], 2e-8, 4000, 5e5)
    assert inband17 <= 1 + 1e-6 and worst17 <= 10.0
    assert worst9 > 10.0


def test_misfit_definition():
    tr = np.array([[[1.0, 2.0, 3.0]]])
    ob = np.array([[[0.0, 2.0, 5.0]]])
    assert stp.misfit(tr, ob, 0.5) == pytest.approx(0.5 * 0.5 * (1 + 0 + 4))


def test_newmark_constants_average_acceleration():
    nm = stp.Newmark(2e-8)
    assert nm.a0 == pytest.approx(4 / 2e-8 ** 2) and nm.a1 == pytest.approx(4 / 2e-8)
    assert nm.a2 == pytest.approx(1.0) and nm.c1 == pytest.approx(2 / 2e-8)
    assert nm.c2 == pytest.approx(-1.0) and nm.c3 == pytest.approx(0.0)
