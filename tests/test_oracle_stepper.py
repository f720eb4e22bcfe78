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
from oracle import element as el
from oracle import stepper as stp
from oracle import stability as stab


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
    g = m.groups[0]
    n, nb, E = g.n, g.n_b, len(g.elem_ids)
    Ae = el.element_system(g.theta, g.phi, g.psi)
    # global unknowns: per element levels -1..n-1, n+1 (internal), then the nodes
    blocks = list(range(0, n + 1)) + [n + 2]
    ic = np.concatenate([np.arange(b * nb, (b + 1) * nb) for b in blocks])
    bc = np.arange((n + 1) * nb, (n + 2) * nb)
    ir = np.arange(0, (n + 2) * nb)
    br = np.arange((n + 2) * nb, (n + 3) * nb)
    NI = ic.size
    N = E * NI + mesh.n_nodes
    A = np.zeros((N, N))
    for e in range(E):
        sl = slice(e * NI, (e + 1) * NI)
        nodes = E * NI + g.loops[e]
        A[sl, sl] = Ae[e][np.ix_(ir, ic)]
        A[sl, nodes] += Ae[e][np.ix_(ir, bc)]
        A[np.ix_(nodes, np.arange(e * NI, (e + 1) * NI))] += Ae[e][np.ix_(br, ic)]
        A[np.ix_(nodes, nodes)] += Ae[e][np.ix_(br, bc)]
    nm = m.nm
    U = V = Acc = np.zeros(mesh.n_nodes)
    u = v = a = np.zeros((E, n, nb))
    for k in range(1, nt + 1):
        Wn = nm.a0 * U + nm.a1 * V + nm.a2 * Acc
        wi = nm.a0 * u + nm.a1 * v + nm.a2 * a
        p = np.einsum("ejab,ejb->eja", g.P, np.concatenate([wi, Wn[g.loops][:, None]], 1))
        b = np.zeros(N)
        for e in range(E):
            b[e * NI + nb:e * NI + (n + 2) * nb] = p[e].ravel()
        b[E * NI + src[0]] += wav[0, k - 1]
        X = np.linalg.solve(A, b)
        Un = X[E * NI:]
        loc = X[:E * NI].reshape(E, n + 2, nb)
        un = loc[:, 1:n + 1]
        U, V, Acc = Un, nm.c1 * (Un - U) + nm.c2 * V + nm.c3 * Acc, nm.a0 * Un - Wn
        u, v, a = un, nm.c1 * (un - u) + nm.c2 * v + nm.c3 * a, nm.a0 * un - wi
        Xd = np.concatenate([loc[:, :n + 1], U[g.loops][:, None], loc[:, n + 1:]], axis=1)
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
