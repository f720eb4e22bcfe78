"""Pins of the bilinear finite element data generator (``oracle.fem``).

* element integrals: the closed-form unit stiffness equals a 2 x 2 Gauss
  quadrature of grad N_a . grad N_b written out from the bilinear shape
  functions (exact for these integrands);
* assembly: K symmetric positive semidefinite with constants in its null
  space (free boundary), lumped masses summing to the total mass;
* dispersion: products of cosines are exact eigenvectors of M^-1 K with the
  textbook symbol of Q1 stiffness over lumped mass, and central differences
  advance such a mode by cos(n theta), cos theta = 1 - dt^2 lambda / 2;
* conservation: without forces the staggered energy of central differences
  stays constant to rounding on a heterogeneous model;
* reciprocity and causality of the driver: swapping source and receiver
  leaves the trace unchanged; the first response at the source node is
  dt^2 w_0 / m and a node d grid steps away stays at rest until u_{d+2};
* convergence (not parity): traces of the scaled boundary oracle approach
  those of a fine finite element run as the scaled boundary mesh refines.
"""

import numpy as np
import pytest

import workloads as W
from oracle import fem
from oracle import stepper as stp


def _shape_grads(hx, hy, s, t):
    """Gradients of the four bilinear shape functions at reference point (s, t) in [0, 1]^2."""
    dNds = np.array([-(1 - t), (1 - t), t, -t])
    dNdt = np.array([-(1 - s), -s, s, (1 - s)])
    return dNds / hx, dNdt / hy


def test_unit_stiffness_equals_gauss_quadrature():
    for hx, hy in [(1.0, 1.0), (0.3, 0.7), (2e-4, 1e-4)]:
        g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
        k = np.zeros((4, 4))
        for s in g:
            for t in g:
                gx, gy = _shape_grads(hx, hy, s, t)
                k += (np.outer(gx, gx) + np.outer(gy, gy)) * hx * hy / 4.0
        np.testing.assert_allclose(fem.unit_stiffness(hx, hy), k, rtol=1e-13, atol=1e-13 * abs(k).max())


def test_assembly_invariants():
    nx, ny, lx, ly = 7, 5, 0.007, 0.004
    rng = np.random.default_rng(3)
    rho = 2700.0 * rng.uniform(1e-3, 2.0, nx * ny)
    K, m = fem.assemble(nx, ny, lx, ly, rho, 3000.0)
    Kd = K.toarray()
    assert abs(Kd - Kd.T).max() <= 1e-14 * abs(Kd).max()
    assert abs(Kd @ np.ones(Kd.shape[0])).max() <= 1e-12 * abs(Kd).max()
    ev = np.linalg.eigvalsh(Kd)
    assert ev.min() >= -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1          # only the constant mode
    np.testing.assert_allclose(m.sum(), rho.sum() * (lx / nx) * (ly / ny), rtol=1e-14)
    # corner node of the grid carries a quarter of its single element's mass
    np.testing.assert_allclose(m[0], rho[0] * (lx / nx) * (ly / ny) / 4.0, rtol=1e-14)


def test_cosine_modes_follow_the_discrete_dispersion_relation():
    nx, ny, lx, ly, c, dt = 12, 8, 0.012, 0.01, 3000.0, 1e-7
    K, m = fem.assemble(nx, ny, lx, ly, np.full(nx * ny, 2700.0), c)
    X = fem.grid_nodes(nx, ny, lx, ly)
    hx, hy = lx / nx, ly / ny
    for p, q in [(1, 0), (0, 3), (3, 2), (5, 7), (12, 8)]:
        phi = np.cos(p * np.pi * X[:, 0] / lx) * np.cos(q * np.pi * X[:, 1] / ly)
        tx, ty = p * np.pi * hx / lx, q * np.pi * hy / ly
        lam = c * c * ((2 - 2 * np.cos(tx)) / hx ** 2 * (2 + np.cos(ty)) / 3
                       + (2 + np.cos(tx)) / 3 * (2 - 2 * np.cos(ty)) / hy ** 2)
        np.testing.assert_allclose(K @ phi / m, lam * phi, atol=1e-12 * lam)
        ct = 1.0 - dt * dt * lam / 2.0
        assert abs(ct) < 1.0
        theta = np.arccos(ct)
        u_prev, u = phi.copy(), ct * phi
        for n in range(2, 60):
            u_prev, u = u, fem.step(K, m, u, u_prev, np.zeros_like(u), dt)
        np.testing.assert_allclose(u, np.cos(59 * theta) * phi, atol=1e-11)


def test_stable_step_bounds_the_spectrum():
    nx, ny, lx, ly, c = 9, 6, 0.009, 0.003, 3000.0
    rho = 2700.0 * np.random.default_rng(4).uniform(1e-5, 2.0, nx * ny)
    K, m = fem.assemble(nx, ny, lx, ly, rho, c)
    lam = np.linalg.eigvals(K.toarray() / m[:, None]).real.max()
    assert lam * fem.stable_dt(nx, ny, lx, ly, c) ** 2 <= 4.0 * (1 + 1e-12)


def test_energy_is_conserved_without_forces():
    nx, ny, lx, ly, c = 10, 6, 0.01, 0.006, 3000.0
    rng = np.random.default_rng(5)
    rho = 2700.0 * rng.uniform(1e-3, 2.0, nx * ny)
    K, m = fem.assemble(nx, ny, lx, ly, rho, c)
    dt = 0.9 * fem.stable_dt(nx, ny, lx, ly, c)
    u_prev = rng.standard_normal(m.shape[0])
    u = u_prev + 0.1 * rng.standard_normal(m.shape[0])

    def energy(u_new, u_old):
        v = (u_new - u_old) / dt
        return 0.5 * v @ (m * v) + 0.5 * u_new @ (K @ u_old)

    e0 = energy(u, u_prev)
    for _ in range(500):
        u_prev, u = u, fem.step(K, m, u, u_prev, np.zeros_like(u), dt)
        np.testing.assert_allclose(energy(u, u_prev), e0, rtol=1e-11)


def test_reciprocity_and_causality():
    nx, ny, lx, ly, c, dt, nt = 16, 9, 0.016, 0.009, 3000.0, 1e-7, 80
    rng = np.random.default_rng(6)
    rho = 2700.0 * rng.uniform(0.2, 2.0, nx * ny)
    w = W.ricker(nt, dt, 5e5, t0=1e-6)[None]
    a = 3 * (nx + 1) + 4
    b = 7 * (nx + 1) + 12
    ab = fem.forward(nx, ny, lx, ly, rho, c, dt, [a], w, [b], nt)
    ba = fem.forward(nx, ny, lx, ly, rho, c, dt, [b], w, [a], nt)
    np.testing.assert_allclose(ab, ba, rtol=0, atol=1e-12 * abs(ab).max())

    _, mass = fem.assemble(nx, ny, lx, ly, rho, c)
    far = a + 5                                       # 5 grid steps along x
    tr = fem.forward(nx, ny, lx, ly, rho, c, dt, [a], w, [a, far], nt)
    assert tr[0, 0, 0] == 0.0
    np.testing.assert_allclose(tr[0, 0, 1], dt * dt * w[0, 0] / mass[a], rtol=1e-14)
    assert np.all(tr[0, 1, :6] == 0.0) and tr[0, 1, 6] != 0.0        # u_7 is its first motion


def test_traces_converge_to_the_scaled_boundary_oracle():
    """Convergence, not parity: both discretise the same wave equation with
    the same source and time conventions."""
    lx = ly = 0.02
    dt, nt = 5e-8, 200
    w = W.ricker(nt, dt, 5e5)[None]
    nf = 128
    diffs = []
    for ne in (8, 16):
        mesh = W.uniform_rect_mesh(lx, ly, ne, ne, segs=2, n_r=16)
        src = np.array([W.nearest_top_node(mesh, 0.01)])
        rec = np.array([W.nearest_top_node(mesh, x) for x in np.linspace(0.00125, 0.01875, 8)])
        tr = stp.forward(stp.Model(mesh, W.homogeneous(mesh), 3000.0, dt), src, w, rec, nt)
        h = lx / nf

        def fnode(n):
            i, j = np.rint(mesh.node_xy[n] / h).astype(int)
            assert np.allclose(mesh.node_xy[n], (i * h, j * h), atol=1e-12)
            return j * (nf + 1) + i

        tf = fem.forward(nf, nf, lx, ly, np.full(nf * nf, 2700.0), 3000.0, dt,
                         [fnode(n) for n in src], w, [fnode(n) for n in rec], nt)
        diffs.append(np.linalg.norm(tf - tr) / np.linalg.norm(tr))
    assert diffs[1] < 0.1 and diffs[1] < 0.5 * diffs[0], diffs
