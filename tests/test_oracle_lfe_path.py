"""Pins of the low-frequency expansion time-domain path (``oracle.lfe``).

* the element K, M from the radial condensation converge to the Riccati and
  Lyapunov solutions (the textbook eigenvalue method and SciPy's Lyapunov
  solver) at second order as the radial levels refine, on a square and on a
  Voronoi polygon;
* K is symmetric with the constants in its null space; M is symmetric
  positive definite and carries the element's mass between xi0 and the
  boundary, 1^T M 1 = (1 - xi0^2) / 2 * 1^T M0 1;
* the assembled Newmark loop conserves 1/2 V^T M V + 1/2 U^T K U to rounding
  once the source has stopped;
* the paper's truncated kernel on this path equals its recomputation from
  nodal velocities obtained by modal superposition (generalised symmetric
  eigenvectors of K and M, every mode advanced by the trapezoidal rule, which
  is average-acceleration Newmark for zero initial state and load), with the
  residual u - d as the back-propagated source; a one-step shift of the
  reversed index must not pass.
"""

import numpy as np
import pytest

import workloads as W
from oracle import element as el
from oracle import lfe


def _elem(kind):
    if kind == "square":
        m = W.uniform_rect_mesh(0.004, 0.004, 1, 1, segs=2, n_r=3)
    else:
        m = W.cvt_mesh(0.01, 0.01, 9, 3, seed=2, lloyd_iters=20)
    lp = m.loop(4 if kind != "square" else 0)
    xy = m.node_xy[lp][None]
    rho = np.full((1, 1, len(lp)), 2700.0)
    rho[0, 0, 1] = 1800.0
    E = [x[0, 0] for x in el.coefficient_matrices(xy, el.polygon_centroid(xy), rho, 3000.0)]
    return xy[0], E


@pytest.mark.parametrize("kind", ["square", "polygon"])
def test_condensed_matrices_converge_to_riccati_and_lyapunov(kind):
    xy, (E0, E1, E2, M0) = _elem(kind)
    K_ref, _ = lfe.lfe_stiffness(E0, E1, E2)
    M_ref = lfe.lfe_mass(K_ref, E0, E1, M0)
    ek, em = [], []
    for nr in (9, 17, 33):
        xi, _ = el.radial_levels(nr, 1e-3)
        K, M = lfe.condensed_matrices(E0, E1, E2, M0, xi)
        ek.append(np.abs(K - K_ref).max() / np.abs(K_ref).max())
        em.append(np.abs(M - M_ref).max() / np.abs(M_ref).max())
    assert ek[2] < 1e-3 and em[2] < 1e-3, (ek, em)
    assert ek[1] < 0.4 * ek[0] and ek[2] < 0.4 * ek[1], ek
    assert em[1] < 0.4 * em[0] and em[2] < 0.4 * em[1], em


def test_condensed_matrices_invariants():
    xy, (E0, E1, E2, M0) = _elem("polygon")
    xi, _ = el.radial_levels(12, 1e-3)
    K, M = lfe.condensed_matrices(E0, E1, E2, M0, xi)
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(K @ np.ones(len(K))).max() <= 1e-10 * np.abs(K).max()
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    # 1^T M 1 = integral of rho over the element between xi0 and 1: (1 - xi0^2) / 2 * 1^T M0 1
    np.testing.assert_allclose(M.sum(), 0.5 * (1.0 - 1e-3 ** 2) * M0.sum(), rtol=1e-12)


def test_lfe_loop_conserves_energy():
    mesh = W.cvt_mesh(0.01, 0.01, 12, 10, seed=4, lloyd_iters=20)
    pts = W.fine_point_positions(mesh)
    rho = W.smooth_random_field(pts, 9, 2700.0, 0.3, wavelength=0.006)
    dt = 1e-7
    model = lfe.LfeModel(mesh, rho, 3000.0, dt)
    nm = model.nm
    src = W.nearest_top_node(mesh, 0.005)
    wav = W.ricker(30, dt, 5e5, t0=1e-6)
    n = mesh.n_nodes
    U, V, A = np.zeros(n), np.zeros(n), np.zeros(n)
    energies = []
    for k in range(1, 231):
        Wv = nm.a0 * U + nm.a1 * V + nm.a2 * A
        F = model.M @ Wv
        if k <= 30:
            F[src] += wav[k - 1]
        Un = model.lu.solve(F)
        V = nm.c1 * (Un - U) + nm.c2 * V + nm.c3 * A
        A = nm.a0 * Un - Wv
        U = Un
        if k > 30:
            energies.append(0.5 * V @ (model.M @ V) + 0.5 * U @ (model.K @ U))
    energies = np.asarray(energies)
    assert energies[0] > 0 and np.abs(energies - energies[0]).max() <= 1e-11 * energies[0]


def test_lfe_paper_kernel_agrees_in_sign_with_finite_differences():
    """The truncated kernel is an approximation (parity unpinned beyond this):
    it must be a direction of increasing misfit and agree in sign with the
    finite-difference derivative along the direction to the data model."""
    wl = W.config_tiny(120)
    m = wl.mesh
    rho = wl.models["random30"]
    rho0 = wl.models["homogeneous"]

    def run(r):
        return lfe.lfe_forward(lfe.LfeModel(m, r, wl.c, wl.dt), wl.src_nodes, wl.wavelets, wl.rec_nodes, 120)

    obs = run(rho0)
    g, _ = lfe.lfe_paper_kernel_gradient(lfe.LfeModel(m, rho, wl.c, wl.dt), wl.src_nodes, wl.wavelets,
                                         wl.rec_nodes, obs, 120)
    J = lambda r: 0.5 * wl.dt * np.sum((run(r) - obs) ** 2)
    offs = m.param_offsets()
    bnd = np.zeros(m.n_params, dtype=bool)
    for e in range(m.n_elem):
        bnd[offs[e] + (m.n_r[e] - 1) * m.n_b()[e]:offs[e + 1]] = True
    assert np.all(g[~bnd] == 0.0) and np.abs(g[bnd]).max() > 0
    h = 1e-4
    d = np.where(bnd, rho0 - rho, 0.0)
    fd_d = (J(rho + h * d) - J(rho - h * d)) / (2 * h)
    assert fd_d < 0 and g @ d < 0
    step = 1e-3 * np.abs(rho).max() / np.abs(g).max()
    fd_g = (J(rho + step * g) - J(rho - step * g)) / (2 * step)
    assert fd_g > 0


def _modal_velocities(K, M, dt, nodes, amps, nt):
    """Nodal velocities of M u'' + K u = f, f^k = amps[:, k - 1] at nodes, zero
    initial state, by modal superposition and the trapezoidal rule per mode."""
    import scipy.linalg as sla
    w2, Phi = sla.eigh(K, M)
    n = K.shape[0]
    eta, deta = np.zeros(n), np.zeros(n)
    g_old = np.zeros(n)
    out = []
    h = 0.5 * dt
    det = 1.0 + h * h * w2
    for k in range(1, nt + 1):
        f = np.zeros(n)
        np.add.at(f, nodes, amps[:, k - 1])
        g = Phi.T @ f
        # (I - h A) x' = (I + h A) x + h (b + b'),  A = [[0, 1], [-w2, 0]], b = [0, g]
        r0 = eta + h * deta
        r1 = deta - h * w2 * eta + h * (g_old + g)
        eta, deta = (r0 + h * r1) / det, (r1 - h * w2 * r0) / det
        g_old = g
        out.append(Phi @ deta)
    return out


def test_lfe_paper_kernel_equals_modal_recomputation():
    wl = W.config_tiny(40)
    m = wl.mesh
    model = lfe.LfeModel(m, wl.models["random30"], wl.c, wl.dt)
    obs = lfe.lfe_forward(lfe.LfeModel(m, wl.models["homogeneous"], wl.c, wl.dt), wl.src_nodes, wl.wavelets,
                          wl.rec_nodes, 40)
    g, tr = lfe.lfe_paper_kernel_gradient(model, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, 40)
    K, M = model.K.toarray(), model.M.toarray()
    K, M = 0.5 * (K + K.T), 0.5 * (M + M.T)
    nt, dt = 40, wl.dt
    vf = _modal_velocities(K, M, dt, wl.src_nodes, wl.wavelets[:, :nt], nt)
    tr_m = np.zeros_like(tr[0])
    # displacements for the residual: integrate the same modal run (u from the trapezoidal rule)
    u = np.zeros(m.n_nodes)
    v_old = np.zeros(m.n_nodes)
    for k in range(nt):
        u = u + 0.5 * dt * (v_old + vf[k])
        v_old = vf[k]
        tr_m[:, k] = u[wl.rec_nodes]
    assert np.abs(tr_m - tr[0]).max() <= 1e-8 * np.abs(tr[0]).max()
    res = tr_m - obs[0]
    vb = _modal_velocities(K, M, dt, wl.rec_nodes, res[:, ::-1], nt)

    def kernel(shift):
        kern = np.zeros(m.n_nodes)
        for kp in range(1, nt + 1):
            kf = nt + 1 - kp - shift
            if 1 <= kf <= nt:
                kern -= dt * vb[kp - 1] * vf[kf - 1]
        out = np.zeros(m.n_params)
        offs = m.param_offsets()
        for e in range(m.n_elem):
            lp = m.loop(e)
            nb, nr = len(lp), int(m.n_r[e])
            out[offs[e] + (nr - 1) * nb:offs[e + 1]] = kern[lp]
        return out

    ref = kernel(0)
    scale = np.abs(ref).max()
    assert scale > 0 and np.abs(g - ref).max() <= 1e-7 * scale
    for sh in (1, -1):
        assert np.abs(g - kernel(sh)).max() > 1e-2 * scale
