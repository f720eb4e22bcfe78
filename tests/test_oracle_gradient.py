"""Pins of the oracle gradient.

* complex step: Im J(rho + i h e_p) / h is the exact derivative of the
  oracle's own forward map (h = 1e-30 rho_p); the adjoint gradient must
  match it to rounding;
* central finite differences with h = 1e-6 relative;
* dot-product test <F dm, dd> = <dm, F^T dd>, F the linearised
  density-to-trace map (F dm by complex step, F^T dd from the adjoint);
* a ragged mesh (several (n_b, N_r) groups);
* the paper's truncated kernel: recomputed from forward and back-propagated
  velocities of the dense uncondensed system (no condensation, no coarse
  assembly), -dt sum_k' v~^{k'} v^{N_t+1-k'} with the residual u - d as the
  back-propagated source, element by element; a one-step shift of the
  reversed index or a dt-weighted source must not pass that comparison; and
  it correlates positively with the exact gradient (the sign reading).
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj
from oracle import stepper as stp

from ._dense import DenseSystem


def _case(mesh=None, nt=14, seed=5):
    if mesh is None:
        mesh = W.uniform_rect_mesh(0.005, 0.005, 2, 2, segs=2, n_r=6)
    pts = W.fine_point_positions(mesh)
    rho = W.smooth_random_field(pts, seed, 2700.0, 0.3, wavelength=0.004)
    dt = 5e-8
    lx = mesh.extent[0]
    src = np.array([W.nearest_top_node(mesh, lx / 2)])
    rec = W.top_edge_nodes(mesh)[::2]
    wav = W.ricker(nt, dt, 5e5, t0=2e-7)[None] * 1e6
    m = stp.Model(mesh, rho, 3000.0, dt)
    tr = stp.forward(m, src, wav, rec, nt)
    obs = 0.8 * tr + 0.05 * np.abs(tr).max() * np.sin(np.arange(tr.size)).reshape(tr.shape)
    return mesh, rho, dt, nt, src, rec, wav, m, tr, obs


def _complex_step(mesh, rho, dt, nt, src, rec, wav, obs, p):
    h = 1e-30 * rho[p]
    rc = rho.astype(complex)
    rc[p] += 1j * h
    mc = stp.Model(mesh, rc, 3000.0, dt)
    return stp.misfit(stp.forward(mc, src, wav, rec, nt), obs, dt).imag / h


def test_exact_gradient_matches_complex_step():
    mesh, rho, dt, nt, src, rec, wav, m, tr, obs = _case()
    grad, J = adj.exact_gradient(m, src, wav, rec, obs, nt)
    assert J == pytest.approx(stp.misfit(tr, obs, dt), rel=1e-14)
    scale = np.abs(grad).max()
    for p in np.random.default_rng(1).choice(mesh.n_params, 8, replace=False):
        cs = _complex_step(mesh, rho, dt, nt, src, rec, wav, obs, p)
        assert abs(grad[p] - cs) <= 1e-9 * scale + 1e-9 * abs(cs)


def test_exact_gradient_matches_central_differences():
    mesh, rho, dt, nt, src, rec, wav, m, tr, obs = _case(seed=9)
    grad, _ = adj.exact_gradient(m, src, wav, rec, obs, nt)
    scale = np.abs(grad).max()
    for p in np.random.default_rng(2).choice(mesh.n_params, 4, replace=False):
        h = 1e-6 * rho[p]
        jp, jm = [], []
        for sgn, acc in ((1, jp), (-1, jm)):
            r = rho.copy()
            r[p] += sgn * h
            acc.append(stp.misfit(stp.forward(stp.Model(mesh, r, 3000.0, dt), src, wav, rec, nt), obs, dt))
        fd = (jp[0] - jm[0]) / (2 * h)
        assert abs(fd - grad[p]) <= 1e-6 * scale


def test_dot_product():
    mesh, rho, dt, nt, src, rec, wav, m, tr, obs = _case(seed=13)
    rng = np.random.default_rng(4)
    dm = rng.standard_normal(mesh.n_params) * rho * 1e-3
    dd = rng.standard_normal(tr.shape)
    # F dm by complex step
    h = 1e-30
    mc = stp.Model(mesh, rho + 1j * h * dm, 3000.0, dt)
    Fdm = stp.forward(mc, src, wav, rec, nt).imag / h
    # F^T dd: gradient of sum dt (u - obs') dd with obs' = u - dd/dt... use J' = sum dd * u
    obs2 = tr - dd / dt
    FTdd, _ = adj.exact_gradient(m, src, wav, rec, obs2, nt)
    lhs = np.sum(Fdm * dd)
    rhs = np.sum(dm * FTdd)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), abs(rhs))


def test_ragged_mesh_gradient():
    mesh = W.quadtree_mesh(0.01, 0.005, base_level=1, max_level=2, refine_centres=[(0.003, 0.002)],
                           refine_radius=0.001, n_r_max=6, n_r_min=3)
    assert len(set(zip(mesh.n_b().tolist(), mesh.n_r.tolist()))) >= 2
    mesh, rho, dt, nt, src, rec, wav, m, tr, obs = _case(mesh=mesh, nt=10)
    grad, _ = adj.exact_gradient(m, src, wav, rec, obs, nt)
    scale = np.abs(grad).max()
    for p in np.random.default_rng(3).choice(mesh.n_params, 6, replace=False):
        cs = _complex_step(mesh, rho, dt, nt, src, rec, wav, obs, p)
        assert abs(grad[p] - cs) <= 1e-9 * scale + 1e-9 * abs(cs)


def test_paper_kernel_correlates_with_exact_gradient():
    cfg = W.config_tiny(n_steps=80)
    m = stp.Model(cfg.mesh, cfg.models["homogeneous"], cfg.c, cfg.dt)
    mv = stp.Model(cfg.mesh, cfg.models["void_floor_half"], cfg.c, cfg.dt)
    obs = stp.forward(mv, cfg.src_nodes, cfg.wavelets, cfg.rec_nodes, cfg.n_steps)
    g, _ = adj.exact_gradient(m, cfg.src_nodes, cfg.wavelets, cfg.rec_nodes, obs, cfg.n_steps)
    gp, _ = adj.paper_kernel_gradient(m, cfg.src_nodes, cfg.wavelets, cfg.rec_nodes, obs,
                                      cfg.n_steps, sign=-1.0)
    assert np.corrcoef(g, gp)[0, 1] > 0.5


def _dense_paper_kernel(dense, src, wav, rec, obs, nt, dt, shift=0, source_weight=1.0):
    fwd = dense.run(src, wav, nt)
    traces = np.stack([f["U"][rec] for f in fwd], axis=-1)          # [n_rec, nt]
    res = source_weight * (traces - obs[0])
    # reversed step k' applies r^{N_t + 1 - k'} = res[:, nt - k']
    bwd = dense.run(rec, res[:, ::-1], nt)
    g = np.zeros_like(fwd[0]["v_fine"])
    for kp in range(1, nt + 1):
        kf = nt + 1 - kp - shift                                    # forward step paired with k'
        if 1 <= kf <= nt:
            g -= dt * bwd[kp - 1]["v_fine"] * fwd[kf - 1]["v_fine"]
    return g, traces


def test_paper_kernel_equals_dense_recomputation():
    mesh, rho, dt, nt, src, rec, wav, m, tr, obs = _case(seed=21)
    gp, tr_o = adj.paper_kernel_gradient(m, src, wav, rec, obs, nt)
    dense = DenseSystem(m)
    g, tr_d = _dense_paper_kernel(dense, src, wav, rec, obs, nt, dt)
    assert np.abs(tr_d - tr_o[0]).max() <= 1e-9 * np.abs(tr_d).max()
    scale = np.abs(g).max()
    assert scale > 0
    assert np.abs(gp - g).max() <= 1e-8 * scale
    # planted mistakes: the reversed index shifted by one step either way, and a
    # back-propagated source weighted by dt, each differ from the oracle far
    # beyond the tolerance above
    for sh in (1, -1):
        gs, _ = _dense_paper_kernel(dense, src, wav, rec, obs, nt, dt, shift=sh)
        assert np.abs(gp - gs).max() > 1e-2 * scale
    gw, _ = _dense_paper_kernel(dense, src, wav, rec, obs, nt, dt, source_weight=dt)
    assert np.abs(gp - gw).max() > 0.5 * scale
