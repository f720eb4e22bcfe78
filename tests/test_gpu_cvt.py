"""Centroidal Voronoi polygon meshes (n_b 4 .. 8 per cell, 5 or 7 radial
intervals) through the GPU path against the oracle, for both radial schemes.

Bars as elsewhere: traces to relative L2 <= 1e-10, gradients <= 1e-8, factors
<= 1e-11.  The full-size case is the 8000-cell plate of the timing-table
workload (7 intervals): the dynamic stiffness of sampled cells against the
oracle one by one and a finite gradient evaluation.
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import element as oel
from oracle import stepper as ostp

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu

SCHEMES = {0: "paper_fd", 1: "radial_galerkin"}


def _small(n_steps):
    m = W.cvt_mesh(0.02, 0.01, 60, 6, seed=5, lloyd_iters=30)
    wl = W.Workload("cvt-small", m, 6000.0, 2700.0, 2e-7, n_steps,
                    np.asarray([W.nearest_top_node(m, 0.007), W.nearest_top_node(m, 0.013)], dtype=np.int64),
                    np.repeat(W.sine_burst(n_steps, 2e-7, 5e5, 2, 1e12)[None], 2, axis=0),
                    W.edge_nodes(m)[::2].copy(), f0=5e5)
    pts = W.fine_point_positions(m)
    wl.models = {"homogeneous": W.homogeneous(m),
                 "random30": W.smooth_random_field(pts, 4 * 1000 + 7, 2700.0, 0.3, wavelength=0.006)}
    return wl


def _om(wl, rho, scheme):
    return ostp.Model(wl.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0, scheme=SCHEMES[scheme])


@pytest.mark.parametrize("scheme", [0, 1])
def test_cvt_forward_and_gradient_parity(scheme):
    wl = _small(120)
    rho = wl.models["random30"]
    log(f"cvt parity, scheme {scheme}: {wl.mesh.n_elem} cells, n_b {wl.mesh.n_b().min()}..{wl.mesh.n_b().max()}")
    g = GpuModel(wl, rho, coarse_solver=1, scheme=scheme)
    tr, _ = g.forward()
    ref = ostp.forward(_om(wl, rho, scheme), wl.src_nodes, wl.wavelets, wl.rec_nodes, wl.n_steps)
    err = rel_l2(tr.cpu().numpy(), ref)
    log(f"  traces relative L2 {err:.3e}")
    assert err <= 1e-10
    steps = 60
    obs = ostp.forward(_om(wl, wl.models["homogeneous"], scheme), wl.src_nodes, wl.wavelets[:, :steps],
                       wl.rec_nodes, steps)
    _, mis, grad, _ = g.gradient(obs, n_steps=steps, n_ckpt=-1, mode=0)
    gref, Jref = oadj.exact_gradient(_om(wl, rho, scheme), wl.src_nodes, wl.wavelets[:, :steps], wl.rec_nodes,
                                     obs, steps)
    gerr = rel_l2(grad, gref)
    log(f"  misfit {mis:.6e} vs {Jref:.6e}, gradient relative L2 {gerr:.3e}")
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)
    assert gerr <= 1e-8


def test_cvt_full_size_8000_cells():
    wl = W.config_cvt(8000, 7)
    mesh = wl.mesh
    log(f"cvt full size: {mesh.n_elem} cells, {mesh.n_nodes} nodes, {len(wl.rec_nodes)} receivers")
    rho = wl.models["hole_floor_half"]
    offs = mesh.param_offsets()
    nb = mesh.n_b().astype(np.int64)
    sample = np.random.default_rng(8).choice(mesh.n_elem, 12, replace=False)
    a0 = 1.0 / (wl.beta * wl.dt ** 2)
    for scheme in (0, 1):
        g = GpuModel(wl, rho, coarse_solver=1, scheme=scheme)
        S_gpu = g.sb.sbfwi_copy_factor_data(g.f, 0, int((nb ** 2).sum()))
        s_off = np.concatenate([[0], np.cumsum(nb ** 2)])
        worst = 0.0
        for e in sample:
            lp = mesh.loop(e)
            grp = oel.ElementGroup([e], lp[None], mesh.node_xy[lp][None],
                                   rho[offs[e]:offs[e + 1]].reshape(1, int(mesh.n_r[e]), int(nb[e])),
                                   wl.c, wl.xi0, a0, scheme=SCHEMES[scheme])
            worst = max(worst, rel_l2(S_gpu[s_off[e]:s_off[e + 1]], grp.f["S"][0].ravel()))
        log(f"  scheme {scheme}: sampled cells, worst S relative L2 {worst:.3e}")
        assert worst <= 1e-11
        tr, ck = g.forward(n_ckpt=-1)
        obs = 0.9 * tr
        _, mis, grad, _ = g.gradient(obs.cpu().numpy(), n_ckpt=-1)
        assert np.isfinite(tr.cpu().numpy()).all() and np.isfinite(grad).all() and mis > 0
