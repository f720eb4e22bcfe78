"""Low-frequency expansion path on the GPU against the oracle.

Scheme 2: K_e from the Riccati equation (device: matrix sign function) and M_e
from the Lyapunov equation (device: Newton iteration), against the oracle's
eigenvalue method and SciPy's Lyapunov solver.  Scheme 3: the condensed
variant (radial Galerkin levels), against the oracle's condensation.
Bars: element K_e, M_e and the assembled K_g + a0 M_g, M_g to 1e-11 relative;
traces to relative L2 <= 1e-10; the paper-kernel gradient (the path's only
gradient) to 1e-8.  Cases: the tiny plate (direct and iterative
coarse solvers), a small Voronoi plate, and on the 8000-cell Voronoi plate
with 33 radial levels sampled cells one by one and a finite 200-step run.
"""

import numpy as np
import pytest

import workloads as W
from oracle import element as oel
from oracle import lfe as olfe

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu

LFE = 2
LFE_CONDENSED = 3
METHOD = {LFE: "riccati", LFE_CONDENSED: "condensed"}


def _cvt_small(n_steps, n_r=12):
    m = W.cvt_mesh(0.02, 0.01, 60, n_r, seed=5, lloyd_iters=30)
    wl = W.Workload("cvt-small", m, 6000.0, 2700.0, 2e-7, n_steps,
                    np.asarray([W.nearest_top_node(m, 0.007), W.nearest_top_node(m, 0.013)], dtype=np.int64),
                    np.repeat(W.sine_burst(n_steps, 2e-7, 5e5, 2, 1e12)[None], 2, axis=0),
                    W.edge_nodes(m)[::2].copy(), f0=5e5)
    pts = W.fine_point_positions(m)
    wl.models = {"random30": W.smooth_random_field(pts, 4 * 1000 + 7, 2700.0, 0.3, wavelength=0.006)}
    return wl


def _per_elem(g, which, mesh):
    nb = mesh.n_b().astype(np.int64)
    return g.sb.sbfwi_copy_factor_data(g.f, which, int((nb ** 2).sum()))


@pytest.mark.parametrize("cfg,scheme", [("tiny", LFE), ("cvt", LFE), ("tiny", LFE_CONDENSED),
                                        ("cvt", LFE_CONDENSED)])
def test_lfe_factor_and_forward_parity(cfg, scheme):
    wl = W.config_tiny(200) if cfg == "tiny" else _cvt_small(120)
    rho = wl.models["random30"]
    log(f"lfe parity {cfg}, scheme {scheme}: {wl.mesh.n_elem} elements, {wl.n_steps} steps")
    om = olfe.LfeModel(wl.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0, method=METHOD[scheme])
    ref = olfe.lfe_forward(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, wl.n_steps)
    for solver in (1, 0):
        g = GpuModel(wl, rho, coarse_solver=solver, scheme=scheme)
        Ke = _per_elem(g, 0, wl.mesh)
        Me = _per_elem(g, 4, wl.mesh)
        eK = max(rel_l2(Ke[o:o + k.size], k.ravel()) for o, k in zip(np.cumsum([0] + [k.size for k in om.Ke]), om.Ke))
        eM = max(rel_l2(Me[o:o + k.size], k.ravel()) for o, k in zip(np.cumsum([0] + [k.size for k in om.Me]), om.Me))
        log(f"  coarse solver {solver}: worst element K_e {eK:.2e}, M_e {eM:.2e}")
        assert eK <= 1e-11 and eM <= 1e-11
        rp, col = g.sb.sbfwi_coarse_pattern(g.mesh)
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        Keff = om.K + om.nm.a0 * om.M
        assert rel_l2(g.sb.sbfwi_copy_factor_data(g.f, 1, len(col)), np.asarray(Keff[rows, col]).ravel()) <= 1e-11
        assert rel_l2(g.sb.sbfwi_copy_factor_data(g.f, 5, len(col)), np.asarray(om.M[rows, col]).ravel()) <= 1e-11
        tr, _ = g.forward()
        err = rel_l2(tr.cpu().numpy(), ref)
        log(f"  coarse solver {solver}: traces relative L2 {err:.3e}")
        assert err <= 1e-10


@pytest.mark.parametrize("scheme", [LFE, LFE_CONDENSED])
def test_lfe_full_size_8000_cells(scheme):
    base = W.config_cvt(8000, 7)
    wl = W.config_cvt(8000, 32, mesh=base.mesh)
    mesh = wl.mesh
    rho = wl.models["hole_floor_half"]
    log(f"lfe full size, scheme {scheme}: {mesh.n_elem} cells, 33 radial levels")
    g = GpuModel(wl, rho, coarse_solver=1, scheme=scheme)
    Ke, Me = _per_elem(g, 0, mesh), _per_elem(g, 4, mesh)
    nb = mesh.n_b().astype(np.int64)
    off = np.concatenate([[0], np.cumsum(nb ** 2)])
    offs = mesh.param_offsets()
    worst = 0.0
    for e in np.random.default_rng(9).choice(mesh.n_elem, 12, replace=False):
        lp = mesh.loop(e)
        xy = mesh.node_xy[lp][None]
        nr = int(mesh.n_r[e])
        rb = rho[offs[e]:offs[e + 1]].reshape(nr, len(lp))[nr - 1][None, None]
        E = [x[0, 0] for x in oel.coefficient_matrices(xy, oel.polygon_centroid(xy), rb, wl.c)]
        if scheme == LFE:
            K = olfe.lfe_stiffness(E[0], E[1], E[2])[0]
            M = olfe.lfe_mass(K, E[0], E[1], E[3])
        else:
            K, M = olfe.condensed_matrices(*E, oel.radial_levels(nr, wl.xi0)[0])
        worst = max(worst, rel_l2(Ke[off[e]:off[e + 1]], K.ravel()), rel_l2(Me[off[e]:off[e + 1]], M.ravel()))
    log(f"  sampled cells: worst K_e, M_e relative L2 {worst:.3e}")
    assert worst <= 1e-11
    tr, _ = g.forward()
    tr = tr.cpu().numpy()
    assert np.isfinite(tr).all() and np.abs(tr).max() > 0


@pytest.mark.parametrize("cfg,scheme", [("tiny", LFE), ("cvt", LFE), ("tiny", LFE_CONDENSED)])
def test_lfe_paper_kernel_gradient_parity(cfg, scheme):
    wl = W.config_tiny(120) if cfg == "tiny" else _cvt_small(100)
    rho = wl.models["random30"]
    om0 = olfe.LfeModel(wl.mesh, rho * 0.9, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0, method=METHOD[scheme])
    obs = olfe.lfe_forward(om0, wl.src_nodes, wl.wavelets, wl.rec_nodes, wl.n_steps)
    log(f"lfe paper-kernel gradient parity {cfg}, scheme {scheme}")
    g = GpuModel(wl, rho, coarse_solver=1, scheme=scheme)
    tr, mis, grad, _ = g.gradient(obs, n_ckpt=-1, mode=1)
    om = olfe.LfeModel(wl.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0, method=METHOD[scheme])
    gref, tref = olfe.lfe_paper_kernel_gradient(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, wl.n_steps)
    err = rel_l2(grad, gref)
    log(f"  traces {rel_l2(tr, tref):.3e}, gradient relative L2 {err:.3e}")
    assert rel_l2(tr, tref) <= 1e-10 and err <= 1e-8
    with pytest.raises(g.sb.SbfwiError, match="paper-kernel gradient only"):
        g.gradient(obs, n_ckpt=-1, mode=0)
