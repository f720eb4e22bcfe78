"""Centroidal Voronoi polygon meshes (``workloads.cvt_mesh``): valid inputs for
the scaled boundary path.

* conforming: every interior segment is shared by exactly two cells, every
  other one lies on the plate's boundary; the cell areas sum to the plate's;
* every loop is counter-clockwise and star-convex about its area centroid
  (every segment has a positive determinant seen from it), with 3 .. 24 nodes;
* no segment is shorter than a tenth of the mean cell size;
* the mesh is reproducible from its seed, and the timing-table workload puts
  its two sources 30 mm apart on the top edge and its receivers on the edges;
* the oracle's radial Galerkin step on such a mesh conserves the energy
  behaviour of a stable scheme (bounded traces over the 200-step window).
"""

import numpy as np

import workloads as W
from oracle import element as el
from oracle import stepper as stp


def _check_mesh(m, lx, ly):
    edges = {}
    area = 0.0
    for e in range(m.n_elem):
        lp = m.loop(e)
        assert 3 <= len(lp) <= 24
        xy = m.node_xy[lp]
        x, y = xy[:, 0], xy[:, 1]
        a = 0.5 * (x * np.roll(y, -1) - np.roll(x, -1) * y).sum()
        assert a > 0
        area += a
        c = el.polygon_centroid(xy[None])[0]
        r = xy - c
        d = np.roll(xy, -1, axis=0) - xy
        assert (r[:, 0] * d[:, 1] - r[:, 1] * d[:, 0] > 0).all()
        for p, q in zip(lp, np.roll(lp, -1)):
            k = (min(p, q), max(p, q))
            edges[k] = edges.get(k, 0) + 1
    assert abs(area - lx * ly) <= 1e-12 * lx * ly
    h = np.sqrt(lx * ly / m.n_elem)
    bnd = set(W.edge_nodes(m).tolist())
    for (p, q), cnt in edges.items():
        assert np.hypot(*(m.node_xy[p] - m.node_xy[q])) >= 0.1 * h
        if cnt == 1:
            assert p in bnd and q in bnd
            xp, xq = m.node_xy[p], m.node_xy[q]
            assert (xp[0] == xq[0] and xp[0] in (0.0, lx)) or (xp[1] == xq[1] and xp[1] in (0.0, ly))
        else:
            assert cnt == 2


def test_cvt_mesh_is_a_valid_polygon_mesh():
    for n in (40, 300):
        m = W.cvt_mesh(0.1, 0.05, n, 6, seed=11 + n, lloyd_iters=25)
        assert m.n_elem == n
        _check_mesh(m, 0.1, 0.05)
    a = W.cvt_mesh(0.1, 0.05, 40, 6, seed=3, lloyd_iters=10)
    b = W.cvt_mesh(0.1, 0.05, 40, 6, seed=3, lloyd_iters=10)
    assert np.array_equal(a.node_xy, b.node_xy) and np.array_equal(a.elem_nodes, b.elem_nodes)


def test_timing_table_workload_shape():
    wl = W.config_cvt(1000, 5, lloyd_iters=10)
    m = wl.mesh
    assert (m.n_r == 6).all() and wl.n_steps == 200 and wl.dt == 2e-7 and wl.c == 6000.0
    xs = m.node_xy[wl.src_nodes]
    assert np.allclose(xs[:, 1], 0.05) and abs(abs(xs[1, 0] - xs[0, 0]) - 0.03) < 0.005
    assert set(wl.rec_nodes.tolist()) <= set(W.edge_nodes(m).tolist()) and len(wl.rec_nodes) > 100
    assert 0.5e12 < np.abs(wl.wavelets).max() <= 1e12


def test_galerkin_traces_stay_bounded_on_a_small_cvt_plate():
    m = W.cvt_mesh(0.02, 0.01, 16, 6, seed=7, lloyd_iters=30)
    top = W.top_edge_nodes(m)
    src = np.array([top[len(top) // 2]])
    wav = W.sine_burst(200, 2e-7, 5e5, 2, 1e12)[None]
    model = stp.Model(m, W.homogeneous(m), 6000.0, 2e-7, scheme="radial_galerkin")
    tr = stp.forward(model, src, wav, top, 200)
    assert np.isfinite(tr).all()
    assert np.abs(tr[..., 150:]).max() < 2.0 * np.abs(tr[..., :150]).max()
