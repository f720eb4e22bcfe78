"""Polygon meshes for scaled-boundary elements (inputs only).

A mesh is a list of global boundary nodes plus, for every element, the
counter-clockwise loop of the global nodes on its boundary.  Straight
segments join consecutive loop nodes; the paper's elements are star-convex
polygons with any number of boundary nodes (Section "Scaled boundary
discretization", the coordinate transformation).  Each element also carries
its number of radial levels N_r.

Two families are produced:

* ``uniform_rect_mesh`` -- a rectangle split into nx x ny equal rectangles,
  each edge split into ``segs`` straight segments (n_b = 4 * segs);
* ``quadtree_mesh`` -- square cells refined around seeded voids, where the
  nodes of finer neighbours become extra boundary nodes of the coarser cell
  (hanging nodes are legal boundary nodes of a polygon element).

Node coordinates are built on an integer lattice so that shared nodes are
bit-identical between elements.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    node_xy: np.ndarray            # [n_nodes, 2] float64
    elem_ptr: np.ndarray           # [n_elem + 1] int64, CSR offsets into elem_nodes
    elem_nodes: np.ndarray         # [sum n_b] int64, CCW loops
    n_r: np.ndarray                # [n_elem] int32, radial levels per element
    extent: tuple = (1.0, 1.0)     # (Lx, Ly) of the plate
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.node_xy.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.elem_ptr.shape[0] - 1)

    def loop(self, e: int) -> np.ndarray:
        return self.elem_nodes[self.elem_ptr[e]:self.elem_ptr[e + 1]]

    def n_b(self) -> np.ndarray:
        return np.diff(self.elem_ptr).astype(np.int32)

    def param_offsets(self) -> np.ndarray:
        """Offsets of each element's [N_r][n_b] block in the fine density grid."""
        sizes = self.n_b().astype(np.int64) * self.n_r.astype(np.int64)
        return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    @property
    def n_params(self) -> int:
        return int(self.param_offsets()[-1])


def _perimeter_ccw(x0: int, y0: int, x1: int, y1: int):
    """Integer lattice points on the perimeter of [x0,x1]x[y0,y1], CCW from (x0,y0)."""
    pts = []
    for x in range(x0, x1):
        pts.append((x, y0))
    for y in range(y0, y1):
        pts.append((x1, y))
    for x in range(x1, x0, -1):
        pts.append((x, y1))
    for y in range(y1, y0, -1):
        pts.append((x0, y))
    return pts


def uniform_rect_mesh(lx: float, ly: float, nx: int, ny: int, segs: int, n_r: int) -> Mesh:
    """nx x ny rectangles over [0,lx]x[0,ly]; every element edge has ``segs`` segments."""
    if nx < 1 or ny < 1 or segs < 1:
        raise ValueError("nx, ny, segs must be positive")
    gx, gy = nx * segs, ny * segs            # lattice size in segment units
    ids = -np.ones((gy + 1, gx + 1), dtype=np.int64)
    coords = []
    # global numbering row-major in (y, x) over lattice points that lie on element edges
    for j in range(gy + 1):
        for i in range(gx + 1):
            if i % segs == 0 or j % segs == 0:
                ids[j, i] = len(coords)
                coords.append((i * lx / gx, j * ly / gy))
    node_xy = np.asarray(coords, dtype=np.float64)
    loops = []
    for ey in range(ny):
        for ex in range(nx):
            pts = _perimeter_ccw(ex * segs, ey * segs, (ex + 1) * segs, (ey + 1) * segs)
            loops.append([ids[y, x] for (x, y) in pts])
    elem_ptr = np.zeros(len(loops) + 1, dtype=np.int64)
    elem_ptr[1:] = np.cumsum([len(l) for l in loops])
    elem_nodes = np.asarray([n for l in loops for n in l], dtype=np.int64)
    assert (elem_nodes >= 0).all()
    return Mesh(node_xy=node_xy, elem_ptr=elem_ptr, elem_nodes=elem_nodes,
                n_r=np.full(nx * ny, n_r, dtype=np.int32), extent=(lx, ly),
                meta={"kind": "uniform", "nx": nx, "ny": ny, "segs": segs})


def quadtree_mesh(lx: float, ly: float, base_level: int, max_level: int, refine_centres,
                  refine_radius: float, n_b_max: int = 24, n_r_max: int = 64,
                  n_r_min: int = 8) -> Mesh:
    """Square cells of side ly/2**level, refined towards ``refine_centres``.

    A cell at level l is split when its centre lies within
    ``refine_radius * 2**(max_level - l) / 2**(max_level - base_level)``
    (a radius that shrinks with depth) of any centre in ``refine_centres``;
    cells keep at most a 4:1 size ratio to their neighbours and at most
    ``n_b_max`` boundary nodes.  Every own edge has two segments.  N_r per
    cell is proportional to its side: clamp(round(n_r_max * side / side_max)).
    """
    side_units = 2 ** (max_level - base_level + 1)      # base-cell side in lattice units
    unit = ly / 2 ** (max_level + 1)                    # lattice spacing
    nbx = int(round(lx / (ly / 2 ** base_level)))
    nby = 2 ** base_level
    # leaves: dict (x0, y0, size) in lattice units
    leaves = {(i * side_units, j * side_units, side_units) for i in range(nbx) for j in range(nby)}
    centres = np.asarray(refine_centres, dtype=np.float64).reshape(-1, 2)

    def wants_split(c):
        x0, y0, s = c
        lvl = base_level + int(round(np.log2(side_units / s)))
        if lvl >= max_level:
            return False
        cx, cy = (x0 + s / 2) * unit, (y0 + s / 2) * unit
        rad = refine_radius * 2.0 ** (-(lvl - base_level) * 0.5)
        d = np.sqrt(((centres - np.array([cx, cy])) ** 2).sum(1)).min() if len(centres) else np.inf
        return d < rad + s * unit

    def split(c):
        x0, y0, s = c
        h = s // 2
        return [(x0, y0, h), (x0 + h, y0, h), (x0, y0 + h, h), (x0 + h, y0 + h, h)]

    changed = True
    while changed:
        changed = False
        for c in list(leaves):
            if c in leaves and wants_split(c):
                leaves.remove(c)
                leaves.update(split(c))
                changed = True

    def build_nodes(lv):
        pts = set()
        for (x0, y0, s) in lv:
            h = s // 2
            for (x, y) in [(x0, y0), (x0 + h, y0), (x0 + s, y0), (x0 + s, y0 + h),
                           (x0 + s, y0 + s), (x0 + h, y0 + s), (x0, y0 + s), (x0, y0 + h)]:
                pts.add((x, y))
        return pts

    # balance: refine any cell whose loop would exceed n_b_max nodes or whose
    # neighbour is more than two levels finer
    while True:
        pts = build_nodes(leaves)
        bad = []
        for c in leaves:
            x0, y0, s = c
            per = _perimeter_ccw(x0, y0, x0 + s, y0 + s)
            nb = sum(1 for p in per if p in pts)
            if nb > n_b_max:
                bad.append(c)
        if not bad:
            break
        for c in bad:
            leaves.remove(c)
            leaves.update(split(c))

    pts = build_nodes(leaves)
    order = sorted(pts, key=lambda p: (p[1], p[0]))
    ids = {p: i for i, p in enumerate(order)}
    node_xy = np.asarray([(p[0] * unit, p[1] * unit) for p in order], dtype=np.float64)
    cells = sorted(leaves, key=lambda c: (c[1], c[0], c[2]))
    loops, n_r = [], []
    for (x0, y0, s) in cells:
        per = _perimeter_ccw(x0, y0, x0 + s, y0 + s)
        loops.append([ids[p] for p in per if p in ids])
        nr = int(round(n_r_max * s / side_units))
        n_r.append(min(max(nr, n_r_min), n_r_max))
    elem_ptr = np.zeros(len(loops) + 1, dtype=np.int64)
    elem_ptr[1:] = np.cumsum([len(l) for l in loops])
    elem_nodes = np.asarray([n for l in loops for n in l], dtype=np.int64)
    return Mesh(node_xy=node_xy, elem_ptr=elem_ptr, elem_nodes=elem_nodes,
                n_r=np.asarray(n_r, dtype=np.int32), extent=(lx, ly),
                meta={"kind": "quadtree", "base_level": base_level, "max_level": max_level})


def top_edge_nodes(mesh: Mesh) -> np.ndarray:
    """Global ids of nodes on the top edge y = Ly, sorted by x."""
    ly = mesh.extent[1]
    on = np.nonzero(np.abs(mesh.node_xy[:, 1] - ly) <= 1e-12 * max(ly, 1.0))[0]
    return on[np.argsort(mesh.node_xy[on, 0])].astype(np.int64)


def nearest_top_node(mesh: Mesh, x: float) -> int:
    top = top_edge_nodes(mesh)
    return int(top[np.argmin(np.abs(mesh.node_xy[top, 0] - x))])


def _bounded_voronoi(pts: np.ndarray, lx: float, ly: float):
    """Voronoi cells of ``pts`` clipped to [0,lx]x[0,ly] (by mirroring the
    generators across the four edges): (vertices, list of vertex-index loops)."""
    from scipy.spatial import Voronoi
    mir = [pts, np.c_[-pts[:, 0], pts[:, 1]], np.c_[2 * lx - pts[:, 0], pts[:, 1]],
           np.c_[pts[:, 0], -pts[:, 1]], np.c_[pts[:, 0], 2 * ly - pts[:, 1]]]
    vor = Voronoi(np.concatenate(mir))
    loops = []
    for i in range(pts.shape[0]):
        reg = vor.regions[vor.point_region[i]]
        if -1 in reg or len(reg) < 3:
            raise RuntimeError("unbounded Voronoi cell")
        loops.append(list(reg))
    return vor.vertices, loops


def cvt_mesh(lx: float, ly: float, n_cells: int, n_r: int, seed: int, lloyd_iters: int = 40,
             merge_frac: float = 0.1) -> Mesh:
    """Centroidal Voronoi tessellation of [0,lx]x[0,ly] with ``n_cells`` polygons.

    Seeded uniform generators are moved ``lloyd_iters`` times to the centroids
    of their (boundary-clipped) Voronoi cells.  Vertices closer than
    ``merge_frac`` times the mean cell size are merged (short edges make
    ill-conditioned segments), vertices on the plate's edges are snapped onto
    them, and every loop is ordered counter-clockwise; each cell edge is one
    straight segment, so n_b is the cell's vertex count.
    """
    rng = np.random.default_rng(seed)
    pts = rng.uniform([0.0, 0.0], [lx, ly], size=(n_cells, 2))
    for _ in range(lloyd_iters):
        verts, loops = _bounded_voronoi(pts, lx, ly)
        for i, lp in enumerate(loops):
            xy = verts[lp]
            ctr = xy.mean(axis=0)
            order = np.argsort(np.arctan2(xy[:, 1] - ctr[1], xy[:, 0] - ctr[0]))
            xy = xy[order]
            x, y = xy[:, 0], xy[:, 1]
            xn, yn = np.roll(x, -1), np.roll(y, -1)
            cr = x * yn - xn * y
            a = cr.sum() / 2.0
            pts[i] = [((x + xn) * cr).sum() / (6 * a), ((y + yn) * cr).sum() / (6 * a)]
    verts, loops = _bounded_voronoi(pts, lx, ly)
    used = sorted({v for lp in loops for v in lp})
    V = verts[used].copy()
    remap = {v: k for k, v in enumerate(used)}
    loops = [[remap[v] for v in lp] for lp in loops]
    tol = 1e-9 * max(lx, ly)
    for d, L in ((0, lx), (1, ly)):
        V[np.abs(V[:, d]) <= tol, d] = 0.0
        V[np.abs(V[:, d] - L) <= tol, d] = L
    # merge close vertices (union-find), preferring vertices on the plate's edges
    h = np.sqrt(lx * ly / n_cells)
    parent = list(range(V.shape[0]))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    on_edge = lambda k: V[k, 0] in (0.0, lx) or V[k, 1] in (0.0, ly)
    corner = lambda k: V[k, 0] in (0.0, lx) and V[k, 1] in (0.0, ly)
    for lp in loops:
        for a, b in zip(lp, lp[1:] + lp[:1]):
            if np.hypot(*(V[a] - V[b])) < merge_frac * h:
                ra, rb = find(a), find(b)
                if ra == rb:
                    continue
                if corner(rb) or (on_edge(rb) and not corner(ra) and not on_edge(ra)):
                    ra, rb = rb, ra
                if corner(rb) and corner(ra):
                    continue
                if on_edge(ra) and on_edge(rb) and not (V[ra, 0] == V[rb, 0] or V[ra, 1] == V[rb, 1]):
                    continue
                parent[rb] = ra
    root = [find(k) for k in range(V.shape[0])]
    keep = sorted(set(root))
    newid = {r: k for k, r in enumerate(keep)}
    node_xy = V[keep]
    out = []
    for lp in loops:
        ids = []
        for v in lp:
            k = newid[root[v]]
            if not ids or ids[-1] != k:
                ids.append(k)
        while len(ids) > 1 and ids[0] == ids[-1]:
            ids.pop()
        xy = node_xy[ids]
        ctr = xy.mean(axis=0)
        order = np.argsort(np.arctan2(xy[:, 1] - ctr[1], xy[:, 0] - ctr[0]))
        out.append([ids[o] for o in order])
    elem_ptr = np.zeros(len(out) + 1, dtype=np.int64)
    elem_ptr[1:] = np.cumsum([len(l) for l in out])
    elem_nodes = np.asarray([n for l in out for n in l], dtype=np.int64)
    return Mesh(node_xy=node_xy, elem_ptr=elem_ptr, elem_nodes=elem_nodes,
                n_r=np.full(len(out), n_r, dtype=np.int32), extent=(lx, ly),
                meta={"kind": "cvt", "n_cells": n_cells, "seed": seed})


def edge_nodes(mesh: Mesh) -> np.ndarray:
    """Global ids of the nodes on the plate's outer boundary."""
    lx, ly = mesh.extent
    x, y = mesh.node_xy[:, 0], mesh.node_xy[:, 1]
    tol = 1e-12 * max(lx, ly)
    on = (np.abs(x) <= tol) | (np.abs(x - lx) <= tol) | (np.abs(y) <= tol) | (np.abs(y - ly) <= tol)
    return np.nonzero(on)[0].astype(np.int64)
