"""Time loop of the condensed scheme: condense, coarse solve, recover, Newmark.

Paper passages followed:

* Newmark updates of velocity and acceleration and the residual source
  (eq. Newmark, eq. ODE_Newmark);
* the forward sweep of the residual source with the pivots rho_i, the
  decoupled last two rows, the effective source f_hat = p_{n+1} - G p_n + f
  and the dynamic stiffness S (Section "Radial discretization");
* assembly of S u_n = f_hat over elements into the global nodal system,
  whose size is that of the boundary mesh (the interior levels are never
  assembled);
* the backward sweep u_i = phi~_i^-1 (p~_i - psi~_i u_{i+1}) and the Newmark
  update at every level;
* the waveform misfit (eq. misfit) sampled at receiver nodes with the
  rectangle rule over the steps.

The coarse solve uses SciPy's sparse LU (exact up to rounding); the paper
does not name its solver.  Zero initial conditions (eq. main) give
u = v = a = 0 at t = 0.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import build_groups


@dataclass
class Newmark:
    """Newmark constants (eq. Newmark): a = a0 (u' - u) - a1 v - a2 a (a2 = 1/(2 beta) - 1),
    v' = c1 (u' - u) + c2 v + c3 a."""
    dt: float
    beta: float = 0.25
    gamma: float = 0.5

    @property
    def a0(self):
        return 1.0 / (self.beta * self.dt ** 2)

    @property
    def a1(self):
        return 1.0 / (self.beta * self.dt)

    @property
    def a2(self):
        return 1.0 / (2.0 * self.beta) - 1.0

    @property
    def c1(self):
        return self.gamma / (self.beta * self.dt)

    @property
    def c2(self):
        return 1.0 - self.gamma / self.beta

    @property
    def c3(self):
        return self.dt * (1.0 - self.gamma / (2.0 * self.beta))


def coarse_matrix(groups, n_nodes):
    """K_g = sum_e L_e^T S_e L_e as a sparse CSC matrix."""
    rows, cols, vals = [], [], []
    for g in groups:
        S = g.f["S"]
        nb = g.n_b
        rows.append(np.repeat(g.loops, nb, axis=1).ravel())
        cols.append(np.tile(g.loops, (1, nb)).ravel())
        vals.append(S.reshape(S.shape[0], -1).ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_nodes, n_nodes))
    return K.tocsc()


class Model:
    """Factored model: element groups, coarse matrix and its LU (once per rho, dt)."""

    def __init__(self, mesh, rho_flat, c, dt, beta=0.25, gamma=0.5, xi0=1e-3, n_gauss=2, scheme="paper_fd"):
        self.mesh = mesh
        self.nm = Newmark(dt, beta, gamma)
        self.c, self.xi0, self.scheme = c, xi0, scheme
        self.groups = build_groups(mesh, rho_flat, c, xi0, self.nm.a0, n_gauss, scheme)
        self.K = coarse_matrix(self.groups, mesh.n_nodes)
        self.lu = spla.splu(self.K)

    def zero_state(self, dtype):
        st = {"U": np.zeros(self.mesh.n_nodes, dtype), "V": np.zeros(self.mesh.n_nodes, dtype),
              "A": np.zeros(self.mesh.n_nodes, dtype), "groups": []}
        for g in self.groups:
            z = np.zeros((len(g.elem_ids), g.n, g.n_b), dtype)
            st["groups"].append({"u": z.copy(), "v": z.copy(), "a": z.copy()})
        return st


def step(model: Model, st, force, keep=False):
    """One time step; ``force`` is the nodal source vector at the new level.

    Returns the new state; with keep=True also the full unknown vector of every
    element (levels -1 .. n+1, ghosts included) and w of the old state, which
    the adjoint gradient needs.
    """
    nm = model.nm
    W = nm.a0 * st["U"] + nm.a1 * st["V"] + nm.a2 * st["A"]
    F = force.astype(np.result_type(force, W)).copy()
    work = []
    for g, gs in zip(model.groups, st["groups"]):
        n = g.n
        w_int = nm.a0 * gs["u"] + nm.a1 * gs["v"] + nm.a2 * gs["a"]
        w = np.concatenate([w_int, W[g.loops][:, None, :]], axis=1)            # levels 0..n
        p = np.einsum("ejab,ejb->eja", g.P, w)
        rho = g.f["rho"]
        pt = np.empty_like(p)
        pt[:, 0] = p[:, 0]                                                    # row -1 has zero RHS
        for i in range(1, n + 1):
            pt[:, i] = p[:, i] - np.einsum("eab,eb->ea", rho[:, i], pt[:, i - 1])
        pt_np1 = -np.einsum("eab,eb->ea", rho[:, n + 1], pt[:, n - 1])
        fhat = pt_np1 - np.einsum("eab,eb->ea", g.f["G"], pt[:, n])
        np.add.at(F, g.loops, fhat)
        work.append((w_int, w, pt))
    U = model.lu.solve(F)
    out = {"U": U, "V": nm.c1 * (U - st["U"]) + nm.c2 * st["V"] + nm.c3 * st["A"],
           "A": nm.a0 * U - W, "groups": []}
    full = []
    for g, gs, (w_int, w, pt) in zip(model.groups, st["groups"], work):
        n = g.n
        phit = g.f["phit"]
        un = U[g.loops]
        u = np.empty_like(gs["u"])
        nxt = un
        for i in range(n - 1, -1, -1):
            rhs = pt[:, i] - np.einsum("eab,eb->ea", g.psit(i), nxt)
            u[:, i] = np.linalg.solve(phit[:, i], rhs[..., None])[..., 0]
            nxt = u[:, i]
        out["groups"].append({"u": u,
                              "v": nm.c1 * (u - gs["u"]) + nm.c2 * gs["v"] + nm.c3 * gs["a"],
                              "a": nm.a0 * u - w_int})
        if keep:
            # ghosts: u_{n+1} from the decoupled row n, u_{-1} from the row at xi0
            psi_n = g.psi[:, n + 1]
            g_hi = np.linalg.solve(psi_n, (pt[:, n] - np.einsum("eab,eb->ea", phit[:, n], un))[..., None])[..., 0]
            r_lo = -(np.einsum("eab,eb->ea", g.phi[:, 0], u[:, 0])
                     + np.einsum("eab,eb->ea", g.psi[:, 0], u[:, 1] if n > 1 else un))
            g_lo = np.linalg.solve(g.theta[:, 0], r_lo[..., None])[..., 0]
            X = np.concatenate([g_lo[:, None], u, un[:, None], g_hi[:, None]], axis=1)
            full.append({"X": X, "w": w})
    if keep:
        return out, full
    return out


def forward(model: Model, src_nodes, wavelets, rec_nodes, n_steps, keep=False, dtype=None):
    """Run all shots; returns traces [n_shots, n_rec, n_steps] (and trajectories)."""
    if dtype is None:
        dtype = model.groups[0].E0.dtype
    n_shots = len(src_nodes)
    traces = np.zeros((n_shots, len(rec_nodes), n_steps), dtype)
    trajs = []
    for s in range(n_shots):
        st = model.zero_state(dtype)
        traj = []
        for k in range(1, n_steps + 1):
            f = np.zeros(model.mesh.n_nodes, dtype)
            f[src_nodes[s]] += wavelets[s][k - 1]
            if keep:
                st, full = step(model, st, f, keep=True)
                traj.append({"full": full, "U": st["U"], "V": st["V"],
                             "groups_v": [gs["v"] for gs in st["groups"]]})
            else:
                st = step(model, st, f)
            traces[s, :, k - 1] = st["U"][rec_nodes]
        trajs.append(traj)
    if keep:
        return traces, trajs
    return traces


def misfit(traces, observed, dt):
    """J = 1/2 sum_shots sum_rec sum_k dt (u - d)^2 (eq. misfit, rectangle rule)."""
    r = traces - observed
    return 0.5 * dt * np.sum(r * r)
