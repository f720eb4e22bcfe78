"""Gradient of the misfit with respect to the fine-grid density.

Two gradients are provided.

``exact_gradient`` -- the exact derivative of the discrete misfit (eq. misfit
with the rectangle rule) with respect to every fine-grid density, i.e. the
discrete counterpart of the Lagrangian/KKT derivation of Section "Adjoint
method" applied to the discretised system.  Step k of the forward model is
the linear solve A X^k = P w^{k-1} + F^k of the uncondensed block system
(eq. system for every element, with the flux rows of all elements summed at
shared boundary nodes), followed by the Newmark updates (eq. Newmark).  The
adjoint runs backwards in time: lambda^k = A^-T (seed^k), where the seed
gathers the misfit residual at the receivers and the adjoints of the later
Newmark updates.  A^-T is applied by plain block elimination of the
element-interior unknowns (a sparse LU per element) and the transposed
coarse system K_g^T = sum_e S_e^T.  Because A and P are linear in the
densities, dA/drho_p is A evaluated with a unit density at p; the gradient
is the zero-lag cross-correlation sum_k [ -lambda^k . (dA/drho_p) X^k
+ lambda^k . (dP/drho_p) w^{k-1} ], accumulated over time first as the
block correlations sum_k lambda_r (X_l)^T.

``paper_kernel_gradient`` -- the paper's truncated Frechet kernel: the
kernel is the time integral of (d_t lambda d_t u - c^2 grad lambda . grad u)
(Section "Adjoint method"); the implementation notes drop the second term
and evaluate the first at the nodal points from forward and back-propagated
wavefields, the back-propagated field being the forward solver driven by
the time-reversed residuals at the receivers.  Readings (the paper gives
only the continuous form):

* source: the residual itself, r = u - d, as a nodal point load (the paper's
  adjoint source is the residual d - u of the misfit's functional derivative;
  with the stepper's sign convention M u'' + K u = f the back-propagated
  system takes u - d);
* time: the kernel's time integral by the rectangle rule of the misfit
  (weight dt at t_k, k = 1 .. N_t); reversed step k' of the back-propagated run
  applies r^{N_t + 1 - k'} and is paired with forward step N_t + 1 - k', the
  pairing of the exact discrete adjoint, whose state at step k is driven by
  the residuals of steps k .. N_t;
* sign: the reversal turns d_t lambda into -d_t lambda~, so
  g = -dt * sum_k' v~^{k'} v^{N_t + 1 - k'} at every (element, level, node);
* no area weight: the paper evaluates the kernel at the nodal points.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import SCHEMES, coefficient_matrices, element_system, row_columns
from .stepper import Model, forward


def _partition(n, n_b):
    """Index sets of eq. system: internal unknowns (levels -1..n-1, n+1), boundary
    unknown (level n); internal rows (-1..n), flux row (n+1)."""
    blocks = list(range(0, n + 1)) + [n + 2]            # block index l + 1
    ic = np.concatenate([np.arange(b * n_b, (b + 1) * n_b) for b in blocks])
    bc = np.arange((n + 1) * n_b, (n + 2) * n_b)
    ir = np.arange(0, (n + 2) * n_b)
    br = np.arange((n + 2) * n_b, (n + 3) * n_b)
    return ic, bc, ir, br


class _ElementBlocks:
    """Per element: the coupling blocks of eq. system between the internal and
    boundary unknowns and a sparse LU of its internal block (built for a few
    hundred elements at a time, so that large meshes fit in memory)."""

    def __init__(self, g, chunk=256):
        n, nb = g.n, g.n_b
        self.ic, self.bc, self.ir, self.br = _partition(n, nb)
        aib, abi, self.lu = [], [], []
        for c0 in range(0, len(g.elem_ids), chunk):
            sl = slice(c0, c0 + chunk)
            A = element_system(g.theta[sl], g.phi[sl], g.psi[sl])
            aib.append(A[:, self.ir][:, :, self.bc])
            abi.append(A[:, self.br][:, :, self.ic])
            self.lu += [spla.splu(sp.csc_matrix(A[e][np.ix_(self.ir, self.ic)])) for e in range(A.shape[0])]
        self.AIB = np.concatenate(aib)
        self.ABI = np.concatenate(abi)


def _basis_rows(g, m, k):
    """d(theta, phi, psi, P)/d rho_{m,k}: the rows built from E-matrices of a unit
    density at level m, node k, less the rows of zero densities (the rows are
    affine in the densities: the radial Galerkin layout has constant identity
    blocks)."""
    E_, nr, nb = len(g.elem_ids), g.n_r, g.n_b
    unit = np.zeros((E_, 1, nb))
    unit[:, 0, k] = 1.0
    bases = coefficient_matrices(g.xy, g.centre, unit, g.c)
    lev = []
    for B in bases:
        Z = np.zeros((E_, nr, nb, nb))
        Z[:, m] = B[:, 0]
        lev.append(Z)
    rows = SCHEMES[g.scheme]
    zero = np.zeros((E_, nr, nb, nb))
    return tuple(a - b for a, b in zip(rows(*lev, g.xi, g.h, g.a0), rows(zero, zero, zero, zero, g.xi, g.h, g.a0)))


def exact_gradient(model: Model, src_nodes, wavelets, rec_nodes, observed, n_steps,
                   elements=None):
    """Exact discrete gradient dJ/drho in the fine-grid layout, and J.

    ``elements`` (optional) restricts the final contraction to a subset of
    global element ids (the adjoint fields are always global); entries of
    other elements are NaN.
    """
    nm = model.nm
    mesh = model.mesh
    traces, trajs = forward(model, src_nodes, wavelets, rec_nodes, n_steps, keep=True)
    res = traces - observed
    J = 0.5 * nm.dt * np.sum(res * res)
    blocks = [_ElementBlocks(g) for g in model.groups]
    corr = [np.zeros((len(g.elem_ids), g.n + 3, 3, g.n_b, g.n_b)) for g in model.groups]
    corr_p = [np.zeros((len(g.elem_ids), g.n + 1, g.n_b, g.n_b)) for g in model.groups]
    n_nodes = mesh.n_nodes
    for s in range(len(src_nodes)):
        ub, vb, ab = np.zeros(n_nodes), np.zeros(n_nodes), np.zeros(n_nodes)
        seeds = [{"u": np.zeros((len(g.elem_ids), g.n, g.n_b)),
                  "v": np.zeros((len(g.elem_ids), g.n, g.n_b)),
                  "a": np.zeros((len(g.elem_ids), g.n, g.n_b))} for g in model.groups]
        for k in range(n_steps, 0, -1):
            np.add.at(ub, rec_nodes, nm.dt * res[s, :, k - 1])
            tB = ub + nm.c1 * vb + nm.a0 * ab
            rhsB = tB.copy()
            zs, tIs = [], []
            for g, blk, sd in zip(model.groups, blocks, seeds):
                n, nb, E_ = g.n, g.n_b, len(g.elem_ids)
                tI_int = sd["u"] + nm.c1 * sd["v"] + nm.a0 * sd["a"]
                tI = np.zeros((E_, (n + 2) * nb))
                tI[:, nb:(n + 1) * nb] = tI_int.reshape(E_, -1)
                z = np.stack([blk.lu[e].solve(tI[e], trans="T") for e in range(E_)])
                gB = np.einsum("eib,ei->eb", blk.AIB, z)
                np.add.at(rhsB, g.loops, -gB)
                tIs.append(tI)
            lamB = model.lu.solve(rhsB, trans="T")
            wbB = np.zeros(n_nodes)
            new_seeds = []
            for gi, (g, blk, sd) in enumerate(zip(model.groups, blocks, seeds)):
                n, nb, E_ = g.n, g.n_b, len(g.elem_ids)
                lb = lamB[g.loops]
                rhs = tIs[gi] - np.einsum("ebi,eb->ei", blk.ABI, lb)
                lamI = np.stack([blk.lu[e].solve(rhs[e], trans="T") for e in range(E_)])
                lam = np.concatenate([lamI.reshape(E_, n + 2, nb), lb[:, None]], axis=1)  # rows -1..n+1
                full = trajs[s][k - 1]["full"][gi]
                X, w = full["X"], full["w"]
                for r in range(-1, n + 2):
                    for t, l in enumerate(row_columns(r, n)):
                        corr[gi][:, r + 1, t] += lam[:, r + 1, :, None] * X[:, l + 1, None, :]
                corr_p[gi] += lam[:, 1:n + 2, :, None] * w[:, :, None, :]
                # w-bar = P^T lambda (rows 0..n) - a-bar
                Pl = np.einsum("ejba,ejb->eja", g.P, lam[:, 1:n + 2])
                np.add.at(wbB, g.loops, Pl[:, n])
                wb = Pl[:, :n] - sd["a"]
                new_seeds.append({"u": -nm.c1 * sd["v"] + nm.a0 * wb,
                                  "v": nm.c2 * sd["v"] + nm.a1 * wb,
                                  "a": nm.c3 * sd["v"] + nm.a2 * wb})
            wbB -= ab
            ub, vb, ab = -nm.c1 * vb + nm.a0 * wbB, nm.c2 * vb + nm.a1 * wbB, nm.c3 * vb + nm.a2 * wbB
            seeds = new_seeds
    grad = np.full(mesh.n_params, np.nan)
    offs = mesh.param_offsets()
    want = None if elements is None else set(int(e) for e in elements)
    for gi, g in enumerate(model.groups):
        sel = np.arange(len(g.elem_ids)) if want is None else \
            np.asarray([i for i, e in enumerate(g.elem_ids) if int(e) in want], dtype=np.int64)
        if sel.size == 0:
            continue
        gsub = _Sub(g, sel)
        ge = np.zeros((sel.size, g.n_r, g.n_b))
        for m in range(g.n_r):
            for kk in range(g.n_b):
                th, ph, ps, P = _basis_rows(gsub, m, kk)
                dA = np.stack([th, ph, ps], axis=2)                    # [E, n+3, 3, nb, nb]
                ge[:, m, kk] = (-np.einsum("ertab,ertab->e", dA, corr[gi][sel])
                                + np.einsum("ejab,ejab->e", P, corr_p[gi][sel]))
        for i, e in zip(sel, g.elem_ids[sel]):
            grad[offs[e]:offs[e + 1]] = ge[list(sel).index(i)].ravel()
    return grad, J


class _Sub:
    """View of an element group restricted to a subset of its elements."""

    def __init__(self, g, sel):
        self.elem_ids = g.elem_ids[sel]
        self.xy, self.centre = g.xy[sel], g.centre[sel]
        self.n_r, self.n_b, self.xi, self.h, self.c, self.a0 = g.n_r, g.n_b, g.xi, g.h, g.c, g.a0
        self.scheme = g.scheme


def paper_kernel_gradient(model: Model, src_nodes, wavelets, rec_nodes, observed, n_steps,
                          sign: float = -1.0):
    """Truncated zero-lag kernel at the nodal points: -dt sum_k' v~^{k'} v^{N_t+1-k'},
    v~ the velocities of the forward stepper driven by the time-reversed residuals
    u - d at the receivers (readings in the module docstring)."""
    nm = model.nm
    mesh = model.mesh
    traces, trajs = forward(model, src_nodes, wavelets, rec_nodes, n_steps, keep=True)
    res = traces - observed
    grad = np.zeros(mesh.n_params)
    offs = mesh.param_offsets()
    for s in range(len(src_nodes)):
        adj_w = np.zeros((len(rec_nodes), n_steps))
        for kp in range(1, n_steps + 1):
            adj_w[:, kp - 1] = res[s, :, n_steps - kp]          # r^{N_t + 1 - k'}
        # back-propagation: the forward stepper with the receivers as sources
        lam_traj = _forward_multi_source(model, rec_nodes, adj_w, n_steps)
        for kp in range(1, n_steps + 1):
            fwd = trajs[s][n_steps - kp]            # state at forward step N_t + 1 - k'
            lam = lam_traj[kp - 1]
            for gi, g in enumerate(model.groups):
                v_f = np.concatenate([fwd["groups_v"][gi], fwd["V"][g.loops][:, None]], axis=1)
                v_l = np.concatenate([lam["groups_v"][gi], lam["V"][g.loops][:, None]], axis=1)
                contrib = sign * nm.dt * v_l * v_f                          # [E, n+1, nb]
                for i, e in enumerate(g.elem_ids):
                    grad[offs[e]:offs[e + 1]] += contrib[i].ravel()
    return grad, traces


def _forward_multi_source(model, nodes, wav, n_steps):
    from .stepper import step
    st = model.zero_state(np.float64)
    out = []
    for k in range(1, n_steps + 1):
        f = np.zeros(model.mesh.n_nodes)
        np.add.at(f, nodes, wav[:, k - 1])
        st = step(model, st, f)
        out.append({"V": st["V"], "groups_v": [gs["v"] for gs in st["groups"]]})
    return out
