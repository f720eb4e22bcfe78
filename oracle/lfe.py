"""Conventional SBFEM by low-frequency expansion (Section "Low-frequency expansion").

For density that does not vary along xi the radial equation reduces to
eq. simplified, whose dynamic stiffness S(omega) is approximated by
K - omega^2 M (eq. S).  K solves the algebraic Riccati equation
(K - E1) E0^-1 (K - E1^T) - E2 = 0 and M the Lyapunov equation
(K - E1) E0^-1 M + M E0^-1 (K - E1^T) + 2 M - M0 = 0.

K is obtained with the textbook eigenvalue method: writing the static radial
equation for [u; q], q = xi E0 u' + E1^T u, as xi d/dxi [u; q] = Z [u; q]
with Z = [[-E0^-1 E1^T, E0^-1], [E2 - E1 E0^-1 E1^T, E1 E0^-1]], the modes
bounded at the scaling centre are those with positive real eigenvalue, plus
the constant mode (u = 1, q = 0); K = Q U^-1.  The Lyapunov equation is
A M + M A^T = M0 with A = (K - E1) E0^-1 + I, solved by SciPy.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lfe_stiffness(E0, E1, E2):
    nb = E0.shape[0]
    E0i = np.linalg.inv(E0)
    Z = np.block([[-E0i @ E1.T, E0i], [E2 - E1 @ E0i @ E1.T, E1 @ E0i]])
    lam, vec = np.linalg.eig(Z)
    order = np.argsort(-lam.real)
    pos = order[:nb - 1]
    U = np.concatenate([vec[:nb, pos], np.ones((nb, 1))], axis=1)
    Q = np.concatenate([vec[nb:, pos], np.zeros((nb, 1))], axis=1)
    K = np.real(Q @ np.linalg.inv(U))
    return K, np.sort(lam.real[pos])


def lfe_mass(K, E0, E1, M0):
    A = (K - E1) @ np.linalg.inv(E0) + np.eye(K.shape[0])
    return sla.solve_continuous_lyapunov(A, M0)


# ---------------------------------------------------------------------------
# The conventional (low-frequency expansion) time-domain path.
#
# For density that does not vary along xi (the boundary values of every
# element, as in eq. simplified) each element contributes a stiffness K_e and
# a mass M_e on its boundary nodes only; the global system K U + M U'' = F is
# stepped with the same Newmark scheme (eq. Newmark).  By default K_e and M_e
# are the paper's: the Riccati solution (lfe_stiffness) and the Lyapunov
# solution (lfe_mass) above.  The alternative ``method="condensed"`` takes
# those of linear radial elements condensed onto the boundary level: K_e the
# static Schur complement, M_e the radial mass seen through the static modes;
# they converge to the Riccati and Lyapunov solutions as the radial levels
# refine (O(h^2)); the tests pin that convergence.
# ---------------------------------------------------------------------------

from . import radial_galerkin as _rg
from .element import coefficient_matrices as _coeffs, polygon_centroid as _centroid, radial_levels as _levels


def condensed_matrices(E0, E1, E2, M0, xi, n_quad=4):
    """K and M of one element with radially constant E0, E1, E2, M0 [n_b, n_b]
    on the radial levels xi."""
    n_r, nb = len(xi), E0.shape[0]
    Er = [np.broadcast_to(E, (n_r,) + E.shape) for E in (E0, E1, E2, M0)]
    K, M = _rg.galerkin_matrices(*Er, xi, n_quad, lumped=True)
    I = np.arange(0, (n_r - 1) * nb)
    B = np.arange((n_r - 1) * nb, n_r * nb)
    X = np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, B)])
    Kc = K[np.ix_(B, B)] - K[np.ix_(B, I)] @ X
    Phi = np.concatenate([-X, np.eye(nb)], axis=0)
    Mc = Phi.T @ M @ Phi
    return Kc, Mc


class LfeModel:
    """Assembled K, M of the low-frequency expansion path and the LU of K + a0 M.

    rho_flat is the fine-grid density; only each element's boundary level
    (level N_r - 1) is used.  method "riccati": K_e, M_e of eq. S (Riccati and
    Lyapunov equations); "condensed": the radial condensation on the element's
    N_r levels."""

    def __init__(self, mesh, rho_flat, c, dt, beta=0.25, gamma=0.5, xi0=1e-3, method="riccati"):
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        from .stepper import Newmark
        self.mesh, self.nm = mesh, Newmark(dt, beta, gamma)
        offs = mesh.param_offsets()
        rows, cols, kv, mv = [], [], [], []
        self.Ke, self.Me = [], []
        for e in range(mesh.n_elem):
            lp = mesh.loop(e)
            nb, nr = len(lp), int(mesh.n_r[e])
            xy = mesh.node_xy[lp][None]
            rb = np.asarray(rho_flat[offs[e]:offs[e + 1]]).reshape(nr, nb)[nr - 1][None, None]
            E0, E1, E2, M0 = [E[0, 0] for E in _coeffs(xy, _centroid(xy), rb, c)]
            if method == "riccati":
                Ke, _ = lfe_stiffness(E0, E1, E2)
                Me = lfe_mass(Ke, E0, E1, M0)
            else:
                xi, _ = _levels(nr, xi0)
                Ke, Me = condensed_matrices(E0, E1, E2, M0, xi)
            self.Ke.append(Ke)
            self.Me.append(Me)
            rows.append(np.repeat(lp, nb))
            cols.append(np.tile(lp, nb))
            kv.append(Ke.ravel())
            mv.append(Me.ravel())
        shape = (mesh.n_nodes, mesh.n_nodes)
        r, cc = np.concatenate(rows), np.concatenate(cols)
        self.K = sp.coo_matrix((np.concatenate(kv), (r, cc)), shape=shape).tocsc()
        self.M = sp.coo_matrix((np.concatenate(mv), (r, cc)), shape=shape).tocsc()
        self.lu = spla.splu((self.K + self.nm.a0 * self.M).tocsc())


def lfe_forward(model: LfeModel, src_nodes, wavelets, rec_nodes, n_steps):
    """Traces [n_shots, n_rec, n_steps] of the Newmark loop on K U + M U'' = F
    (force sample k - 1 at step k, zero initial state)."""
    nm, n = model.nm, model.mesh.n_nodes
    out = np.zeros((len(src_nodes), len(rec_nodes), n_steps))
    for s in range(len(src_nodes)):
        U, V, A = np.zeros(n), np.zeros(n), np.zeros(n)
        for k in range(1, n_steps + 1):
            W = nm.a0 * U + nm.a1 * V + nm.a2 * A
            F = model.M @ W
            F[src_nodes[s]] += wavelets[s][k - 1]
            Un = model.lu.solve(F)
            V = nm.c1 * (Un - U) + nm.c2 * V + nm.c3 * A
            A = nm.a0 * Un - W
            U = Un
            out[s, :, k - 1] = U[rec_nodes]
    return out


def _lfe_velocities(model: LfeModel, nodes, amps, n_steps):
    """Nodal velocities of every step of the loop driven by point forces
    amps[c][k - 1] at nodes[c] (one run)."""
    nm, n = model.nm, model.mesh.n_nodes
    U, V, A = np.zeros(n), np.zeros(n), np.zeros(n)
    out = []
    for k in range(1, n_steps + 1):
        W = nm.a0 * U + nm.a1 * V + nm.a2 * A
        F = model.M @ W
        np.add.at(F, nodes, amps[:, k - 1])
        Un = model.lu.solve(F)
        V = nm.c1 * (Un - U) + nm.c2 * V + nm.c3 * A
        A = nm.a0 * Un - W
        U = Un
        out.append(V.copy())
    return out


def lfe_paper_kernel_gradient(model: LfeModel, src_nodes, wavelets, rec_nodes, observed, n_steps,
                              sign: float = -1.0):
    """The paper's truncated kernel on the expansion path: sign * dt * sum_k'
    v~^{k'} v^{N_t + 1 - k'} at every node (sign -1), the back-propagated run v~
    driven by the time-reversed residuals u - d at the receivers (the readings
    of ``adjoint.paper_kernel_gradient``); every element's boundary-level
    density at a node takes that node's value."""
    nm, mesh = model.nm, model.mesh
    traces = lfe_forward(model, src_nodes, wavelets, rec_nodes, n_steps)
    res = traces - observed
    kern = np.zeros(mesh.n_nodes)
    for s in range(len(src_nodes)):
        v_f = _lfe_velocities(model, np.asarray([src_nodes[s]]), np.asarray(wavelets)[s:s + 1], n_steps)
        adj_w = res[s][:, ::-1]                      # amplitude at reversed step k' is r^{N_t + 1 - k'}
        v_b = _lfe_velocities(model, np.asarray(rec_nodes), adj_w, n_steps)
        for kp in range(1, n_steps + 1):
            kern += sign * nm.dt * v_b[kp - 1] * v_f[n_steps - kp]
    grad = np.zeros(mesh.n_params)
    offs = mesh.param_offsets()
    for e in range(mesh.n_elem):
        lp = mesh.loop(e)
        nb, nr = len(lp), int(mesh.n_r[e])
        grad[offs[e] + (nr - 1) * nb:offs[e + 1]] = kern[lp]
    return grad, traces
