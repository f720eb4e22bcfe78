"""Element-level oracle: geometry, coefficient matrices, radial rows, condensation.

Everything here works on a *group* of elements that share the boundary-node
count n_b and the number of radial levels N_r; arrays carry the element index
first.  The scalar type follows the density array (float64, or complex128 for
complex-step derivative checks).

Paper passages followed (Section "Scaled boundary discretization"):

* scaling-centre coordinate transformation and boundary interpolation
  (eq. transformation), the boundary Jacobian and the vectors b1, b2
  (eq. partial3, eq. b1b2), area element det(J_b) xi dxi deta;
* coefficient matrices E0, E1, E2, M0 as functions of xi with the density
  interpolated along the boundary from nodal values (eq. Es);
* the Newmark residual source p = -xi^2 M0 (a0 u + a1 v + a2 a)
  (eq. ODE_Newmark);
* central differences in xi (eq. FD), the three-point block rows
  (theta_i, phi_i, psi_i), one-sided differences of E0, E1 at i = 0 and
  i = n, the ghost rows from the internal-flux boundary conditions at xi0 and
  xi = 1, and the assembled block system (eq. system);
* the condensation by block Gauss elimination (pivot rho_0, Thomas sweep,
  rho_{n+1}, the 2 x 2 block system and the dynamic stiffness S).
"""

from __future__ import annotations

import numpy as np


def T(x: np.ndarray) -> np.ndarray:
    """Transpose of the last two axes (plain transpose, never conjugate)."""
    return np.swapaxes(x, -1, -2)


def right_divide(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """x @ inv(y) for stacks of square matrices."""
    return T(np.linalg.solve(T(y), T(x)))


def polygon_centroid(xy: np.ndarray) -> np.ndarray:
    """Area centroid of each CCW polygon (the default scaling centre); xy [E, n_b, 2]."""
    x, y = xy[..., 0], xy[..., 1]
    xn, yn = np.roll(x, -1, axis=-1), np.roll(y, -1, axis=-1)
    cr = x * yn - xn * y
    area = cr.sum(-1) / 2.0
    cx = ((x + xn) * cr).sum(-1) / (6.0 * area)
    cy = ((y + yn) * cr).sum(-1) / (6.0 * area)
    return np.stack([cx, cy], axis=-1)


def radial_levels(n_r: int, xi0: float = 1e-3):
    """Uniform levels xi_i = xi0 + i h, h = (1 - xi0) / n, n = N_r - 1, so xi_n = 1.

    The centre is moved from xi = 0 to a small xi0 (the paper suggests 1e-3)
    to avoid the singular point of the radial equation.
    """
    n = n_r - 1
    h = (1.0 - xi0) / n
    return xi0 + h * np.arange(n_r, dtype=np.float64), h


def segment_jacobian_terms(xy: np.ndarray, centre: np.ndarray, n_gauss: int = 2):
    """Per segment and Gauss point: (k0, k1, weight, N, dN, detJ_b, b1, b2).

    Linear boundary segments between consecutive loop nodes, eta in [-1, 1]:
    x_b(eta) = N1 x_k0 + N2 x_k1, J_b = [[x_b - x0, y_b - y0], [dx_b, dy_b]],
    b1 = [dy_b, -dx_b] / det J_b, b2 = [-(y_b - y0), x_b - x0] / det J_b.
    """
    n_b = xy.shape[1]
    pts, wts = np.polynomial.legendre.leggauss(n_gauss)
    out = []
    for s in range(n_b):
        k0, k1 = s, (s + 1) % n_b
        xa, xb_ = xy[:, k0], xy[:, k1]
        dxb = (xb_ - xa) / 2.0
        for eta, w in zip(pts, wts):
            N = np.array([(1.0 - eta) / 2.0, (1.0 + eta) / 2.0])
            dN = np.array([-0.5, 0.5])
            xb = N[0] * xa + N[1] * xb_
            r = xb - centre
            det = r[:, 0] * dxb[:, 1] - r[:, 1] * dxb[:, 0]
            b1 = np.stack([dxb[:, 1], -dxb[:, 0]], axis=-1) / det[:, None]
            b2 = np.stack([-r[:, 1], r[:, 0]], axis=-1) / det[:, None]
            out.append((k0, k1, w, N, dN, det, b1, b2))
    return out


def coefficient_matrices(xy, centre, rho, c, n_gauss: int = 2):
    """E0, E1, E2, M0 at every level (eq. Es), each [E, N_r, n_b, n_b].

    rho[E, N_r, n_b] holds the nodal densities of each level; along a segment
    the density is interpolated with the same linear shape functions as the
    geometry.  E0 = int rho c^2 phi^T b1.b1 phi detJ, E1 = int rho c^2
    dphi^T b2.b1 phi detJ, E2 = int rho c^2 dphi^T b2.b2 dphi detJ,
    M0 = int rho phi^T phi detJ.  Two Gauss points per segment integrate the
    cubic integrands exactly.
    """
    E, n_r, n_b = rho.shape
    dt_ = np.result_type(rho.dtype, np.float64)
    E0 = np.zeros((E, n_r, n_b, n_b), dt_)
    E1 = np.zeros_like(E0)
    E2 = np.zeros_like(E0)
    M0 = np.zeros_like(E0)
    c2 = c * c
    for (k0, k1, w, N, dN, det, b1, b2) in segment_jacobian_terms(xy, centre, n_gauss):
        rho_g = N[0] * rho[:, :, k0] + N[1] * rho[:, :, k1]          # [E, N_r]
        f = (w * det)[:, None] * rho_g
        b11 = (b1 * b1).sum(-1)[:, None]
        b21 = (b2 * b1).sum(-1)[:, None]
        b22 = (b2 * b2).sum(-1)[:, None]
        idx = (k0, k1)
        for a in range(2):
            for b in range(2):
                ia, ib = idx[a], idx[b]
                E0[:, :, ia, ib] += c2 * b11 * f * N[a] * N[b]
                E1[:, :, ia, ib] += c2 * b21 * f * dN[a] * N[b]
                E2[:, :, ia, ib] += c2 * b22 * f * dN[a] * dN[b]
                M0[:, :, ia, ib] += f * N[a] * N[b]
    return E0, E1, E2, M0


def radial_derivative(Em: np.ndarray, h: float) -> np.ndarray:
    """d/dxi of a level-indexed matrix field [E, N_r, ...]: central differences
    inside, forward difference at i = 0 and backward difference at i = n."""
    D = np.empty_like(Em)
    D[:, 0] = (Em[:, 1] - Em[:, 0]) / h
    D[:, -1] = (Em[:, -1] - Em[:, -2]) / h
    D[:, 1:-1] = (Em[:, 2:] - Em[:, :-2]) / (2.0 * h)
    return D


def block_rows(E0, E1, E2, M0, xi, h, a0):
    """Block rows of the radially discretised, Newmark-discretised element system.

    Returns (theta, phi, psi, P).  theta/phi/psi have shape [E, n + 3, n_b, n_b]
    where index r + 1 holds row r for r = -1 .. n + 1; P[E, n + 1, n_b, n_b]
    holds -xi_i^2 M0_i for rows i = 0 .. n (p_i = P_i w_i).

    Rows i = 0 .. n (discretised eq. ODE_Newmark):
      theta_i = xi^2 E0 / h^2 - xi C / (2h),  psi_i = xi^2 E0 / h^2 + xi C / (2h),
      phi_i = -2 xi^2 E0 / h^2 - E2 + xi dE1^T - a0 xi^2 M0,
      C = E0 + E1^T - E1 + xi dE0.
    Ghost rows (central-difference internal flux q = xi E0 u' + E1^T u):
      row -1 at xi0:   (-xi0 E0_0 / 2h, E1_0^T, xi0 E0_0 / 2h) on (u_-1, u_0, u_1), RHS 0;
      row n+1 at xi=1: (-xi_n E0_n / 2h, E1_n^T, xi_n E0_n / 2h) on (u_n-1, u_n, u_n+1),
                       RHS the external nodal source f.
    """
    n = E0.shape[1] - 1
    D0 = radial_derivative(E0, h)
    D1 = radial_derivative(E1, h)
    x = xi[None, :, None, None]
    C = E0 + T(E1) - E1 + x * D0
    th_i = x ** 2 * E0 / h ** 2 - x * C / (2.0 * h)
    ph_i = -2.0 * x ** 2 * E0 / h ** 2 - E2 + x * T(D1) - a0 * x ** 2 * M0
    ps_i = x ** 2 * E0 / h ** 2 + x * C / (2.0 * h)
    P = -(x ** 2) * M0
    E_, n_b = E0.shape[0], E0.shape[-1]
    shape = (E_, n + 3, n_b, n_b)
    theta = np.zeros(shape, E0.dtype)
    phi = np.zeros(shape, E0.dtype)
    psi = np.zeros(shape, E0.dtype)
    theta[:, 1:n + 2], phi[:, 1:n + 2], psi[:, 1:n + 2] = th_i, ph_i, ps_i
    theta[:, 0] = -xi[0] * E0[:, 0] / (2.0 * h)
    phi[:, 0] = T(E1[:, 0])
    psi[:, 0] = xi[0] * E0[:, 0] / (2.0 * h)
    theta[:, n + 2] = -xi[n] * E0[:, n] / (2.0 * h)
    phi[:, n + 2] = T(E1[:, n])
    psi[:, n + 2] = xi[n] * E0[:, n] / (2.0 * h)
    return theta, phi, psi, P


def galerkin_rows(E0, E1, E2, M0, xi, h, a0, n_quad: int = 4):
    """Block rows of the radial Galerkin scheme, in the layout of ``block_rows``.

    Linear finite elements between consecutive levels replace the central
    differences (a deviation from the paper's eq. FD, which is not symmetric
    and loses stability at large density contrast).  From the semi-weak
    radial equation integrated by parts in xi with the internal flux
    q = xi E0 u' + E1^T u (natural conditions q(xi0) = 0 and q(1) = f), the
    stiffness block of levels (r, l) collects, over the intervals
    [xi_j, xi_j+1] that contain both,
        int [ xi N_r' N_l' E0 + N_r' N_l E1^T + N_r N_l' E1 + N_r N_l E2 / xi ] dxi,
    with every E interpolated linearly between its two levels and n_quad-point
    Gauss-Legendre quadrature per interval.  The radial mass is lumped:
    M_r = sum over its intervals of int xi N_r M0 dxi.  Newmark turns
    K u + M a = f into (K + a0 M) u = f + M w.

    Layout (rows r = -1 .. n + 1 at index r + 1, as in ``block_rows``):
      rows 0 .. n-1: the negated Galerkin rows (theta = -K_{r,r-1},
        phi = -(K_rr + a0 M_r), psi = -K_{r,r+1}, P = -M_r);
      row n: the identity on the unused level n + 1 with P_n = M_n, so that
        u_{n+1} = M_n w_n;
      row n + 1: the boundary row (K_{n,n-1}, K_nn + a0 M_n, -I) with the
        nodal force on its right-hand side, so that it reads
        K_{n,n-1} u_{n-1} + (K_nn + a0 M_n) u_n = f + M_n w_n;
      row -1: the identity on the unused level -1 (u_{-1} = 0).
    The elimination of ``condense`` then yields G = -I and the Schur
    complement of the interior levels as S.
    """
    E_, nr, nb, _ = E0.shape
    n = nr - 1
    dt_ = E0.dtype
    Kd = np.zeros((E_, nr, nb, nb), dt_)
    Kl = np.zeros_like(Kd)    # block (r, r - 1)
    Ku = np.zeros_like(Kd)    # block (r, r + 1)
    Ml = np.zeros_like(Kd)
    gp, gw = np.polynomial.legendre.leggauss(n_quad)
    for j in range(n):
        a, b = xi[j], xi[j + 1]
        for t, w in zip(gp, gw):
            x = (a + b) / 2 + (b - a) / 2 * t
            ww = w * (b - a) / 2
            Nf = ((b - x) / (b - a), (x - a) / (b - a))
            dN = (-1.0 / (b - a), 1.0 / (b - a))
            e0, e1, e2, m0 = [Nf[0] * E[:, j] + Nf[1] * E[:, j + 1] for E in (E0, E1, E2, M0)]
            for p in range(2):
                for q in range(2):
                    blk = ww * (x * dN[p] * dN[q] * e0 + dN[p] * Nf[q] * T(e1) + Nf[p] * dN[q] * e1
                                + Nf[p] * Nf[q] * e2 / x)
                    if p == q:
                        Kd[:, j + p] += blk
                    elif q < p:
                        Kl[:, j + p] += blk
                    else:
                        Ku[:, j + p] += blk
                Ml[:, j + p] += ww * x * Nf[p] * m0
    eye = np.broadcast_to(np.eye(nb, dtype=dt_), (E_, nb, nb))
    shape = (E_, n + 3, nb, nb)
    theta = np.zeros(shape, dt_)
    phi = np.zeros(shape, dt_)
    psi = np.zeros(shape, dt_)
    P = np.zeros((E_, n + 1, nb, nb), dt_)
    theta[:, 1:n + 1] = -Kl[:, :n]
    phi[:, 1:n + 1] = -(Kd[:, :n] + a0 * Ml[:, :n])
    psi[:, 1:n + 1] = -Ku[:, :n]
    P[:, :n] = -Ml[:, :n]
    psi[:, n + 1] = eye
    P[:, n] = Ml[:, n]
    theta[:, n + 2] = Kl[:, n]
    phi[:, n + 2] = Kd[:, n] + a0 * Ml[:, n]
    psi[:, n + 2] = -eye
    theta[:, 0] = eye
    return theta, phi, psi, P


SCHEMES = {"paper_fd": block_rows, "radial_galerkin": galerkin_rows}


def row_columns(r: int, n: int):
    """Levels of the three unknowns that row r couples (eq. system)."""
    if r == -1:
        return (-1, 0, 1)
    if r == n + 1:
        return (n - 1, n, n + 1)
    return (r - 1, r, r + 1)


def element_system(theta, phi, psi):
    """Dense matrix of eq. system, [E, (n+3) n_b, (n+3) n_b]; block (r+1, l+1) for
    row r and unknown level l, both running over -1 .. n+1."""
    E_, m, n_b, _ = theta.shape
    n = m - 3
    A = np.zeros((E_, m * n_b, m * n_b), theta.dtype)
    for r in range(-1, n + 2):
        for blk, l in zip((theta, phi, psi), row_columns(r, n)):
            A[:, (r + 1) * n_b:(r + 2) * n_b, (l + 1) * n_b:(l + 2) * n_b] += blk[:, r + 1]
    return A


def condense(theta, phi, psi):
    """The paper's condensation sweep (block Gauss elimination of eq. system).

    rho_0 = theta_0 theta_-1^-1; phi~_0 = phi_0 - rho_0 phi_-1; psi~_0 = psi_0 - rho_0 psi_-1;
    rho_i = theta_i phi~_{i-1}^-1, phi~_i = phi_i - rho_i psi~_{i-1} (i = 1 .. n);
    rho_{n+1} = theta_{n+1} phi~_{n-1}^-1, phi~_{n+1} = phi_{n+1} - rho_{n+1} psi~_{n-1};
    G = psi_{n+1} psi_n^-1, S = phi~_{n+1} - G phi~_n.

    Only psi_0 is modified by the sweep (psi~_i = psi_i for i >= 1); psi_n is
    used unmodified in G.  Returns a dict with rho [E, n+2] (index i for
    rho_i, i = 0 .. n+1), phit [E, n+2] (phi~_i, i = 0 .. n+1), psit0, G, S.
    """
    m = theta.shape[1]
    n = m - 3
    R = lambda r: r + 1   # row r -> array index
    E_, _, n_b, _ = theta.shape
    rho = np.zeros((E_, n + 2, n_b, n_b), theta.dtype)
    phit = np.zeros((E_, n + 2, n_b, n_b), theta.dtype)
    rho[:, 0] = right_divide(theta[:, R(0)], theta[:, R(-1)])
    phit[:, 0] = phi[:, R(0)] - rho[:, 0] @ phi[:, R(-1)]
    psit0 = psi[:, R(0)] - rho[:, 0] @ psi[:, R(-1)]
    psit = lambda i: psit0 if i == 0 else psi[:, R(i)]
    for i in range(1, n + 1):
        rho[:, i] = right_divide(theta[:, R(i)], phit[:, i - 1])
        phit[:, i] = phi[:, R(i)] - rho[:, i] @ psit(i - 1)
    rho[:, n + 1] = right_divide(theta[:, R(n + 1)], phit[:, n - 1])
    phit[:, n + 1] = phi[:, R(n + 1)] - rho[:, n + 1] @ psit(n - 1)
    G = right_divide(psi[:, R(n + 1)], psi[:, R(n)])
    S = phit[:, n + 1] - G @ phit[:, n]
    return {"rho": rho, "phit": phit, "psit0": psit0, "G": G, "S": S}


class ElementGroup:
    """All oracle data of a group of elements with one (n_b, N_r)."""

    def __init__(self, elem_ids, loops, xy, rho, c, xi0, a0, centre=None, n_gauss=2, scheme="paper_fd"):
        self.elem_ids = np.asarray(elem_ids, dtype=np.int64)
        self.loops = np.asarray(loops, dtype=np.int64)          # [E, n_b]
        self.xy = xy
        self.centre = polygon_centroid(xy) if centre is None else centre
        self.n_r = rho.shape[1]
        self.n = self.n_r - 1
        self.n_b = rho.shape[2]
        self.xi, self.h = radial_levels(self.n_r, xi0)
        self.c, self.a0, self.scheme = c, a0, scheme
        self.E0, self.E1, self.E2, self.M0 = coefficient_matrices(xy, self.centre, rho, c, n_gauss)
        self.theta, self.phi, self.psi, self.P = SCHEMES[scheme](
            self.E0, self.E1, self.E2, self.M0, self.xi, self.h, a0)
        self.f = condense(self.theta, self.phi, self.psi)

    def psit(self, i):
        return self.f["psit0"] if i == 0 else self.psi[:, i + 1]


def group_elements(mesh):
    """Split a mesh into groups of equal (n_b, N_r); returns [(ids, n_b, n_r)]."""
    nb = mesh.n_b()
    keys = {}
    for e in range(mesh.n_elem):
        keys.setdefault((int(nb[e]), int(mesh.n_r[e])), []).append(e)
    return [(np.asarray(v, dtype=np.int64), k[0], k[1]) for k, v in sorted(keys.items())]


def build_groups(mesh, rho_flat, c, xi0, a0, n_gauss=2, scheme="paper_fd"):
    """ElementGroup per (n_b, N_r) from the fine-grid density (level-major per element)."""
    offs = mesh.param_offsets()
    groups = []
    for ids, n_b, n_r in group_elements(mesh):
        loops = np.stack([mesh.loop(e) for e in ids])
        xy = mesh.node_xy[loops]
        rho = np.stack([rho_flat[offs[e]:offs[e + 1]].reshape(n_r, n_b) for e in ids])
        groups.append(ElementGroup(ids, loops, xy, rho, c, xi0, a0, n_gauss=n_gauss, scheme=scheme))
    return groups
