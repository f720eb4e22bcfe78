"""Radial Galerkin reference for the dynamic stiffness of one element.

Used only as an independent check of the radial finite-difference scheme.
Starting from the semi-weak radial equation (the xi-integral that precedes
eq. ODE) and integrating by parts in xi with the internal flux
q = xi E0 u' + E1^T u (eq. internal), the bilinear form of the element is

    a(w, u) = int [ xi w'^T E0 u' + w'^T E1^T u + w^T E1 u' + w^T E2 u / xi
                    + a0 xi w^T M0 u ] dxi,

with the flux q(1) = f at the boundary and q(xi0) = 0 at the centre
(natural conditions).  With linear finite elements between the radial levels
and E(xi) interpolated linearly between them, condensing onto the boundary
level gives a stiffness that converges, as the levels refine, to the same
limit as the paper's finite-difference S.  The finite-difference terms
xi dE0/dxi and xi dE1^T/dxi of the strong form are exactly what this weak
form produces on integration by parts, so the two limits agree only if
those terms are right.
"""

from __future__ import annotations

import numpy as np


def galerkin_matrices(E0, E1, E2, M0, xi, n_quad=4, lumped=False):
    """Assembled stiffness K and mass M over all levels, dense [N_r n_b]^2, for
    level matrices E*[N_r, n_b, n_b]; ``lumped`` sums each mass row over the
    levels (one n_b x n_b block per level)."""
    n_r, nb = E0.shape[0], E0.shape[1]
    N = n_r * nb
    dt_ = np.result_type(E0, np.float64)
    K = np.zeros((N, N), dt_)
    M = np.zeros((N, N), dt_)
    gp, gw = np.polynomial.legendre.leggauss(n_quad)
    for j in range(n_r - 1):
        a, b = xi[j], xi[j + 1]
        for t, w in zip(gp, gw):
            x = (a + b) / 2 + (b - a) / 2 * t
            ww = w * (b - a) / 2
            Nf = np.array([(b - x) / (b - a), (x - a) / (b - a)])
            dN = np.array([-1.0 / (b - a), 1.0 / (b - a)])
            e0, e1, e2, m0 = [Nf[0] * E[j] + Nf[1] * E[j + 1] for E in (E0, E1, E2, M0)]
            for p in range(2):
                for q in range(2):
                    blk = ww * (x * dN[p] * dN[q] * e0 + dN[p] * Nf[q] * e1.T
                                + Nf[p] * dN[q] * e1 + Nf[p] * Nf[q] * e2 / x)
                    K[(j + p) * nb:(j + p + 1) * nb, (j + q) * nb:(j + q + 1) * nb] += blk
                    mq = j + p if lumped else j + q
                    M[(j + p) * nb:(j + p + 1) * nb, mq * nb:(mq + 1) * nb] += ww * x * Nf[p] * Nf[q] * m0
    return K, M


def galerkin_stiffness(E0, E1, E2, M0, xi, a0, n_quad=4, lumped=False):
    """Condensed boundary stiffness for level matrices E*[N_r, n_b, n_b] on levels xi."""
    n_r, nb = E0.shape[0], E0.shape[1]
    N = n_r * nb
    K, M = galerkin_matrices(E0, E1, E2, M0, xi, n_quad, lumped)
    K = K + a0 * M
    I = np.arange(0, (n_r - 1) * nb)
    B = np.arange((n_r - 1) * nb, N)
    return K[np.ix_(B, B)] - K[np.ix_(B, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, B)])
