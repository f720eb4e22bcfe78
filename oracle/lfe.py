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
