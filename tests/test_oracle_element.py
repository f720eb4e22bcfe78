"""Pins of the element-level oracle against facts fixed by the paper and by mathematics.

* coefficient-matrix invariants (eq. Es): a constant field has no
  circumferential gradient, so E2 1 = 0 and E1^T 1 = 0; E0, E2, M0 are
  symmetric and E0 is positive definite; 1^T M0 1 = sum over segments of
  rho * 2 * area(triangle) (the segment integral of rho det J_b); two-point
  and four-point Gauss rules agree (the integrands are cubic in eta);
* the condensation sweep equals the dense Schur complement of eq. system
  onto the boundary level (brute force);
* a constant field carries no flux in statics: S(a0 = 0) 1 = 0;
* radially constant density: S(a0 = 0) -> K and dS/da0 -> M of the
  conventional low-frequency expansion (Riccati + Lyapunov) at O(h^2);
* radially varying density: the finite-difference S and a radial-Galerkin
  discretisation of the same semi-weak form converge to one limit at O(h^2),
  which fails if the d/dxi terms of the radial equation are dropped.
"""

import numpy as np
import pytest

import workloads as W
from oracle import element as el
from oracle import lfe
from oracle.radial_galerkin import galerkin_stiffness


def _square(n_r, segs=2, side=0.0025):
    mesh = W.uniform_rect_mesh(side, side, 1, 1, segs=segs, n_r=n_r)
    xy = mesh.node_xy[mesh.loop(0)][None]
    return mesh, xy, el.polygon_centroid(xy)


def _skewed_polygon():
    """A star-convex pentagon-like loop with 7 nodes (not a square)."""
    ang = np.sort(np.random.default_rng(7).uniform(0, 2 * np.pi, 7))
    r = 0.002 * (1 + 0.3 * np.sin(3 * ang))
    return np.stack([0.01 + r * np.cos(ang), 0.02 + r * np.sin(ang)], -1)[None]


@pytest.mark.parametrize("shape", ["square", "polygon"])
def test_e_matrix_invariants(shape):
    if shape == "square":
        _, xy, ctr = _square(5, segs=3)
    else:
        xy = _skewed_polygon()
        ctr = el.polygon_centroid(xy)
    nb = xy.shape[1]
    rng = np.random.default_rng(3)
    rho = rng.uniform(1000, 4000, size=(1, 4, nb))
    E0, E1, E2, M0 = el.coefficient_matrices(xy, ctr, rho, 3000.0)
    one = np.ones(nb)
    for j in range(4):
        s = np.abs(E0[0, j]).max()
        assert np.abs(E2[0, j] @ one).max() <= 1e-13 * np.abs(E2[0, j]).max()
        assert np.abs(E1[0, j].T @ one).max() <= 1e-13 * np.abs(E1[0, j]).max()
        for M in (E0, E2, M0):
            assert np.abs(M[0, j] - M[0, j].T).max() <= 1e-15 * np.abs(M[0, j]).max()
        assert np.linalg.eigvalsh(E0[0, j]).min() > 1e-6 * s
        # 1^T M0 1 = sum_seg 2 * rho_mean_seg * area(centre, A, B)
        area = 0.0
        for k in range(nb):
            a, b = xy[0, k] - ctr[0], xy[0, (k + 1) % nb] - ctr[0]
            area += (rho[0, j, k] + rho[0, j, (k + 1) % nb]) / 2 * (a[0] * b[1] - a[1] * b[0]) / 2 * 2
        assert one @ M0[0, j] @ one == pytest.approx(area, rel=1e-14)
    E4 = el.coefficient_matrices(xy, ctr, rho, 3000.0, n_gauss=4)
    for A, B in zip((E0, E1, E2, M0), E4):
        assert np.abs(A - B).max() <= 1e-14 * np.abs(A).max()


def test_homogeneous_mass_equals_rho_area():
    # int xi dxi over (0, 1) times 1^T M0 1 is the element mass rho * area
    _, xy, ctr = _square(3)
    E0, E1, E2, M0 = el.coefficient_matrices(xy, ctr, np.full((1, 1, 8), 2700.0), 3000.0)
    assert 0.5 * M0[0, 0].sum() == pytest.approx(2700.0 * 0.0025 ** 2, rel=1e-14)


@pytest.mark.parametrize("a0", [0.0, 1.6e15])
def test_sweep_equals_dense_schur_complement(a0):
    _, xy, ctr = _square(9)
    rho = np.random.default_rng(11).uniform(1500, 3500, size=(1, 9, 8))
    E = el.coefficient_matrices(xy, ctr, rho, 3000.0)
    xi, h = el.radial_levels(9)
    th, ph, ps, P = el.block_rows(*E, xi, h, a0)
    f = el.condense(th, ph, ps)
    A = el.element_system(th, ph, ps)[0]
    n, nb = 8, 8
    bidx = np.arange((n + 1) * nb, (n + 2) * nb)
    iidx = np.setdiff1d(np.arange((n + 3) * nb), bidx)
    ridx = np.arange(0, (n + 2) * nb)
    fidx = np.arange((n + 2) * nb, (n + 3) * nb)
    S = A[np.ix_(fidx, bidx)] - A[np.ix_(fidx, iidx)] @ np.linalg.solve(A[np.ix_(ridx, iidx)], A[np.ix_(ridx, bidx)])
    tol = 1e-9 if a0 == 0.0 else 1e-13
    assert np.linalg.norm(f["S"][0] - S) <= tol * np.linalg.norm(S)


def test_static_constant_mode_has_no_flux():
    _, xy, ctr = _square(17)
    rho = np.random.default_rng(5).uniform(1500, 3500, size=(1, 17, 8))
    xi, h = el.radial_levels(17)
    th, ph, ps, P = el.block_rows(*el.coefficient_matrices(xy, ctr, rho, 3000.0), xi, h, 0.0)
    S = el.condense(th, ph, ps)["S"][0]
    assert np.abs(S @ np.ones(8)).max() <= 1e-10 * np.abs(S).max()


def _lfe_errors(n_r):
    _, xy, ctr = _square(n_r)
    rho = np.full((1, n_r, 8), 2700.0)
    rho[0, :, ::2] = 2000.0          # varies along eta only
    E = el.coefficient_matrices(xy, ctr, rho, 3000.0)
    xi, h = el.radial_levels(n_r)
    S0 = el.condense(*el.block_rows(*E, xi, h, 0.0)[:3])["S"][0]
    da = 1e6
    S1 = el.condense(*el.block_rows(*E, xi, h, da)[:3])["S"][0]
    K, _ = lfe.lfe_stiffness(E[0][0, 0], E[1][0, 0], E[2][0, 0])
    M = lfe.lfe_mass(K, E[0][0, 0], E[1][0, 0], E[3][0, 0])
    return (np.linalg.norm(S0 - K) / np.linalg.norm(K),
            np.linalg.norm((S1 - S0) / da - M) / np.linalg.norm(M))


def test_low_frequency_expansion_limit():
    errs = [_lfe_errors(n) for n in (9, 17, 33)]
    for (k1, m1), (k2, m2) in zip(errs[:-1], errs[1:]):
        assert 3.5 < k1 / k2 < 4.5          # O(h^2)
        assert 3.5 < m1 / m2 < 4.5
    assert errs[-1][0] < 2e-3 and errs[-1][1] < 2e-3


def test_lfe_solution_invariants():
    _, xy, ctr = _square(2)
    E = el.coefficient_matrices(xy, ctr, np.full((1, 1, 8), 2700.0), 3000.0)
    K, lam = lfe.lfe_stiffness(E[0][0, 0], E[1][0, 0], E[2][0, 0])
    M = lfe.lfe_mass(K, E[0][0, 0], E[1][0, 0], E[3][0, 0])
    one = np.ones(8)
    assert np.abs(K @ one).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-10 * np.abs(K).max()
    assert one @ M @ one == pytest.approx(2700.0 * 0.0025 ** 2, rel=1e-12)
    # linear fields are reproduced exactly: two modes with exponent 1
    np.testing.assert_allclose(lam[:2], [1.0, 1.0], rtol=1e-10)


def _fd_vs_galerkin(n_r, drop_radial_terms=False, monkeypatch=None):
    _, xy, ctr = _square(n_r)
    xi, h = el.radial_levels(n_r)
    prof = 2700.0 * (1 + 0.4 * np.sin(2.5 * xi))
    rho = np.repeat(prof[None, :, None], 8, axis=2)
    rho[0, :, 1::2] *= 0.8
    E = el.coefficient_matrices(xy, ctr, rho, 3000.0)
    a0 = 1e9
    S_fd = el.condense(*el.block_rows(*E, xi, h, a0)[:3])["S"][0]
    S_rg = galerkin_stiffness(E[0][0], E[1][0], E[2][0], E[3][0], xi, a0)
    return np.linalg.norm(S_fd - S_rg) / np.linalg.norm(S_rg)


def test_radial_terms_against_galerkin_limit():
    e = [_fd_vs_galerkin(n) for n in (17, 33, 65)]
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5
    assert e[2] < 5e-4


def test_planted_mistake_in_radial_terms_is_caught(monkeypatch):
    # dropping the d/dxi terms of E0, E1 (the variable-density terms of eq. ODE)
    monkeypatch.setattr(el, "radial_derivative", lambda Em, h: np.zeros_like(Em))
    e = [_fd_vs_galerkin(n) for n in (33, 65)]
    assert min(e) > 1e-2
