"""Pins of the radial Galerkin scheme (``oracle.element.galerkin_rows``).

* the paper's condensation sweep applied to the Galerkin rows (in the block
  layout of the finite-difference rows, with identity rows on the unused
  levels) yields exactly the Schur complement of an independently assembled
  dense element matrix, at a0 = 0 and at a Newmark a0, and it is symmetric;
* energy: with the radial mass lumped, the coupled time loop conserves
  1/2 v^T M v + 1/2 u^T K u of the assembled Galerkin matrices to rounding
  once the source has stopped, also with a void at the 1e-5 density floor;
* stability: on a coarse radial grid where the finite-difference scheme's
  step map has eigenvalues outside the unit circle, every eigenvalue of the
  Galerkin step map has modulus 1 (to 1e-9), with and without the void;
* the exact adjoint gradient matches the complex-step derivative of the
  Galerkin forward map.
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj
from oracle import element as el
from oracle import radial_galerkin as rg
from oracle import stability as stab
from oracle import stepper as stp

RG = "radial_galerkin"


def _void_model(mesh, floor):
    pts = W.fine_point_positions(mesh)
    lx, ly = mesh.extent
    void = [(0.55 * lx, 0.45 * ly, 0.2 * lx, 0.15 * ly, 0.3)]
    return W.smoothed_voids(pts, void, 2700.0, floor, 0.05 * lx)


@pytest.mark.parametrize("a0", [0.0, 1.0 / (0.25 * 2e-8 ** 2)])
def test_condensed_stiffness_is_the_dense_schur_complement(a0):
    mesh = W.uniform_rect_mesh(0.005, 0.0025, 2, 1, segs=2, n_r=7)
    rho = W.smooth_random_field(W.fine_point_positions(mesh), 5, 2700.0, 0.3, wavelength=0.004)
    g = el.build_groups(mesh, rho, 3000.0, 1e-3, a0, scheme=RG)[0]
    for e in range(len(g.elem_ids)):
        ref = rg.galerkin_stiffness(g.E0[e], g.E1[e], g.E2[e], g.M0[e], g.xi, a0, lumped=True)
        S = g.f["S"][e]
        assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
        np.testing.assert_array_equal(g.f["G"][e], -np.eye(g.n_b))


def _energy(model, st):
    E = 0.0
    for g, gs in zip(model.groups, st["groups"]):
        for e in range(len(g.elem_ids)):
            K, M = rg.galerkin_matrices(g.E0[e], g.E1[e], g.E2[e], g.M0[e], g.xi, lumped=True)
            lp = g.loops[e]
            u = np.concatenate([gs["u"][e].ravel(), st["U"][lp]])
            v = np.concatenate([gs["v"][e].ravel(), st["V"][lp]])
            E += 0.5 * v @ M @ v + 0.5 * u @ K @ u
    return E


@pytest.mark.parametrize("floor", [1.0, 1e-5])
def test_energy_is_conserved_after_the_source(floor):
    mesh = W.uniform_rect_mesh(0.005, 0.005, 2, 2, segs=2, n_r=6)
    rho = _void_model(mesh, floor)
    dt = 5e-8
    m = stp.Model(mesh, rho, 3000.0, dt, scheme=RG)
    st = m.zero_state(np.float64)
    src = W.nearest_top_node(mesh, 0.002)
    wav = W.ricker(40, dt, 5e5, t0=1e-6)
    energies = []
    for k in range(1, 241):
        f = np.zeros(mesh.n_nodes)
        if k <= 40:
            f[src] = wav[k - 1]
        st = stp.step(m, st, f)
        if k > 40:
            energies.append(_energy(m, st))
    energies = np.asarray(energies)
    assert energies[0] > 0
    assert np.abs(energies - energies[0]).max() <= 1e-11 * energies[0]


@pytest.mark.parametrize("floor", [1.0, 1e-5])
def test_step_map_has_unit_modulus_where_finite_differences_grow(floor):
    mesh = W.uniform_rect_mesh(0.005, 0.005, 2, 2, segs=2, n_r=9)
    rho = _void_model(mesh, floor)
    mu_fd = stab.step_map_eigenvalues(stp.Model(mesh, rho, 3000.0, 2e-8))
    mu_rg = stab.step_map_eigenvalues(stp.Model(mesh, rho, 3000.0, 2e-8, scheme=RG))
    assert np.abs(mu_fd).max() > 1.0 + 1e-6
    assert np.abs(mu_rg).max() <= 1.0 + 1e-9


def test_exact_gradient_matches_complex_step():
    mesh = W.uniform_rect_mesh(0.005, 0.005, 2, 2, segs=2, n_r=6)
    rho = _void_model(mesh, 1e-5)
    dt, nt = 5e-8, 14
    src = np.array([W.nearest_top_node(mesh, 0.0025)])
    rec = W.top_edge_nodes(mesh)[::2]
    wav = W.ricker(nt, dt, 5e5, t0=2e-7)[None] * 1e6
    m = stp.Model(mesh, rho, 3000.0, dt, scheme=RG)
    tr = stp.forward(m, src, wav, rec, nt)
    obs = 0.8 * tr + 0.05 * np.abs(tr).max() * np.sin(np.arange(tr.size)).reshape(tr.shape)
    grad, J = adj.exact_gradient(m, src, wav, rec, obs, nt)
    assert J == pytest.approx(stp.misfit(tr, obs, dt), rel=1e-14)
    scale = np.abs(grad).max()
    for p in np.random.default_rng(3).choice(mesh.n_params, 8, replace=False):
        h = 1e-30 * rho[p]
        rc = rho.astype(complex)
        rc[p] += 1j * h
        mc = stp.Model(mesh, rc, 3000.0, dt, scheme=RG)
        cs = stp.misfit(stp.forward(mc, src, wav, rec, nt), obs, dt).imag / h
        assert abs(grad[p] - cs) <= 1e-9 * scale + 1e-9 * abs(cs)
