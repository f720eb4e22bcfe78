"""Differentiation through the autograd Function (backward = the library's adjoint run).

Checks: the backward equals the library gradient call and the oracle's exact
gradient; central finite differences (a seeded direction and single seeded
parameters, h = 1e-6 relative); the dot-product test <J dm, dd> = <dm, J^T dd>
with J dm from central differences of the traces; sqrt(T)-checkpointed versus
full-storage backward; and the L-BFGS outer loop on the density scaling field.
"""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as oadj
from oracle import stepper as ostp

from ._gpu import log, rel_l2

pytestmark = pytest.mark.gpu


def _problem(wl, n_steps, n_ckpt=-1, mode=0, coarse_solver=1):
    import paper_2501_06748_amd as sb
    from paper_2501_06748_amd.autograd import WaveProblem
    m = wl.mesh
    mesh = sb.sbfwi_build_mesh(m.node_xy, m.elem_ptr, m.elem_nodes, m.n_r, xi0=wl.xi0)
    dev = "cuda"
    return WaveProblem(mesh=mesh, c=wl.c, dt=wl.dt,
                       src=torch.tensor(wl.src_nodes, dtype=torch.int64, device=dev),
                       wavelet=torch.tensor(np.ascontiguousarray(wl.wavelets[:, :n_steps]), dtype=torch.float64,
                                            device=dev),
                       rec=torch.tensor(wl.rec_nodes, dtype=torch.int64, device=dev),
                       beta=wl.beta, gamma=wl.gamma, n_ckpt=n_ckpt, mode=mode, coarse_solver=coarse_solver)


def _objective(prob, observed):
    from paper_2501_06748_amd.autograd import misfit, simulate

    def J(rho):
        return misfit(simulate(rho, prob), observed, prob.dt)
    return J


def _value_and_grad(J, rho):
    r = rho.detach().clone().requires_grad_(True)
    val = J(r)
    val.backward()
    return float(val.item()), r.grad.detach().clone()


def _data(prob, rho_true):
    from paper_2501_06748_amd.autograd import simulate
    with torch.no_grad():
        return simulate(torch.tensor(rho_true, dtype=torch.float64, device="cuda"), prob)


@pytest.mark.parametrize("coarse_solver", [1, 0])
def test_backward_equals_library_gradient_and_oracle(coarse_solver):
    import paper_2501_06748_amd as sb
    wl = W.config_tiny(n_steps=48)
    prob = _problem(wl, 48, coarse_solver=coarse_solver)
    rho = torch.tensor(wl.models["random30"], dtype=torch.float64, device="cuda")
    obs = _data(prob, wl.models["void_floor_half"])
    log(f"autograd backward vs sbfwi_gradient vs oracle (tiny, 48 steps, coarse solver {coarse_solver})")
    J = _objective(prob, obs)
    val, g = _value_and_grad(J, rho)
    f = sb.sbfwi_factor_elements(prob.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, coarse_solver=coarse_solver)
    tr = torch.zeros(prob.trace_shape(), dtype=torch.float64, device="cuda")
    ck = sb.sbfwi_forward(f, prob.src, prob.wavelet, prob.rec, tr, n_ckpt=-1)
    mis = torch.zeros(1, dtype=torch.float64, device="cuda")
    g_lib = torch.zeros_like(rho)
    sb.sbfwi_gradient(f, ck, obs, tr, sb.GRAD_EXACT, mis, g_lib)
    torch.cuda.synchronize()
    assert val == pytest.approx(float(mis.item()), rel=1e-12, abs=0)
    assert rel_l2(g.cpu().numpy(), g_lib.cpu().numpy()) <= 1e-12
    om = ostp.Model(wl.mesh, wl.models["random30"], wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets[:, :48], wl.rec_nodes, obs.cpu().numpy(), 48)
    err = rel_l2(g.cpu().numpy(), gref)
    log(f"  misfit {val:.6e} vs oracle {Jref:.6e}; gradient relative L2 vs oracle {err:.3e}")
    assert val == pytest.approx(Jref, rel=1e-10, abs=0)
    assert err <= 1e-8


def test_finite_differences():
    wl = W.config_small(n_steps=40)
    prob = _problem(wl, 40)
    rho0 = torch.tensor(wl.models["random30"], dtype=torch.float64, device="cuda")
    obs = _data(prob, wl.models["homogeneous"])
    J = _objective(prob, obs)
    val, g = _value_and_grad(J, rho0)
    rng = np.random.default_rng(2 * 1000 + 11)
    # directional derivative along a seeded relative direction
    d = torch.tensor(rng.standard_normal(rho0.numel()), dtype=torch.float64, device="cuda") * rho0
    h = 1e-6
    with torch.no_grad():
        fd = (float(J(rho0 + h * d)) - float(J(rho0 - h * d))) / (2 * h)
    ad = float(torch.dot(g, d))
    log(f"directional FD {fd:.12e} vs adjoint {ad:.12e}: rel {abs(fd - ad) / abs(ad):.2e}")
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    # single seeded parameters with a gradient of at least 1 % of the largest
    gn = g.cpu().numpy()
    cand = np.flatnonzero(np.abs(gn) >= 1e-2 * np.abs(gn).max())
    picks = rng.choice(cand, size=min(16, cand.size), replace=False)
    worst = 0.0
    for p in picks:
        e = torch.zeros_like(rho0)
        hp = 1e-6 * float(rho0[p])
        e[p] = hp
        with torch.no_grad():
            fdp = (float(J(rho0 + e)) - float(J(rho0 - e))) / (2 * hp)
        worst = max(worst, abs(fdp - gn[p]) / abs(gn[p]))
    log(f"single-parameter FD on {len(picks)} parameters: worst relative error {worst:.2e}")
    assert worst <= 1e-5


def test_dot_product():
    from paper_2501_06748_amd.autograd import simulate
    wl = W.config_small(n_steps=40)
    prob = _problem(wl, 40)
    rho0 = torch.tensor(wl.models["random30"], dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(2 * 1000 + 12)
    dm = torch.tensor(rng.standard_normal(rho0.numel()), dtype=torch.float64, device="cuda") * rho0
    r = rho0.clone().requires_grad_(True)
    tr = simulate(r, prob)
    dd = torch.tensor(rng.standard_normal(tuple(tr.shape)), dtype=torch.float64, device="cuda") * tr.detach().abs().max()
    tr.backward(dd)
    rhs = float(torch.dot(dm, r.grad))
    h = 1e-5
    with torch.no_grad():
        jdm = (simulate(rho0 + h * dm, prob) - simulate(rho0 - h * dm, prob)) / (2 * h)
    lhs = float((jdm * dd).sum())
    log(f"dot product <J dm, dd> {lhs:.12e} vs <dm, J^T dd> {rhs:.12e}: rel {abs(lhs - rhs) / abs(rhs):.2e}")
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)


def test_checkpointed_backward_equals_full_storage():
    wl = W.config_small(n_steps=30)
    rho0 = torch.tensor(wl.models["random30"], dtype=torch.float64, device="cuda")
    grads = []
    for n_ckpt in (-1, 30):
        prob = _problem(wl, 30, n_ckpt=n_ckpt)
        obs = _data(prob, wl.models["homogeneous"])
        _, g = _value_and_grad(_objective(prob, obs), rho0)
        grads.append(g.cpu().numpy())
    log(f"sqrt(T) vs full storage: rel {rel_l2(grads[0], grads[1]):.2e}")
    assert rel_l2(grads[0], grads[1]) <= 1e-13


def test_lbfgs_on_scaling_field():
    from paper_2501_06748_amd import lbfgs
    wl = W.config_tiny(n_steps=200)
    prob = _problem(wl, 200)
    obs = _data(prob, wl.models["void_floor_half"])
    rho0 = float(wl.rho0)
    J = _objective(prob, obs)
    J0, _ = _value_and_grad(J, torch.full((wl.mesh.n_params,), rho0, dtype=torch.float64, device="cuda"))

    def fg(m):
        v, g = _value_and_grad(J, rho0 * m)
        return v / J0, g * (rho0 / J0)
    m0 = torch.ones(wl.mesh.n_params, dtype=torch.float64, device="cuda")
    res = lbfgs.minimize_box(fg, m0, 1e-6, 2.0, iters=10, memory=10, first_step=0.05)
    log(f"L-BFGS normalised misfit: {[round(h, 5) for h in res.history]} "
        f"({res.evaluations} evaluations, {res.rejected} rejected)")
    assert len(res.history) >= 6
    assert all(h1 <= h0 for h0, h1 in zip(res.history, res.history[1:]))
    assert res.history[-1] < 0.25 * res.history[0]
    assert float(res.x.min()) >= 1e-6 and float(res.x.max()) <= 2.0


def test_library_misfit_matches_the_oracle():
    """sbfwi_misfit (what autograd.misfit calls) against the oracle's misfit on seeded
    traces, and its residual against dt (u - d); the autograd Function's gradient with
    respect to the traces is that residual."""
    import torch
    import paper_2501_06748_amd as sb
    from paper_2501_06748_amd.autograd import misfit
    rng = np.random.default_rng(17)
    tr = rng.standard_normal((3, 7, 41))
    ob = rng.standard_normal((3, 7, 41))
    dt = 2e-8
    t = torch.tensor(tr, device="cuda", requires_grad=True)
    o = torch.tensor(ob, device="cuda")
    val = torch.zeros(1, dtype=torch.float64, device="cuda")
    res = torch.empty_like(o)
    sb.sbfwi_misfit(o, t.detach(), dt, val, residual=res)
    J = misfit(t, o, dt)
    J.backward()
    ref = ostp.misfit(tr, ob, dt)
    assert float(val.item()) == pytest.approx(ref, rel=1e-13)
    assert float(J.item()) == pytest.approx(ref, rel=1e-13)
    assert np.allclose(res.cpu().numpy(), dt * (tr - ob), rtol=1e-15, atol=0)
    assert np.allclose(t.grad.cpu().numpy(), dt * (tr - ob), rtol=1e-15, atol=0)
