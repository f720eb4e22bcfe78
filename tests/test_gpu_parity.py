"""GPU path (HIP kernels through the C ABI) against the CPU oracle, element by element.

Bars (from the FP64 arithmetic of both sides): factor data and coarse matrix
to 1e-11 relative, wavefield traces to relative L2 <= 1e-10, gradients to
relative L2 <= 1e-8.  Inputs are the seeded synthetic workloads; the cases
span several element tiles, ragged (n_b, N_r) mixes, several shots and the
boundary / ghost levels.
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import element as oel
from oracle import stepper as ostp

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu


def _oracle_model(wl, rho, dt=None):
    return ostp.Model(wl.mesh, rho, wl.c, wl.dt if dt is None else dt, wl.beta, wl.gamma, wl.xi0)


def _per_element(mesh, groups, key):
    """Oracle per-element dense blocks in element order."""
    out = [None] * mesh.n_elem
    for g in groups:
        for i, e in enumerate(g.elem_ids):
            out[e] = key(g, i)
    return out


@pytest.mark.parametrize("cfg", ["tiny", "quadtree"])
def test_factor_parity(cfg):
    wl = W.config_tiny() if cfg == "tiny" else W.config_quadtree_tiny()
    rho = wl.models["random30"]
    log(f"factor parity {cfg}: {wl.mesh.n_elem} elements")
    g = GpuModel(wl, rho)
    om = _oracle_model(wl, rho)
    mesh = wl.mesh
    nb = mesh.n_b()
    S_gpu = g.sb.sbfwi_copy_factor_data(g.f, 0, int((nb.astype(np.int64) ** 2).sum()))
    G_gpu = g.sb.sbfwi_copy_factor_data(g.f, 3, int((nb.astype(np.int64) ** 2).sum()))
    nfinv = int(((mesh.n_r - 1).astype(np.int64) * nb.astype(np.int64) ** 2).sum())
    F_gpu = g.sb.sbfwi_copy_factor_data(g.f, 2, nfinv)
    S_or = _per_element(mesh, om.groups, lambda gr, i: gr.f["S"][i])
    G_or = _per_element(mesh, om.groups, lambda gr, i: gr.f["G"][i])
    F_or = _per_element(mesh, om.groups, lambda gr, i: np.linalg.inv(gr.f["phit"][i, :gr.n]))
    off = fo = 0
    worst = 0.0
    for e in range(mesh.n_elem):
        k = int(nb[e]) ** 2
        worst = max(worst, rel_l2(S_gpu[off:off + k], S_or[e].ravel()), rel_l2(G_gpu[off:off + k], G_or[e].ravel()))
        kf = (int(mesh.n_r[e]) - 1) * k
        worst = max(worst, rel_l2(F_gpu[fo:fo + kf], F_or[e].ravel()))
        off += k
        fo += kf
    log(f"  worst per-element relative L2 (S, G, phi~^-1): {worst:.3e}")
    assert worst <= 1e-11
    rp, col = g.sb.sbfwi_coarse_pattern(g.mesh)
    Kv = g.sb.sbfwi_copy_factor_data(g.f, 1, len(col))
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    K_or = np.asarray(om.K[rows, col]).ravel()
    assert rel_l2(Kv, K_or) <= 1e-11


@pytest.mark.parametrize("cfg,model,steps,solver", [("tiny", "homogeneous", 200, 1), ("tiny", "random30", 120, 1),
                                                    ("small", "random30", 60, 1), ("quadtree", "random30", 40, 1),
                                                    ("tiny", "random30", 120, 0), ("quadtree", "random30", 40, 0)])
def test_forward_parity(cfg, model, steps, solver):
    wl = {"tiny": W.config_tiny, "small": W.config_small, "quadtree": W.config_quadtree_tiny}[cfg]()
    rho = wl.models[model]
    log(f"forward parity {cfg}/{model}: {wl.mesh.n_elem} el, {wl.n_shots} shots, {steps} steps, "
        f"coarse solver {solver}")
    g = GpuModel(wl, rho, coarse_solver=solver)
    tr, _ = g.forward(n_steps=steps)
    tr = tr.cpu().numpy()
    om = _oracle_model(wl, rho)
    ref = ostp.forward(om, wl.src_nodes, wl.wavelets[:, :steps], wl.rec_nodes, steps)
    err = rel_l2(tr, ref)
    log(f"  traces relative L2 = {err:.3e}")
    assert np.isfinite(tr).all()
    assert err <= 1e-10


def test_shots_batched_equal_alone_and_rerun_bitwise():
    wl = W.config_small()
    rho = wl.models["random30"]
    log("batch invariance: 3 shots together vs alone")
    g = GpuModel(wl, rho)
    tr_all, _ = g.forward(n_steps=30)
    tr_all = tr_all.cpu().numpy()
    tr_again, _ = g.forward(n_steps=30)
    assert np.array_equal(tr_all, tr_again.cpu().numpy())
    for s in range(wl.n_shots):
        tr1, _ = g.forward(n_steps=30, shots=[s])
        assert rel_l2(tr1.cpu().numpy()[0], tr_all[s]) <= 1e-13


def _observed(wl, steps):
    om = _oracle_model(wl, wl.models["void_floor_half"] if "void_floor_half" in wl.models else wl.models["homogeneous"] * 0.9)
    return ostp.forward(om, wl.src_nodes, wl.wavelets[:, :steps], wl.rec_nodes, steps)


@pytest.mark.parametrize("ckpt,solver", [(-1, 1), (7, 1), (-1, 0)])
def test_exact_gradient_parity(ckpt, solver):
    wl = W.config_tiny(n_steps=48)
    steps = 48
    rho = wl.models["random30"]
    obs = _observed(wl, steps)
    log(f"exact gradient parity tiny, {steps} steps, n_ckpt={ckpt}, coarse solver {solver}")
    g = GpuModel(wl, rho, coarse_solver=solver)
    tr, mis, grad, _ = g.gradient(obs, n_steps=steps, n_ckpt=ckpt, mode=0)
    om = _oracle_model(wl, rho)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets[:, :steps], wl.rec_nodes, obs, steps)
    err = rel_l2(grad, gref)
    log(f"  misfit {mis:.6e} vs {Jref:.6e}; gradient relative L2 = {err:.3e}")
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)
    assert err <= 1e-8


def test_checkpointed_equals_full_storage():
    wl = W.config_tiny(n_steps=30)
    rho = wl.models["random30"]
    obs = _observed(wl, 30)
    g = GpuModel(wl, rho)
    log("sqrt(T) checkpoints vs full storage")
    _, _, g_ck, _ = g.gradient(obs, n_steps=30, n_ckpt=-1)
    _, _, g_full, _ = g.gradient(obs, n_steps=30, n_ckpt=30)
    assert rel_l2(g_ck, g_full) <= 1e-13


def test_paper_kernel_parity():
    wl = W.config_tiny(n_steps=48)
    rho = wl.models["random30"]
    obs = _observed(wl, 48)
    log("paper-kernel gradient parity tiny")
    g = GpuModel(wl, rho)
    _, _, grad, _ = g.gradient(obs, n_steps=48, n_ckpt=-1, mode=1)
    om = _oracle_model(wl, rho)
    gref, _ = oadj.paper_kernel_gradient(om, wl.src_nodes, wl.wavelets[:, :48], wl.rec_nodes, obs, 48)
    err = rel_l2(grad, gref)
    log(f"  paper kernel relative L2 = {err:.3e}")
    assert err <= 1e-8


def test_exact_gradient_ragged_multishot():
    wl = W.config_small(nx=4, ny=2, segs=2, n_r=7, n_steps=24, n_shots=2)
    rho = wl.models["random30"]
    om = _oracle_model(wl, rho)
    obs = ostp.forward(_oracle_model(wl, rho * 0.95), wl.src_nodes, wl.wavelets, wl.rec_nodes, 24)
    log("exact gradient parity, 2 shots")
    g = GpuModel(wl, rho)
    _, mis, grad, _ = g.gradient(obs, n_steps=24, n_ckpt=5)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, 24)
    err = rel_l2(grad, gref)
    log(f"  gradient relative L2 = {err:.3e}")
    assert err <= 1e-8


def test_full_size_sampled_parity():
    """The benchmark's plate at full size (128 x 64 elements, n_b 16, N_r 32,
    4 shots, the launch configuration bench.py times): factor data of 32
    seeded elements and the whole nodal wavefield of the first 3 steps.  The
    wavelets are seeded N(0, 1) samples so that the first steps carry signal."""
    steps = 3
    wl = W.config_paper(n_steps=steps, n_shots=4)
    rng = np.random.default_rng(1000 * 1 + 7)
    wl.wavelets = rng.standard_normal((wl.n_shots, steps))
    wl.rec_nodes = np.arange(wl.mesh.n_nodes, dtype=np.int64)
    rho = wl.models["random30"]
    log(f"full-size sampled parity: {wl.mesh.n_elem} el, {wl.mesh.n_nodes} nodes, {steps} steps")
    g = GpuModel(wl, rho)
    tr, _ = g.forward(n_steps=steps)
    tr = tr.cpu().numpy()
    om = _oracle_model(wl, rho)
    mesh = wl.mesh
    nb = mesh.n_b().astype(np.int64)
    S_gpu = g.sb.sbfwi_copy_factor_data(g.f, 0, int((nb ** 2).sum()))
    nfinv = int(((mesh.n_r - 1).astype(np.int64) * nb ** 2).sum())
    F_gpu = g.sb.sbfwi_copy_factor_data(g.f, 2, nfinv)
    S_or = _per_element(mesh, om.groups, lambda gr, i: gr.f["S"][i])
    F_or = _per_element(mesh, om.groups, lambda gr, i: np.linalg.inv(gr.f["phit"][i, :gr.n]))
    soff = np.concatenate([[0], np.cumsum(nb ** 2)])
    foff = np.concatenate([[0], np.cumsum((mesh.n_r - 1).astype(np.int64) * nb ** 2)])
    worst = 0.0
    for e in rng.choice(mesh.n_elem, size=32, replace=False):
        worst = max(worst, rel_l2(S_gpu[soff[e]:soff[e + 1]], S_or[e].ravel()),
                    rel_l2(F_gpu[foff[e]:foff[e + 1]], F_or[e].ravel()))
    log(f"  sampled elements: worst relative L2 (S, phi~^-1) = {worst:.3e}")
    assert worst <= 1e-11
    ref = ostp.forward(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, steps)
    err = rel_l2(tr, ref)
    log(f"  nodal wavefield relative L2 = {err:.3e}")
    assert np.isfinite(tr).all()
    assert err <= 1e-10
