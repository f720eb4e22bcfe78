"""Edge cases of the GPU path against the oracle.

- the largest radial level count the mesh accepts (N_r = 128: 127 intervals
  per element, eight chunks of the gradient contraction, the longest level
  loops of every sweep), forward traces and exact gradient with sqrt(T)
  checkpoints (segment recompute overlapped with the adjoint), driven by a
  pulse that peaks within the run;
- a run of a single time step (one checkpoint segment of one step);
- a run without receivers: no data, so the misfit and its gradient are
  exactly zero in every gradient mode, and the forward run records nothing.
Bars as in the parity tests: traces to relative L2 <= 1e-10, gradients to
relative L2 <= 1e-8.
"""

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import stepper as ostp

from ._gpu import GpuModel, log, rel_l2

pytestmark = pytest.mark.gpu


def _om(wl, rho):
    return ostp.Model(wl.mesh, rho, wl.c, wl.dt, wl.beta, wl.gamma, wl.xi0)


def test_max_radial_levels():
    steps = 40
    wl = W.config_small(nx=2, ny=1, segs=2, n_r=128, n_steps=steps, n_shots=2)
    assert int(wl.mesh.n_r.max()) == 128
    # a 2 MHz pulse that peaks inside the 40 steps (the workload's 500 kHz one would not)
    f0 = 2e6
    wl.wavelets = np.stack([W.ricker(steps, wl.dt, f0, t0=(1.2 + 0.1 * s) / f0) for s in range(2)])
    rho = wl.models["random30"]
    obs = ostp.forward(_om(wl, rho * 0.95), wl.src_nodes, wl.wavelets, wl.rec_nodes, steps)
    log(f"N_r = 128: {wl.mesh.n_elem} elements, n_b {int(wl.mesh.n_b().max())}, {steps} steps, 2 shots")
    g = GpuModel(wl, rho)
    tr, mis, grad, _ = g.gradient(obs, n_steps=steps, n_ckpt=-1)
    om = _om(wl, rho)
    tref = ostp.forward(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, steps)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets, wl.rec_nodes, obs, steps)
    et, eg = rel_l2(tr, tref), rel_l2(grad, gref)
    log(f"  traces relative L2 = {et:.3e}; misfit {mis:.6e} vs {Jref:.6e}; gradient relative L2 = {eg:.3e}")
    assert np.abs(tref).max() > 0 and np.abs(gref).max() > 0
    assert et <= 1e-10
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)
    assert eg <= 1e-8


def test_single_time_step():
    wl = W.config_tiny(n_steps=1)
    rho = wl.models["random30"]
    obs = np.zeros((wl.n_shots, len(wl.rec_nodes), 1))
    log("a single time step: traces, misfit and exact gradient")
    g = GpuModel(wl, rho)
    tr, mis, grad, _ = g.gradient(obs, n_steps=1, n_ckpt=-1)
    om = _om(wl, rho)
    tref = ostp.forward(om, wl.src_nodes, wl.wavelets[:, :1], wl.rec_nodes, 1)
    gref, Jref = oadj.exact_gradient(om, wl.src_nodes, wl.wavelets[:, :1], wl.rec_nodes, obs, 1)
    et, eg = rel_l2(tr, tref), rel_l2(grad, gref)
    log(f"  traces relative L2 = {et:.3e}; gradient relative L2 = {eg:.3e}")
    assert np.abs(tref).max() > 0 and Jref > 0
    assert et <= 1e-10
    assert mis == pytest.approx(Jref, rel=1e-10, abs=0)
    assert eg <= 1e-8


@pytest.mark.parametrize("mode", [0, 1, 16])   # exact, paper kernel, exact per shot
def test_no_receivers(mode):
    import torch
    wl = W.config_tiny(n_steps=12)
    wl.rec_nodes = np.zeros(0, dtype=np.int64)
    g = GpuModel(wl, wl.models["random30"])
    sb = g.sb
    S, N = wl.n_shots, 12
    src, wav, rec, tr = g.tensors(N)
    assert tr.numel() == 0
    ck = sb.sbfwi_forward(g.f, src, wav, rec, tr, n_ckpt=-1)
    per_shot = bool(mode & sb.GRAD_PER_SHOT)
    n = S if per_shot else 1
    mis = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    grad = torch.full((n * g.info["n_params"],), np.nan, dtype=torch.float64, device="cuda")
    sb.sbfwi_gradient(g.f, ck, torch.zeros_like(tr), tr, mode, mis, grad)
    torch.cuda.synchronize()
    log(f"no receivers, mode {mode}: misfit {mis.cpu().numpy()}, max |grad| {grad.abs().max().item()}")
    assert np.array_equal(mis.cpu().numpy(), np.zeros(n))
    assert np.array_equal(grad.cpu().numpy(), np.zeros(n * g.info["n_params"]))
    ck.close()
